"""Seeded synthetic workloads for the SC-LBM hot path.

This module is the only code shared by the CPU oracle side and the GPU side.
It produces *inputs* only: box sizes, boundary-face kinds, solid masks of
seeded building arrays, probe cell lists and the numeric constants of each
workload.  It performs none of the method's arithmetic (no lattice, no
collision, no quadrature, no inflow evaluation).

The paper's inputs (the Reutlingen building geometry and the measured hourly
wind series, Sec. 3 and the data-availability statement) are not available;
the seeded building arrays and the parametric log-law inflow of this module
stand in for them.  Geometry follows these rules:

* the building region is x in [nx/8, 3nx/4), y in [ny/8, 7ny/8), split into
  n_bx x n_by pitches;
* each pitch holds one square building of footprint
  F = min(16, floor(2 * min(pitch) / 3)), centred in the pitch, standing on
  the ground (z = 0);
* heights are integers drawn uniformly from {8, ..., min(40, nz - 8)} with a
  splitmix64 stream, one draw per building in row-major (y, then x) order.

Seeds are ``1000 * config_number + case_number``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

MASK64 = (1 << 64) - 1

# Face order used by every workload description: -x, +x, -y, +y, -z, +z.
FACE_NAMES = ("wall", "inlet", "outlet", "freeslip", "periodic")


class SplitMix64:
    """splitmix64 (Steele, Lea, Flood 2014): a counter-based 64-bit generator."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform_int(self, lo: int, hi: int) -> int:
        """Integer in [lo, hi] (inclusive)."""
        return lo + self.next() % (hi - lo + 1)

    def uniform01(self) -> float:
        return (self.next() >> 11) * (1.0 / (1 << 53))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One lattice case plus its collocation and QoI recipe (all plain data)."""

    name: str
    nx: int
    ny: int
    nz: int
    faces: Tuple[str, str, str, str, str, str]
    model: str                      # "bgk" or "smagorinsky"
    tau0: float                     # molecular relaxation time
    cs: float                       # Smagorinsky constant (0 for BGK)
    inflow: str                     # "uniform", "loglaw" or "series"
    # inflow parameter recipe: value = base * (1 + rel * xi_1); angle = deg * xi_2
    # (series: speed multiplier 1 + rel * xi_1 on the hourly speeds)
    speed_base: float               # U (uniform) or u* (log-law)
    speed_rel: float
    angle_deg: float                # direction spread in degrees (0: none)
    z0: float                       # log-law roughness length in cells
    quadrature: str                 # "gauss_legendre" or "smolyak_cc"
    quad_level: int                 # points (GL) or level (Smolyak)
    quad_dim: int
    steps: int
    avg_start: int                  # time average over steps n in (avg_start, steps]
    ramp: int                       # inflow ramp length T_r in steps (0: none)
    n_cases: int = 1
    seed_base: int = 0
    buildings: Optional[Tuple[int, int]] = None   # (n_bx, n_by) array, None: the single block
    probe_kind: Optional[str] = None              # "plane" or "points", see probe_cells
    ckpt_every: int = 0
    # hourly measured-series inflow ("series"): ((U_H, Theta[rad]), ...) per
    # hour, steps per hour, blending steps at each hour change, reference
    # height H of the normalised log profile (cells)
    series: Tuple[Tuple[float, float], ...] = ()
    hour_steps: int = 0
    blend_steps: int = 0
    ref_height: float = 0.0
    # cylindrical domain: radius of the vertical cylinder about the box centre
    # (cells); 0 for the plain box
    cylinder_radius: float = 0.0

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def seed(self, case: int = 0) -> int:
        return self.seed_base + case


def _int_div_centre(lo: int, hi: int, n: int, i: int) -> int:
    """Integer centre of the i-th of n equal pitches of [lo, hi)."""
    return lo + ((2 * i + 1) * (hi - lo)) // (2 * n)


def building_array_mask(nx: int, ny: int, nz: int, nbx: int, nby: int,
                        seed: int) -> np.ndarray:
    """Solid mask [nz, ny, nx] (uint8, 1 = solid) of a seeded building array."""
    x0, x1 = nx // 8, (3 * nx) // 4
    y0, y1 = ny // 8, (7 * ny) // 8
    pitch = min((x1 - x0) // nbx, (y1 - y0) // nby)
    F = min(16, (2 * pitch) // 3)
    hmax = min(40, nz - 8)
    rng = SplitMix64(seed)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    for by in range(nby):
        for bx in range(nbx):
            h = rng.uniform_int(8, hmax)
            cx = _int_div_centre(x0, x1, nbx, bx)
            cy = _int_div_centre(y0, y1, nby, by)
            xs, ys = cx - F // 2, cy - F // 2
            mask[0:h, ys:ys + F, xs:xs + F] = 1
    return mask


def small_block_mask(nx: int = 32, ny: int = 16, nz: int = 16) -> np.ndarray:
    """The single 6x6x8 block of the small case: x in [10,16), y in [5,11), z in [0,8)."""
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[0:8, 5:11, 10:16] = 1
    return mask


def cylinder_mask(nx: int, ny: int, nz: int, radius: float, nbx: int, nby: int,
                  seed: int) -> np.ndarray:
    """Mask [nz, ny, nx] of a cylindrical domain: 2 (mantle region) for every
    column whose centre (x + 1/2, y + 1/2) lies farther than `radius` from the
    box centre (nx/2, ny/2), 1 for a seeded n_bx x n_by block array in the
    central square of side `radius` (the building-array rule of this module
    on that square, footprint max(2, min(radius / 6, 2 pitch / 3)), heights
    up to nz / 2 below 16 layers), 0 fluid."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    r2 = (xx + 0.5 - nx / 2.0) ** 2 + (yy + 0.5 - ny / 2.0) ** 2
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[:, r2 > radius * radius] = 2
    if nbx * nby == 0:
        return mask
    half = int(radius) // 2
    x0, x1 = nx // 2 - half, nx // 2 + half
    y0, y1 = ny // 2 - half, ny // 2 + half
    pitch = min((x1 - x0) // nbx, (y1 - y0) // nby)
    F = max(2, min(int(radius) // 6, (2 * pitch) // 3))
    hmax = min(40, nz - 8) if nz >= 16 else nz // 2
    rng = SplitMix64(seed)
    for by in range(nby):
        for bx in range(nbx):
            h = rng.uniform_int(min(8, hmax), hmax)
            cx = _int_div_centre(x0, x1, nbx, bx)
            cy = _int_div_centre(y0, y1, nby, by)
            xs, ys = cx - F // 2, cy - F // 2
            mask[0:h, ys:ys + F, xs:xs + F] = 1
    return mask


def solid_mask(w: Workload, case: int = 0) -> np.ndarray:
    if w.cylinder_radius > 0:
        nbx, nby = w.buildings if w.buildings is not None else (0, 0)
        return cylinder_mask(w.nx, w.ny, w.nz, w.cylinder_radius, nbx, nby, w.seed(case))
    if w.buildings is None:
        return small_block_mask(w.nx, w.ny, w.nz)
    return building_array_mask(w.nx, w.ny, w.nz, w.buildings[0], w.buildings[1],
                               w.seed(case))


def probe_cells(w: Workload, mask: np.ndarray) -> np.ndarray:
    """Sorted linear cell indices (x fastest) of the probe set, int64, fluid cells only.

    * "plane": the y-z plane at x = 3nx/4, y in [ny/4, 3ny/4), z in [0, nz/3),
      i.e. 32 x 16 cells at the 128x64x48 size; solid cells are left out.
    * "points": an 8 x 8 grid at z = 10 over the building region; a probe that
      lands in a solid cell moves to the nearest fluid cell of that plane
      (smallest squared distance, ties broken by smaller y, then smaller x).
    * "lines": vertical profiles, the fluid cells of the four columns
      x in {3nx/8, 5nx/8}, y in {ny/4, 3ny/4}.
    """
    nx, ny, nz = w.nx, w.ny, w.nz
    if w.probe_kind is None:
        return np.zeros(0, dtype=np.int64)
    if w.probe_kind == "plane":
        xp = (3 * nx) // 4
        out = []
        for z in range(0, nz // 3):
            for y in range(ny // 4, (3 * ny) // 4):
                if not mask[z, y, xp]:
                    out.append((z * ny + y) * nx + xp)
        return np.asarray(out, dtype=np.int64)
    if w.probe_kind == "points":
        zp = 10
        x0, x1 = nx // 8, (3 * nx) // 4
        y0, y1 = ny // 8, (7 * ny) // 8
        plane = mask[zp]
        fy, fx = np.nonzero(plane == 0)
        out = []
        for j in range(8):
            for i in range(8):
                px = _int_div_centre(x0, x1, 8, i)
                py = _int_div_centre(y0, y1, 8, j)
                if not plane[py, px]:
                    out.append((zp * ny + py) * nx + px)
                    continue
                d2 = (fx - px) ** 2 + (fy - py) ** 2
                order = np.lexsort((fx, fy, d2))
                k = order[0]
                out.append((zp * ny + int(fy[k])) * nx + int(fx[k]))
        return np.sort(np.asarray(out, dtype=np.int64))
    if w.probe_kind == "lines":
        # vertical profiles (the paper's probe lines): four columns at
        # x in {3nx/8, 5nx/8}, y in {ny/4, 3ny/4}, every fluid cell of z
        out = []
        for px in ((3 * nx) // 8, (5 * nx) // 8):
            for py in (ny // 4, (3 * ny) // 4):
                for z in range(nz):
                    if not mask[z, py, px]:
                        out.append((z * ny + py) * nx + px)
        return np.sort(np.asarray(out, dtype=np.int64))
    raise ValueError(f"unknown probe kind {w.probe_kind!r}")


BOX_FACES = ("inlet", "outlet", "wall", "wall", "wall", "wall")
URBAN_FACES = ("inlet", "outlet", "periodic", "periodic", "wall", "freeslip")

# Molecular relaxation time of the LES cases (nu = 5e-4 in lattice units).  The
# workload descriptions leave it open; with Cs = 0.1 this value keeps the FP64
# reference finite through 2000 steps of the 256x128x64 urban case.
LES_TAU0 = 0.5015


def small_block() -> Workload:
    """Small plain SC-LBM case: BGK tau=0.6, 32x16x16 box, one block, 5 GL nodes."""
    return Workload(name="small_block_bgk_32x16x16", nx=32, ny=16, nz=16, faces=BOX_FACES,
                    model="bgk", tau0=0.6, cs=0.0, inflow="uniform",
                    speed_base=0.05, speed_rel=0.1, angle_deg=0.0, z0=0.0,
                    quadrature="gauss_legendre", quad_level=5, quad_dim=1,
                    steps=1000, avg_start=1000, ramp=0, seed_base=1000)


def urban_les(steps: int = 20000, avg_len: int = 5000) -> Workload:
    """Urban-like LES ensemble: Smagorinsky Cs=0.1, 256x128x64, 6x4 buildings, 13 Smolyak nodes."""
    return Workload(name="urban_les_256x128x64", nx=256, ny=128, nz=64, faces=URBAN_FACES,
                    model="smagorinsky", tau0=LES_TAU0, cs=0.1, inflow="loglaw",
                    speed_base=0.004, speed_rel=0.15, angle_deg=5.0, z0=0.5,
                    quadrature="smolyak_cc", quad_level=2, quad_dim=2,
                    steps=steps, avg_start=steps - avg_len, ramp=1000,
                    seed_base=2000, buildings=(6, 4))


UNEVEN_SIZES = ((128, 64, 32), (192, 96, 48), (256, 128, 64))


def uneven_cases(steps: int = 5000, per_size: int = 16) -> List[Workload]:
    """48 uneven cases (16 per size) of the batched run; each gets 13 Smolyak nodes."""
    out = []
    case = 0
    for (nx, ny, nz) in UNEVEN_SIZES:
        for _ in range(per_size):
            out.append(Workload(name=f"uneven_{nx}x{ny}x{nz}_{case}", nx=nx, ny=ny, nz=nz,
                                faces=URBAN_FACES, model="smagorinsky", tau0=LES_TAU0,
                                cs=0.1, inflow="loglaw", speed_base=0.004,
                                speed_rel=0.15, angle_deg=5.0, z0=0.5,
                                quadrature="smolyak_cc", quad_level=2, quad_dim=2,
                                steps=steps, avg_start=steps, ramp=1000,
                                seed_base=3000 + case, buildings=(6, 4)))
            case += 1
    return out


def adjoint_case(steps: int = 2000, avg_len: int = 500) -> Workload:
    """Adjoint case: BGK tau=0.6, 128x64x48, 4x3 buildings, probe-plane QoI, 13 nodes."""
    return Workload(name="adjoint_bgk_128x64x48", nx=128, ny=64, nz=48, faces=URBAN_FACES,
                    model="bgk", tau0=0.6, cs=0.0, inflow="loglaw",
                    speed_base=0.004, speed_rel=0.15, angle_deg=5.0, z0=0.5,
                    quadrature="smolyak_cc", quad_level=2, quad_dim=2,
                    steps=steps, avg_start=steps - avg_len, ramp=0,
                    seed_base=4000, buildings=(4, 3), probe_kind="plane",
                    ckpt_every=100)


def assimilation_case(steps: int = 2000, avg_len: int = 500) -> Workload:
    """Data-assimilation scale: Smagorinsky, 512x256x128, 10x6 buildings, 64 probes."""
    return Workload(name="assimilation_les_512x256x128", nx=512, ny=256, nz=128, faces=URBAN_FACES,
                    model="smagorinsky", tau0=LES_TAU0, cs=0.1, inflow="loglaw",
                    speed_base=0.004, speed_rel=0.15, angle_deg=5.0, z0=0.5,
                    quadrature="smolyak_cc", quad_level=2, quad_dim=2,
                    steps=steps, avg_start=steps - avg_len, ramp=1000,
                    seed_base=5000, buildings=(10, 6), probe_kind="points",
                    ckpt_every=100)


def hourly_series(hours: int, seed: int, speed_mean: float = 0.016, speed_amp: float = 0.006,
                  dir0_deg: float = 0.0, dir_step_deg: float = 12.0) -> Tuple[Tuple[float, float], ...]:
    """Synthetic hourly reference wind (lattice speed, direction in rad) in
    place of the station record: speeds from a smoothed seeded sequence around
    speed_mean, directions a seeded random walk from dir0_deg."""
    g = SplitMix64(seed)
    out = []
    s = 0.0
    d = math.radians(dir0_deg)
    for _ in range(hours):
        s = 0.7 * s + 0.3 * (2.0 * g.uniform01() - 1.0)
        d += math.radians(dir_step_deg) * (2.0 * g.uniform01() - 1.0)
        out.append((speed_mean + speed_amp * s, d))   # |s| <= 1
    return tuple(out)


def urban_series(hours: int = 8, hour_steps: int = 500, blend_steps: int = 100) -> Workload:
    """Urban LES driven by an hourly wind series (the paper's time-dependent
    inflow): speed multiplier 1 + 0.1 xi_1 and direction offset 6 deg xi_2 on
    the series, normalised log profile with z0 = 0.1 cells and H = nz."""
    nz = 64
    return Workload(name="urban_series_256x128x64", nx=256, ny=128, nz=nz, faces=URBAN_FACES,
                    model="smagorinsky", tau0=LES_TAU0, cs=0.1, inflow="series",
                    speed_base=1.0, speed_rel=0.1, angle_deg=6.0, z0=0.1,
                    quadrature="smolyak_cc", quad_level=2, quad_dim=2,
                    steps=1000 + hours * hour_steps, avg_start=1000 + hours * hour_steps, ramp=1000,
                    seed_base=6000, buildings=(6, 4),
                    series=hourly_series(hours, 6000), hour_steps=hour_steps, blend_steps=blend_steps,
                    ref_height=float(nz))


def urban_gpc(hours: int = 8, hour_steps: int = 500, blend_steps: int = 100) -> Workload:
    """The paper's stochastic set-up on the urban box: zeta_1 ~ N(1, 0.1^2) on
    the hourly speeds and zeta_2 ~ N(0, (6 deg)^2) on the directions, dense
    11 x 11 Gauss-Hermite rule (121 nodes), normalised log profile with
    z0 = 0.1 cells and H = nz, time-averaged u_x on vertical probe lines for
    the gPC expansion (order 5)."""
    w = urban_series(hours, hour_steps, blend_steps)
    steps = w.steps
    return dataclasses.replace(w, name="urban_gpc_256x128x64", quadrature="gauss_hermite", quad_level=11,
                               quad_dim=2, avg_start=steps - hours * hour_steps // 2, probe_kind="lines",
                               seed_base=7000, series=hourly_series(hours, 7000))


CYLINDER_FACES = ("wall", "wall", "wall", "wall", "wall", "freeslip")


def cylinder_gpc(radius: int = 270, height: int = 40, hours: int = 8, hour_steps: int = 500,
                 blend_steps: int = 100) -> Workload:
    """The paper's domain class: a vertical cylinder of radius 270 and height
    40 cells (1 m cells) whose mantle carries the wind, bounce-back ground, a
    free-slip sky, two seeded blocks in the centre in place of the real
    buildings; Smagorinsky LES driven by an hourly series with the reference
    speed at Ma = 0.0346 (0.02 in lattice units), zeta_1 ~ N(1, 0.1^2) on the
    speeds and zeta_2 ~ N(0, (6 deg)^2) on the directions, 11 x 11
    Gauss-Hermite nodes, normalised log profile with z0 = 0.1 cells and
    H = height.  The box is 2 radius + 4 cells wide so that a ring of mantle
    cells surrounds the disk everywhere."""
    n = 2 * radius + 4
    steps = 1000 + hours * hour_steps
    return Workload(name=f"cylinder_gpc_r{radius}_h{height}", nx=n, ny=n, nz=height,
                    faces=CYLINDER_FACES, model="smagorinsky", tau0=LES_TAU0, cs=0.1,
                    inflow="series", speed_base=1.0, speed_rel=0.1, angle_deg=6.0, z0=0.1,
                    quadrature="gauss_hermite", quad_level=11, quad_dim=2,
                    steps=steps, avg_start=steps - hours * hour_steps // 2, ramp=1000,
                    seed_base=8000, buildings=(2, 1), probe_kind="lines",
                    series=hourly_series(hours, 8000, speed_mean=0.02, speed_amp=0.006,
                                         dir0_deg=225.0, dir_step_deg=20.0),
                    hour_steps=hour_steps, blend_steps=blend_steps, ref_height=float(height),
                    cylinder_radius=float(radius))


def scaled(w: Workload, nx: int, ny: int, nz: int, **kw) -> Workload:
    """The same recipe on another box size (used for small parity cases)."""
    return dataclasses.replace(w, nx=nx, ny=ny, nz=nz, name=f"{w.name}_{nx}x{ny}x{nz}", **kw)


def random_populations(shape, seed: int, scale: float = 1e-3) -> np.ndarray:
    """Seeded small perturbation field (float64) for invariance tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal(shape)


def da_truth() -> Tuple[float, float]:
    """Hidden truth (mean multiplier, spread) of the data-assimilation workload."""
    return 1.08, 0.22


def da_start() -> Tuple[float, float]:
    """First guess (mean multiplier, spread) of the data-assimilation workload."""
    return 1.0, 0.15


def da_noise(n: int, seed: int = 5099) -> np.ndarray:
    """Standard-normal draws for the 5 % multiplicative observation noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n)


def mask_hash(mask: np.ndarray) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(mask, dtype=np.uint8).tobytes()).hexdigest()
