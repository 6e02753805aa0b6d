"""Python side of the FP64 CPU oracle of the SC-LBM hot path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the GPU library (it links only ``liblbm_oracle.so``,
built from ``lbm_oracle.c`` in this folder).

Contents, each following arXiv 2508.18202:

* ``gauss_legendre``  -- n-point Gauss-Legendre rule for a uniform variable on
  [-1, 1] (probability weights), by Newton iteration on the Legendre
  three-term recurrence; the tensor/ sparse collocation grids of Sec. 2.3
  (Eq. coef_discrete uses nodes Z^(j) and weights a_j).
* ``clenshaw_curtis`` / ``smolyak_cc`` -- nested Clenshaw-Curtis rules and
  their Smolyak combination (sparse-grid collocation, Sec. 2.3/2.4 step 3).
* ``node_params``     -- collocation node -> inflow parameters (Sec. 3: the
  measured speed times a relative perturbation, the direction plus an
  additive perturbation; here with uniform xi on [-1, 1]).
* ``moments``         -- Eq. (quad_moments): E = sum a_j Q_j,
  Var = sum a_j (Q_j - E)^2, two passes in float64.
* ``gauss_hermite`` / ``tensor_gauss_hermite`` -- the probabilists' Gauss-
  Hermite rule (numpy's hermegauss, weights normalised to probabilities) and
  its tensor product, for the Gaussian germ of Sec. 3 (11 x 11 = 121 nodes).
* ``gpc_multi_indices`` / ``hermite_he`` / ``gpc_basis`` / ``gpc`` -- the
  orthonormal Hermite chaos of total degree <= order and the projection of
  Sec. 2.3 (coefficients by quadrature, mean, variance, 95 % band).
* ``equilibrium`` / ``equilibrium3`` / ``rr3_basis`` / ``tau_eff`` -- the
  second- and third-order equilibria, the Hermite basis orthogonal on D3Q19
  and the Smagorinsky relaxation time of Sec. 2.2 (from the C oracle).
* ``Case`` / ``run`` / ``adjoint`` -- drive the C oracle: time stepping with
  QoI capture (final fields, time averages, probe means; Sec. 2.4 step 6),
  the hourly-series inflow of Sec. 3, the cylindrical domain, and the
  discrete adjoint with checkpointed recomputation.

Every function is pinned by tests/test_oracle_*.py to closed forms,
invariants or brute force; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

NQ = 19
FACE_CODES = {"wall": 0, "inlet": 1, "outlet": 2, "freeslip": 3, "periodic": 4}
MODEL_CODES = {"bgk": 0, "smagorinsky": 1, "rr3": 2}
INFLOW_CODES = {"uniform": 0, "loglaw": 1, "series": 2}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP over cells)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Case(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("face", ctypes.c_int * 6), ("solid", ctypes.POINTER(ctypes.c_uint8)),
                ("model", ctypes.c_int), ("tau0", ctypes.c_double), ("cs", ctypes.c_double),
                ("inflow", ctypes.c_int), ("theta", ctypes.c_double * 3),
                ("ramp", ctypes.c_int), ("force", ctypes.c_double * 3),
                ("series", ctypes.POINTER(ctypes.c_double)), ("series_len", ctypes.c_int),
                ("hour_steps", ctypes.c_int), ("blend_steps", ctypes.c_int), ("ref_height", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        L.orc_lattice.argtypes = [P(ctypes.c_int), dp, P(ctypes.c_int)]
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_equilibrium3.argtypes = [ctypes.c_double, dp, dp]
        L.orc_rr3_basis.argtypes = [dp, dp]
        L.orc_tau_eff.argtypes = [ctypes.c_double] * 4
        L.orc_tau_eff.restype = ctypes.c_double
        L.orc_check_case.argtypes = [P(_Case)]
        L.orc_init.argtypes = [P(_Case), dp]
        L.orc_macros.argtypes = [P(_Case), dp, dp, dp]
        L.orc_collide_cell.argtypes = [P(_Case), dp, dp]
        L.orc_step.argtypes = [P(_Case), ctypes.c_long, dp, dp]
        L.orc_link_rules.argtypes = [P(_Case), P(ctypes.c_int)]
        L.orc_collision_jacobian.argtypes = [P(_Case), dp, dp]
        L.orc_adjoint_step.argtypes = [P(_Case), ctypes.c_long, dp, dp, dp, dp]
        L.orc_inflow_velocity.argtypes = [P(_Case), ctypes.c_int, ctypes.c_long, dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's loops over cells (n <= 0: leave as is); returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------- lattice

def lattice():
    """(c [19,3] int, w [19], opp [19]) as the oracle defines them."""
    c = (ctypes.c_int * (3 * NQ))()
    w = np.zeros(NQ)
    o = (ctypes.c_int * NQ)()
    lib().orc_lattice(c, _dp(w), o)
    return np.array(list(c)).reshape(NQ, 3), w, np.array(list(o))


def equilibrium(rho: float, u: Sequence[float]) -> np.ndarray:
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(NQ)
    lib().orc_equilibrium(rho, _dp(uu), _dp(out))
    return out


def equilibrium3(rho: float, u: Sequence[float]) -> np.ndarray:
    """Third-order equilibrium in the Hermite polynomials orthogonal on D3Q19
    (Sec. 2.2, the equilibrium expanded to order three)."""
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(NQ)
    lib().orc_equilibrium3(rho, _dp(uu), _dp(out))
    return out


def rr3_basis():
    """(P [16, 19], N [16]): the D3Q19-orthogonal Hermite polynomials up to
    third order at the velocities, and their norms sum_i w_i P_k(c_i)^2."""
    P = np.zeros(16 * NQ)
    N = np.zeros(16)
    lib().orc_rr3_basis(_dp(P), _dp(N))
    return P.reshape(16, NQ), N


def tau_eff(tau0: float, cs: float, rho: float, q: float) -> float:
    return lib().orc_tau_eff(tau0, cs, rho, q)


# --------------------------------------------------------------------------- quadrature

def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes and probability weights for xi ~ U(-1, 1).

    Nodes are the roots of P_n, found by Newton iteration on the recurrence
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; weights 2 / ((1-x^2) P_n'(x)^2),
    halved to integrate against the density 1/2.
    """
    x = np.cos(np.pi * (np.arange(1, n + 1) - 0.25) / (n + 0.5))
    for _ in range(100):
        p0, p1 = np.ones_like(x), x.copy()
        for k in range(1, n):
            p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
        dp = n * (x * p1 - p0) / (x * x - 1.0)
        dx = p1 / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p0, p1 = np.ones_like(x), x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], 0.5 * w[order]


def clenshaw_curtis(m: int):
    """m-point Clenshaw-Curtis rule on [-1, 1] with probability weights.

    Nodes cos(j pi / (m-1)); weights by the explicit cosine-sum formula
    w_j = c_j/(m-1) [1 - sum_{k=1}^{(m-1)/2} b_k cos(2 k j pi/(m-1)) / (4k^2-1)],
    c_0 = c_{m-1} = 1, c_j = 2 otherwise, b_k = 1 at k = (m-1)/2, else 2.
    """
    if m == 1:
        return np.zeros(1), np.ones(1)
    n = m - 1
    th = np.pi * np.arange(m) / n
    w = np.zeros(m)
    for j in range(m):
        s = 0.0
        for k in range(1, n // 2 + 1):
            b = 1.0 if 2 * k == n else 2.0
            s += b * math.cos(2 * k * th[j]) / (4 * k * k - 1)
        c = 1.0 if j in (0, n) else 2.0
        w[j] = c / n * (1.0 - s)
    return np.cos(th), 0.5 * w


def smolyak_cc(level: int, dim: int):
    """Smolyak sparse grid of nested CC rules (m(0)=1, m(l)=2^l+1).

    A(L, d) = sum over multi-indices l >= 0 with L-d+1 <= |l| <= L of
    (-1)^(L-|l|) binom(d-1, L-|l|) Q_{l_1} x ... x Q_{l_d}; coincident nodes
    are merged by summing their weights.
    """
    def m_of(l):
        return 1 if l == 0 else 2 ** l + 1

    acc: Dict[tuple, float] = {}
    pts: Dict[tuple, np.ndarray] = {}
    for l in itertools.product(range(level + 1), repeat=dim):
        s = sum(l)
        if s < level - dim + 1 or s > level:
            continue
        coef = (-1) ** (level - s) * math.comb(dim - 1, level - s)
        rules = [clenshaw_curtis(m_of(li)) for li in l]
        for combo in itertools.product(*[range(len(r[0])) for r in rules]):
            x = np.array([rules[k][0][combo[k]] for k in range(dim)])
            w = coef * np.prod([rules[k][1][combo[k]] for k in range(dim)])
            key = tuple(np.round(x, 12) + 0.0)
            acc[key] = acc.get(key, 0.0) + w
            pts[key] = x
    keys = sorted(acc)
    return np.array([pts[k] for k in keys]), np.array([acc[k] for k in keys])


def gauss_hermite(n: int):
    """n-point Gauss-Hermite rule for z ~ N(0, 1) (probabilists' polynomials):
    numpy's hermegauss nodes, weights divided by their sum sqrt(2 pi)."""
    x, w = np.polynomial.hermite_e.hermegauss(n)
    return x, w / w.sum()


def tensor_gauss_hermite(n: int, dim: int):
    """Dense tensor product of the n-point rule (Sec. 3): node (i_1 .. i_d)
    in lexicographic order (last coordinate fastest), weight the product."""
    x, w = gauss_hermite(n)
    idx = list(itertools.product(range(n), repeat=dim))
    nodes = np.array([[x[i] for i in t] for t in idx])
    weights = np.array([np.prod([w[i] for i in t]) for t in idx])
    return nodes, weights


def collocation(w) -> tuple:
    """(nodes [N_q, d], weights [N_q]) of a workload's collocation rule."""
    if w.quadrature == "gauss_legendre":
        x, a = gauss_legendre(w.quad_level)
        return x.reshape(-1, 1), a
    if w.quadrature == "smolyak_cc":
        return smolyak_cc(w.quad_level, w.quad_dim)
    if w.quadrature == "gauss_hermite":
        return tensor_gauss_hermite(w.quad_level, w.quad_dim)
    raise ValueError(w.quadrature)


# --------------------------------------------------------------------------- gPC

def gpc_multi_indices(dim: int, order: int) -> np.ndarray:
    """Multi-indices of total degree <= order, graded (degree 0, 1, ...),
    within a degree the first variable's power descending."""
    out = []
    for deg in range(order + 1):
        def rec(prefix, left, k):
            if k == dim - 1:
                out.append(prefix + [left])
                return
            for a in range(left, -1, -1):
                rec(prefix + [a], left - a, k + 1)
        rec([], deg, 0)
    return np.array(out, dtype=np.int64).reshape(-1, dim)


def hermite_he(n: int, z: np.ndarray) -> np.ndarray:
    """Probabilists' Hermite polynomial He_n(z) by He_{k+1} = z He_k - k He_{k-1}."""
    z = np.asarray(z, dtype=np.float64)
    h0, h1 = np.ones_like(z), z.copy()
    if n == 0:
        return h0
    for k in range(1, n):
        h0, h1 = h1, z * h1 - k * h0
    return h1


def gpc_basis(nodes: np.ndarray, order: int):
    """Phi [N_q, P] of the orthonormal Hermite chaos prod_k He_{a_k}(z_k)/sqrt(a_k!)
    at the nodes, and the multi-indices [P, d]."""
    nodes = np.asarray(nodes, dtype=np.float64)
    alpha = gpc_multi_indices(nodes.shape[1], order)
    phi = np.ones((nodes.shape[0], alpha.shape[0]))
    for p, a in enumerate(alpha):
        for k, ak in enumerate(a):
            phi[:, p] *= hermite_he(int(ak), nodes[:, k]) / math.sqrt(math.factorial(int(ak)))
    return phi, alpha


def gpc(q: np.ndarray, nodes: np.ndarray, weights: np.ndarray, order: int) -> dict:
    """gPC coefficients by projection with the collocation rule (Sec. 2.3):
    c_alpha = sum_j a_j Q_j Phi_alpha(Z^(j)); mean c_0, variance
    sum_{alpha != 0} c_alpha^2, 95 % band mean -+ 1.96 std (float64)."""
    q = np.asarray(q, dtype=np.float64)
    phi, alpha = gpc_basis(nodes, order)
    coef = np.zeros((phi.shape[1],) + q.shape[1:])
    for j in range(q.shape[0]):
        for p in range(phi.shape[1]):
            coef[p] += weights[j] * phi[j, p] * q[j]
    var = (coef[1:] ** 2).sum(0)
    sd = np.sqrt(var)
    return {"coef": coef, "alpha": alpha, "mean": coef[0], "var": var,
            "band": np.stack([coef[0] - 1.96 * sd, coef[0] + 1.96 * sd])}


def node_params(w, xi: Sequence[float]) -> np.ndarray:
    """Inflow parameters theta of one node: (speed, direction [rad], z0).

    speed = base * (1 + rel * xi_1) (relative perturbation of the measured
    speed, Sec. 3); direction = angle_deg * xi_2 in radians (additive
    perturbation of the measured direction)."""
    speed = w.speed_base * (1.0 + w.speed_rel * xi[0])
    phi = math.radians(w.angle_deg * xi[1]) if len(xi) > 1 else 0.0
    return np.array([speed, phi, w.z0])


def moments(q: np.ndarray, a: np.ndarray):
    """Eq. (quad_moments): E = sum_j a_j Q_j, Var = sum_j a_j (Q_j - E)^2 (float64)."""
    q = np.asarray(q, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    e = np.zeros(q.shape[1:])
    for j in range(q.shape[0]):
        e += a[j] * q[j]
    v = np.zeros(q.shape[1:])
    for j in range(q.shape[0]):
        v += a[j] * (q[j] - e) ** 2
    return e, v


# --------------------------------------------------------------------------- lattice runs

class Case:
    """One deterministic lattice case at one collocation node."""

    def __init__(self, nx, ny, nz, faces, solid, model="bgk", tau0=0.6, cs=0.0,
                 inflow="uniform", theta=(0.0, 0.0, 0.0), ramp=0, force=(0.0, 0.0, 0.0),
                 series=(), hour_steps=0, blend_steps=0, ref_height=0.0):
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(nz, ny, nx)
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        c = _Case()
        c.nx, c.ny, c.nz = nx, ny, nz
        for k, f in enumerate(faces):
            c.face[k] = FACE_CODES[f] if isinstance(f, str) else int(f)
        c.solid = self.solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        c.model = MODEL_CODES[model] if isinstance(model, str) else int(model)
        c.tau0, c.cs = tau0, cs
        c.inflow = INFLOW_CODES[inflow] if isinstance(inflow, str) else int(inflow)
        for k in range(3):
            c.theta[k] = float(theta[k])
            c.force[k] = float(force[k])
        c.ramp = ramp
        # hourly series inflow: [hours][2] (U_H, Theta in rad)
        self.series = np.ascontiguousarray(np.asarray(series, dtype=np.float64).reshape(-1, 2))
        if len(self.series):
            c.series = self.series.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        c.series_len, c.hour_steps, c.blend_steps = len(self.series), int(hour_steps), int(blend_steps)
        c.ref_height = float(ref_height)
        self.c = c
        err = lib().orc_check_case(ctypes.byref(c))
        if err:
            raise ValueError(f"oracle rejects the case (code {err})")

    @classmethod
    def from_workload(cls, w, solid, theta):
        return cls(w.nx, w.ny, w.nz, w.faces, solid, w.model, w.tau0, w.cs, w.inflow,
                   theta, w.ramp, series=w.series, hour_steps=w.hour_steps, blend_steps=w.blend_steps,
                   ref_height=w.ref_height)

    def with_theta(self, theta):
        nz, ny, nx = self.shape
        c = self.c
        return Case(nx, ny, nz, list(c.face), self.solid, c.model, c.tau0, c.cs, c.inflow,
                    theta, c.ramp, list(c.force), self.series, c.hour_steps, c.blend_steps, c.ref_height)

    def init(self) -> np.ndarray:
        f = np.zeros((NQ, self.n))
        lib().orc_init(ctypes.byref(self.c), _dp(f))
        return f

    def step(self, n: int, f: np.ndarray) -> np.ndarray:
        out = np.empty_like(f)
        lib().orc_step(ctypes.byref(self.c), n, _dp(f), _dp(out))
        return out

    def macros(self, f: np.ndarray):
        rho = np.zeros(self.n)
        u = np.zeros((3, self.n))
        lib().orc_macros(ctypes.byref(self.c), _dp(f), _dp(rho), _dp(u))
        return rho, u

    def link_rules(self) -> np.ndarray:
        r = np.zeros((NQ, self.n), dtype=np.int32)
        lib().orc_link_rules(ctypes.byref(self.c), r.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return r

    def collide_cell(self, f19) -> np.ndarray:
        f = np.ascontiguousarray(f19, dtype=np.float64)
        out = np.zeros(NQ)
        lib().orc_collide_cell(ctypes.byref(self.c), _dp(f), _dp(out))
        return out

    def collision_jacobian(self, f19) -> np.ndarray:
        f = np.ascontiguousarray(f19, dtype=np.float64)
        J = np.zeros(NQ * NQ)
        lib().orc_collision_jacobian(ctypes.byref(self.c), _dp(f), _dp(J))
        return J.reshape(NQ, NQ)

    def adjoint_step(self, n: int, f_n, lam_next):
        lam = np.empty_like(lam_next)
        g = np.zeros(3)
        lib().orc_adjoint_step(ctypes.byref(self.c), n, _dp(f_n), _dp(lam_next), _dp(lam), _dp(g))
        return lam, g

    def inflow_velocity(self, z: int, n: int) -> np.ndarray:
        u = np.zeros(3)
        lib().orc_inflow_velocity(ctypes.byref(self.c), z, n, _dp(u))
        return u


def qoi_fields(case: Case, f: np.ndarray) -> np.ndarray:
    """[4, cells]: u_x, u_y, u_z, |u| of a state (solid cells: 0)."""
    _, u = case.macros(f)
    return np.concatenate([u, np.sqrt((u * u).sum(0))[None]], axis=0)


def run(case: Case, steps: int, avg_start: Optional[int] = None,
        probes: Optional[np.ndarray] = None, f0: Optional[np.ndarray] = None,
        start_step: int = 0, keep: Optional[Sequence[int]] = None):
    """Advance ``steps`` steps from f0 (default: rest equilibrium) at step ``start_step``.

    QoIs (Sec. 2.4 step 6), measured on the pre-collision state f^n:
      * ``final``: u_x, u_y, u_z, |u| of the last state;
      * ``avg``:   time averages over n in (avg_start, end] of u and of |u|;
      * ``probe``: per-probe time average of u_x over the same window.
    """
    f = case.init() if f0 is None else f0.copy()
    out = {}
    keep = set(keep or ())
    kept = {}
    if start_step in keep:
        kept[start_step] = f.copy()
    acc = np.zeros((4, case.n))
    pacc = np.zeros(len(probes)) if probes is not None else None
    cnt = 0
    end = start_step + steps
    for n in range(start_step, end):
        f = case.step(n, f)
        t = n + 1
        if t in keep:
            kept[t] = f.copy()
        if avg_start is not None and t > avg_start:
            q = qoi_fields(case, f)
            acc += q
            if pacc is not None:
                pacc += q[0, probes]
            cnt += 1
    out["f"] = f
    out["final"] = qoi_fields(case, f)
    if cnt:
        out["avg"] = acc / cnt
        if pacc is not None:
            out["probe"] = pacc / cnt
    out["count"] = cnt
    out["kept"] = kept
    return out


def probe_source(case: Case, f: np.ndarray, probes: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """d/df of sum_p weights_p * u_x(f, p): (c_kx - u_x) / rho at each probe cell."""
    c, _, _ = lattice()
    rho, u = case.macros(f)
    s = np.zeros((NQ, case.n))
    for p, wp in zip(probes, weights):
        for k in range(NQ):
            s[k, p] += wp * (c[k, 0] - u[0, p]) / rho[p]
    return s


def probe_objective(case: Case, steps: int, avg_start: int, probes: np.ndarray,
                    pweights: np.ndarray) -> float:
    """J = sum_p pweights_p * (time average over (avg_start, steps] of u_x at probe p)."""
    r = run(case, steps, avg_start=avg_start, probes=probes)
    return float(np.dot(pweights, r["probe"]))


def adjoint(case: Case, steps: int, avg_start: int, probes: np.ndarray,
            pweights: np.ndarray, ckpt: int = 100):
    """dJ/dtheta of J = sum_p pweights_p <u_x(p)>_(avg_start, steps], by the discrete adjoint.

    lambda^N = dj_N/df^N; lambda^n = J_C(f^n)^T P^T lambda^{n+1} + dj_n/df^n;
    dJ/dtheta = sum_n (db(theta, n)/dtheta)^T lambda^{n+1}.  States are
    recomputed per segment of ``ckpt`` steps from stored checkpoints.
    """
    cnt = steps - avg_start
    wsrc = np.asarray(pweights, dtype=np.float64) / cnt
    marks = list(range(0, steps + 1, ckpt))
    r = run(case, steps, keep=marks)
    ckpts = r["kept"]
    lam = probe_source(case, r["f"], probes, wsrc) if steps > avg_start else np.zeros((NQ, case.n))
    grad = np.zeros(3)
    seg_starts = sorted(m for m in marks if m < steps)
    for s0 in reversed(seg_starts):
        s1 = min(s0 + ckpt, steps)
        states = [ckpts[s0]]
        for n in range(s0, s1 - 1):
            states.append(case.step(n, states[-1]))
        for n in range(s1 - 1, s0 - 1, -1):
            fn = states[n - s0]
            lam, g = case.adjoint_step(n, fn, lam)
            grad += g
            if n > avg_start:
                lam += probe_source(case, fn, probes, wsrc)
    return grad, lam
