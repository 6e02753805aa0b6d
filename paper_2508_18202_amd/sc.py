"""Non-intrusive stochastic-collocation driver over the C ABI (Sec. 2.4 of
arXiv 2508.18202, steps 2-7 on synthetic inputs).

PyTorch provides device memory and the stream; every computation runs in the
library: collocation rule and node parameters (``lbm_quadrature``,
``lbm_node_params``), geometry (``lbm_init_geometry``), the batched
deterministic runs of all nodes of all cases in one plan
(``lbm_collide_stream``), QoI capture and window averages, and the
quadrature moments (``lbm_sc_moments``).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import lbmsc as L
from .inputs import Workload


def stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


def collocation(w: Workload):
    """(nodes [N_q, d], weights [N_q], thetas [N_q, 3]) of a workload."""
    x, a = L.lbm_quadrature(w.quadrature, w.quad_level, w.quad_dim)
    th = np.stack([L.lbm_node_params(xi, w.speed_base, w.speed_rel, w.angle_deg, w.z0) for xi in x])
    return x, a, th


@dataclasses.dataclass
class CaseGeometry:
    """Geometry buffer of one lattice case (shared by all of its nodes)."""
    w: Workload
    solid: np.ndarray
    probes: np.ndarray
    dom: L.lbm_domain
    qs: int
    geom: torch.Tensor

    @property
    def ncells(self) -> int:
        return self.w.nx * self.w.ny * self.w.nz

    @property
    def fluid(self) -> np.ndarray:
        return self.solid.reshape(-1) == 0


def make_geometry(w: Workload, solid: np.ndarray, probes: Optional[np.ndarray] = None) -> CaseGeometry:
    """Allocate the geometry buffer of a case; it is filled (and every node's
    populations set to rest) by ``lbm_init_geometry`` when an ensemble is built."""
    probes = np.zeros(0, np.int32) if probes is None else np.asarray(probes, np.int32)
    dom = L.domain(w.nx, w.ny, w.nz, w.faces)
    qs = L.lbm_population_stride(dom)
    geom = torch.empty(L.lbm_geometry_bytes(dom, len(probes)), dtype=torch.uint8, device="cuda")
    return CaseGeometry(w, np.ascontiguousarray(solid, np.uint8), probes, dom, qs, geom)


def init_populations(cg: CaseGeometry, f: torch.Tensor):
    """Geometry flags of the case and the rest equilibrium in f."""
    L.lbm_init_geometry(cg.dom, cg.solid, cg.probes, cg.geom.data_ptr(), f.data_ptr(), stream_handle())


class Ensemble:
    """Every (case, node) pair of a batch advanced together by one plan."""

    def __init__(self, cases: Sequence[CaseGeometry], thetas: Sequence[Sequence[Sequence[float]]],
                 avg_begin: int = 0, avg_end: int = 0, fields: bool = True, probe_sums: bool = True,
                 use_graph: bool = True, block: int = 0, variant: Optional[Sequence[int]] = None,
                 cache_block: Optional[int] = None):
        self.cases = list(cases)
        self.index: List[Tuple[int, int]] = []
        self.f: List[torch.Tensor] = []
        self.qpart: List[Optional[torch.Tensor]] = []
        self.qsum: List[Optional[torch.Tensor]] = []
        self.psum: List[Optional[torch.Tensor]] = []
        self.avg_begin, self.avg_end = avg_begin, avg_end
        window = avg_end > avg_begin
        insts = []
        self.series: List[Optional[torch.Tensor]] = []   # per case: hourly series on the device
        for ci, (cg, ths) in enumerate(zip(self.cases, thetas)):
            w = cg.w
            ser = None
            if w.inflow == "series":
                ser = torch.tensor(w.series, dtype=torch.float32, device="cuda").reshape(-1).contiguous()
            self.series.append(ser)
            for j, th in enumerate(ths):
                f = torch.empty(19 * cg.qs, dtype=torch.float32, device="cuda")
                init_populations(cg, f)
                qp = qsm = ps = None
                if window and fields:
                    qp = torch.empty(4 * cg.ncells, dtype=torch.float32, device="cuda")
                    qsm = torch.empty(4 * cg.ncells, dtype=torch.float64, device="cuda")
                if window and probe_sums and len(cg.probes):
                    ps = torch.empty(len(cg.probes), dtype=torch.float64, device="cuda")
                inst = L.lbm_instance()
                inst.dom = cg.dom
                inst.geom_dev = cg.geom.data_ptr()
                inst.n_probes = len(cg.probes)
                inst.f_dev = f.data_ptr()
                inst.model = L.MODELS[w.model]
                inst.tau0 = w.tau0
                inst.cs = w.cs
                inst.inflow = L.INFLOWS[w.inflow]
                for k in range(3):
                    inst.theta[k] = float(th[k])
                inst.ramp = w.ramp
                inst.qoi_part_dev = qp.data_ptr() if qp is not None else None
                inst.qoi_sum_dev = qsm.data_ptr() if qsm is not None else None
                inst.probe_sum_dev = ps.data_ptr() if ps is not None else None
                if ser is not None:
                    inst.series_dev = ser.data_ptr()
                    inst.series_len = len(w.series)
                    inst.hour_steps = w.hour_steps
                    inst.blend_steps = w.blend_steps
                    inst.ref_height = w.ref_height
                insts.append(inst)
                self.index.append((ci, j))
                self.f.append(f)
                self.qpart.append(qp)
                self.qsum.append(qsm)
                self.psum.append(ps)
        self.instances = insts
        v = tuple(variant) if variant is not None else (block, 0, 1, 0)
        v = v + (0,) * (4 - len(v))
        self.plan = L.lbm_plan_create(insts, avg_begin, avg_end, use_graph, *v)
        if cache_block is not None:          # bytes per instance block (0: the whole batch per step)
            L.lbm_plan_set_cache_block(self.plan, cache_block)
        L.lbm_plan_reset_qoi(self.plan, stream_handle())

    def reset(self):
        """Every node back to rest at step 0 with cleared QoI sums."""
        for (ci, _), f in zip(self.index, self.f):
            init_populations(self.cases[ci], f)
        L.lbm_plan_set_step(self.plan, 0)
        L.lbm_plan_reset_qoi(self.plan, stream_handle())

    def __len__(self):
        return len(self.instances)

    def close(self):
        if self.plan is not None:
            L.lbm_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step(self) -> int:
        return L.lbm_plan_step(self.plan)

    def advance(self, n_steps: int):
        L.lbm_collide_stream(self.plan, n_steps, stream_handle())

    def health(self) -> int:
        """-1 if every instance is healthy, else the first unstable instance."""
        return L.lbm_check_health(self.plan, stream_handle())

    def fields_into(self, i: int, out: torch.Tensor):
        L.lbm_read_fields(self.plan, i, out.data_ptr(), stream_handle())

    def fields(self, i: int) -> torch.Tensor:
        cg = self.cases[self.index[i][0]]
        out = torch.empty(cg.ncells, 4, dtype=torch.float32, device="cuda")
        self.fields_into(i, out)
        return out

    def populations(self, i: int) -> torch.Tensor:
        cg = self.cases[self.index[i][0]]
        out = torch.empty(19, cg.qs, dtype=torch.float32, device="cuda")
        L.lbm_read_populations(self.plan, i, out.data_ptr(), stream_handle())
        return out[:, :cg.ncells]

    def averages_into(self, i: int, out: Optional[torch.Tensor], pout: Optional[torch.Tensor] = None):
        L.lbm_qoi_average(self.plan, i, out.data_ptr() if out is not None else None,
                          pout.data_ptr() if pout is not None else None, stream_handle())

    def instances_of(self, case: int) -> List[int]:
        return [k for k, (c, _) in enumerate(self.index) if c == case]


def moments(q: torch.Tensor, weights: np.ndarray, count_negative: bool = False):
    """Eq. (quad_moments) over the leading (node) axis of a float32 tensor."""
    n_nodes = q.shape[0]
    n = q[0].numel()
    q = q.contiguous()
    mean = torch.empty(q.shape[1:], dtype=torch.float64, device=q.device)
    var = torch.empty(q.shape[1:], dtype=torch.float64, device=q.device)
    neg = torch.zeros(1, dtype=torch.int64, device=q.device) if count_negative else None
    L.lbm_sc_moments(q.data_ptr(), weights, n_nodes, n, mean.data_ptr(), var.data_ptr(),
                     neg.data_ptr() if neg is not None else None, stream_handle())
    if count_negative:
        return mean, var, int(neg.item())
    return mean, var


def gpc(q: torch.Tensor, nodes: np.ndarray, weights: np.ndarray, order: int):
    """gPC expansion (Sec. 2.3) of q [N_q, ...] (float32, node-major) in the
    orthonormal Hermite chaos of total degree <= order at the collocation
    nodes: coefficients [P, ...], multi-indices [P, d], mean (coef 0),
    variance (sum of the squared higher coefficients) and the 95 % band
    mean -+ 1.96 std, all FP64 from one kernel."""
    wphi_h, alpha = L.lbm_gpc_basis(nodes, order, weights)
    wphi = torch.from_numpy(wphi_h).to(q.device).contiguous()
    q = q.contiguous()
    n = q[0].numel()
    P = wphi_h.shape[1]
    coef = torch.empty((P,) + tuple(q.shape[1:]), dtype=torch.float64, device=q.device)
    var = torch.empty(tuple(q.shape[1:]), dtype=torch.float64, device=q.device)
    band = torch.empty((2,) + tuple(q.shape[1:]), dtype=torch.float64, device=q.device)
    L.lbm_gpc_coefficients(q.data_ptr(), wphi.data_ptr(), q.shape[0], P, n, coef.data_ptr(), var.data_ptr(),
                           band.data_ptr(), stream_handle())
    return {"coef": coef, "alpha": alpha, "mean": coef[0], "var": var, "band": band}


def run_sc(w: Workload, solid: np.ndarray, steps: Optional[int] = None, avg_start: Optional[int] = None,
           probes: Optional[np.ndarray] = None, use_graph: bool = True, block: int = 0,
           check_every: int = 0, variant: Optional[Sequence[int]] = None):
    """One SC-LBM pass of one case: every collocation node advanced together,
    then the quadrature mean and variance of the QoI fields.

    QoI: time averages of (u_x, u_y, u_z, |u|) over states n in
    (avg_start, steps] when avg_start < steps, else the final fields."""
    steps = w.steps if steps is None else steps
    avg_start = w.avg_start if avg_start is None else avg_start
    x, a, th = collocation(w)
    cg = make_geometry(w, solid, probes)
    window = avg_start < steps
    ens = Ensemble([cg], [th], avg_begin=avg_start if window else 0, avg_end=steps if window else 0,
                   use_graph=use_graph, block=block, variant=variant)
    try:
        if check_every:
            done = 0
            while done < steps:
                k = min(check_every, steps - done)
                ens.advance(k)
                done += k
                bad = ens.health()
                if bad >= 0:
                    raise L.LbmError(L.LBM_E_UNSTABLE, f"node {bad} unstable by step {ens.step}")
        else:
            ens.advance(steps)
        q = torch.empty(len(ens), cg.ncells, 4, dtype=torch.float32, device="cuda")
        pq = None
        if window and len(cg.probes):
            pq = torch.empty(len(ens), len(cg.probes), dtype=torch.float32, device="cuda")
        for j in range(len(ens)):
            if window:
                ens.averages_into(j, q[j], pq[j] if pq is not None else None)
            else:
                ens.fields_into(j, q[j])
        mean, var, nneg = moments(q, a, count_negative=True)
        return {"nodes": x, "weights": a, "thetas": th, "q": q, "mean": mean, "var": var,
                "n_negative": nneg, "probe_q": pq, "ensemble": ens, "geometry": cg}
    except Exception:
        ens.close()
        raise
