"""Thin ctypes binding of ``liblbmsc.so`` (C ABI in ``include/lbm_sc.h``).

Argument marshalling only: every function forwards to the C function of the
same name and raises :class:`LbmError` with ``lbm_last_error()`` on failure.
Device pointers are plain integers (``tensor.data_ptr()``); streams are HIP
stream handles (``torch.cuda.current_stream().cuda_stream``).  There is no
fallback: importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmsc.so")

LBM_OK, LBM_E_INVALID, LBM_E_HIP, LBM_E_UNSTABLE, LBM_E_UNSUPPORTED = 0, -1, -2, -3, -4
WALL, INLET, OUTLET, FREESLIP, PERIODIC = 0, 1, 2, 3, 4
FACES = {"wall": WALL, "inlet": INLET, "outlet": OUTLET, "freeslip": FREESLIP, "periodic": PERIODIC}
BGK, SMAGORINSKY, RR3 = 0, 1, 2
MODELS = {"bgk": BGK, "smagorinsky": SMAGORINSKY, "rr3": RR3}
INFLOW_UNIFORM, INFLOW_LOGLAW, INFLOW_SERIES = 0, 1, 2
INFLOWS = {"uniform": INFLOW_UNIFORM, "loglaw": INFLOW_LOGLAW, "series": INFLOW_SERIES}
QUAD_GAUSS_LEGENDRE, QUAD_SMOLYAK_CC, QUAD_GAUSS_HERMITE = 0, 1, 2
QUADS = {"gauss_legendre": QUAD_GAUSS_LEGENDRE, "smolyak_cc": QUAD_SMOLYAK_CC, "gauss_hermite": QUAD_GAUSS_HERMITE}
RECORD_MACROS, RECORD_POPULATIONS, RECORD_RR3_STATE = 1, 2, 3
RR3_STATE_VALUES = 16             # per cell in a record of kind 3


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbmsc error {code}: {msg}")
        self.code = code


class lbm_domain(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("face", ctypes.c_int32 * 6)]


class lbm_instance(ctypes.Structure):
    _fields_ = [("dom", lbm_domain), ("geom_dev", ctypes.c_void_p), ("n_probes", ctypes.c_int32),
                ("f_dev", ctypes.c_void_p), ("model", ctypes.c_int32), ("tau0", ctypes.c_float),
                ("cs", ctypes.c_float), ("inflow", ctypes.c_int32), ("theta", ctypes.c_float * 3),
                ("ramp", ctypes.c_int32), ("qoi_part_dev", ctypes.c_void_p),
                ("qoi_sum_dev", ctypes.c_void_p), ("probe_sum_dev", ctypes.c_void_p),
                ("series_dev", ctypes.c_void_p), ("series_len", ctypes.c_int32),
                ("hour_steps", ctypes.c_int32), ("blend_steps", ctypes.c_int32),
                ("ref_height", ctypes.c_float)]


class lbm_plan_opts(ctypes.Structure):
    _fields_ = [("avg_begin", ctypes.c_int64), ("avg_end", ctypes.c_int64),
                ("use_graph", ctypes.c_int32), ("block", ctypes.c_int32),
                ("cells_per_thread", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("xcd_order", ctypes.c_int32)]


_lib = None

# (name, restype, argtypes) of every function in include/lbm_sc.h
_P = ctypes.c_void_p
_SIGS = [
    ("lbm_last_error", ctypes.c_char_p, []),
    ("lbm_version", ctypes.c_char_p, []),
    ("lbm_quadrature", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    ("lbm_node_params", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_float * 3]),
    ("lbm_geometry_bytes", ctypes.c_int64, [ctypes.POINTER(lbm_domain), ctypes.c_int32]),
    ("lbm_population_stride", ctypes.c_int64, [ctypes.POINTER(lbm_domain)]),
    ("lbm_init_geometry", ctypes.c_int, [ctypes.POINTER(lbm_domain), _P, _P, ctypes.c_int32, _P, _P, _P]),
    ("lbm_plan_create", ctypes.c_int, [ctypes.POINTER(lbm_instance), ctypes.c_int32,
                                       ctypes.POINTER(lbm_plan_opts), ctypes.POINTER(_P)]),
    ("lbm_plan_destroy", None, [_P]),
    ("lbm_plan_step", ctypes.c_int64, [_P]),
    ("lbm_plan_set_step", ctypes.c_int, [_P, ctypes.c_int64]),
    ("lbm_plan_set_cache_block", ctypes.c_int, [_P, ctypes.c_int64]),
    ("lbm_plan_cache_blocks", ctypes.c_int32, [_P]),
    ("lbm_plan_set_theta", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_float * 3]),
    ("lbm_plan_reset_qoi", ctypes.c_int, [_P, _P]),
    ("lbm_sync", ctypes.c_int, [_P, _P]),
    ("lbm_check_health", ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int32)]),
    ("lbm_plan_variant", ctypes.c_int, [_P, ctypes.c_int32 * 4]),
    ("lbm_plan_autotune", ctypes.c_int, [_P, _P, ctypes.c_int32 * 4]),
    ("lbm_collide_stream", ctypes.c_int, [_P, ctypes.c_int32, _P]),
    ("lbm_collide_stream_record", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P,
                                                 ctypes.c_int32, _P]),
    ("lbm_collide_stream_record_qoi", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P,
                                                 ctypes.c_int32, _P]),
    ("lbm_read_fields", ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    ("lbm_read_populations", ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    ("lbm_qoi_average", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    ("lbm_sc_moments", ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P]),
    ("lbm_gpc_basis", ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int32,
                                     _P]),
    ("lbm_gpc_coefficients", ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P, _P,
                                            _P]),
    ("lbm_adjoint_step", ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, ctypes.c_int32,
                                        ctypes.c_int32, _P, _P, _P]),
    ("lbm_adjoint_step_inplace", ctypes.c_int, [_P, ctypes.c_int64, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                                _P, _P, _P]),
    ("lbm_adjoint_step_inplace_noalloc", ctypes.c_int, [_P, ctypes.c_int64, _P, _P, ctypes.c_int32,
                                                        ctypes.c_int32, _P, _P, _P]),
    ("lbm_adjoint_init", ctypes.c_int, [_P, _P, _P, _P]),
]

EXPORTED = [s[0] for s in _SIGS]


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2508_18202_amd.build` (no fallback path exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, lbm_last_error())
    return rc


def _ptr_array(ptrs: Sequence[Optional[int]]):
    arr = (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])
    return arr


def lbm_last_error() -> str:
    return lib().lbm_last_error().decode()


def lbm_version() -> str:
    return lib().lbm_version().decode()


def domain(nx: int, ny: int, nz: int, faces: Sequence) -> lbm_domain:
    d = lbm_domain()
    d.nx, d.ny, d.nz = nx, ny, nz
    for k, f in enumerate(faces):
        d.face[k] = FACES[f] if isinstance(f, str) else int(f)
    return d


def lbm_quadrature(kind, level: int, dim: int):
    """(nodes [n, dim], weights [n]) as float64 numpy arrays."""
    k = QUADS[kind] if isinstance(kind, str) else int(kind)
    n = ctypes.c_int32(0)
    _check(lib().lbm_quadrature(k, level, dim, None, None, 0, ctypes.byref(n)))
    x = np.zeros((n.value, dim))
    w = np.zeros(n.value)
    _check(lib().lbm_quadrature(k, level, dim, x.ctypes.data, w.ctypes.data, n.value, ctypes.byref(n)))
    return x, w


def lbm_gpc_basis(nodes: np.ndarray, order: int, weights: Optional[np.ndarray] = None):
    """(phi [n, P], alpha [P, dim]) of the orthonormal Hermite chaos basis;
    with weights, phi holds the weighted basis a_j Phi_p(Z^(j))."""
    x = np.ascontiguousarray(nodes, dtype=np.float64)
    n, dim = x.shape
    wt = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if wt is not None and wt.shape != (n,):
        raise ValueError("one weight per node")
    P = ctypes.c_int32(0)
    _check(lib().lbm_gpc_basis(None, None, n, dim, order, None, None, 0, ctypes.byref(P)))
    phi = np.zeros((n, P.value))
    alpha = np.zeros((P.value, dim), dtype=np.int32)
    _check(lib().lbm_gpc_basis(x.ctypes.data, wt.ctypes.data if wt is not None else None, n, dim, order,
                               phi.ctypes.data, alpha.ctypes.data, n, ctypes.byref(P)))
    return phi, alpha


def lbm_gpc_coefficients(q_dev: int, wphi_dev: int, n_nodes: int, n_basis: int, n_elems: int, coef_dev: int,
                         var_dev, band_dev, stream: int) -> None:
    _check(lib().lbm_gpc_coefficients(q_dev, wphi_dev, n_nodes, n_basis, n_elems, coef_dev, var_dev, band_dev,
                                      stream))


def lbm_node_params(xi: Sequence[float], base: float, rel: float, angle_deg: float, z0: float):
    x = np.ascontiguousarray(xi, dtype=np.float64)
    out = (ctypes.c_float * 3)()
    _check(lib().lbm_node_params(x.ctypes.data, len(x), base, rel, angle_deg, z0, out))
    return np.array(list(out), dtype=np.float32)


def lbm_geometry_bytes(dom: lbm_domain, n_probes: int) -> int:
    v = lib().lbm_geometry_bytes(ctypes.byref(dom), n_probes)
    if v < 0:
        raise LbmError(LBM_E_INVALID, lbm_last_error())
    return int(v)


def lbm_population_stride(dom: lbm_domain) -> int:
    v = lib().lbm_population_stride(ctypes.byref(dom))
    if v < 0:
        raise LbmError(LBM_E_INVALID, lbm_last_error())
    return int(v)


def lbm_init_geometry(dom: lbm_domain, solid: np.ndarray, probes: np.ndarray, geom_dev: int,
                      f_dev: int, stream: int):
    s = np.ascontiguousarray(solid, dtype=np.uint8)
    p = np.ascontiguousarray(probes, dtype=np.int32)
    _check(lib().lbm_init_geometry(ctypes.byref(dom), s.ctypes.data, p.ctypes.data if p.size else None,
                                   int(p.size), geom_dev, f_dev, stream))


def lbm_plan_create(instances: Sequence[lbm_instance], avg_begin: int = 0, avg_end: int = 0,
                    use_graph: bool = False, block: int = 0, cells_per_thread: int = 0,
                    nontemporal: int = 0, xcd_order: int = 0):
    arr = (lbm_instance * len(instances))(*instances)
    o = lbm_plan_opts()
    o.avg_begin, o.avg_end, o.use_graph, o.block = avg_begin, avg_end, int(use_graph), block
    o.cells_per_thread, o.nontemporal, o.xcd_order = cells_per_thread, nontemporal, xcd_order
    h = ctypes.c_void_p()
    _check(lib().lbm_plan_create(arr, len(instances), ctypes.byref(o), ctypes.byref(h)))
    return h


def lbm_plan_destroy(plan):
    lib().lbm_plan_destroy(plan)


def lbm_plan_step(plan) -> int:
    return int(lib().lbm_plan_step(plan))


def lbm_plan_set_step(plan, step: int):
    _check(lib().lbm_plan_set_step(plan, step))


def lbm_plan_set_theta(plan, inst: int, theta):
    t = (ctypes.c_float * 3)(*[float(v) for v in theta])
    _check(lib().lbm_plan_set_theta(plan, inst, t))


def lbm_plan_reset_qoi(plan, stream: int):
    _check(lib().lbm_plan_reset_qoi(plan, stream))


def lbm_sync(plan, stream: int):
    _check(lib().lbm_sync(plan, stream))


def lbm_check_health(plan, stream: int) -> int:
    bad = ctypes.c_int32(-1)
    rc = lib().lbm_check_health(plan, stream, ctypes.byref(bad))
    if rc not in (LBM_OK, LBM_E_UNSTABLE):
        _check(rc)
    return bad.value


def lbm_plan_variant(plan):
    """(block, cells_per_thread, nontemporal, xcd_order) of a plan."""
    v = (ctypes.c_int32 * 4)()
    _check(lib().lbm_plan_variant(plan, v))
    return tuple(v)


def lbm_plan_autotune(plan, stream: int):
    """Fastest (block, cells_per_thread, nontemporal, xcd_order) for the plan's batch."""
    v = (ctypes.c_int32 * 4)()
    _check(lib().lbm_plan_autotune(plan, stream, v))
    return tuple(v)


def lbm_plan_set_cache_block(plan, nbytes: int):
    """Byte budget of the instance blocks that take plain stretches one at a time (0: off)."""
    _check(lib().lbm_plan_set_cache_block(plan, int(nbytes)))


def lbm_plan_cache_blocks(plan) -> int:
    return int(lib().lbm_plan_cache_blocks(plan))


def lbm_collide_stream(plan, n_steps: int, stream: int):
    _check(lib().lbm_collide_stream(plan, n_steps, stream))


def lbm_collide_stream_record(plan, n_steps: int, kind: int, rec_ptrs: Sequence[int], n_slots: int,
                              stream: int):
    _check(lib().lbm_collide_stream_record(plan, n_steps, kind, _ptr_array(rec_ptrs), n_slots, stream))


def lbm_collide_stream_record_qoi(plan, n_steps: int, kind: int, rec_ptrs: Sequence[int], n_slots: int,
                                  stream: int):
    _check(lib().lbm_collide_stream_record_qoi(plan, n_steps, kind, _ptr_array(rec_ptrs), n_slots, stream))


def lbm_read_fields(plan, inst: int, out_dev: int, stream: int):
    _check(lib().lbm_read_fields(plan, inst, out_dev, stream))


def lbm_read_populations(plan, inst: int, out_dev: int, stream: int):
    _check(lib().lbm_read_populations(plan, inst, out_dev, stream))


def lbm_qoi_average(plan, inst: int, out_dev: Optional[int], probe_out_dev: Optional[int], stream: int):
    _check(lib().lbm_qoi_average(plan, inst, out_dev, probe_out_dev, stream))


def lbm_sc_moments(q_dev: int, weights: np.ndarray, n_nodes: int, n_elems: int, mean_dev: int,
                   var_dev: int, n_negative_dev: Optional[int], stream: int):
    w = np.ascontiguousarray(weights, dtype=np.float64)
    _check(lib().lbm_sc_moments(q_dev, w.ctypes.data, n_nodes, n_elems, mean_dev, var_dev,
                                n_negative_dev, stream))


def lbm_adjoint_step(plan, step: int, lam_in: Sequence[int], lam_out: Sequence[int],
                     rec: Sequence[int], kind: int, n_slots: int, pw: Sequence[Optional[int]],
                     grad_dev: int, stream: int):
    _check(lib().lbm_adjoint_step(plan, step, _ptr_array(lam_in), _ptr_array(lam_out), _ptr_array(rec),
                                  kind, n_slots, _ptr_array(pw), grad_dev, stream))


def lbm_adjoint_step_inplace(plan, step: int, lam: Sequence[int], rec: Sequence[int], kind: int, n_slots: int,
                             pw: Sequence[Optional[int]], grad_dev: int, stream: int):
    _check(lib().lbm_adjoint_step_inplace(plan, step, _ptr_array(lam), _ptr_array(rec), kind, n_slots,
                                          _ptr_array(pw), grad_dev, stream))


def lbm_adjoint_step_inplace_noalloc(plan, step: int, lam: Sequence[int], rec: Sequence[int], kind: int,
                                     n_slots: int, pw: Sequence[Optional[int]], grad_dev: int, stream: int):
    _check(lib().lbm_adjoint_step_inplace_noalloc(plan, step, _ptr_array(lam), _ptr_array(rec), kind, n_slots,
                                                  _ptr_array(pw), grad_dev, stream))


def lbm_adjoint_init(plan, lam_out: Sequence[int], pw: Sequence[Optional[int]], stream: int):
    _check(lib().lbm_adjoint_init(plan, _ptr_array(lam_out), _ptr_array(pw), stream))
