"""Shared helpers of the GPU parity tests (comparison norms, oracle runs)."""
import numpy as np

from oracle import oracle as orc


def rel_l2(a, b, mask=None, floor=1e-30):
    """||a - b|| / ||b|| over the masked entries (float64)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if mask is not None:
        a = a[..., mask]
        b = b[..., mask]
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor))


def per_channel_rel(gpu_c4, ora_4c, fluid):
    """Relative L2 of each of the 4 QoI channels; gpu [cells, 4], oracle [4, cells]."""
    g = np.asarray(gpu_c4, np.float64).T
    return [rel_l2(g[k], ora_4c[k], fluid) for k in range(4)]


def per_channel_maxrel(gpu_c4, ora_4c, fluid):
    """Element-wise maximum error of each channel relative to the channel's
    largest oracle value (a localised error cannot hide in the L2 norm)."""
    g = np.asarray(gpu_c4, np.float64).T
    out = []
    for k in range(4):
        a, b = g[k][fluid], np.asarray(ora_4c[k], np.float64)[fluid]
        out.append(float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)))
    return out


def oracle_case(w, solid, theta, **over):
    kw = dict(model=w.model, tau0=w.tau0, cs=w.cs, inflow=w.inflow, theta=theta, ramp=w.ramp,
              series=w.series, hour_steps=w.hour_steps, blend_steps=w.blend_steps, ref_height=w.ref_height)
    kw.update(over)
    return orc.Case(w.nx, w.ny, w.nz, list(w.faces), solid, **kw)


def shifted_populations(f_oracle, w_lat):
    """Oracle populations [19, cells] as f - w (the library's stored form)."""
    return f_oracle - w_lat[:, None]
