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


# A velocity component that the oracle holds at zero by symmetry (a wind
# along x before the flow reaches the first building) has no scale of its
# own: FP32 rounding leaves noise of about 1e-8 of the speed there.  Each
# channel is measured against its own size, but at least this fraction of
# the speed channel's (components of 1 % of the speed or more keep their
# own scale).
SPEED_FLOOR = 1e-2


def per_channel_rel(gpu_c4, ora_4c, fluid):
    """Relative L2 of each of the 4 QoI channels (u_x, u_y, u_z, |u|); gpu
    [cells, 4], oracle [4, cells]; the denominator of a component is at least
    SPEED_FLOOR times the norm of |u|."""
    g = np.asarray(gpu_c4, np.float64).T
    o = [np.asarray(ora_4c[k], np.float64)[fluid] for k in range(4)]
    speed = np.linalg.norm(o[3])
    out = []
    for k in range(4):
        d = np.linalg.norm(g[k][fluid] - o[k])
        out.append(float(d / max(np.linalg.norm(o[k]), SPEED_FLOOR * speed, 1e-30)))
    return out


def per_channel_maxrel(gpu_c4, ora_4c, fluid):
    """Element-wise maximum error of each channel relative to the channel's
    largest oracle value (a localised error cannot hide in the L2 norm); the
    denominator of a component is at least SPEED_FLOOR times the largest
    |u|."""
    g = np.asarray(gpu_c4, np.float64).T
    o = [np.asarray(ora_4c[k], np.float64)[fluid] for k in range(4)]
    speed = np.abs(o[3]).max()
    out = []
    for k in range(4):
        d = np.abs(g[k][fluid] - o[k]).max()
        out.append(float(d / max(np.abs(o[k]).max(), SPEED_FLOOR * speed, 1e-30)))
    return out


def oracle_case(w, solid, theta, **over):
    kw = dict(model=w.model, tau0=w.tau0, cs=w.cs, inflow=w.inflow, theta=theta, ramp=w.ramp,
              series=w.series, hour_steps=w.hour_steps, blend_steps=w.blend_steps, ref_height=w.ref_height)
    kw.update(over)
    return orc.Case(w.nx, w.ny, w.nz, list(w.faces), solid, **kw)


def shifted_populations(f_oracle, w_lat):
    """Oracle populations [19, cells] as f - w (the library's stored form)."""
    return f_oracle - w_lat[:, None]
