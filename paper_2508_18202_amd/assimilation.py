"""Gradient-based assimilation of the inflow noise model through the adjoint.

The paper (arXiv 2508.18202, Sec. 2.4 step 5 and Sec. 3) injects uncertain
hourly measurements into the inflow; here the same uncertain-inflow model is
fitted to probe observations by gradient descent.  The speed multiplier of
the friction velocity is m = mu + s * xi_1 (xi_1 ~ U(-1, 1)), so node j of the
collocation rule runs with u*_j = u*_base (mu + s xi_1^(j)) and direction
angle_deg * xi_2^(j).  Observations are the collocation mean and standard
deviation of the probe time averages of u_x under a hidden (mu, s), each
perturbed by 5 % relative Gaussian noise.  The loss is

  L(mu, s) = sum_p [(E_p - E^obs_p)^2 + (S_p - S^obs_p)^2] / (0.05 E^obs_p)^2

with E, S from Eq. (quad_moments) over the nodes.  Its gradient chains the
per-node probe adjoint (ProbeQoI) through the quadrature sums and the
parameter map; steps use gradient descent with Armijo backtracking, each
first trial capped at the step where the loss's linearisation vanishes.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from . import inputs
from .adjoint import CheckpointedAdjoint, probe_qoi
from .sc import Ensemble, collocation, make_geometry


def node_thetas(w, xi: torch.Tensor, params: torch.Tensor) -> torch.Tensor:
    """theta [N_q, 3] (FP64, differentiable in params = (mu, s))."""
    mu, s = params[0], params[1]
    ustar = w.speed_base * (mu + s * xi[:, 0])
    phi = torch.deg2rad(w.angle_deg * xi[:, 1]) if xi.shape[1] > 1 else torch.zeros_like(ustar)
    z0 = torch.full_like(ustar, w.z0)
    return torch.stack([ustar, phi, z0], dim=1)


def sc_stats(q: torch.Tensor, a: torch.Tensor, floor: float = 1e-30):
    """Collocation mean and standard deviation over nodes (FP64)."""
    e = (a[:, None] * q).sum(0)
    v = (a[:, None] * (q - e) ** 2).sum(0)
    return e, torch.sqrt(torch.clamp(v, min=floor))


class Assimilation:
    def __init__(self, w, steps: int, avg_len: int, ckpt: int = 100, group_size: Optional[int] = None,
                 solid: Optional[np.ndarray] = None, probes: Optional[np.ndarray] = None):
        self.w = w
        solid = inputs.solid_mask(w) if solid is None else solid
        probes = inputs.probe_cells(w, solid) if probes is None else probes
        x, a, th = collocation(w)
        self.xi = torch.tensor(x, dtype=torch.float64)
        self.a = torch.tensor(a, dtype=torch.float64)
        cg = make_geometry(w, solid, probes)
        self.ens = Ensemble([cg], [th], avg_begin=steps - avg_len, avg_end=steps, fields=False,
                            use_graph=True)
        self.runner = CheckpointedAdjoint(self.ens, steps, ckpt, group_size)
        self.obs: Optional[Tuple[torch.Tensor, torch.Tensor]] = None

    def close(self):
        self.runner.close()
        self.ens.close()

    def qoi(self, params: torch.Tensor) -> torch.Tensor:
        return probe_qoi(node_thetas(self.w, self.xi, params), self.runner).cpu()

    def observe(self, truth: Tuple[float, float], noise: np.ndarray, rel: float = 0.05):
        with torch.no_grad():
            q = self.qoi(torch.tensor(truth, dtype=torch.float64))
            e, s = sc_stats(q, self.a)
        n = e.numel()
        eps = torch.tensor(noise[: 2 * n], dtype=torch.float64)
        self.obs = (e * (1 + rel * eps[:n]), s * (1 + rel * eps[n:]))
        return self.obs

    def loss(self, params: torch.Tensor, rel: float = 0.05) -> torch.Tensor:
        eo, so = self.obs
        q = self.qoi(params)
        e, s = sc_stats(q, self.a)
        scale = (rel * eo) ** 2
        return (((e - eo) ** 2 + (s - so) ** 2) / scale).sum()

    def run(self, start: Tuple[float, float], iters: int, step0: float = 1e-3,
            max_backtrack: int = 6) -> List[Dict]:
        params = torch.tensor(start, dtype=torch.float64)
        hist = []
        step = step0
        for it in range(iters):
            t0 = time.perf_counter()
            p = params.clone().requires_grad_(True)
            L = self.loss(p)
            (g,) = torch.autograd.grad(L, p)
            g = g.detach()
            lval = float(L.detach())
            gn2 = float((g * g).sum())
            if gn2 == 0.0:
                # a stationary point (with exact observations, the truth)
                hist.append({"iter": it, "mu": float(params[0]), "s": float(params[1]), "loss": lval,
                             "grad": [0.0, 0.0], "step": step, "accepted": False, "trials": 0,
                             "wall_s": round(time.perf_counter() - t0, 2)})
                break
            # the loss is a sum of squares (never below zero): along -g its
            # linearisation reaches zero at the step L / |g|^2, a step no
            # trial exceeds, whatever the scale of the observations
            step = min(step, lval / gn2)
            accepted = False
            trials = 0
            for _ in range(max_backtrack):
                trial = params - step * g
                if float(trial[1]) <= 0.0:
                    step *= 0.5
                    continue
                with torch.no_grad():
                    lt = float(self.loss(trial))
                trials += 1
                if lt <= lval - 1e-4 * step * gn2:
                    params = trial
                    accepted = True
                    step *= 1.5
                    break
                step *= 0.5
            hist.append({"iter": it, "mu": float(params[0]), "s": float(params[1]), "loss": lval,
                         "grad": [float(v) for v in g], "step": step, "accepted": accepted, "trials": trials,
                         "wall_s": round(time.perf_counter() - t0, 2)})
        return hist
