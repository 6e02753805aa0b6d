"""Checkpointed discrete adjoint of a batched run and its autograd wrapper.

The gradient of probe QoIs with respect to the inflow parameters is not part
of arXiv 2508.18202; it differentiates the paper's deterministic solver
(Sec. 2.2) with respect to the uncertain boundary data of Sec. 3 and feeds a
gradient-based assimilation of the inflow noise model.

Schedule for a run of N steps with snapshots every C steps:
  forward   advance 0 -> N, copying the populations at steps 0, C, 2C, ...
  init      lam^N = dj_N/df^N                               (lbm_adjoint_init)
  segments  for each segment [s0, s1) from last to first:
              restore the snapshot of s0, re-run s0 -> s1 recording the state
              of every step (rho, u for BGK; populations for Smagorinsky; the
              16 state values of the regularised collision), then lam^n from
              lam^{n+1} for n = s1-1 ... s0  (lbm_adjoint_step)
dJ/dtheta accumulates in FP64 inside the adjoint kernel.

With ``group_size`` set, the forward pass advances the whole batch without
snapshots, and the reverse sweep runs group by group (each group re-runs its
own forward with snapshots on a plan of its own), so snapshot and record
memory scale with the group, not the batch.

Without groups the forward run records its last steps itself
(lbm_collide_stream_record_qoi), as many whole segments as fit in a fraction
of the free device memory (every step when they all fit: ``store_all``), and
the sweep takes those segments without a re-run.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import lbmsc as L
from .sc import Ensemble, stream_handle


def stored_tail(steps: int, ckpt: int, grouped: bool, store_all: Optional[bool], stored_steps: Optional[int],
                per_step: int, free: Optional[int], memory_fraction: float = 0.6) -> int:
    """Number of last steps the forward run records itself (host logic of
    CheckpointedAdjoint): stored_steps if given (the run length or a multiple
    of ckpt below it), every step or one segment for store_all True/False,
    one segment for grouped sweeps, else as many whole segments as
    memory_fraction of `free` bytes holds at `per_step` bytes per step (at
    least one segment, at most the run)."""
    if grouped:
        if store_all:
            raise ValueError("store_all needs the whole batch in one sweep (no group_size)")
        return ckpt
    if stored_steps is not None:
        if stored_steps != steps and (stored_steps % ckpt or not ckpt <= stored_steps < steps):
            raise ValueError("stored_steps must be the run length or a multiple of ckpt below it")
        return stored_steps
    if store_all is not None:
        return steps if store_all else min(ckpt, steps)
    return min(steps, max(ckpt, int(memory_fraction * free // per_step) // ckpt * ckpt))


class CheckpointedAdjoint:
    """Forward run with snapshots and the reverse sweep over one Ensemble.

    The ensemble's plan window (avg_begin, avg_end] defines the objective
    j_n = sum_p pw[p] u_x(f^n, p) / count; avg_end must equal the run length.
    """

    def __init__(self, ens: Ensemble, steps: int, ckpt: int = 100, group_size: Optional[int] = None,
                 inplace: bool = False, record_kind: Optional[int] = None,
                 store_all: Optional[bool] = None, memory_fraction: float = 0.6,
                 stored_steps: Optional[int] = None):
        if steps % 2 or ckpt % 2:
            raise ValueError("run length and checkpoint spacing must be even")
        if ens.avg_end != steps:
            raise ValueError("the QoI window must end at the last step")
        self.ens = ens
        self.steps = steps
        self.ckpt = ckpt
        self.model = ens.instances[0].model
        # lambda layout: two alternating buffers (lbm_adjoint_step) by
        # default, for every model as fast as or faster than one buffer
        # updated in place (lbm_adjoint_step_inplace, half the lambda memory)
        # on the 13 x 128x64x48 adjoint case (BGK 4-7 %, regularised 0-3 %)
        self.inplace = bool(inplace)
        n = len(ens)
        self.groups = [list(range(n))] if not group_size else \
            [list(range(k, min(n, k + group_size))) for k in range(0, n, group_size)]
        self.grouped = bool(group_size) and group_size < n
        # what the recording re-runs save per cell and step: (rho, u) for BGK,
        # the populations for Smagorinsky, the 16 state values of the
        # regularised collision for it (record_kind overrides, e.g. 2)
        default = {L.BGK: L.RECORD_MACROS, L.RR3: L.RECORD_RR3_STATE}.get(self.model, L.RECORD_POPULATIONS)
        self.kind = default if record_kind is None else int(record_kind)
        self.marks = list(range(0, steps, ckpt))
        self.snaps: List[List[torch.Tensor]] = []
        gmax = max(len(g) for g in self.groups)

        def per_slot_of(cg):
            if self.kind == L.RECORD_MACROS:
                return 4 * cg.ncells
            return (L.RR3_STATE_VALUES if self.kind == L.RECORD_RR3_STATE else 19) * cg.qs

        # stored tail: the forward run records its last `stored` steps (a
        # multiple of ckpt), whose segments the sweep then takes without a
        # re-run; the earlier segments keep their snapshots and are re-run
        # with recording into the same slots (slot n % stored) once the tail
        # is consumed.  By default as many steps as fit in memory_fraction of
        # the free device memory (all of them for BGK's 16-byte records of the
        # 13 x 128x64x48 adjoint case, 164 GB); store_all=True asks for every
        # step, False for one segment; grouped sweeps store one segment.
        per_step = 4 * sum(per_slot_of(ens.cases[ens.index[i][0]]) for i in range(n))
        free = None
        if not self.grouped and stored_steps is None and store_all is None:
            free = torch.cuda.mem_get_info()[0] + torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
        stored = stored_tail(steps, ckpt, self.grouped, store_all, stored_steps, per_step, free, memory_fraction)
        self.stored = stored
        self.store_all = stored >= steps
        self.n_slots = stored
        self.head = steps - stored         # steps before the stored tail
        # record and adjoint buffers for the largest group (reused group after group)
        self.rec: List[torch.Tensor] = []
        self.lam = [[], []]
        for k in range(gmax):
            cgs = [ens.cases[ens.index[g[k]][0]] for g in self.groups if k < len(g)]
            per_slot = max(per_slot_of(cg) for cg in cgs)
            lam_len = max(19 * cg.qs for cg in cgs)
            self.rec.append(torch.empty(self.n_slots * per_slot, dtype=torch.float32, device="cuda"))
            for b in range(1 if self.inplace else 2):
                self.lam[b].append(torch.empty(lam_len, dtype=torch.float32, device="cuda"))
        self.grad = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
        self._subplans = {}

    # ------------------------------------------------------------------ forward
    def _advance_with_snapshots(self, plan, fs: Sequence[torch.Tensor], upto: Optional[int] = None):
        """Advance to step `upto` (default N), copying the populations at the
        marks before it."""
        upto = self.steps if upto is None else upto
        self.snaps = []
        for s0 in self.marks:
            if s0 >= upto:
                break
            self.snaps.append([f.clone() for f in fs])
            L.lbm_collide_stream(plan, min(self.ckpt, upto - s0), stream_handle())

    def forward(self):
        """Advance the batch from rest to step N; returns the probe averages per instance."""
        ens = self.ens
        ens.reset()
        if self.grouped:
            ens.advance(self.steps)
        else:
            # snapshots up to the stored tail, then the tail with its records
            self._advance_with_snapshots(ens.plan, ens.f, upto=self.head)
            L.lbm_collide_stream_record_qoi(ens.plan, self.stored, self.kind, [t.data_ptr() for t in self.rec],
                                            self.n_slots, stream_handle())
        out = []
        for i in range(len(ens)):
            cg = ens.cases[ens.index[i][0]]
            p = torch.empty(len(cg.probes), dtype=torch.float32, device="cuda")
            ens.averages_into(i, None, p)
            out.append(p)
        return out

    # ----------------------------------------------------------------- backward
    def _subplan(self, gi: int):
        if gi not in self._subplans:
            insts = []
            for i in self.groups[gi]:
                inst = L.lbm_instance.from_buffer_copy(self.ens.instances[i])
                inst.qoi_part_dev = None
                inst.qoi_sum_dev = None
                inst.probe_sum_dev = None
                insts.append(inst)
            self._subplans[gi] = L.lbm_plan_create(insts, self.ens.avg_begin, self.ens.avg_end,
                                                   use_graph=False)
        return self._subplans[gi]

    def _sweep(self, plan, members: Sequence[int], pw_ptr, grad: torch.Tensor):
        s = stream_handle()
        k = len(members)
        lam_ptr = [[t.data_ptr() for t in self.lam[b][:k]] for b in range(1 if self.inplace else 2)]
        rec_ptr = [t.data_ptr() for t in self.rec[:k]]
        fs = [self.ens.f[i] for i in members]
        N = self.steps
        L.lbm_adjoint_init(plan, lam_ptr[0 if self.inplace else N % 2], pw_ptr, s)

        def adjoint_steps(s1, s0):
            for n in range(s1 - 1, s0 - 1, -1):
                if self.inplace:
                    L.lbm_adjoint_step_inplace(plan, n, lam_ptr[0], rec_ptr, self.kind, self.n_slots, pw_ptr,
                                               grad.data_ptr(), s)
                else:
                    L.lbm_adjoint_step(plan, n, lam_ptr[(n + 1) % 2], lam_ptr[n % 2], rec_ptr,
                                       self.kind, self.n_slots, pw_ptr, grad.data_ptr(), s)

        # segments of the stored tail still have their records from the
        # forward run; the earlier ones are re-run from their snapshots
        tail_from = N if self.grouped else self.head
        for m in reversed(range(len(self.marks))):
            s0 = self.marks[m]
            s1 = min(s0 + self.ckpt, N)
            if s0 < tail_from:
                for f, snap in zip(fs, self.snaps[m]):
                    f.copy_(snap)
                L.lbm_plan_set_step(plan, s0)
                L.lbm_collide_stream_record(plan, s1 - s0, self.kind, rec_ptr, self.n_slots, s)
            adjoint_steps(s1, s0)

    def backward(self, pweights: Sequence[Optional[torch.Tensor]]):
        """dJ/dtheta [n_inst, 3] (FP64) of J_i = sum_p pweights[i][p] <u_x(p)>.

        Leaves every instance at step 0 in the rest state, with cleared QoI
        sums (the populations are re-initialised after the sweep)."""
        ens = self.ens
        pw = [p.to(torch.float64).contiguous() if p is not None else None for p in pweights]
        pw_ptr = [p.data_ptr() if p is not None else None for p in pw]
        self.grad.zero_()
        if not self.grouped:
            if L.lbm_plan_step(ens.plan) != self.steps:
                raise RuntimeError("backward needs the state of the last forward step (call forward first)")
            self._sweep(ens.plan, self.groups[0], pw_ptr, self.grad)
        else:
            for gi, members in enumerate(self.groups):
                plan = self._subplan(gi)
                for i in members:
                    L.lbm_plan_set_theta(plan, members.index(i), list(ens.instances[i].theta))
                    ens.f[i].zero_()          # the rest state (f - w = 0); geometry unchanged
                L.lbm_plan_set_step(plan, 0)
                self._advance_with_snapshots(plan, [ens.f[i] for i in members])
                g = torch.zeros(len(members), 3, dtype=torch.float64, device="cuda")
                self._sweep(plan, members, [pw_ptr[i] for i in members], g)
                self.grad[members[0]:members[-1] + 1] = g
                self.snaps = []
        # the sweep leaves the populations at the end of the first segment's
        # re-run (and, grouped, in the subplans' state): back to the rest
        # state, which is f - w = 0 in every slot, at step 0
        for f in ens.f:
            f.zero_()
        L.lbm_plan_set_step(ens.plan, 0)
        L.lbm_plan_reset_qoi(ens.plan, stream_handle())
        return self.grad.clone()

    def close(self):
        for p in self._subplans.values():
            L.lbm_plan_destroy(p)
        self._subplans = {}


def set_thetas(runner: CheckpointedAdjoint, theta) -> None:
    """Inflow parameters [n_inst, 3] of every instance of the runner's batch."""
    ens = runner.ens
    for i in range(len(ens)):
        t = [float(v) for v in theta[i]]
        L.lbm_plan_set_theta(ens.plan, i, t)
        for k in range(3):
            ens.instances[i].theta[k] = t[k]


class ProbeQoI(torch.autograd.Function):
    """theta [n_inst, 3] (FP64) -> probe time averages of u_x [n_inst, n_probes].

    The backward pass is the checkpointed discrete adjoint: the incoming
    gradient becomes the probe weights of the adjoint source.  Requires every
    instance to share one probe count."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, runner: CheckpointedAdjoint):
        set_thetas(runner, theta.detach().cpu().numpy())
        q = runner.forward()
        ctx.runner = runner
        ctx.theta_device = theta.device
        return torch.stack(q).to(torch.float64)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        runner = ctx.runner
        g = grad_out.to(torch.float64)
        pw = [g[i].contiguous() for i in range(g.shape[0])]
        dth = runner.backward(pw)
        return dth.to(ctx.theta_device), None


def probe_qoi(theta: torch.Tensor, runner: CheckpointedAdjoint) -> torch.Tensor:
    return ProbeQoI.apply(theta, runner)
