"""Differentiable N-step rollout: J(amp) and dJ/d amp through the HIP adjoint.

J = wk * KE(f*_N) + wl * (L_u + L_d)(f*_N) for f*_N = step^N(init_rt3(amp)),
with the mixing lengths of Sec. IV (eq. 3L).  The backward pass runs the
library's adjoint kernels (lbm_objective seed; lbm_adjoint_collide, then
lbm_adjoint_gather per step, or lbm_adjoint_step per step in push form;
lbm_init_rt3_vjp); this module only schedules them and manages memory.

Memory schedule (two levels):
* level 1 -- the state f*_t is checkpointed every ``ckpt_every`` steps during
  the forward pass (the initial state is checkpoint 0), also where every
  step's moments are kept and no segment will be recomputed; ``ckpt_every =
  0`` sets the interval to the number of kept steps, the largest segment the
  kept buffer can hold, which needs the fewest checkpoints;
* level 2 -- the adjoint of step t needs the 4 pre-collision moments of that
  step (double, or float with ``mom_precision="f32"``).  The forward pass
  keeps them for the last ``keep`` steps (as many as ``moment_budget_bytes``
  allows); for earlier steps each checkpoint segment is recomputed from its
  checkpoint, storing its moments, just before the backward sweep crosses it.
  The recomputed moments go into the kept buffer, whose contents the sweep
  has consumed by then (a separate segment buffer only when fewer than
  ``ckpt_every`` steps are kept).
With every step's moments kept the backward pass needs no recomputation; in
general it recomputes nsteps - keep steps, each once.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import abi
from .workload import Workload


@dataclass
class RolloutConfig:
    lx: int
    lz: int
    tau: float
    g: float
    t_d: float
    t_m: float
    t_u: float
    width: float
    k: np.ndarray
    phase: np.ndarray
    nsteps: int
    ckpt_every: int = 100
    precision: str = "f64"
    wk: float = 1.0
    wl: float = 1.0
    moment_budget_bytes: int = 64 << 30
    adj_precision: str = "f64"     # "f32": adjoint buffers in float (LBM_ADJ_F32)
    wall: str = "dirichlet"        # or "diffuse" (LBM_WALL_DIFFUSE)
    mom_precision: str = "f64"     # "f32": stored moments in float (LBM_MOM_F32)
    # "gather" (lbm_adjoint_collide, lbm_adjoint_gather), "push" (lbm_adjoint_step)
    # or "auto" (= gather, the faster form on MI355X: 2048 x 6144 all-float
    # 0.693 ms vs 0.82 ms push; 512 x 1536 double 0.082 ms vs 0.103 ms)
    adjoint_form: str = "auto"
    collide_f64: bool = False      # FP32-dev forward steps collide in double (LBM_COLLIDE_F64)

    @classmethod
    def from_workload(cls, wl: Workload, modes, nsteps=None, **kw):
        kw.setdefault("ckpt_every", wl.ckpt_every)
        kw.setdefault("precision", wl.precision)
        kw.setdefault("adj_precision", wl.adj_precision)
        kw.setdefault("wall", wl.wall)
        kw.setdefault("mom_precision", wl.mom_precision)
        return cls(wl.lx, wl.lz, wl.tau, wl.g, wl.t_d, wl.t_m, wl.t_u, wl.width, modes.k,
                   modes.phase, wl.steps if nsteps is None else nsteps, **kw)


def checkpoint_steps(nsteps, keep, ckpt_every):
    """Steps after which the forward pass stores the state (0 = the initial
    state): every ``ckpt_every`` steps of the run, whether or not the
    backward sweep will recompute from them (with every step's moments kept
    none is needed for the gradient; they are the run's restart points).
    ``keep`` does not change the schedule; it is taken for symmetry with
    backward_plan."""
    del keep
    return [0] + list(range(ckpt_every, nsteps, ckpt_every))


def backward_plan(nsteps, keep, ckpt_every):
    """The backward sweep as a list of operations, in order:
    ("adjoint", t, "kept", i)   adjoint of step t with the moments in kept[i];
    ("recompute", a, b)         restore checkpoint a, recompute steps a+1..b,
                                moments of step s into segment slot s-a-1;
    ("adjoint", t, "seg", i)    adjoint of step t with segment slot i."""
    first_kept = nsteps - keep + 1
    plan, t = [], nsteps
    while t >= 1:
        if t >= first_kept:
            plan.append(("adjoint", t, "kept", t - first_kept))
            t -= 1
            continue
        a = ((t - 1) // ckpt_every) * ckpt_every     # the checkpoint segment (a, t]
        plan.append(("recompute", a, t))
        plan.extend(("adjoint", s, "seg", s - a - 1) for s in range(t, a, -1))
        t = a
    return plan


class Rollout:
    """Forward/backward driver with checkpointing (one GPU)."""

    def __init__(self, cfg: RolloutConfig, device="cuda"):
        self.cfg = c = cfg
        self.device = torch.device(device)
        self.params = abi.make_params(c.lx, c.lz, c.tau, c.g,
                                      abi.F64 if c.precision == "f64" else abi.F32_DEV,
                                      (abi.ADJ_F32 if c.adj_precision == "f32" else 0)
                                      | (abi.MOM_F32 if c.mom_precision == "f32" else 0)
                                      | (abi.COLLIDE_F64 if c.collide_f64 else 0)
                                      | abi.wall_flag(c.wall))
        self.ldtype = torch.float32 if c.adj_precision == "f32" else torch.float64
        self.desc = abi.RT3Desc(c.t_d, c.t_m, c.t_u, c.width, c.k, c.phase)
        self.sdtype = torch.float64 if c.precision == "f64" else torch.float32
        self.buf = [abi.empty_populations(self.params, self.sdtype, self.device) for _ in range(2)]
        self.ghost = torch.empty((2, 3, abi.Q), dtype=self.sdtype, device=self.device)
        self.scratch = torch.empty(max(abi.lbm_scratch_bytes(self.params), 256), dtype=torch.uint8,
                                   device=self.device)
        mdtype = torch.float32 if c.mom_precision == "f32" else torch.float64
        mbytes = 4 * c.lx * c.lz * (4 if c.mom_precision == "f32" else 8)
        self.keep = int(min(c.nsteps, c.moment_budget_bytes // mbytes))
        self.first_kept = c.nsteps - self.keep + 1          # steps >= this keep their moments
        self.kept = torch.empty((self.keep, 4, c.lx, c.lz), dtype=mdtype, device=self.device)
        self.ckpt_every = c.ckpt_every if c.ckpt_every > 0 else (self.keep if self.keep > 0 else 100)
        if self.keep >= c.nsteps:
            self.segbuf = self.kept[:0]
        elif self.keep >= self.ckpt_every:
            self.segbuf = self.kept[:self.ckpt_every]       # reused once the sweep has passed it
        else:
            self.segbuf = torch.empty((self.ckpt_every, 4, c.lx, c.lz), dtype=mdtype, device=self.device)
        if c.adjoint_form not in ("gather", "push", "auto"):
            raise ValueError(f"unknown adjoint form {c.adjoint_form!r}")
        self.form = "gather" if c.adjoint_form == "auto" else c.adjoint_form
        p = self.params
        self.params_stream = abi.make_params(c.lx, c.lz, c.tau, c.g, p.precision, p.flags | abi.NO_COLLIDE)
        self.ckpt = {}
        self.recomputed_steps = 0

    # ---- forward ----------------------------------------------------------
    def _step(self, src, dst, mom=None):
        abi.lbm_step(self.params, self.ghost, src, dst, mom)

    def _save(self, t, state):
        # checkpoint slots are allocated by the first forward pass and reused
        if t not in self.ckpt:
            self.ckpt[t] = torch.empty_like(state)
        self.ckpt[t].copy_(state)

    def _mom_slot(self, t):
        return self.kept[t - self.first_kept] if t >= self.first_kept else None

    def forward(self, amp):
        c = self.cfg
        self.amp = amp.detach().to(self.device, torch.float64).contiguous()
        abi.lbm_init_rt3(self.params, self.desc, self.amp, self.buf[0], self.ghost)
        cur = 0
        saves = set(checkpoint_steps(c.nsteps, self.keep, self.ckpt_every))
        self._save(0, self.buf[0])
        for t in range(1, c.nsteps + 1):
            self._step(self.buf[cur], self.buf[1 - cur], self._mom_slot(t))
            cur = 1 - cur
            if t in saves:
                self._save(t, self.buf[cur])
        self.final = self.buf[cur]
        self.j = torch.empty(5, dtype=torch.float64, device=self.device)
        self.lam = [abi.empty_populations(self.params, self.ldtype, self.device) for _ in range(2)]
        abi.lbm_objective(self.params, self.desc, self.final, c.wk, c.wl, self.j, self.lam[0],
                          self.scratch)
        return self.j

    # ---- backward ---------------------------------------------------------
    def backward(self):
        """dJ/d amp [2, nmodes] (device float64)."""
        c = self.cfg
        li = 0
        for op in backward_plan(c.nsteps, self.keep, self.ckpt_every):
            if op[0] == "recompute":
                _, a, b = op
                self.buf[0].copy_(self.ckpt[a])
                cur = 0
                for s in range(a + 1, b + 1):
                    self._step(self.buf[cur], self.buf[1 - cur], self.segbuf[s - a - 1])
                    cur = 1 - cur
                self.recomputed_steps += b - a
                continue
            _, t, where, i = op
            mom = self.kept[i] if where == "kept" else self.segbuf[i]
            src, dst = self.lam[li], self.lam[1 - li]
            if self.form == "push":
                # lam_{t-1} = S^T C_t^T lam_t
                abi.lbm_adjoint_step(self.params, self.ghost, mom, src, dst)
            elif t == c.nsteps:
                # mu_N = C_N^T lam_N
                abi.lbm_adjoint_collide(self.params, mom, src, dst)
            else:
                # mu_t = C_t^T S^T mu_{t+1}
                abi.lbm_adjoint_gather(self.params, self.ghost, mom, src, dst)
            li = 1 - li
        if self.form == "gather" and c.nsteps > 0:
            # lam_0 = S^T mu_1
            abi.lbm_adjoint_gather(self.params_stream, self.ghost, None, self.lam[li], self.lam[1 - li])
            li = 1 - li
        d_amp = torch.empty_like(self.amp)
        abi.lbm_init_rt3_vjp(self.params, self.desc, self.amp, self.lam[li], d_amp, self.scratch)
        return d_amp


class RTRollout(torch.autograd.Function):
    """J = RTRollout.apply(amp, rollout): autograd entry point; the backward
    pass returns grad_J * dJ/d amp from the HIP adjoint."""

    @staticmethod
    def forward(ctx, amp, rollout):
        ctx.rollout = rollout
        return rollout.forward(amp)[0].clone()

    @staticmethod
    def backward(ctx, grad):
        d_amp = ctx.rollout.backward()
        return grad * d_amp, None
