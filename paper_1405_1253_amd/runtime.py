"""Lattice: device buffers and stream plumbing around the C entry points.

Population buffers are in the library's tiled layout; ``state_soa()``,
``populations()`` and ``set_state()`` convert from and to [37, Lx, Lz].

Owns the prv/nxt pair of population buffers (Sec. III.B) -- or, with
``inplace=True``, a single buffer stepped by lbm_step_inplace -- the wall
table and the diagnostics scratch, all as torch tensors on one GPU; every
computation is a call into liblbm.so on the current torch stream.
"""
import numpy as np
import torch

from . import abi
from .workload import Workload, draw_modes


class Lattice:
    def __init__(self, lx, lz, tau, g, precision="f64", flags=0, device="cuda", inplace=False):
        if precision not in ("f64", "f32dev"):
            raise ValueError(precision)
        self.lx, self.lz, self.tau, self.g = lx, lz, tau, g
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.params = abi.make_params(lx, lz, tau, g,
                                      abi.F64 if precision == "f64" else abi.F32_DEV, flags)
        self.device = torch.device(device)
        self.inplace = inplace
        self.buf = [abi.empty_populations(self.params, self.dtype, self.device)
                    for _ in range(1 if inplace else 2)]
        self.cur = 0
        self.kind = abi.INPLACE_FROM_STATE   # in place: what the buffer holds
        self.ghost = torch.zeros((2, 3, abi.Q), dtype=self.dtype, device=self.device)
        nbytes = max(abi.lbm_scratch_bytes(self.params), 256)
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.steps_done = 0

    # ---- construction -----------------------------------------------------
    @classmethod
    def from_workload(cls, wl: Workload, modes=None, amp=None, device="cuda", **kw):
        kw["flags"] = kw.get("flags", 0) | abi.wall_flag(wl.wall)
        kw.setdefault("inplace", wl.inplace)
        lat = cls(wl.lx, wl.lz, wl.tau, wl.g, precision=wl.precision, device=device, **kw)
        modes = modes if modes is not None else draw_modes(wl.seed)
        a = modes.amp if amp is None else amp
        lat.init_rt3(wl.t_d, wl.t_m, wl.t_u, wl.width, modes.k, modes.phase, a, wl.z_lo, wl.z_hi)
        if wl.t_m_diag is not None:
            lat.diag_desc = abi.RT3Desc(wl.t_d, wl.t_m_diag, wl.t_u, wl.width)
        return lat

    def init_rt3(self, t_d, t_m, t_u, width, k, phase, amp, z_lo=None, z_hi=None):
        if not torch.is_tensor(amp):
            amp = torch.as_tensor(np.asarray(amp, dtype=np.float64), device=self.device)
        amp = amp.to(device=self.device, dtype=torch.float64).contiguous()
        self.desc = abi.RT3Desc(t_d, t_m, t_u, width, k, phase, z_lo, z_hi)
        self.diag_desc = self.desc     # temperatures of the tent-map diagnostics
        abi.lbm_init_rt3(self.params, self.desc, amp, self.buf[0], self.ghost)
        self.cur = 0
        self.kind = abi.INPLACE_FROM_STATE
        self.steps_done = 0
        self._amp = amp   # keep alive until the stream has consumed it

    # ---- time stepping ----------------------------------------------------
    @property
    def state(self):
        """The post-collision state buffer (library's tiled layout)."""
        if self.kind != abi.INPLACE_FROM_STATE:
            raise RuntimeError("the single buffer holds the streamed form after an odd number of "
                               "in-place steps; step once more to get the post-collision state")
        return self.buf[self.cur]

    def state_soa(self):
        """The stored state in the plain layout [37, lx, lz], element type of
        the state (FP32 deviation storage: f - w); a bit-exact copy."""
        return abi.to_soa(self.params, self.state)

    def set_state(self, f):
        """Set the post-collision state from a plain-layout [37, lx, lz] array
        of the state's element type, or copy a tiled buffer of this lattice."""
        if tuple(f.shape) == (abi.Q, self.lx, self.lz):
            abi.lbm_pack(self.params, torch.as_tensor(f).to(self.device, self.dtype).contiguous(),
                         self.buf[self.cur])
        else:
            self.buf[self.cur].copy_(f)
        self.kind = abi.INPLACE_FROM_STATE

    def step(self, n=1, moments_out=None):
        """Advance n steps; moments_out (optional) receives the last step's
        pre-collision moments [4, lx, lz]."""
        for i in range(n):
            mo = moments_out if i == n - 1 else None
            if self.inplace:
                abi.lbm_step_inplace(self.params, self.ghost, self.buf[0], self.kind, mo, self.scratch)
                self.kind ^= 1
            else:
                abi.lbm_step(self.params, self.ghost, self.buf[self.cur], self.buf[1 - self.cur], mo)
                self.cur = 1 - self.cur
        self.steps_done += n

    # ---- placement ----------------------------------------------------------
    def tune_placement(self, trials=12, steps=12):
        """Re-allocate the population buffers and keep the allocation on
        which the step runs fastest.

        A step's rate depends on where its buffers land in physical memory,
        which the caller cannot choose: on MI355X at 4096 x 12288 (FP64) fresh
        allocations in one process ran at 4.9-5.4 ms per step, each stable to
        about 0.5 %.  This times ``steps`` steps (HIP events, after two
        warm-up steps) on the current buffers and on ``trials - 1`` fresh
        allocations, keeps the fastest and returns the state unchanged; the
        trial steps do not count as steps of the lattice.  Needs free device
        memory for one state copy and one more set of buffers, else returns
        None without doing anything.  Returns the ms per step of each trial,
        the current allocation's first."""
        nbuf = len(self.buf)
        nbytes = self.buf[0].numel() * self.buf[0].element_size()
        free, _ = torch.cuda.mem_get_info(self.device)
        if trials < 1 or free < (nbuf + 1) * nbytes + (1 << 30):
            return None
        saved = self.buf[self.cur].clone()      # the state (in place: the buffer as it is)
        stream = torch.cuda.current_stream(self.device)

        def run(bufs, n):
            for i in range(n):
                if self.inplace:
                    abi.lbm_step_inplace(self.params, self.ghost, bufs[0], (self.kind + i) % 2, None,
                                         self.scratch)
                else:
                    abi.lbm_step(self.params, self.ghost, bufs[i % 2], bufs[1 - i % 2])

        def time_on(bufs):
            bufs[0].copy_(saved)
            run(bufs, 2)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run(bufs, 2 * ((steps + 1) // 2))
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / (2 * ((steps + 1) // 2))

        best = time_on(self.buf)
        times = [round(best, 4)]
        for _ in range(trials - 1):
            cand = [abi.empty_populations(self.params, self.dtype, self.device) for _ in range(nbuf)]
            t = time_on(cand)
            times.append(round(t, 4))
            if t < best:
                best, self.buf = t, cand          # the previous buffers lose their last reference
            del cand
            torch.cuda.empty_cache()              # hand the loser's pages back before the next try
        self.buf[0].copy_(saved)
        self.cur = 0
        del saved
        torch.cuda.synchronize(self.device)
        torch.cuda.empty_cache()
        return times

    # ---- diagnostics ------------------------------------------------------
    def fields(self):
        out = torch.empty((4, self.lx, self.lz), dtype=torch.float64, device=self.device)
        abi.lbm_moments(self.params, self.state, fields=out, scratch=self.scratch)
        return out

    def tbar(self):
        out = torch.empty(self.lz, dtype=torch.float64, device=self.device)
        abi.lbm_moments(self.params, self.state, tbar=out, scratch=self.scratch)
        return out

    def profiles(self):
        """[4, Lz]: mean and rms fluctuation over x of T^H and of E_k."""
        out = torch.empty((4, self.lz), dtype=torch.float64, device=self.device)
        abi.lbm_profiles(self.params, self.state, out, self.scratch)
        return out

    def objective(self, wk=1.0, wl=1.0):
        """[5]: J = wk KE + wl (L_u + L_d), KE, L_u + L_d, L_u, L_d of the current state."""
        out = torch.empty(5, dtype=torch.float64, device=self.device)
        abi.lbm_objective(self.params, self.diag_desc, self.state, wk, wl, out, None, self.scratch)
        return out

    def sums(self, check=True):
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        abi.lbm_moments(self.params, self.state, sums=out, scratch=self.scratch)
        if check:
            host = out.cpu()
            if not torch.isfinite(host).all():
                raise FloatingPointError(f"non-finite global sums {host.tolist()}: state diverged")
        return out

    # ---- checkpoint / restore ---------------------------------------------
    def state_dict(self):
        """Everything needed to continue the run bitwise: state, wall table,
        parameters and step count (host tensors)."""
        return {"lx": self.lx, "lz": self.lz, "tau": self.tau, "g": self.g,
                "precision": self.precision, "flags": int(self.params.flags),
                "steps_done": self.steps_done, "state": self.state_soa().cpu(),
                "ghost": self.ghost.cpu()}

    def save(self, path):
        torch.save(self.state_dict(), path)

    @classmethod
    def from_state_dict(cls, d, device="cuda"):
        lat = cls(d["lx"], d["lz"], d["tau"], d["g"], precision=d["precision"],
                  flags=d["flags"], device=device)
        lat.cur = 0
        lat.set_state(d["state"])
        lat.ghost.copy_(d["ghost"])
        lat.steps_done = d["steps_done"]
        return lat

    @classmethod
    def load(cls, path, device="cuda"):
        return cls.from_state_dict(torch.load(path, weights_only=True), device=device)

    def populations(self):
        """Full populations f_l as float64, plain layout [37, lx, lz] (adds the
        weights back in FP32 mode)."""
        f = self.state_soa().to(torch.float64)
        if self.precision == "f32dev":
            _, w, _ = abi.lbm_lattice()
            f = f + torch.as_tensor(w, device=self.device)[:, None, None]
        return f
