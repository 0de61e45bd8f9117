"""GPU adjoint against the oracle's hand-written adjoint and against finite
differences of the GPU forward path.

Bars: adjoint step, objective seed and init VJP within 1e-12 of the oracle
(relative to the largest entry); the N-step gradient at 128 x 384 within
1e-10 of the oracle; the 512 x 1536, 2000-step gradient within 1e-6 of
central finite differences (h = 1e-6) on 8 seeded modes.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as A
from oracle import lbm as O
from paper_1405_1253_amd import workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def abi():
    from paper_1405_1253_amd import abi as mod
    mod.load()
    return mod


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _pop(abi, a):
    """Plain-layout [37, lx, lz] array -> tiled device buffer."""
    return abi.to_tiled(abi.make_params(a.shape[1], a.shape[2], 0.7, 0.0), a)


def _np(abi, lx, lz, t):
    """Tiled device buffer -> plain-layout [37, lx, lz] numpy array."""
    return abi.to_soa(abi.make_params(lx, lz, 0.7, 0.0), t).cpu().numpy()


def _rel_max(got, want):
    return float(np.abs(got - want).max() / np.abs(want).max())


def _state(lx, lz, tau, g, seed, steps=3, periodic=False):
    m = W.draw_modes(seed, 6)
    p = O.Params(lx, lz, tau, g, periodic_z=periodic)
    desc = O.RT3(1.05, 1.0, 0.95, 3.0, m.k, m.phase)
    f0, ghost = O.init_rt3(O.Params(lx, lz, tau, g), desc, m.amp * 2)
    return p, O.run(f0, ghost, p, steps), ghost


@pytest.mark.parametrize("lx,lz", [(128, 384), (37, 300), (5, 7), (2, 3)])
@pytest.mark.parametrize("mode", ["walls", "periodic", "nocollide", "diffuse", "diffuse_nocollide"])
def test_adjoint_step_parity(abi, lx, lz, mode):
    p, f, ghost = _state(lx, lz, 0.7, 2e-3, lx + lz, periodic=(mode == "periodic"))
    p.no_collide = mode.endswith("nocollide")
    p.wall = "diffuse" if mode.startswith("diffuse") else "dirichlet"
    lam = np.random.default_rng(lx * lz).standard_normal((37, lx, lz))
    want = A.step_vjp(lam, f, ghost, p)
    flags = ((abi.PERIODIC_Z if p.periodic_z else 0) | (abi.NO_COLLIDE if p.no_collide else 0)
             | abi.wall_flag(p.wall))
    params = abi.make_params(lx, lz, p.tau, p.g, flags=flags)
    fin, gh = _pop(abi, f), _t(ghost)
    fout = torch.empty_like(fin)
    mom = torch.empty((4, lx, lz), dtype=torch.float64, device=DEV)
    abi.lbm_step(params, gh, fin, fout, mom)
    lam_out = torch.full_like(fin, float("nan"))
    abi.lbm_adjoint_step(params, gh, mom, _pop(abi, lam), lam_out)
    got = _np(abi, lx, lz, lam_out)
    assert np.isfinite(got).all()
    assert _rel_max(got, want) <= 1e-12


def test_objective_and_seed_parity(abi):
    lx, lz = 64, 192
    p, f, _ = _state(lx, lz, 0.7, 1e-3, 3, steps=5)
    desc = abi.RT3Desc(1.05, 1.0, 0.95, 3.0)
    params = abi.make_params(lx, lz, p.tau, p.g)
    j = torch.empty(5, dtype=torch.float64, device=DEV)
    seed = abi.empty_populations(params, torch.float64)
    scratch = torch.empty(abi.lbm_scratch_bytes(params), dtype=torch.uint8, device=DEV)
    abi.lbm_objective(params, desc, _pop(abi, f), 2.0, 0.5, j, seed, scratch)
    Jo, ke, L = O.objective(f, p, 0.95, 1.0, 1.05, 2.0, 0.5)
    got = j.cpu().numpy()
    assert L > 1.0 and ke > 0.0
    assert abs(got[0] / Jo - 1) <= 1e-12 and abs(got[1] / ke - 1) <= 1e-12 and abs(got[2] / L - 1) <= 1e-12
    Lu, Ld = O.mixing_lengths(O.tbar(O.hydro_fields(f, p)[2]), 0.95, 1.0, 1.05)
    assert Lu > 0.5 and Ld > 0.5
    assert abs(got[3] / Lu - 1) <= 1e-12 and abs(got[4] / Ld - 1) <= 1e-12
    want = A.objective_vjp(f, p, 0.95, 1.0, 1.05, 2.0, 0.5)
    assert _rel_max(_np(abi, lx, lz, seed), want) <= 1e-12


def test_init_vjp_parity(abi):
    for lx, lz, nm in ((48, 150, 16), (7, 30, 3)):
        m = W.draw_modes(lx, nm)
        p = O.Params(lx, lz, 0.7, 1e-3)
        desc = O.RT3(1.05, 1.0, 0.95, 4.0, m.k, m.phase)
        lam = np.random.default_rng(lz).standard_normal((37, lx, lz))
        want = A.init_vjp(lam, p, desc, m.amp)
        params = abi.make_params(lx, lz, p.tau, p.g)
        d_amp = torch.empty((2, nm), dtype=torch.float64, device=DEV)
        scratch = torch.empty(abi.lbm_scratch_bytes(params), dtype=torch.uint8, device=DEV)
        abi.lbm_init_rt3_vjp(params, abi.RT3Desc(1.05, 1.0, 0.95, 4.0, m.k, m.phase), _t(m.amp),
                             _pop(abi, lam), d_amp, scratch)
        assert _rel_max(d_amp.cpu().numpy(), want) <= 1e-12, (lx, lz)


def _rollout(wl, modes, nsteps, **kw):
    from paper_1405_1253_amd.rollout import Rollout, RolloutConfig
    return Rollout(RolloutConfig.from_workload(wl, modes, nsteps=nsteps, **kw))


@pytest.mark.parametrize("wall", ["dirichlet", "diffuse"])
def test_rollout_gradient_vs_oracle_128x384(abi, wall):
    from paper_1405_1253_amd.rollout import RTRollout
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    n = 20
    J_o, g_o = A.rollout_gradient(O.Params(wl.lx, wl.lz, wl.tau, wl.g, wall=wall),
                                  O.RT3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase), m.amp, n)
    amp = torch.tensor(m.amp, device=DEV, requires_grad=True)
    J = RTRollout.apply(amp, _rollout(wl, m, n, wall=wall))
    J.backward()
    got = amp.grad.cpu().numpy()
    print(f"J gpu {J.item():.15e} oracle {J_o:.15e}; grad rel err {_rel_max(got, g_o):.2e}")
    assert abs(J.item() / J_o - 1) <= 1e-12
    assert _rel_max(got, g_o) <= 1e-10
    # recomputing from checkpoints gives the bitwise same gradient
    r2 = _rollout(wl, m, n, ckpt_every=7, moment_budget_bytes=3 * 4 * wl.lx * wl.lz * 8, wall=wall)
    r2.forward(torch.as_tensor(m.amp, device=DEV))
    g2 = r2.backward().cpu().numpy()
    assert r2.recomputed_steps == n - 3
    assert np.array_equal(g2, got)


def test_rollout_with_the_double_collision(abi):
    """RolloutConfig(collide_f64=True) on an FP32-dev state (float adjoint
    buffers and moments): the forward steps and the recomputed ones take the
    same kernel, so recomputing from checkpoints gives the bitwise same
    gradient; J lies closer to the all-FP64 rollout's than with the float
    collision, and the gradient within the float forms' bar of 1e-3 of its
    largest entry (128 x 384, 20 steps)."""
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    amp = torch.as_tensor(m.amp, device=DEV)
    kw = dict(precision="f32dev", adj_precision="f32", mom_precision="f32")
    res = {}
    for key, extra in (("f64", dict()), ("f32", kw), ("c64", dict(kw, collide_f64=True)),
                       ("c64_recompute", dict(kw, collide_f64=True, ckpt_every=7,
                                              moment_budget_bytes=3 * 4 * wl.lx * wl.lz * 4))):
        r = _rollout(wl, m, 20, **extra)
        J = r.forward(amp)[0].item()
        res[key] = (J, r.backward().cpu().numpy(), r.recomputed_steps)
    (J64, g64, _), (J32, g32, _) = res["f64"], res["f32"]
    (Jc, gc, _), (Jr, gr, nr) = res["c64"], res["c64_recompute"]
    assert nr == 17 and Jr == Jc and np.array_equal(gr, gc)
    e32, ec = _rel_max(g32, g64), _rel_max(gc, g64)
    print(f"vs FP64: J {abs(J32 / J64 - 1):.2e} / {abs(Jc / J64 - 1):.2e}, gradient {e32:.2e} / {ec:.2e} "
          "(float / double collision)")
    assert abs(Jc / J64 - 1) <= abs(J32 / J64 - 1) and ec <= 1e-3


@pytest.mark.parametrize("name", ["rt3_512x1536_adj", "rt3_512x1536_adj_diffuse"])
def test_gradient_vs_finite_differences_512x1536(abi, name):
    """Central differences of the GPU forward at h = 1e-6 carry a rounding
    noise of about |dJ_noise| / (2h) with |dJ_noise| ~ 1e-12 (J ~ 30 after
    2000 steps of sums over 786k sites): the bar at h = 1e-6 is an absolute
    1e-6.  Larger h lowers that noise until the h^2 truncation takes over;
    at h = 1e-4 the adjoint must agree to 1e-6 relative to the largest
    gradient, showing that the remaining difference is the FD's own."""
    wl = W.WORKLOADS[name]
    m = W.draw_modes(wl.seed)
    r = _rollout(wl, m, wl.steps)
    amp0 = torch.as_tensor(m.amp, device=DEV)
    J0 = r.forward(amp0)[0].item()
    grad = r.backward().cpu().numpy().ravel()
    idx = W.fd_mode_indices()

    def fd(h):
        out = []
        for i in idx:
            Js = []
            for s in (1.0, -1.0):
                a = m.amp.copy().ravel()
                a[i] += s * h
                Js.append(r.forward(torch.as_tensor(a.reshape(2, -1), device=DEV))[0].item())
            out.append((Js[0] - Js[1]) / (2 * h))
        return np.array(out)

    errs = {}
    for h in (1e-6, 1e-5, 1e-4, 1e-3):
        d = fd(h)
        errs[h] = np.abs(grad[idx] - d)
        print(f"h={h:.0e}: max abs err {errs[h].max():.2e}, max err / max|grad| "
              f"{errs[h].max() / np.abs(d).max():.2e}")
    print(f"J = {J0:.12e}; adjoint dJ/damp at modes {idx.tolist()}: {grad[idx]}")
    gmax = np.abs(grad[idx]).max()
    assert errs[1e-6].max() <= 1e-6
    assert errs[1e-4].max() <= 1e-6 * gmax


@pytest.mark.parametrize("wall", ["dirichlet", "diffuse"])
def test_adjoint_step_float_buffers(abi, wall):
    """LBM_ADJ_F32: float adjoint buffers, double arithmetic.  Against the
    oracle fed the same float-rounded input, the only extra error is the
    final rounding to float: <= 2^-24 relative to each entry, bounded here
    by 2^-23 of the largest entry.  The diffuse wall's parked values are
    rounded to float once more before the wall pass sums them: at most
    another 2^-24 of the largest entry."""
    lx, lz = 128, 384
    p, f, ghost = _state(lx, lz, 0.7, 2e-3, 9)
    p.wall = wall
    lam = np.random.default_rng(8).standard_normal((37, lx, lz)).astype(np.float32)
    want = A.step_vjp(lam.astype(np.float64), f, ghost, p)
    params = abi.make_params(lx, lz, p.tau, p.g, flags=abi.ADJ_F32 | abi.wall_flag(wall))
    fout = abi.empty_populations(params, torch.float64)
    mom = torch.empty((4, lx, lz), dtype=torch.float64, device=DEV)
    gh = _t(ghost)
    abi.lbm_step(params, gh, _pop(abi, f), fout, mom)
    out = abi.empty_populations(params, torch.float32)
    abi.lbm_adjoint_step(params, gh, mom, _pop(abi, lam), out)
    assert _rel_max(_np(abi, lx, lz, out).astype(np.float64), want) <= (2.0 ** -23 if wall == "dirichlet"
                                                                   else 3 * 2.0 ** -24)


def test_gradient_float_storage_and_adjoint_vs_f64(abi):
    """Gradient error of the FP32 forms (the all-float adjoint among them)
    against the all-FP64 gradient, 128 x 384, 100 steps (stated; bar 1e-3
    relative to the largest entry)."""
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    amp = torch.as_tensor(m.amp, device=DEV)
    out = {}
    for prec, adj, mom in (("f64", "f64", "f64"), ("f64", "f32", "f64"), ("f32dev", "f64", "f64"),
                           ("f32dev", "f32", "f64"), ("f32dev", "f32", "f32")):
        r = _rollout(wl, m, wl.steps, precision=prec, adj_precision=adj, mom_precision=mom)
        J = r.forward(amp)[0].item()
        out[prec, adj, mom] = (J, r.backward().cpu().numpy())
    J64, g64 = out["f64", "f64", "f64"]
    for key, (J, g) in out.items():
        err = _rel_max(g, g64)
        print(f"state {key[0]}, adjoint {key[1]}, moments {key[2]}: J rel err {abs(J / J64 - 1):.2e}, "
              f"grad max err / max|grad| {err:.2e}")
        assert err <= 1e-3


def test_float_moments(abi):
    """LBM_MOM_F32: lbm_step writes the moments rounded to float (bit for bit
    the double moments' rounding); the adjoint step reading them differs from
    the one reading double moments by the effect of that rounding, bounded
    here by 1e-6 of the largest entry (the float rounding is 6e-8 relative)."""
    lx, lz = 128, 384
    p, f, ghost = _state(lx, lz, 0.7, 2e-3, 21)
    lam = np.random.default_rng(22).standard_normal((37, lx, lz))
    fin, gh = _pop(abi, f), _t(ghost)
    fout = torch.empty_like(fin)
    m64 = torch.empty((4, lx, lz), dtype=torch.float64, device=DEV)
    m32 = torch.empty((4, lx, lz), dtype=torch.float32, device=DEV)
    p64 = abi.make_params(lx, lz, p.tau, p.g)
    p32 = abi.make_params(lx, lz, p.tau, p.g, flags=abi.MOM_F32)
    abi.lbm_step(p64, gh, fin, fout, m64)
    abi.lbm_step(p32, gh, fin, fout, m32)
    assert torch.equal(m32, m64.float())
    out64 = torch.empty_like(fin)
    out32 = torch.empty_like(fin)
    abi.lbm_adjoint_step(p64, gh, m64, _pop(abi, lam), out64)
    abi.lbm_adjoint_step(p32, gh, m32, _pop(abi, lam), out32)
    err = _rel_max(_np(abi, lx, lz, out32), _np(abi, lx, lz, out64))
    print(f"adjoint step with float moments: {err:.2e} of max")
    assert err <= 1e-6


@pytest.mark.parametrize("wall", ["dirichlet", "diffuse"])
def test_adjoint_step_all_float(abi, wall):
    """LBM_ADJ_F32 | LBM_MOM_F32: float buffers, float moments, and float
    arithmetic for the 15 per-site sums and the outputs G.  The arithmetic
    alone, against the double-arithmetic step on the same float inputs
    (double lam holding the float values, the same float moments): bounded
    by 32 float roundings of the largest entry (the sums accumulate 18 pair
    terms rounded about three times each; G adds four roundings).  Against
    the oracle: that bound plus the float moments' effect (1e-6 of the
    largest entry, as in test_float_moments)."""
    lx, lz = 128, 384
    p, f, ghost = _state(lx, lz, 0.7, 2e-3, 23)
    p.wall = wall
    lam = np.random.default_rng(24).standard_normal((37, lx, lz)).astype(np.float32)
    want = A.step_vjp(lam.astype(np.float64), f, ghost, p)
    flags = abi.MOM_F32 | abi.wall_flag(wall)
    fin, gh = _pop(abi, f), _t(ghost)
    fout = torch.empty_like(fin)
    m32 = torch.empty((4, lx, lz), dtype=torch.float32, device=DEV)
    abi.lbm_step(abi.make_params(lx, lz, p.tau, p.g, flags=flags), gh, fin, fout, m32)
    out_f = abi.empty_populations(abi.make_params(lx, lz, p.tau, p.g), torch.float32)
    abi.lbm_adjoint_step(abi.make_params(lx, lz, p.tau, p.g, flags=flags | abi.ADJ_F32), gh, m32, _pop(abi, lam),
                         out_f)
    out_d = abi.empty_populations(abi.make_params(lx, lz, p.tau, p.g), torch.float64)
    abi.lbm_adjoint_step(abi.make_params(lx, lz, p.tau, p.g, flags=flags), gh, m32,
                         _pop(abi, lam.astype(np.float64)), out_d)
    got = _np(abi, lx, lz, out_f).astype(np.float64)
    arith = _rel_max(got, _np(abi, lx, lz, out_d))
    err = _rel_max(got, want)
    print(f"all-float adjoint step ({wall}): float arithmetic {arith:.2e} of max "
          f"({arith / 2.0 ** -24:.1f} roundings), vs oracle {err:.2e}")
    assert arith <= 32 * 2.0 ** -24
    assert err <= 32 * 2.0 ** -24 + 1e-6


def test_rollout_float_moments_vs_oracle(abi):
    """20-step gradient at 128 x 384 with float moments (and the segment
    buffer inside the kept buffer: keep 10, checkpoints every 5) against the
    oracle adjoint: 1e-5 of the largest entry."""
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    n = 20
    _, g_o = A.rollout_gradient(O.Params(wl.lx, wl.lz, wl.tau, wl.g),
                                O.RT3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase), m.amp, n)
    r = _rollout(wl, m, n, mom_precision="f32", ckpt_every=5, moment_budget_bytes=10 * 4 * wl.lx * wl.lz * 4)
    assert r.keep == 10 and r.segbuf.data_ptr() == r.kept.data_ptr()
    r.forward(torch.as_tensor(m.amp, device=DEV))
    got = r.backward().cpu().numpy()
    err = _rel_max(got, g_o)
    print(f"float moments: gradient {err:.2e} of max; recomputed {r.recomputed_steps}")
    assert r.recomputed_steps == 10
    assert err <= 1e-5
    # checkpoint interval = kept steps (ckpt_every = 0): the same gradient
    r0 = _rollout(wl, m, n, mom_precision="f32", ckpt_every=0, moment_budget_bytes=10 * 4 * wl.lx * wl.lz * 4)
    assert r0.ckpt_every == 10
    r0.forward(torch.as_tensor(m.amp, device=DEV))
    assert np.array_equal(r0.backward().cpu().numpy(), got)
