"""The adjoint in gather form (lbm_adjoint_collide, lbm_adjoint_gather)
against the oracle's factors of the step's transpose: the collision
transpose C^T (collide_vjp, Sec. III.A eq. LBE) and the streaming
transpose S^T (pull_transpose: a gather y <- y + e_l, zero or the diffuse
wall's ghost-site sum beyond the walls).  Bars as for lbm_adjoint_step:
1e-12 of the largest entry in double; the float bounds of test_gpu_adjoint
otherwise.  A rollout in gather form gives the push form's gradient to
rounding.  Shapes include interior 256-row blocks (Lz >= 515) and ragged
tails."""
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


def _rel_max(got, want):
    return float(np.abs(got - want).max() / np.abs(want).max())


def _state(lx, lz, seed, periodic=False, tau=0.7, g=2e-3):
    m = W.draw_modes(seed, 6)
    p = O.Params(lx, lz, tau, g, periodic_z=periodic)
    desc = O.RT3(1.05, 1.0, 0.95, 3.0, m.k, m.phase)
    f0, ghost = O.init_rt3(O.Params(lx, lz, tau, g), desc, m.amp * 2)
    return p, O.run(f0, ghost, p, 3), ghost


MODES = ["walls", "periodic", "diffuse"]
SHAPES = [(16, 1040), (5, 777), (37, 300), (2, 3)]


def _case(abi, lx, lz, mode, seed):
    p, f, ghost = _state(lx, lz, seed, periodic=(mode == "periodic"))
    p.wall = "diffuse" if mode == "diffuse" else "dirichlet"
    flags = (abi.PERIODIC_Z if p.periodic_z else 0) | abi.wall_flag(p.wall)
    return p, f, ghost, flags


def _moments(abi, params, f, ghost, mflags=0):
    """The GPU step's pre-collision moments of the step from f."""
    lx, lz = params.lx, params.lz
    mp = abi.make_params(lx, lz, params.tau, params.g, params.precision, params.flags | mflags)
    fin = abi.to_tiled(mp, f)
    mom = torch.empty((4, lx, lz), dtype=torch.float32 if mflags else torch.float64, device=DEV)
    abi.lbm_step(mp, _t(ghost), fin, torch.empty_like(fin), mom)
    return mom


@pytest.mark.parametrize("lx,lz", SHAPES)
@pytest.mark.parametrize("mode", MODES)
def test_collide_and_gather_parity(abi, lx, lz, mode):
    p, f, ghost, flags = _case(abi, lx, lz, mode, 17 * lx + lz)
    params = abi.make_params(lx, lz, p.tau, p.g, flags=flags)
    mom = _moments(abi, params, f, ghost)
    g = O.pull(f, ghost, p)                            # the step's pre-collision populations
    rng = np.random.default_rng(lx + 3 * lz)
    lam = rng.standard_normal((37, lx, lz))
    mu = rng.standard_normal((37, lx, lz))
    # C^T alone
    out = abi.empty_populations(params, torch.float64)
    abi.lbm_adjoint_collide(params, mom, abi.to_tiled(params, lam), out)
    e_c = _rel_max(abi.to_soa(params, out).cpu().numpy(), A.collide_vjp(lam, g, p))
    # S^T alone (NO_COLLIDE)
    p_nc = abi.make_params(lx, lz, p.tau, p.g, flags=flags | abi.NO_COLLIDE)
    abi.lbm_adjoint_gather(p_nc, _t(ghost), None, abi.to_tiled(params, mu), out)
    st = A.pull_transpose(mu, p, ghost)
    got_s = abi.to_soa(params, out).cpu().numpy()
    inner = slice(3, max(lz - 3, 3))
    e_s = _rel_max(got_s, st)
    # C^T S^T
    abi.lbm_adjoint_gather(params, _t(ghost), mom, abi.to_tiled(params, mu), out)
    e_cs = _rel_max(abi.to_soa(params, out).cpu().numpy(), A.collide_vjp(st, g, p))
    print(f"{mode} {lx}x{lz}: C^T {e_c:.2e}, S^T {e_s:.2e}, C^T S^T {e_cs:.2e}")
    assert e_c <= 1e-12 and e_cs <= 1e-12
    # streaming alone is a permutation away from the walls, a plain sum at them
    assert np.array_equal(got_s[:, :, inner], st[:, :, inner]) and e_s <= 1e-14


@pytest.mark.parametrize("lx,lz", [(16, 1040), (37, 300)])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("form", ["float_buffers", "all_float"])
def test_gather_float_forms(abi, lx, lz, mode, form):
    """Float adjoint buffers (double arithmetic): 2^-23 of the largest entry
    (3 x 2^-24 with the diffuse wall's float-rounded ghost sums); all-float
    (float moments too): 32 float roundings plus 1e-6 (the moments' rounding)."""
    p, f, ghost, flags = _case(abi, lx, lz, mode, 29 * lx + lz)
    mflags = abi.MOM_F32 if form == "all_float" else 0
    params = abi.make_params(lx, lz, p.tau, p.g, flags=flags | mflags | abi.ADJ_F32)
    mom = _moments(abi, abi.make_params(lx, lz, p.tau, p.g, flags=flags), f, ghost, mflags)
    g = O.pull(f, ghost, p)
    mu = np.random.default_rng(5 * lx + lz).standard_normal((37, lx, lz)).astype(np.float32)
    want = A.collide_vjp(A.pull_transpose(mu.astype(np.float64), p, ghost), g, p)
    out = abi.empty_populations(params, torch.float32)
    abi.lbm_adjoint_gather(params, _t(ghost), mom, abi.to_tiled(params, mu), out)
    got = abi.to_soa(params, out).cpu().numpy().astype(np.float64)
    err = _rel_max(got, want)
    if form == "float_buffers":
        bound = 2.0 ** -23 if mode != "diffuse" else 3 * 2.0 ** -24
    else:
        bound = 32 * 2.0 ** -24 + 1e-6
    print(f"gather {form} {mode} {lx}x{lz}: {err:.2e} of max (bar {bound:.1e})")
    assert np.isfinite(got).all() and err <= bound


@pytest.mark.parametrize("wall", ["dirichlet", "diffuse"])
@pytest.mark.parametrize("prec,adj,mom", [("f64", "f64", "f64"), ("f32dev", "f32", "f32")])
def test_gather_rollout_equals_push_rollout(abi, wall, prec, adj, mom):
    """The gather chain regroups the same per-site arithmetic, so the
    gradient equals the push form's to rounding (the compiler may contract
    multiply-adds differently in the two kernels): 1e-12 of the largest
    entry in double, 1e-5 in the all-float form (128 x 384, 20 steps, with a
    recomputed checkpoint segment)."""
    from paper_1405_1253_amd.rollout import Rollout, RolloutConfig
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    mbytes = 4 * wl.lx * wl.lz * (4 if mom == "f32" else 8)
    grads = {}
    for form in ("gather", "push"):
        r = Rollout(RolloutConfig.from_workload(wl, m, nsteps=20, ckpt_every=7, moment_budget_bytes=5 * mbytes,
                                                wall=wall, precision=prec, adj_precision=adj, mom_precision=mom,
                                                adjoint_form=form))
        r.forward(torch.as_tensor(m.amp, device=DEV))
        grads[form] = r.backward().cpu().numpy()
        assert r.recomputed_steps == 15
    assert np.isfinite(grads["gather"]).all()
    err = _rel_max(grads["gather"], grads["push"])
    print(f"{prec}/{adj}/{mom} {wall}: gather vs push gradient {err:.2e} of max")
    assert err <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("wall", ["dirichlet", "diffuse"])
def test_gather_rollout_gradient_vs_oracle(abi, wall):
    """The gather chain's 20-step gradient at 128 x 384 (double) against the
    oracle's adjoint (pinned by complex step): 1e-10 of the largest entry."""
    from paper_1405_1253_amd.rollout import Rollout, RolloutConfig
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    _, g_o = A.rollout_gradient(O.Params(wl.lx, wl.lz, wl.tau, wl.g, wall=wall),
                                O.RT3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase), m.amp, 20)
    r = Rollout(RolloutConfig.from_workload(wl, m, nsteps=20, wall=wall, adjoint_form="gather"))
    assert r.form == "gather"
    r.forward(torch.as_tensor(m.amp, device=DEV))
    err = _rel_max(r.backward().cpu().numpy(), g_o)
    print(f"gather rollout ({wall}) vs oracle: {err:.2e} of max")
    assert err <= 1e-10
