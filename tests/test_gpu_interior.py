"""GPU parity through the branch-free interior tiles, against the oracle.

The step kernel gives a tile the branch-free (interior) code only when none
of its rows pulls from within 3 rows of a wall or of the lattice end: tile
rows [z0, z0 + BS) with z0 >= 3 and z0 + BS + 3 <= Lz, BS = 512 rows in both
precisions.  The adjoint kernels' blocks are 256 rows (push form and gather
form).  So interior tiles need Lz >= 1027 (step) and Lz >= 515 (adjoint);
every large lattice spends almost all of its time in them.  These tests
take shapes with several interior tiles and a ragged tail:

* streaming (LBM_NO_COLLIDE), walled and periodic, both precisions: bit-exact
  (a pure permutation, Sec. III.B propagate);
* the FP64 step (Sec. III.A eq. LBE), 1 and 100 steps: 1e-12 relative;
* the FP32 deviation step against the FP64 oracle: the bound derived in
  test_gpu_f32 (5e-7 per step, linear growth);
* the adjoint step in every mode, with double, float and all-float buffers:
  1e-12 of the largest entry (double), the float bounds of test_gpu_adjoint.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as A
from oracle import lbm as O
from oracle.lattice import lattice
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


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _rel_max(got, want):
    return float(np.abs(got - want).max() / np.abs(want).max())


def interior_tiles(lz, bs):
    """Tile origins that take the branch-free path (the kernels' own test)."""
    return [z0 for z0 in range(0, lz, bs) if z0 >= 3 and z0 + bs + 3 <= lz]


def test_shapes_reach_interior_tiles():
    # the shapes below must exercise the interior path of every kernel
    assert interior_tiles(1100, 512) == [512]
    assert interior_tiles(2051, 512) == [512, 1024, 1536]
    assert interior_tiles(2560, 512) == [512, 1024, 1536]
    assert len(interior_tiles(1100, 256)) == 3 and len(interior_tiles(777, 256)) == 2
    assert interior_tiles(1040, 256) == [256, 512, 768] and interior_tiles(515, 256) == [256]


# ---------------------------------------------------------------------------
# streaming: bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lx,lz", [(9, 1100), (7, 2051), (3, 515)])
@pytest.mark.parametrize("prec", ["f64", "f32dev"])
@pytest.mark.parametrize("periodic", [False, True])
def test_propagate_bit_exact_interior(abi, lx, lz, prec, periodic):
    np_dt = np.float64 if prec == "f64" else np.float32
    f = W.random_populations(300 + lx, lx, lz).astype(np_dt)
    ghost = W.random_ghost(400 + lz).astype(np_dt)
    flags = abi.NO_COLLIDE | (abi.PERIODIC_Z if periodic else 0)
    params = abi.make_params(lx, lz, 0.7, 1e-4, abi.F64 if prec == "f64" else abi.F32_DEV, flags)
    fin = abi.to_tiled(params, f)
    fout = torch.full_like(fin, float("nan"))
    abi.lbm_step(params, _t(ghost), fin, fout)
    torch.cuda.synchronize()
    want = O.pull(f, ghost, O.Params(lx, lz, 0.7, 1e-4, periodic_z=periodic, no_collide=True))
    assert np.array_equal(abi.to_soa(params, fout).cpu().numpy(), want)


# ---------------------------------------------------------------------------
# FP64 and FP32 steps: 1 and 100 steps
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def interior_run():
    """Oracle trajectory of a 24 x 2560 three-layer lattice (three interior
    FP64 tiles per column, eight FP32 ones): steps 0, 1, 100."""
    lx, lz, tau, g = 24, 2560, 0.7, 1.5e-5
    m = W.draw_modes(2560, 8)
    p = O.Params(lx, lz, tau, g)
    desc = O.RT3(1.05, 1.0, 0.95, 4.0, m.k, m.phase)
    f0, ghost = O.init_rt3(p, desc, m.amp * 4)
    f1 = O.step(f0, ghost, p)
    f100 = O.run(f1, ghost, p, 99)
    return m, p, f0, ghost, f1, f100


def _gpu_run(abi, p, m, prec, steps, flags=0):
    dt = torch.float64 if prec == "f64" else torch.float32
    params = abi.make_params(p.lx, p.lz, p.tau, p.g, abi.F64 if prec == "f64" else abi.F32_DEV, flags)
    fa = abi.empty_populations(params, dt)
    gh = torch.empty((2, 3, 37), dtype=dt, device=DEV)
    abi.lbm_init_rt3(params, abi.RT3Desc(1.05, 1.0, 0.95, 4.0, m.k, m.phase), _t(m.amp * 4), fa, gh)
    fb = torch.empty_like(fa)
    out = []
    for s in range(1, steps + 1):
        abi.lbm_step(params, gh, fa, fb)
        fa, fb = fb, fa
        if s in (1, steps):
            out.append(abi.to_soa(params, fa).double().cpu().numpy())
    return out


def _full(f):
    # FP32 deviation storage holds f_l - w_l
    return f + lattice()[2][:, None, None]


def test_step_parity_f64_interior_1_and_100_steps(abi, interior_run):
    m, p, _, _, f1, f100 = interior_run
    got1, got100 = _gpu_run(abi, p, m, "f64", 100)
    e1, e100 = _rel(got1, f1), _rel(got100, f100)
    print(f"FP64 24x2560 max rel err: 1 step {e1:.3e}, 100 steps {e100:.3e}")
    assert e1 <= 1e-12 and e100 <= 1e-12


def test_step_parity_f32dev_interior_1_and_100_steps(abi, interior_run):
    m, p, _, _, f1, f100 = interior_run
    got1, got100 = _gpu_run(abi, p, m, "f32dev", 100)
    e1, e100 = _rel(_full(got1), f1), _rel(_full(got100), f100)
    print(f"FP32-dev 24x2560 max rel err vs FP64 oracle: 1 step {e1:.3e}, 100 steps {e100:.3e}")
    assert e1 <= 5e-7 and e100 <= 100 * 3e-7


# ---------------------------------------------------------------------------
# adjoint step: every mode, interior 256-row tiles
# ---------------------------------------------------------------------------
def _adj_state(lx, lz, tau, g, seed, periodic=False):
    m = W.draw_modes(seed, 6)
    p = O.Params(lx, lz, tau, g, periodic_z=periodic)
    desc = O.RT3(1.05, 1.0, 0.95, 3.0, m.k, m.phase)
    f0, ghost = O.init_rt3(O.Params(lx, lz, tau, g), desc, m.amp * 2)
    return p, O.run(f0, ghost, p, 3), ghost


MODES = ["walls", "periodic", "nocollide", "diffuse", "diffuse_nocollide"]


def _adj_case(abi, lx, lz, mode, seed):
    p, f, ghost = _adj_state(lx, lz, 0.7, 2e-3, seed, periodic=(mode == "periodic"))
    p.no_collide = mode.endswith("nocollide")
    p.wall = "diffuse" if mode.startswith("diffuse") else "dirichlet"
    flags = ((abi.PERIODIC_Z if p.periodic_z else 0) | (abi.NO_COLLIDE if p.no_collide else 0)
             | abi.wall_flag(p.wall))
    return p, f, ghost, flags


@pytest.mark.parametrize("lx,lz", [(16, 1040), (5, 777)])
@pytest.mark.parametrize("mode", MODES)
def test_adjoint_step_parity_interior(abi, lx, lz, mode):
    p, f, ghost, flags = _adj_case(abi, lx, lz, mode, 11 * lx + lz)
    lam = np.random.default_rng(lx + 7 * lz).standard_normal((37, lx, lz))
    want = A.step_vjp(lam, f, ghost, p)
    params = abi.make_params(lx, lz, p.tau, p.g, flags=flags)
    fin, gh = abi.to_tiled(params, f), _t(ghost)
    mom = torch.empty((4, lx, lz), dtype=torch.float64, device=DEV)
    abi.lbm_step(params, gh, fin, torch.empty_like(fin), mom)
    lam_out = torch.full_like(fin, float("nan"))
    abi.lbm_adjoint_step(params, gh, mom, abi.to_tiled(params, lam), lam_out)
    got = abi.to_soa(params, lam_out).cpu().numpy()
    assert np.isfinite(got).all()
    err = _rel_max(got, want)
    print(f"adjoint {mode} {lx}x{lz}: {err:.2e} of max")
    assert err <= 1e-12


@pytest.mark.parametrize("lx,lz", [(16, 1040), (5, 777)])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("form", ["float_buffers", "float_moments", "all_float"])
def test_adjoint_step_float_forms_interior(abi, lx, lz, mode, form):
    """Float adjoint buffers (double arithmetic): 2^-23 of the largest entry
    (3 x 2^-24 with the diffuse wall's extra rounding of parked values).
    Float moments (double buffers): 1e-6 of the largest entry (the moments'
    float rounding, as in test_gpu_adjoint).  All-float: the float
    arithmetic within 32 float roundings of the largest entry of the
    double-arithmetic step on the same float inputs, and that plus 1e-6
    against the oracle."""
    p, f, ghost, flags = _adj_case(abi, lx, lz, mode, 13 * lx + lz)
    lam = np.random.default_rng(3 * lx + lz).standard_normal((37, lx, lz)).astype(np.float32)
    want = A.step_vjp(lam.astype(np.float64), f, ghost, p)
    pp = abi.make_params(lx, lz, p.tau, p.g)   # lattice shape for the layout conversions
    fin, gh = abi.to_tiled(pp, f), _t(ghost)
    mflags = abi.MOM_F32 if form != "float_buffers" else 0
    mdt = torch.float32 if mflags else torch.float64
    mom = torch.empty((4, lx, lz), dtype=mdt, device=DEV)
    abi.lbm_step(abi.make_params(lx, lz, p.tau, p.g, flags=flags | mflags), gh, fin, torch.empty_like(fin), mom)
    if form == "float_moments":
        out = abi.empty_populations(pp, torch.float64)
        abi.lbm_adjoint_step(abi.make_params(lx, lz, p.tau, p.g, flags=flags | mflags), gh, mom,
                             abi.to_tiled(pp, lam.astype(np.float64)), out)
        err = _rel_max(abi.to_soa(pp, out).cpu().numpy(), want)
        bound = 1e-6
    else:
        out = abi.empty_populations(pp, torch.float32)
        abi.lbm_adjoint_step(abi.make_params(lx, lz, p.tau, p.g, flags=flags | mflags | abi.ADJ_F32), gh, mom,
                             abi.to_tiled(pp, lam), out)
        got = abi.to_soa(pp, out).cpu().numpy().astype(np.float64)
        err = _rel_max(got, want)
        if form == "float_buffers":
            bound = 2.0 ** -23 if not mode.startswith("diffuse") else 3 * 2.0 ** -24
        else:
            ref = abi.empty_populations(pp, torch.float64)
            abi.lbm_adjoint_step(abi.make_params(lx, lz, p.tau, p.g, flags=flags | mflags), gh, mom,
                                 abi.to_tiled(pp, lam.astype(np.float64)), ref)
            arith = _rel_max(got, abi.to_soa(pp, ref).cpu().numpy())
            print(f"all-float {mode} {lx}x{lz}: float arithmetic {arith / 2.0 ** -24:.1f} roundings")
            assert arith <= 32 * 2.0 ** -24
            bound = 32 * 2.0 ** -24 + 1e-6
    assert np.isfinite(abi.to_soa(pp, out).cpu().numpy()).all()
    print(f"adjoint {form} {mode} {lx}x{lz}: {err:.2e} of max (bar {bound:.1e})")
    assert err <= bound
