"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars:
* streaming (LBM_NO_COLLIDE) and the wall table: bit-exact, both precisions;
* FP64 init and step: max |f_gpu - f_oracle| / f_oracle <= 1e-12 after 1 and
  after 100 steps (the oracle evaluates the equilibrium as a tensor
  contraction, the kernel as a factored polynomial: only rounding differs);
* FP32 deviation storage against the FP64 oracle: the error bound derived in
  the FP32 tests below.
Sizes span ragged tails and lattices smaller than the
velocity reach.
"""
import numpy as np
import pytest
import torch

from oracle import lbm as O
from paper_1405_1253_amd import workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def abi():
    from paper_1405_1253_amd import abi as mod
    mod.load()
    return mod


def _oracle_setup(lx, lz, tau, g, seed, nmodes=16, t=(1.05, 1.0, 0.95), width=4.0):
    m = W.draw_modes(seed, nmodes)
    p = O.Params(lx, lz, tau, g)
    desc = O.RT3(t[0], t[1], t[2], width, m.k, m.phase)
    return m, p, desc


def _gpu_init(abi, lat_p, m, t=(1.05, 1.0, 0.95), width=4.0, dtype=torch.float64):
    f = abi.empty_populations(lat_p, dtype)
    ghost = torch.empty((2, 3, 37), dtype=dtype, device=DEV)
    amp = torch.as_tensor(m.amp, device=DEV)
    abi.lbm_init_rt3(lat_p, abi.RT3Desc(t[0], t[1], t[2], width, m.k, m.phase), amp, f, ghost)
    return f, ghost


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


# ---------------------------------------------------------------------------
# streaming and walls: bit-exact
# ---------------------------------------------------------------------------
SHAPES = [(128, 384), (37, 300), (9, 513), (5, 7), (3, 2), (1, 5)]


@pytest.mark.parametrize("lx,lz", SHAPES)
@pytest.mark.parametrize("prec", ["f64", "f32dev"])
@pytest.mark.parametrize("periodic", [False, True])
def test_propagate_bit_exact(abi, lx, lz, prec, periodic):
    np_dt = np.float64 if prec == "f64" else np.float32
    f = W.random_populations(100 + lx, lx, lz).astype(np_dt)
    ghost = W.random_ghost(200 + lz).astype(np_dt)
    flags = abi.NO_COLLIDE | (abi.PERIODIC_Z if periodic else 0)
    params = abi.make_params(lx, lz, 0.7, 1e-4, abi.F64 if prec == "f64" else abi.F32_DEV, flags)
    fin = abi.to_tiled(params, f)
    fout = torch.full_like(fin, float("nan"))
    abi.lbm_step(params, torch.as_tensor(ghost, device=DEV), fin, fout)
    torch.cuda.synchronize()
    want = O.pull(f, ghost, O.Params(lx, lz, 0.7, 1e-4, periodic_z=periodic, no_collide=True))
    assert np.array_equal(abi.to_soa(params, fout).cpu().numpy(), want)


# ---------------------------------------------------------------------------
# FP64 init, step, moments
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_oracle():
    """Oracle trajectory of the 128 x 384 three-layer workload: steps 0, 1, 100."""
    wl = W.WORKLOADS["rt3_128x384"]
    m, p, desc = _oracle_setup(wl.lx, wl.lz, wl.tau, wl.g, wl.seed)
    f0, ghost = O.init_rt3(p, desc, m.amp)
    f1 = O.step(f0, ghost, p)
    f100 = O.run(f1, ghost, p, 99)
    return wl, m, p, desc, f0, ghost, f1, f100


def test_init_parity_f64(abi, c1_oracle):
    wl, m, p, desc, f0, ghost, _, _ = c1_oracle
    params = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g)
    f, gh = _gpu_init(abi, params, m)
    assert _rel(abi.to_soa(params, f).cpu().numpy(), f0) <= 1e-13
    assert _rel(gh.cpu().numpy(), ghost) <= 1e-13


def test_step_parity_f64_1_and_100_steps(abi, c1_oracle):
    wl, m, p, desc, f0, ghost, f1, f100 = c1_oracle
    params = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g)
    fa, gh = _gpu_init(abi, params, m)
    fb = torch.empty_like(fa)
    abi.lbm_step(params, gh, fa, fb)
    e1 = _rel(abi.to_soa(params, fb).cpu().numpy(), f1)
    for _ in range(99):
        abi.lbm_step(params, gh, fb, fa)
        fa, fb = fb, fa
    e100 = _rel(abi.to_soa(params, fb).cpu().numpy(), f100)
    print(f"FP64 max rel err: 1 step {e1:.3e}, 100 steps {e100:.3e}")
    assert e1 <= 1e-12 and e100 <= 1e-12


def test_step_parity_f64_ragged(abi):
    lx, lz, steps = 37, 300, 12      # 2 tiles along z, ragged tail, odd Lx
    m, p, desc = _oracle_setup(lx, lz, 0.6, 3e-4, 7, nmodes=5)
    f0, ghost = O.init_rt3(p, desc, m.amp)
    want = O.run(f0, ghost, p, steps)
    params = abi.make_params(lx, lz, 0.6, 3e-4)
    fa, gh = _gpu_init(abi, params, m)
    fb = torch.empty_like(fa)
    for _ in range(steps):
        abi.lbm_step(params, gh, fa, fb)
        fa, fb = fb, fa
    assert _rel(abi.to_soa(params, fa).cpu().numpy(), want) <= 1e-12


def test_step_parity_tiny_lattices(abi):
    """Lattices narrower/shorter than the 3-site reach: multiple wraps in x,
    every row is a wall row."""
    for lx, lz in ((2, 3), (1, 1), (4, 6)):
        m, p, desc = _oracle_setup(lx, lz, 0.8, 1e-3, 3, nmodes=2, width=1.0)
        f0, ghost = O.init_rt3(p, desc, m.amp)
        want = O.run(f0, ghost, p, 3)
        params = abi.make_params(lx, lz, 0.8, 1e-3)
        fa, gh = _gpu_init(abi, params, m, width=1.0)
        fb = torch.empty_like(fa)
        for _ in range(3):
            abi.lbm_step(params, gh, fa, fb)
            fa, fb = fb, fa
        assert _rel(abi.to_soa(params, fa).cpu().numpy(), want) <= 1e-12, (lx, lz)


def test_moments_parity(abi, c1_oracle):
    wl, m, p, desc, f0, ghost, f1, f100 = c1_oracle
    params = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g)
    f = abi.to_tiled(params, f100)
    fields = torch.empty((4, wl.lx, wl.lz), dtype=torch.float64, device=DEV)
    tbar = torch.empty(wl.lz, dtype=torch.float64, device=DEV)
    sums = torch.empty(4, dtype=torch.float64, device=DEV)
    scratch = torch.empty(abi.lbm_scratch_bytes(params), dtype=torch.uint8, device=DEV)
    abi.lbm_moments(params, f, fields, tbar, sums, scratch)
    rho, uH, TH = O.hydro_fields(f100, p)
    got = fields.cpu().numpy()
    assert _rel(got[0], rho) <= 1e-13
    assert np.abs(got[1] - uH[..., 0]).max() <= 1e-15
    assert np.abs(got[2] - uH[..., 1]).max() <= 1e-15
    assert _rel(got[3], TH) <= 1e-13
    assert _rel(tbar.cpu().numpy(), O.tbar(TH)) <= 1e-13
    s = O.global_sums(f100)
    gs = sums.cpu().numpy()
    assert abs(gs[0] / s[0] - 1) <= 1e-13 and abs(gs[3] / s[3] - 1) <= 1e-13
    assert np.abs(gs[1:3] - s[1:3]).max() <= 1e-13 * s[0]


def test_step_moments_out(abi, c1_oracle):
    wl, m, p, desc, f0, ghost, f1, _ = c1_oracle
    params = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g)
    fa, gh = _gpu_init(abi, params, m)
    fb = torch.empty_like(fa)
    mom = torch.empty((4, wl.lx, wl.lz), dtype=torch.float64, device=DEV)
    abi.lbm_step(params, gh, fa, fb, mom)
    rho, u, T = O.moments(O.pull(f0, ghost, p))
    got = mom.cpu().numpy()
    assert _rel(got[0], rho) <= 1e-13
    assert np.abs(got[1] - u[..., 0]).max() <= 1e-15
    assert np.abs(got[2] - u[..., 1]).max() <= 1e-15
    assert _rel(got[3], T) <= 1e-13


def test_bitwise_reproducible(abi):
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    params = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g)
    outs = []
    for _ in range(2):
        fa, gh = _gpu_init(abi, params, m)
        fb = torch.empty_like(fa)
        for _ in range(20):
            abi.lbm_step(params, gh, fa, fb)
            fa, fb = fb, fa
        sums = torch.empty(4, dtype=torch.float64, device=DEV)
        scratch = torch.empty(abi.lbm_scratch_bytes(params), dtype=torch.uint8, device=DEV)
        abi.lbm_moments(params, fa, sums=sums, scratch=scratch)
        outs.append((abi.to_soa(params, fa).cpu().numpy(), sums.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_runtime_errors(abi):
    params = abi.make_params(16, 16, 0.7, 1e-4)
    f = abi.empty_populations(params, torch.float64).zero_()
    gh = torch.zeros((2, 3, 37), dtype=torch.float64, device=DEV)
    with pytest.raises(abi.LbmError, match="EALIAS"):
        abi.lbm_step(params, gh, f, f)
    with pytest.raises(abi.LbmError, match="EINVAL"):
        abi.lbm_step(abi.make_params(16, 16, 0.4, 1e-4), gh, f, torch.empty_like(f))
    abi.lbm_step(abi.make_params(0, 16, 0.7, 1e-4), gh, f, torch.empty_like(f))   # empty: no-op


# ---------------------------------------------------------------------------
# physics invariants on the GPU path
# ---------------------------------------------------------------------------
def test_gpu_x_uniform_state_stays_x_uniform(abi):
    lx, lz = 16, 384
    params = abi.make_params(lx, lz, 0.7, 1e-4)
    m = W.draw_modes(1)
    m.amp[:] = 0.0
    fa, gh = _gpu_init(abi, params, m)
    fb = torch.empty_like(fa)
    for _ in range(200):
        abi.lbm_step(params, gh, fa, fb)
        fa, fb = fb, fa
    f = abi.to_soa(params, fa).cpu().numpy()
    assert all(np.array_equal(f[:, x], f[:, 0]) for x in range(lx))


def test_gpu_periodic_momentum_and_mass(abi):
    rng = np.random.default_rng(5)
    lx, lz, g = 32, 40, 2e-3
    rho = rng.uniform(0.9, 1.1, (lx, lz))
    u = rng.uniform(-0.05, 0.05, (lx, lz, 2))
    T = rng.uniform(0.95, 1.05, (lx, lz))
    f0 = O.equilibrium(rho, u, T)
    params = abi.make_params(lx, lz, 0.9, g, flags=abi.PERIODIC_Z)
    fa = abi.to_tiled(params, f0)
    fb = torch.empty_like(fa)
    sums = torch.empty(4, dtype=torch.float64, device=DEV)
    scratch = torch.empty(abi.lbm_scratch_bytes(params), dtype=torch.uint8, device=DEV)
    abi.lbm_moments(params, fa, sums=sums, scratch=scratch)
    s0 = sums.cpu().numpy()
    for t in range(1, 11):
        abi.lbm_step(params, None, fa, fb)
        fa, fb = fb, fa
    abi.lbm_moments(params, fa, sums=sums, scratch=scratch)
    s = sums.cpu().numpy()
    assert abs(s[0] / s0[0] - 1) <= 1e-14
    assert abs(s[1] - s0[1]) <= 1e-13 * s0[0]
    assert abs(s[2] - (s0[2] - 10 * g * s0[0])) <= 1e-12 * s0[0]
