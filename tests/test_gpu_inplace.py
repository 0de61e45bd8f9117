"""Single-buffer step (lbm_step_inplace) against the two-buffer step and the
oracle.

Bars: streaming only, the streamed form after one step is the layout
include/lbm.h defines and two steps equal two two-buffer steps, bit for bit;
with collisions the two in-place kinds in turn give, after every even number
of steps, the two-buffer state to rounding (the same formulas per site; the
compiler may contract them to FMAs differently in the two instantiations):
1e-13 relative in FP64, 2^-20 of the largest deviation in FP32, moments to
1e-13 (FP64) / 1e-6 (FP32) absolute, and the oracle within 1e-12 (FP64);
both wall rules, both precisions, periodic z, ragged and tiny lattices.
"""
import numpy as np
import pytest
import torch

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


def _opp():
    E = lattice()[0]
    return [int(np.nonzero((E[:, 0] == -E[l, 0]) & (E[:, 1] == -E[l, 1]))[0][0]) for l in range(37)]


def _scratch(abi, params):
    return torch.empty(max(abi.lbm_scratch_bytes(params), 256), dtype=torch.uint8, device=DEV)


def _two_buffer(abi, params, ghost, f0, steps, mom=False):
    fa, fb = f0.clone(), torch.empty_like(f0)
    moms = []
    for _ in range(steps):
        m = torch.empty((4, params.lx, params.lz), dtype=torch.float64, device=DEV) if mom else None
        abi.lbm_step(params, ghost, fa, fb, m)
        fa, fb = fb, fa
        moms.append(m)
    return fa, moms


def _in_place(abi, params, ghost, f0, steps, mom=False):
    f = f0.clone()
    scratch = _scratch(abi, params)
    moms = []
    for t in range(steps):
        m = torch.empty((4, params.lx, params.lz), dtype=torch.float64, device=DEV) if mom else None
        abi.lbm_step_inplace(params, ghost, f, t % 2, m, scratch)
        moms.append(m)
    return f, moms


@pytest.mark.parametrize("prec", ["f64", "f32dev"])
@pytest.mark.parametrize("mode", ["dirichlet", "diffuse", "periodic"])
@pytest.mark.parametrize("lx,lz", [(64, 200), (37, 300), (5, 7), (2, 3)])
def test_streaming_in_place(abi, prec, mode, lx, lz):
    """Streaming only: after one step the buffer holds the streamed form of
    include/lbm.h; after two it equals two two-buffer steps, bit for bit."""
    dt = np.float64 if prec == "f64" else np.float32
    f = W.random_populations(500 + lx, lx, lz).astype(dt)
    ghost = W.random_ghost(600 + lz).astype(dt)
    flags = abi.NO_COLLIDE | {"dirichlet": 0, "diffuse": abi.WALL_DIFFUSE, "periodic": abi.PERIODIC_Z}[mode]
    params = abi.make_params(lx, lz, 0.7, 1e-4, abi.F64 if prec == "f64" else abi.F32_DEV, flags)
    f0, gh = abi.to_tiled(params, f), torch.as_tensor(ghost, device=DEV)
    one, _ = _in_place(abi, params, gh, f0, 1)
    pulled, _ = _two_buffer(abi, params, gh, f0, 1)
    got, g = abi.to_soa(params, one).cpu().numpy(), abi.to_soa(params, pulled).cpu().numpy()
    E, opp = lattice()[0], _opp()
    want = np.empty_like(got)
    for l in range(37):
        # the step's output g, streamed once more: slot -l at x holds g_l(x - e_l)
        ex, ez = int(E[l, 0]), int(E[l, 1])
        want[opp[l]] = np.roll(g[l], shift=(ex, ez), axis=(0, 1))
        if mode == "periodic":
            continue
        # rows whose source lies beyond a wall hold the parked population -l
        for z in range(lz):
            if not 0 <= z - ez < lz:
                want[opp[l], :, z] = g[opp[l], :, z]
    assert np.array_equal(got, want)
    two, _ = _in_place(abi, params, gh, f0, 2)
    ref, _ = _two_buffer(abi, params, gh, f0, 2)
    assert torch.equal(abi.to_soa(params, two), abi.to_soa(params, ref))


def _init(abi, params, seed, width=4.0, nmodes=16):
    m = W.draw_modes(seed, nmodes)
    dt = torch.float64 if params.precision == abi.F64 else torch.float32
    f = abi.empty_populations(params, dt)
    gh = torch.empty((2, 3, 37), dtype=dt, device=DEV)
    abi.lbm_init_rt3(params, abi.RT3Desc(1.05, 1.0, 0.95, width, m.k, m.phase),
                     torch.as_tensor(m.amp, device=DEV), f, gh)
    return m, f, gh


@pytest.mark.parametrize("prec", ["f64", "f32dev"])
@pytest.mark.parametrize("wall", ["dirichlet", "diffuse"])
def test_in_place_equals_two_buffers(abi, prec, wall):
    """128 x 384 three-layer workload, 2 and 20 steps: the two-buffer state
    and moments_out of every step, to rounding."""
    params = abi.make_params(128, 384, 0.7, 2.6e-4, abi.F64 if prec == "f64" else abi.F32_DEV,
                             abi.wall_flag(wall))
    _, f0, gh = _init(abi, params, 1405)
    for steps in (2, 20):
        a, ma = _in_place(abi, params, gh, f0, steps, mom=True)
        b, mb = _two_buffer(abi, params, gh, f0, steps, mom=True)
        a, b = abi.to_soa(params, a).double(), abi.to_soa(params, b).double()
        if prec == "f64":
            err = float(((a - b).abs() / b.abs()).max())
            bar = 1e-13
        else:   # deviations f - w: relative to the largest one
            err = float((a - b).abs().max() / b.abs().max())
            bar = 2.0 ** -20
        # absolute: rho and T are ~1, the velocities ~1e-4 (their relative
        # rounding is amplified by the cancellation in sum_l xi_l f_l)
        merr = max(float((x - y).abs().max()) for x, y in zip(ma[1:], mb[1:]))
        print(f"{prec} {wall}, {steps} steps: in place vs two buffers: state {err:.2e}, "
              f"moments {merr:.2e}, first step's moments equal: {torch.equal(ma[0], mb[0])}")
        assert err <= bar, (steps, err)
        assert torch.equal(ma[0], mb[0])         # same input, same moment sums
        assert merr <= (1e-13 if prec == "f64" else 1e-6), (steps, merr)


@pytest.mark.parametrize("prec", ["f64", "f32dev", "f32dev_collide_f64"])
@pytest.mark.parametrize("wall", ["dirichlet", "diffuse"])
@pytest.mark.parametrize("lx,lz", [(3, 6), (2, 3), (100, 5), (5, 7), (16, 2051), (1024, 4100)])
def test_in_place_equals_two_buffers_tiny_and_ragged(abi, prec, wall, lx, lz):
    """Lattices whose rows are all wall rows (Lz < 7), the smallest with an
    interior row, a ragged one of several tiles (wall blocks and tile blocks
    in one launch) and a ragged FP64 one of 2^22 sites or more (tiles and
    wall rows in two launches): 4 steps against the two-buffer step, same
    bars."""
    params = abi.make_params(lx, lz, 0.6, 3e-4, abi.F64 if prec == "f64" else abi.F32_DEV,
                             abi.wall_flag(wall) | (abi.COLLIDE_F64 if prec == "f32dev_collide_f64" else 0))
    _, f0, gh = _init(abi, params, 11, width=1.0 if lz < 64 else 4.0, nmodes=2)
    a, _ = _in_place(abi, params, gh, f0, 4)
    b, _ = _two_buffer(abi, params, gh, f0, 4)
    a, b = abi.to_soa(params, a).double(), abi.to_soa(params, b).double()
    if prec == "f64":
        err, bar = float(((a - b).abs() / b.abs()).max()), 1e-13
    else:
        err, bar = float((a - b).abs().max() / b.abs().max()), 2.0 ** -20
    print(f"{prec} {wall} {lx}x{lz}: in place vs two buffers {err:.2e}")
    assert torch.isfinite(a).all() and err <= bar


def test_in_place_parity_with_oracle_ragged_and_tiny(abi):
    for lx, lz, steps, width, wall in ((37, 300, 12, 4.0, "dirichlet"), (37, 300, 12, 4.0, "diffuse"),
                                       (2, 3, 4, 1.0, "diffuse"), (4, 6, 4, 1.0, "dirichlet"),
                                       (1, 1, 2, 1.0, "diffuse")):
        params = abi.make_params(lx, lz, 0.6, 3e-4, flags=abi.wall_flag(wall))
        m, f0, gh = _init(abi, params, 7, width=width, nmodes=2)
        p = O.Params(lx, lz, 0.6, 3e-4, wall=wall)
        f_o, ghost_o = O.init_rt3(p, O.RT3(1.05, 1.0, 0.95, width, m.k, m.phase), m.amp)
        want = O.run(f_o, ghost_o, p, steps)
        got, _ = _in_place(abi, params, gh, f0, steps)
        err = float(np.max(np.abs(abi.to_soa(params, got).cpu().numpy() - want) / want))
        assert err <= 1e-12, (lx, lz, wall, err)


def test_lattice_in_place_runtime(abi):
    """Lattice(inplace=True): one buffer; the state is readable after an even
    number of steps and refused after an odd one."""
    from paper_1405_1253_amd.runtime import Lattice
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    lat = Lattice.from_workload(wl, modes=m, inplace=True)
    ref = Lattice.from_workload(wl, modes=m)
    assert len(lat.buf) == 1
    lat.step(3)
    with pytest.raises(RuntimeError):
        lat.sums()
    lat.step(1)
    ref.step(4)
    a, b = lat.state_soa(), ref.state_soa()
    assert float(((a - b).abs() / b.abs()).max()) <= 1e-13
    a, b = lat.sums(), ref.sums()              # mass, momentum (~0 in x), energy
    assert float((a - b).abs().max()) <= 1e-12 * float(b[0])


def _oracle_column(wl, m, x, nsteps):
    # a site after n steps depends on columns within 3n of it (Dirichlet
    # walls): step a periodic window of 6n + 1 columns around x
    half = 3 * nsteps
    cols = (np.arange(x - half, x + half + 1)) % wl.lx
    desc = O.RT3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase)
    f, ghost = O.init_rt3(O.Params(wl.lx, wl.lz, wl.tau, wl.g), desc, m.amp, columns=cols)
    return O.run(f, ghost, O.Params(len(cols), wl.lz, wl.tau, wl.g), nsteps)[:, half, :]


def test_largest_lattice_single_buffer(abi):
    """16384 x 32768 = 2^29 sites, the largest lattice the library accepts, in
    FP64 on one 159 GB buffer (two buffers would need 318 GB): sampled
    columns, both wrap-around edges among them, against the oracle's windowed
    columns after the initial state and after 2 steps (1e-12 relative), and
    the mass lbm_moments reports against a plain sum of the buffer; the rate
    of 10 more steps is printed."""
    from paper_1405_1253_amd.runtime import Lattice
    wl = W.WORKLOADS["rt3_16384x32768_inplace"]
    assert wl.sites == 1 << 29
    torch.cuda.empty_cache()
    need = 37 * 8 * wl.sites
    free = torch.cuda.mem_get_info()[0]
    if free < need + (8 << 30):
        pytest.skip(f"needs {need / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")
    m = W.draw_modes(wl.seed)
    lat = Lattice.from_workload(wl, modes=m)
    assert lat.inplace and len(lat.buf) == 1
    samples = (0, 8191, 16383)
    got = {0: {x: abi.column(lat.params, lat.state, x).cpu().numpy() for x in samples}}
    lat.step(2)
    got[2] = {x: abi.column(lat.params, lat.state, x).cpu().numpy() for x in samples}
    assert wl.lz % abi.TILE == 0          # no padding rows: the raw sum is the lattice's
    mass, total = lat.sums()[0].item(), lat.state.sum().item()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    lat.step(10)
    stop.record()
    stop.synchronize()
    ms = start.elapsed_time(stop) / 10
    del lat
    torch.cuda.empty_cache()
    worst = {}
    for n, cols in got.items():
        for x, g in cols.items():
            want = _oracle_column(wl, m, x, n)
            worst[n] = max(worst.get(n, 0.0), float(np.max(np.abs(g - want) / want)))
    gbs = 2 * need / (ms * 1e-3) / 1e9
    print(f"2^29 sites, one FP64 buffer: max rel err init {worst[0]:.2e}, 2 steps {worst[2]:.2e}; "
          f"lbm_moments mass vs a plain sum {abs(mass / total - 1):.1e}; {ms:.1f} ms/step, {gbs:.0f} GB/s")
    assert worst[0] <= 1e-12 and worst[2] <= 1e-12
    assert abs(mass / total - 1) <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32dev"])
def test_in_place_float_moments(abi, prec):
    """LBM_MOM_F32 on a single buffer: the first step's float moments equal
    the two-buffer step's bit for bit (same input), and they are the double
    moments rounded to float."""
    base = abi.F64 if prec == "f64" else abi.F32_DEV
    p32 = abi.make_params(64, 200, 0.7, 2.6e-4, base, abi.MOM_F32)
    p64 = abi.make_params(64, 200, 0.7, 2.6e-4, base, 0)
    _, f0, gh = _init(abi, p32, 77)
    m_in = torch.empty((4, 64, 200), dtype=torch.float32, device=DEV)
    f = f0.clone()
    abi.lbm_step_inplace(p32, gh, f, abi.INPLACE_FROM_STATE, m_in, _scratch(abi, p32))
    m_two = torch.empty_like(m_in)
    m_dbl = torch.empty((4, 64, 200), dtype=torch.float64, device=DEV)
    out = torch.empty_like(f0)
    abi.lbm_step(p32, gh, f0, out, m_two)
    abi.lbm_step(p64, gh, f0, out, m_dbl)
    assert torch.equal(m_in, m_two)
    assert torch.equal(m_in, m_dbl.float())
