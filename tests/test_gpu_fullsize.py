"""Parity at the full 4096 x 12288 lattice, in the launch configuration the
benchmark times, on sampled columns.

The oracle cannot step 50 M sites, but a site after n steps depends only on
columns within 3n of it: the oracle builds the initial state of a window of
6n + 1 columns around a sampled column (columns wrap at the lattice edge),
steps the window as a periodic strip, and its centre column is then exact.
Sampled columns include both wrap-around edges.
"""
import numpy as np
import pytest
import torch

from oracle import lbm as O
from paper_1405_1253_amd import workload as W

pytestmark = pytest.mark.gpu
SAMPLES = (0, 1, 2, 1365, 2048, 4093, 4095)


def _oracle_column(wl, m, x, nsteps):
    half = 3 * nsteps
    cols = (np.arange(x - half, x + half + 1)) % wl.lx
    p_full = O.Params(wl.lx, wl.lz, wl.tau, wl.g)
    desc = O.RT3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase)
    f, ghost = O.init_rt3(p_full, desc, m.amp, columns=cols)
    p = O.Params(len(cols), wl.lz, wl.tau, wl.g)
    f = O.run(f, ghost, p, nsteps)
    return f[:, half, :], ghost


@pytest.mark.parametrize("name,tol", [("rt3_4096x12288", 1e-12), ("rt3_4096x12288_f32", 5e-7),
                                      ("rt3_4096x12288_inplace", 1e-12), ("rt3_4096x12288_f32_inplace", 5e-7)])
def test_fullsize_sampled_columns(name, tol):
    """Both storage forms, on two buffers and on one (the single buffer holds
    the state only after an even number of steps: sampled after 0 and 2)."""
    from paper_1405_1253_amd.runtime import Lattice
    wl = W.WORKLOADS[name]
    m = W.draw_modes(wl.seed)
    lat = Lattice.from_workload(wl)
    ghost_gpu = lat.ghost.to(torch.float64).cpu().numpy()
    w = None
    if wl.precision == "f32dev":
        from paper_1405_1253_amd import abi as _abi
        w = _abi.lbm_lattice()[1]

    from paper_1405_1253_amd import abi

    def column(x):
        c = abi.column(lat.params, lat.state, x).to(torch.float64).cpu().numpy()
        return c + w[:, None] if w is not None else c

    got = {0: {x: column(x) for x in SAMPLES}}
    if wl.inplace:
        lat.step(2)
        got[2] = {x: column(x) for x in SAMPLES}
    else:
        lat.step(1)
        got[1] = {x: column(x) for x in SAMPLES}
        lat.step(1)
        got[2] = {x: column(x) for x in (0, 2048, 4095)}
    lat.sums()
    del lat
    torch.cuda.empty_cache()

    worst = {}
    for n, cols in got.items():
        for x, g in cols.items():
            want, ghost = _oracle_column(wl, m, x, n)
            worst[n] = max(worst.get(n, 0.0), float(np.max(np.abs(g - want) / want)))
    ghost_full = ghost_gpu + (w[None, None, :] if w is not None else 0.0)
    print(f"{name}: max rel err over sampled columns: "
          + ", ".join(f"{n} steps {e:.2e}" for n, e in sorted(worst.items())))
    assert float(np.max(np.abs(ghost_full - ghost) / ghost)) <= (1e-13 if w is None else 2.0 ** -24)
    for n, e in worst.items():
        # FP32: the per-step deviation bound, growing at most linearly
        assert e <= tol * (max(n, 1) if w is not None else 1), (n, e)


def test_fullsize_bitwise_reproducible():
    from paper_1405_1253_amd.runtime import Lattice
    wl = W.WORKLOADS["rt3_4096x12288"]
    cols = []
    for _ in range(2):
        lat = Lattice.from_workload(wl)
        lat.step(20)
        from paper_1405_1253_amd import abi
        cols.append(abi.tiled_view(lat.params, lat.state)[:, ::511, :, ::97].cpu().numpy())
        del lat
        torch.cuda.empty_cache()
    assert np.array_equal(cols[0], cols[1])


@pytest.mark.parametrize("name,form", [("rt3_2048x6144_adj", "gather"), ("rt3_512x1536_adj", "push")])
def test_fullsize_adjoint_step_sampled_columns(name, form):
    """One adjoint step at the rollouts' full lattices, in the form and
    precision the rollouts run there (2048 x 6144: lbm_adjoint_gather with
    float buffers and float moments from an FP32-dev forward step;
    512 x 1536: lbm_adjoint_step in double), on sampled columns (both wrap
    edges included) against the oracle's factors of the step's transpose
    (collide_vjp, pull_transpose).  A column y of C^T S^T mu depends on mu at
    columns y..y+3 and on the pre-collision populations of column y, pulled
    from columns y-3..y; a column of S^T C^T lam on lam and the pulled
    populations of columns y..y+3, i.e. the state at y-3..y+6.  So a window
    of 13 columns around y (periodic in x within the window) gives the
    centre column exactly.  Bars: the all-float bound (32 float roundings
    plus 1e-6 for the moments' float rounding) and 1e-12, of the column's
    largest entry."""
    from oracle import adjoint as A
    from paper_1405_1253_amd import abi
    wl = W.WORKLOADS[name]
    m = W.draw_modes(wl.seed)
    f32 = form == "gather"
    prec = abi.F32_DEV if f32 else abi.F64
    sdt = torch.float32 if f32 else torch.float64
    mflag = abi.MOM_F32 if f32 else 0
    p_fwd = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, prec, mflag)
    p_adj = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, prec, mflag | (abi.ADJ_F32 if f32 else 0))
    f = abi.empty_populations(p_fwd, sdt)
    gh = torch.empty((2, 3, abi.Q), dtype=sdt, device="cuda")
    abi.lbm_init_rt3(p_fwd, abi.RT3Desc(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase),
                     torch.as_tensor(m.amp, device="cuda"), f, gh)
    mom = torch.empty((4, wl.lx, wl.lz), dtype=sdt, device="cuda")
    abi.lbm_step(p_fwd, gh, f, torch.empty_like(f), mom)
    gen = torch.Generator(device="cuda").manual_seed(wl.seed)
    lam = torch.randn(f.shape, dtype=sdt, device="cuda", generator=gen)
    out = torch.empty_like(f)
    if f32:
        abi.lbm_adjoint_gather(p_adj, gh, mom, lam, out)
    else:
        abi.lbm_adjoint_step(p_adj, gh, mom, lam, out)
    w = abi.lbm_lattice()[1] if f32 else np.zeros(abi.Q)
    ghost = gh.double().cpu().numpy() + w                    # the FP32 table holds f - w

    def window(t, cols, full):
        c = np.stack([abi.column(p_adj, t, int(x)).double().cpu().numpy() for x in cols], axis=1)
        return c + w[:, None, None] if full else c

    p13 = O.Params(13, wl.lz, wl.tau, wl.g)
    worst = 0.0
    for y in (0, 1, wl.lx // 2, wl.lx - 2, wl.lx - 1):
        cols = np.arange(y - 6, y + 7) % wl.lx
        g = O.pull(window(f, cols, True), ghost, p13)
        lw = window(lam, cols, False)
        if f32:
            want = A.collide_vjp(A.pull_transpose(lw, p13, ghost), g, p13)[:, 6, :]
        else:
            want = A.pull_transpose(A.collide_vjp(lw, g, p13), p13, ghost)[:, 6, :]
        got = abi.column(p_adj, out, y).double().cpu().numpy()
        worst = max(worst, float(np.abs(got - want).max() / np.abs(want).max()))
    bound = 32 * 2.0 ** -24 + 1e-6 if f32 else 1e-12
    print(f"{name} {form}: max error over sampled columns {worst:.2e} of the column's largest entry (bar {bound:.1e})")
    assert worst <= bound
