"""lbm_moments_noalloc: the diagnostics entry point that allocates nothing.

Through the C ABI, against lbm_moments with a caller scratch buffer (same
kernels and order of sums, so the results must agree bit for bit), on two
calls in a row with the second on a smaller lattice (the static array keeps
the first call's partial sums, which the second must not see).  The host
check that refuses lattices whose scratch exceeds the static array runs
without a GPU.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1405_1253_amd import workload as W

DEV = "cuda"


@pytest.fixture(scope="module")
def abi():
    from paper_1405_1253_amd import abi as mod
    mod.load()
    return mod


def _state(abi, lx, lz, prec, seed, steps=3):
    dt = torch.float64 if prec == "f64" else torch.float32
    params = abi.make_params(lx, lz, 0.7, 2e-4, abi.F64 if prec == "f64" else abi.F32_DEV)
    m = W.draw_modes(seed, 6)
    f = abi.empty_populations(params, dt)
    gh = torch.empty((2, 3, 37), dtype=dt, device=DEV)
    abi.lbm_init_rt3(params, abi.RT3Desc(1.05, 1.0, 0.95, 4.0, m.k, m.phase),
                     torch.as_tensor(m.amp * 3, device=DEV), f, gh)
    g = torch.empty_like(f)
    for _ in range(steps):
        abi.lbm_step(params, gh, f, g)
        f, g = g, f
    return params, f


def _outputs(lx, lz):
    return (torch.full((4, lx, lz), float("nan"), dtype=torch.float64, device=DEV),
            torch.full((lz,), float("nan"), dtype=torch.float64, device=DEV),
            torch.full((4,), float("nan"), dtype=torch.float64, device=DEV))


@pytest.mark.gpu
def test_noalloc_matches_moments_on_two_calls(abi):
    for lx, lz, prec, seed in ((300, 1100, "f64", 1), (70, 200, "f32dev", 2)):
        params, f = _state(abi, lx, lz, prec, seed)
        fields, tbar, sums = _outputs(lx, lz)
        scratch = torch.empty(abi.lbm_scratch_bytes(params), dtype=torch.uint8, device=DEV)
        abi.lbm_moments(params, f, fields, tbar, sums, scratch)
        fields2, tbar2, sums2 = _outputs(lx, lz)
        abi.lbm_moments_noalloc(params, f, fields2, tbar2, sums2)
        torch.cuda.synchronize()
        assert torch.isfinite(tbar).all() and torch.isfinite(sums).all()
        assert torch.equal(fields2, fields), (lx, lz)
        assert torch.equal(tbar2, tbar), (lx, lz)
        assert torch.equal(sums2, sums), (lx, lz)
        # the mass is the plain sum of the populations (independent of both)
        soa = abi.to_soa(params, f).double()
        full = soa if prec == "f64" else soa + torch.as_tensor(abi.lbm_lattice()[1], device=DEV)[:, None, None]
        assert abs(sums2[0].item() / full.sum().item() - 1) <= 1e-12


@pytest.mark.gpu
def test_noalloc_outputs_one_at_a_time(abi):
    # tbar alone, sums alone, fields alone: each equals the full call's
    params, f = _state(abi, 33, 517, "f64", 3)
    fields, tbar, sums = _outputs(33, 517)
    abi.lbm_moments_noalloc(params, f, fields, tbar, sums)
    for which in ("fields", "tbar", "sums"):
        out = _outputs(33, 517)
        kw = {which: out[("fields", "tbar", "sums").index(which)]}
        abi.lbm_moments_noalloc(params, f, **kw)
        ref = {"fields": fields, "tbar": tbar, "sums": sums}[which]
        assert torch.equal(kw[which], ref), which


def test_noalloc_refuses_lattices_beyond_the_static_array():
    """tbar or sums on a lattice whose partial sums need more than the
    static array: LBM_ESTATIC before any HIP call (fake device addresses)."""
    from paper_1405_1253_amd import abi as A
    lib = A.load()
    big = A.make_params(16384, 32768, 0.7, 1e-4)
    f, tb, su = 1 << 32, 1 << 40, 1 << 41
    assert lib.lbm_moments_noalloc(ctypes.byref(big), f, None, tb, None, None) == -7
    assert lib.lbm_moments_noalloc(ctypes.byref(big), f, None, None, su, None) == -7
    assert "static scratch" in lib.lbm_strerror(-7).decode()
    # one GPU's production share (4096 x 12288) needs 8 ceil(Lx/64) Lz bytes
    # of row partials plus 32 B per (strip, 256-row block): within the array
    assert A.STATIC_SCRATCH_BYTES == 16 << 20
    assert 8 * 64 * 12288 + 32 * 64 * 48 < A.STATIC_SCRATCH_BYTES
    c2 = A.make_params(4096, 12288, 0.7, 1e-4)
    assert lib.lbm_moments_noalloc(ctypes.byref(c2), 3, None, tb, None, None) == -3   # misaligned f
    assert np.int32(lib.lbm_moments_noalloc(ctypes.byref(big), f, None, None, None, None)) == 0
