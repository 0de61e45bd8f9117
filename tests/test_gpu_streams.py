"""The boundary's stream contract on the GPU: every entry point only enqueues
on the stream it is given, so work on a side stream, on two streams at once,
or captured in a HIP graph and replayed gives the same bits as the same
calls made eagerly on the current stream.

The graph test replays its capture several times with eager work and
synchronisations between the replays and checks every replay against the
eager result (the library records no memset or copy, only kernels).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def abi():
    from paper_1405_1253_amd import abi as mod
    mod.load()
    return mod


def _setup(abi, lx=24, lz=1100, precision=0, flags=0, seed=1405):
    from paper_1405_1253_amd import workload as W
    p = abi.make_params(lx, lz, 0.7, 1e-4, precision, flags)
    m = W.draw_modes(seed)
    dt = torch.float64 if precision == abi.F64 else torch.float32
    f = abi.empty_populations(p, dt)
    gh = torch.empty((2, 3, abi.Q), dtype=dt, device=DEV)
    abi.lbm_init_rt3(p, abi.RT3Desc(1.05, 1.0, 0.95, 4.0, m.k, m.phase), torch.as_tensor(m.amp, device=DEV), f, gh)
    return p, f, gh


def _run(abi, p, gh, f0, n, stream=None):
    bufs = [f0.clone(), torch.empty_like(f0)]
    for i in range(n):
        abi.lbm_step(p, gh, bufs[i % 2], bufs[1 - i % 2], stream=stream)
    return bufs[n % 2]


def _bits(t):
    return t.cpu().numpy().view(np.uint8).copy()


@pytest.mark.parametrize("prec", ["f64", "f32dev"])
def test_side_stream_equals_current_stream(abi, prec):
    p, f0, gh = _setup(abi, precision=abi.F64 if prec == "f64" else abi.F32_DEV)
    torch.cuda.synchronize()
    ref = _run(abi, p, gh, f0, 20)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bufs = [f0.clone(), torch.empty_like(f0)]
    for i in range(20):
        abi.lbm_step(p, gh, bufs[i % 2], bufs[1 - i % 2], stream=s)
    s.synchronize()
    assert np.array_equal(_bits(abi.to_soa(p, bufs[0])), _bits(abi.to_soa(p, ref)))


def test_two_streams_at_once(abi):
    """Two lattices stepped concurrently on two streams, interleaved call by
    call, end bitwise where each ends alone."""
    pa, fa, gha = _setup(abi, lx=20, lz=1300, seed=1405)
    pb, fb, ghb = _setup(abi, lx=33, lz=777, precision=abi.F32_DEV, flags=abi.WALL_DIFFUSE, seed=1406)
    torch.cuda.synchronize()
    ref_a = _run(abi, pa, gha, fa, 16)
    ref_b = _run(abi, pb, ghb, fb, 16)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    a = [fa.clone(), torch.empty_like(fa)]
    b = [fb.clone(), torch.empty_like(fb)]
    torch.cuda.synchronize()
    for i in range(16):
        abi.lbm_step(pa, gha, a[i % 2], a[1 - i % 2], stream=sa)
        abi.lbm_step(pb, ghb, b[i % 2], b[1 - i % 2], stream=sb)
    sa.synchronize()
    sb.synchronize()
    assert np.array_equal(_bits(abi.to_soa(pa, a[0])), _bits(abi.to_soa(pa, ref_a)))
    assert np.array_equal(_bits(abi.to_soa(pb, b[0])), _bits(abi.to_soa(pb, ref_b)))


def test_graph_capture_and_replay(abi):
    """Ten steps and the allocation-free global sums captured in one graph;
    three replays from the same start, eager work between them, each equal
    bit for bit to the eager sequence."""
    p, f0, gh = _setup(abi, lx=24, lz=1100)
    sums_ref = torch.empty(4, dtype=torch.float64, device=DEV)
    ref = _run(abi, p, gh, f0, 10)
    abi.lbm_moments_noalloc(p, ref, sums=sums_ref)      # also sets up the static scratch
    torch.cuda.synchronize()
    ref_bits, sums_bits = _bits(abi.to_soa(p, ref)), _bits(sums_ref)

    bufs = [torch.empty_like(f0), torch.empty_like(f0)]
    sums = torch.empty(4, dtype=torch.float64, device=DEV)
    bufs[0].copy_(f0)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        # one eager pass on the capture stream before capturing (no lazy set-up inside)
        for i in range(10):
            abi.lbm_step(p, gh, bufs[i % 2], bufs[1 - i % 2])
        abi.lbm_moments_noalloc(p, bufs[0], sums=sums)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        for i in range(10):
            abi.lbm_step(p, gh, bufs[i % 2], bufs[1 - i % 2])
        abi.lbm_moments_noalloc(p, bufs[0], sums=sums)
    other = [f0.clone(), torch.empty_like(f0)]
    for rep in range(3):
        bufs[0].copy_(f0)
        bufs[1].fill_(float("nan"))
        sums.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_bits(abi.to_soa(p, bufs[0])), ref_bits), rep
        assert np.array_equal(_bits(sums), sums_bits), rep
        # eager work of the program between replays
        for i in range(3):
            abi.lbm_step(p, gh, other[i % 2], other[1 - i % 2])
        torch.cuda.synchronize()
