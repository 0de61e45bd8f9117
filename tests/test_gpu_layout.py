"""The tiled population layout on the GPU: lbm_pack / lbm_unpack against the
index formula of include/lbm.h written out in numpy (bit-exact: a pure
permutation, padding rows packed as zero bits), for both element sizes,
ragged and tiny lattices."""
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


def _tiled_numpy(soa, tile=512):
    """[37, lx, lz] -> flat tiled array: element (l, x, z) at
    (((z // tile) lx + x) 37 + l) tile + z % tile, padding rows zero."""
    q, lx, lz = soa.shape
    nt = -(-lz // tile)
    out = np.zeros((nt, lx, q, tile), dtype=soa.dtype)
    pad = np.zeros((q, lx, nt * tile), dtype=soa.dtype)
    pad[:, :, :lz] = soa
    out[:] = pad.reshape(q, lx, nt, tile).transpose(2, 1, 0, 3)
    return out.ravel()


@pytest.mark.parametrize("lx,lz", [(1, 1), (3, 7), (5, 513), (2, 1100), (64, 1024)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_pack_unpack_bit_exact(abi, lx, lz, dtype):
    rng = np.random.default_rng(lx * 1000 + lz)
    soa = rng.standard_normal((37, lx, lz)).astype(dtype)
    params = abi.make_params(lx, lz, 0.7, 0.0)
    tiled = abi.empty_populations(params, torch.float64 if dtype == np.float64 else torch.float32)
    tiled.fill_(float("nan"))
    abi.lbm_pack(params, torch.as_tensor(soa, device=DEV), tiled)
    got = tiled.cpu().numpy()
    want = _tiled_numpy(soa)
    assert got.view(np.uint8).tobytes() == want.view(np.uint8).tobytes()
    back = torch.full((37, lx, lz), float("nan"), dtype=tiled.dtype, device=DEV)
    abi.lbm_unpack(params, tiled, back)
    assert np.array_equal(back.cpu().numpy(), soa)
    # the binding's column view reads the same elements
    x = lx - 1
    assert np.array_equal(abi.column(params, tiled, x).cpu().numpy(), soa[:, x, :])


def test_pack_refuses_overlap_and_bad_element_size(abi):
    params = abi.make_params(4, 600, 0.7, 0.0)
    t = abi.empty_populations(params, torch.float64)
    soa = torch.zeros((37, 4, 600), dtype=torch.float64, device=DEV)
    with pytest.raises(abi.LbmError, match="EALIAS"):
        abi.lbm_pack(params, t, t)
    import ctypes
    lib = abi.load()
    assert lib.lbm_pack(ctypes.byref(params), soa.data_ptr(), t.data_ptr(), 2, None) == -1
    assert lib.lbm_unpack(ctypes.byref(params), t.data_ptr(), soa.data_ptr() + 4, 8, None) == -3
