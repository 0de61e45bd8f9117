"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every entry point include/lbm.h declares, its compiled constants
agree with the oracle's independent quadrature solve, the constant header is
reproducible from its generator, and invalid arguments are refused before
anything is launched."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from oracle import lattice as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_1405_1253_amd import abi as mod
    mod.load()
    return mod


def test_exports_every_declared_symbol(abi):
    names = declared_functions()
    assert "lbm_step" in names and "lbm_init_rt3" in names and "lbm_moments" in names
    lib = ctypes.CDLL(abi.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_library_constants_match_oracle(abi):
    r, w, e = abi.lbm_lattice()
    E, _, w_o, r_o = L.lattice()
    assert np.array_equal(e, E)                  # documented population order
    assert abs(r - r_o) <= 1e-14
    assert np.abs(w / w_o - 1).max() <= 1e-13


def test_constant_header_is_generated():
    csrc = os.path.join(ROOT, "paper_1405_1253_amd", "csrc")
    out = subprocess.run([sys.executable, os.path.join(csrc, "gen_lattice.py")],
                         check=True, capture_output=True, text=True).stdout
    assert out.strip() == open(os.path.join(csrc, "lattice_constants.h")).read().strip()


def _call_step(abi, params, ghost=1 << 20, f_in=2 << 30, f_out=4 << 30, mom=None):
    return abi.load().lbm_step(ctypes.byref(params), ghost, f_in, f_out, mom, None)


def test_step_rejects_bad_arguments(abi):
    mk = abi.make_params
    assert _call_step(abi, mk(16, 16, 0.5, 0.0)) == -1           # tau <= 1/2
    assert _call_step(abi, mk(16, 16, 0.7, -1e-3)) == -1         # g < 0
    assert _call_step(abi, mk(-1, 16, 0.7, 0.0)) == -1
    assert _call_step(abi, mk(1 << 15, 1 << 15, 0.7, 0.0)) == -1  # too many sites
    assert _call_step(abi, mk(16, 16, 0.7, 0.0, precision=7)) == -1
    assert _call_step(abi, mk(16, 16, 0.7, 0.0, flags=64)) == -1          # unknown flag
    assert _call_step(abi, mk(16, 16, 0.7, 0.0, flags=abi.PERIODIC_Z | abi.WALL_DIFFUSE)) == -1
    assert _call_step(abi, mk(16, 16, 0.7, 0.0, flags=abi.WALL_DIFFUSE), ghost=None) == -1
    p = mk(16, 16, 0.7, 0.0)
    p.abi_version = 99
    assert _call_step(abi, p) == -6
    assert _call_step(abi, mk(16, 16, 0.7, 0.0), ghost=None) == -1   # walls need a table
    assert _call_step(abi, mk(16, 16, 0.7, 0.0), f_in=None) == -1
    assert _call_step(abi, mk(16, 16, 0.7, 0.0), f_out=(2 << 30) + 8) == -3
    # output overlapping the input
    assert _call_step(abi, mk(16, 16, 0.7, 0.0), f_out=(2 << 30) + 4096) == -2
    assert _call_step(abi, mk(16, 16, 0.7, 0.0), mom=(2 << 30) + 4096) == -2


def test_step_inplace_rejects_bad_arguments(abi):
    lib = abi.load()
    mk = abi.make_params
    p = mk(16, 16, 0.7, 0.0)
    f, gh, mom = 2 << 30, 1 << 20, 3 << 30

    def call(params, ghost=gh, f=f, kind=0, mom=None, scratch=None, nbytes=0):
        return lib.lbm_step_inplace(ctypes.byref(params), ghost, f, kind, mom, scratch, nbytes, None)

    assert call(p, kind=2) == -1
    assert call(p, f=None) == -1
    assert call(p, ghost=None) == -1                          # walls need a table
    assert call(p, f=f + 8) == -3
    assert call(p, mom=f + 4096) == -2                        # moments inside the state
    pd = mk(16, 16, 0.7, 0.0, flags=abi.WALL_DIFFUSE)
    assert call(pd) == -5                                     # diffuse walls need scratch
    need = abi.lbm_scratch_bytes(pd)
    assert need >= 6 * 16 * 8
    assert call(pd, scratch=4 << 30, nbytes=6 * 16 * 8 - 8) == -5
    assert call(pd, scratch=f + 64, nbytes=need) == -2        # scratch inside the state
    assert call(mk(0, 16, 0.7, 0.0)) == 0                     # empty lattice


def test_empty_lattice_is_a_no_op(abi):
    for lx, lz in ((0, 16), (16, 0)):
        assert _call_step(abi, abi.make_params(lx, lz, 0.7, 0.0)) == 0
        assert abi.lbm_scratch_bytes(abi.make_params(lx, lz, 0.7, 0.0)) == 0


def test_every_entry_point_accepts_an_empty_lattice(abi):
    """Lx = 0 or Lz = 0 is a valid lattice with nothing to do: every entry
    point that takes params returns LBM_OK without touching the (here
    fictitious, never dereferenced) device buffers or the HIP runtime, and
    lbm_population_elems / lbm_scratch_bytes return 0."""
    lib = abi.load()
    desc = abi.RT3Desc(1.05, 1.0, 0.95, 4.0, np.ones((2, 2), np.int32), np.zeros((2, 2)))
    a, b, c, d, e = (1 << 30), (3 << 30), (5 << 30), (7 << 30), (9 << 30)
    for lx, lz in ((0, 16), (16, 0), (0, 0)):
        for flags in (0, abi.WALL_DIFFUSE, abi.ADJ_F32 | abi.MOM_F32):
            p = abi.make_params(lx, lz, 0.7, 1e-4, flags=flags)
            r = ctypes.byref(p)
            assert lib.lbm_population_elems(r) == 0 and lib.lbm_scratch_bytes(r) == 0
            calls = {
                "init_rt3": lib.lbm_init_rt3(r, ctypes.byref(desc.c), a, b, c, None),
                "step": lib.lbm_step(r, a, b, c, None, None),
                "step_inplace": lib.lbm_step_inplace(r, a, b, 0, None, None, 0, None),
                "pack": lib.lbm_pack(r, a, b, 8, None),
                "unpack": lib.lbm_unpack(r, a, b, 4, None),
                "moments": lib.lbm_moments(r, a, b, None, None, None, 0, None),
                "moments_noalloc": lib.lbm_moments_noalloc(r, a, b, None, None, None),
                "profiles": lib.lbm_profiles(r, a, b, c, 0, None),
                "objective": lib.lbm_objective(r, ctypes.byref(desc.c), a, 1.0, 1.0, b, None, c, 0, None),
                "adjoint_step": lib.lbm_adjoint_step(r, a, b, c, d, None),
                "adjoint_collide": lib.lbm_adjoint_collide(r, b, c, d, None),
                "adjoint_gather": lib.lbm_adjoint_gather(r, a, b, c, d, None),
                "init_rt3_vjp": lib.lbm_init_rt3_vjp(r, ctypes.byref(desc.c), a, b, c, d, 0, None),
            }
            assert all(v == 0 for v in calls.values()), (lx, lz, flags, calls)


def test_moments_and_init_reject_bad_arguments(abi):
    lib = abi.load()
    p = abi.make_params(64, 64, 0.7, 1e-4)
    need = abi.lbm_scratch_bytes(p)
    assert need > 0
    # sums requested with a scratch buffer that is too small
    st = lib.lbm_moments(ctypes.byref(p), 1 << 30, None, None, 1 << 20, 3 << 30, 64, None)
    assert st == -5
    st = lib.lbm_moments(ctypes.byref(p), 1 << 30, None, None, 1 << 20, None, 0, None)
    assert st == -5
    k = np.ones((2, 40), np.int32)
    ph = np.zeros((2, 40))
    desc = abi.lbm_rt3_desc(1.05, 1.0, 0.95, 4.0, 40, 0,
                            k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), -1.0, -1.0)
    assert lib.lbm_init_rt3(ctypes.byref(p), ctypes.byref(desc), 1 << 20, 1 << 30, 3 << 30, None) == -1
    desc.nmodes = 16
    desc.width = 0.0
    assert lib.lbm_init_rt3(ctypes.byref(p), ctypes.byref(desc), 1 << 20, 1 << 30, 3 << 30, None) == -1
    desc.width = 4.0
    desc.z_lo = float("nan")
    assert lib.lbm_init_rt3(ctypes.byref(p), ctypes.byref(desc), 1 << 20, 1 << 30, 3 << 30, None) == -1
    desc.z_lo = -1.0
    # objective needs t_d > t_m > t_u and scratch; adjoint needs moments unless NO_COLLIDE
    bad = abi.lbm_rt3_desc(0.95, 1.0, 1.05, 4.0, 0, 0, None, None, -1.0, -1.0)
    assert lib.lbm_objective(ctypes.byref(p), ctypes.byref(bad), 1 << 30, 1.0, 1.0, 1 << 20, None,
                             3 << 30, need, None) == -1
    assert lib.lbm_objective(ctypes.byref(p), ctypes.byref(desc), 1 << 30, 1.0, 1.0, 1 << 20, None,
                             3 << 30, 64, None) == -5
    assert lib.lbm_adjoint_step(ctypes.byref(p), None, None, 1 << 30, 3 << 30, None) == -1
    assert lib.lbm_adjoint_step(ctypes.byref(p), None, 1 << 20, 1 << 30, (1 << 30) + 4096, None) == -2
    # the diffuse wall's adjoint needs the wall table, which must not overlap lam_out
    pd = abi.make_params(64, 64, 0.7, 1e-4, flags=abi.WALL_DIFFUSE)
    assert lib.lbm_adjoint_step(ctypes.byref(pd), None, 1 << 20, 1 << 30, 3 << 30, None) == -1
    assert lib.lbm_adjoint_step(ctypes.byref(pd), (3 << 30) + 64, 1 << 20, 1 << 30, 3 << 30, None) == -2
    assert lib.lbm_init_rt3_vjp(ctypes.byref(p), ctypes.byref(desc), 1 << 20, 1 << 30, 1 << 19,
                                3 << 30, 8, None) == -5


def test_error_strings(abi):
    lib = abi.load()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.lbm_strerror(code)


def test_missing_library_fails_loudly(tmp_path):
    """Without liblbm.so every entry into the product raises: there is no CPU
    fallback (run in a fresh interpreter so the loaded library of the other
    tests is untouched)."""
    code = f"""
import sys
sys.path.insert(0, {ROOT!r})
from paper_1405_1253_amd import abi
abi._LIB = None
abi.LIB_PATH = {str(tmp_path / "liblbm.so")!r}
p = abi.make_params(8, 8, 0.7, 1e-4)          # a host struct: no library needed
for call in (abi.load, lambda: abi.lbm_scratch_bytes(p), lambda: abi.lbm_step(p, None, None, None)):
    try:
        call()
    except ImportError as e:
        assert "no CPU fallback" in str(e), e
    else:
        raise SystemExit("no error without the library")
from paper_1405_1253_amd.runtime import Lattice
try:
    Lattice(8, 8, 0.7, 1e-4, device="cpu")
except ImportError:
    pass
else:
    raise SystemExit("Lattice built without the library")
print("ok")
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def header_constants():
    """#define and enum values of include/lbm.h (comments stripped)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {k: int(v) for k, v in re.findall(r"#define\s+(LBM_[A-Z0-9_]+)\s+(-?\d+)u?\b", text)}
    for body in re.findall(r"enum\s+\w+\s*\{(.*?)\}", text, flags=re.S):
        for k, v in re.findall(r"(LBM_[A-Z0-9_]+)\s*=\s*(-?\d+)u?", body):
            out[k] = int(v)
    return out


def test_binding_constants_match_the_header():
    """The ctypes binding's numbers are the header's: ABI version, sizes,
    precisions, flags, in-place kinds and status codes."""
    from paper_1405_1253_amd import abi as mod
    h = header_constants()
    assert h["LBM_ABI_VERSION"] == mod.ABI_VERSION and h["LBM_Q"] == mod.Q
    assert h["LBM_MAX_MODES"] == mod.MAX_MODES and h["LBM_TILE"] == mod.TILE
    for name in ("F64", "F32_DEV", "PERIODIC_Z", "NO_COLLIDE", "ADJ_F32", "WALL_DIFFUSE", "MOM_F32", "COLLIDE_F64",
                 "INPLACE_FROM_STATE", "INPLACE_FROM_STREAMED"):
        assert h["LBM_" + name] == getattr(mod, name), name
    status = {v: k for k, v in h.items() if k in ("LBM_OK",) or (k.startswith("LBM_E") and v < 0)}
    assert status == mod.STATUS


def test_binding_rejects_mismatched_buffers():
    """The binding checks each tensor's element type and size against the
    parameters before the library sees its address: a float32 state with
    FP64 parameters, float moments without LBM_MOM_F32, a short buffer or a
    double adjoint buffer with LBM_ADJ_F32 raise ValueError (no launch; CPU
    tensors suffice because the check comes first)."""
    import torch

    from paper_1405_1253_amd import abi as A
    lx, lz = 4, 9
    p64 = A.make_params(lx, lz, 0.7, 1e-4)
    p32 = A.make_params(lx, lz, 0.7, 1e-4, A.F32_DEV)
    n = A.population_elems(p64)
    assert n == 37 * lx * 512                 # one tile of 512 rows per column
    st64 = torch.zeros(n, dtype=torch.float64)
    st32 = torch.zeros(n, dtype=torch.float32)
    gh64 = torch.zeros((2, 3, 37), dtype=torch.float64)
    gh32 = torch.zeros((2, 3, 37), dtype=torch.float32)
    mom64 = torch.zeros((4, lx, lz), dtype=torch.float64)
    mom32 = torch.zeros((4, lx, lz), dtype=torch.float32)
    cases = [
        lambda: A.lbm_step(p64, gh64, st32, st64),                     # float state, FP64 params
        lambda: A.lbm_step(p32, gh32, st32, st64),                     # double output, FP32 params
        lambda: A.lbm_step(p64, gh32, st64, st64.clone()),             # float wall table
        lambda: A.lbm_step(p64, gh64, st64, st64.clone(), mom32),      # float moments, no MOM_F32
        lambda: A.lbm_step(A.make_params(lx, lz, 0.7, 1e-4, flags=A.MOM_F32), gh64, st64, st64.clone(), mom64),
        lambda: A.lbm_step(p64, gh64, st64[:-1].contiguous(), st64.clone()),      # too short
        lambda: A.lbm_step(p64, gh64, torch.zeros((37, lx, lz), dtype=torch.float64), st64.clone()),  # plain layout
        lambda: A.lbm_pack(p64, torch.zeros((37, lx, lz), dtype=torch.float64), st32),  # element sizes differ
        lambda: A.lbm_unpack(p64, st64[:100].contiguous(), torch.zeros((37, lx, lz), dtype=torch.float64)),
        lambda: A.lbm_step_inplace(p64, gh64, st32, A.INPLACE_FROM_STATE),
        lambda: A.lbm_moments(p64, st64, fields=mom32),
        lambda: A.lbm_moments(p64, st64, tbar=torch.zeros(lz - 1, dtype=torch.float64)),
        lambda: A.lbm_moments(p64, st64, sums=torch.zeros(3, dtype=torch.float64)),
        lambda: A.lbm_adjoint_step(A.make_params(lx, lz, 0.7, 1e-4, flags=A.ADJ_F32), gh64, mom64, st64,
                                   st64.clone()),                       # double lam with ADJ_F32
        lambda: A.lbm_adjoint_step(p64, gh64, mom64, st32, st32.clone()),
        lambda: A.lbm_adjoint_step(p64, gh64, mom64[:3].contiguous(), st64, st64.clone()),
        lambda: A.lbm_profiles(p64, st64, torch.zeros((4, lz - 1), dtype=torch.float64), None),
        lambda: A.lbm_objective(p64, A.RT3Desc(1.05, 1.0, 0.95, 4.0), st64, 1.0, 1.0,
                                torch.zeros(4, dtype=torch.float64)),
        lambda: A.lbm_init_rt3(p64, A.RT3Desc(1.05, 1.0, 0.95, 4.0, np.ones((2, 3)), np.zeros((2, 3))),
                               torch.zeros((2, 3), dtype=torch.float32), st64, gh64),
        lambda: A.lbm_init_rt3(p32, A.RT3Desc(1.05, 1.0, 0.95, 4.0), None, st64, gh32),
        lambda: A.lbm_init_rt3_vjp(p64, A.RT3Desc(1.05, 1.0, 0.95, 4.0, np.ones((2, 3)), np.zeros((2, 3))),
                                   torch.zeros((2, 3), dtype=torch.float64), st64,
                                   torch.zeros((2, 2), dtype=torch.float64), None),
    ]
    for i, call in enumerate(cases):
        with pytest.raises(ValueError):
            call()
    # matching buffers pass the check and reach the GPU-tensor check instead
    with pytest.raises(ValueError, match="GPU tensors"):
        A.lbm_step(p64, gh64, st64, st64.clone(), mom64)


def test_population_buffer_size_and_layout_index():
    """lbm_population_elems against the binding's formula, and the tiled
    index of include/lbm.h (element (l, x, z) at ((zt Lx + x) 37 + l) 512 +
    z - 512 zt) as a bijection of the [37][Lx][Lz] elements onto the buffer
    minus its padding rows."""
    from paper_1405_1253_amd import abi as A
    lib = A.load()
    for lx, lz in ((1, 1), (3, 7), (4, 512), (5, 513), (2, 1100), (4096, 12288), (16384, 32768)):
        p = A.make_params(lx, lz, 0.7, 0.0)
        assert lib.lbm_population_elems(ctypes.byref(p)) == A.population_elems(p) == 37 * lx * (-(-lz // 512)) * 512
    lx, lz = 3, 1100
    l, x, z = np.meshgrid(np.arange(37), np.arange(lx), np.arange(lz), indexing="ij")
    idx = (((z // 512) * lx + x) * 37 + l) * 512 + z % 512
    assert len(np.unique(idx)) == idx.size
    assert idx.max() < A.population_elems(A.make_params(lx, lz, 0.7, 0.0))
    # the tiled_view / column helpers read the same index
    import torch
    t = torch.arange(A.population_elems(A.make_params(lx, lz, 0.7, 0.0)), dtype=torch.float64)
    p = A.make_params(lx, lz, 0.7, 0.0)
    assert np.array_equal(A.column(p, t, 2).numpy(), idx[:, 2, :].astype(np.float64))
