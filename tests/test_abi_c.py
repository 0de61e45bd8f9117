"""The boundary from plain C (no GPU needed): a C99 program that includes
include/lbm.h, compiled by gcc with -pedantic -Werror and linked against the
library, calls the host-only entry points and the argument checks that
return before any launch, and agrees with the Python binding on what it
prints.  This pins that the header needs no C++ and no HIP header, and that
the exported symbols have C linkage."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_SOURCE = r"""
#include <stdio.h>
#include <string.h>
#include "lbm.h"

static lbm_params make(int lx, int lz, int precision, unsigned flags) {
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.abi_version = LBM_ABI_VERSION;
    p.lx = lx;
    p.lz = lz;
    p.precision = precision;
    p.flags = flags;
    p.tau = 0.7;
    p.g = 1e-4;
    return p;
}

int main(void) {
    double r = 0.0, w[LBM_Q];
    int32_t e[2 * LBM_Q];
    int l, st;
    lbm_params p;
    if (lbm_lattice(&r, w, e) != LBM_OK) return 1;
    printf("r %.17g\n", r);
    for (l = 0; l < LBM_Q; ++l) printf("w %d %.17g %d %d\n", l, w[l], (int)e[2 * l], (int)e[2 * l + 1]);
    p = make(16, 1040, LBM_F64, 0u);
    printf("elems %lu\n", (unsigned long)lbm_population_elems(&p));
    printf("scratch %lu\n", (unsigned long)lbm_scratch_bytes(&p));
    p = make(33, 777, LBM_F32_DEV, LBM_WALL_DIFFUSE);
    printf("elems_f32 %lu\n", (unsigned long)lbm_population_elems(&p));
    printf("scratch_diffuse %lu\n", (unsigned long)lbm_scratch_bytes(&p));
    p.abi_version = LBM_ABI_VERSION + 1u;
    st = lbm_step(&p, NULL, NULL, NULL, NULL, NULL);
    printf("version %d %s\n", st, lbm_strerror(st));
    p = make(16, 1040, LBM_F64, 0u);
    p.tau = 0.5;
    st = lbm_step(&p, NULL, NULL, NULL, NULL, NULL);
    printf("tau %d %s\n", st, lbm_strerror(st));
    p = make(16, 1040, LBM_F64, 0u);
    st = lbm_adjoint_gather(&p, NULL, NULL, NULL, NULL, NULL);
    printf("null %d\n", st);
    st = lbm_step(&p, (void *)0x100000, (void *)0x200008, (void *)0x400000, NULL, NULL);
    printf("align %d\n", st);
    printf("hip [%s]\n", lbm_last_hip_error());
    return 0;
}
"""


@pytest.fixture(scope="module")
def abi():
    from paper_1405_1253_amd import abi as mod
    mod.load()
    return mod


@pytest.fixture(scope="module")
def c_output(abi, tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    d = tmp_path_factory.mktemp("cabi")
    src, exe = d / "use_lbm.c", d / "use_lbm"
    src.write_text(C_SOURCE)
    libdir = os.path.dirname(abi.LIB_PATH)
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                    "-L", libdir, "-l:" + os.path.basename(abi.LIB_PATH), "-Wl,-rpath," + libdir],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=120).stdout
    lines = {}
    for ln in out.splitlines():
        key, rest = ln.split(" ", 1)
        if key == "w":                     # "w <l> <w_l> <e_x> <e_z>"
            key, rest = f"w{rest.split(' ', 1)[0]}", rest
        lines[key] = rest
    return lines


def test_c_program_sees_the_bindings_lattice(abi, c_output):
    r, w, e = abi.lbm_lattice()
    assert float(c_output["r"]) == r
    for l in range(abi.Q):
        _, wl, ex, ez = c_output[f"w{l}"].split(" ")
        assert float(wl) == w[l] and (int(ex), int(ez)) == tuple(e[l])


def test_c_program_sizes_match_the_binding(abi, c_output):
    p = abi.make_params(16, 1040, 0.7, 1e-4)
    q = abi.make_params(33, 777, 0.7, 1e-4, abi.F32_DEV, abi.WALL_DIFFUSE)
    assert int(c_output["elems"]) == abi.population_elems(p) == 37 * 16 * 3 * 512
    assert int(c_output["elems_f32"]) == abi.population_elems(q) == 37 * 33 * 2 * 512
    assert int(c_output["scratch"]) == abi.lbm_scratch_bytes(p)
    assert int(c_output["scratch_diffuse"]) == abi.lbm_scratch_bytes(q)


def test_c_program_argument_errors(abi, c_output):
    st, msg = c_output["version"].split(" ", 1)
    assert int(st) == -6 and "version" in msg.lower()
    st, msg = c_output["tau"].split(" ", 1)
    assert int(st) == -1 and msg
    assert int(c_output["null"]) == -1
    assert int(c_output["align"]) == -3
    assert c_output["hip"] == "[]"          # refused on the host: no HIP call was made
