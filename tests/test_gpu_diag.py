"""Diagnostics and the paper-geometry initial states on the GPU path:
row profiles (Figs. 8-9) and the objective against the oracle; the
double-front (middle layer delta) and single-front states of Sec. IV."""
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


@pytest.fixture(scope="module")
def state():
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    p = O.Params(wl.lx, wl.lz, wl.tau, wl.g)
    f0, ghost = O.init_rt3(p, O.RT3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase), m.amp * 3)
    return wl, p, O.run(f0, ghost, p, 60)


@pytest.mark.parametrize("prec", ["f64", "f32dev"])
def test_profiles_parity(abi, state, prec):
    wl, p, f = state
    w = abi.lbm_lattice()[1]
    if prec == "f32dev":
        d = (f - w[:, None, None]).astype(np.float32)
        f = d.astype(np.float64) + w[:, None, None]          # the state the GPU sees
    params = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, abi.F64 if prec == "f64" else abi.F32_DEV)
    buf = abi.to_tiled(params, d if prec == "f32dev" else f)
    prof = torch.empty((4, wl.lz), dtype=torch.float64, device=DEV)
    scratch = torch.empty(abi.lbm_scratch_bytes(params), dtype=torch.uint8, device=DEV)
    abi.lbm_profiles(params, buf, prof, scratch)
    got = prof.cpu().numpy()
    want = O.profiles(f, p)
    assert want[1].max() > 1e-4 and want[3].max() > 0
    for i in range(4):
        assert np.abs(got[i] - want[i]).max() <= 1e-12 * np.abs(want[i]).max(), i


@pytest.mark.parametrize("single", [False, True])
def test_paper_geometry_init_and_objective(abi, single):
    """Reduced copy of the Table II runs: middle layer of width 20 rows
    centred in a 300-row box (double front) or one interface at mid-height
    (single front, no jump at the lower interface; diagnostics use the
    virtual T_m = 1)."""
    lx, lz, tau, g = 96, 300, 0.55, 5e-4
    t_d, t_m, t_u = 1.025, (1.025 if single else 1.0), 0.975
    z_lo, z_hi = (75.0, 150.0) if single else (140.0, 160.0)
    m = W.draw_modes(3)
    p = O.Params(lx, lz, tau, g)
    desc = O.RT3(t_d, t_m, t_u, 4.0, m.k, m.phase, z_lo, z_hi)
    f0, ghost = O.init_rt3(p, desc, m.amp)
    f5 = O.run(f0, ghost, p, 5)
    from paper_1405_1253_amd.runtime import Lattice
    lat = Lattice(lx, lz, tau, g)
    lat.init_rt3(t_d, t_m, t_u, 4.0, m.k, m.phase, m.amp, z_lo, z_hi)
    assert np.max(np.abs(lat.state_soa().cpu().numpy() / f0 - 1)) <= 1e-13
    assert np.max(np.abs(lat.ghost.cpu().numpy() / ghost - 1)) <= 1e-13
    lat.step(5)
    assert np.max(np.abs(lat.state_soa().cpu().numpy() / f5 - 1)) <= 1e-12
    lat.diag_desc = abi.RT3Desc(t_d, 1.0, t_u, 4.0)
    j = lat.objective().cpu().numpy()
    Jo, ke, L = O.objective(f5, p, t_u, 1.0, t_d)
    assert L > 5.0
    assert abs(j[0] / Jo - 1) <= 1e-12 and abs(j[2] / L - 1) <= 1e-12
