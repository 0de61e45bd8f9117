"""Host-side analysis of the long runs (Sec. IV)."""
import numpy as np

from paper_1405_1253_amd import campaign as C
from paper_1405_1253_amd import workload as W


def test_alpha_recovers_quadratic_growth():
    """L = alpha At g t^2 (eq. eqL) gives Ldot^2 / (4 At g L) = alpha (eq. eqL2)."""
    t = np.linspace(0.0, 5e4, 201)
    for alpha in (0.02, 0.07):
        L = alpha * 0.025 * 1.5e-5 * t ** 2
        a = C.alpha_tot(t, L, 0.025, 1.5e-5)
        assert np.allclose(a[1:-1], alpha, rtol=1e-12)


def test_paper_workloads():
    """Table II: At = 0.025, g = 1.5e-5, 2400 x 6144, delta = 500; the RT time
    unit sqrt(Lx / (g At)) with Lx in length units (one column = r)."""
    r = 1.196979770393074
    for name in ("rt3_2400x6144_paper", "rt2_2400x6144_paper"):
        wl = W.WORKLOADS[name]
        assert abs(wl.atwood - 0.025) < 1e-12 and wl.g == 1.5e-5
        assert (wl.lx, wl.lz) == (2400, 6144)
        assert abs(C.rt_time(wl, r) - np.sqrt(r * 2400 / (1.5e-5 * 0.025))) < 1e-6
    d = W.WORKLOADS["rt3_2400x6144_paper"]
    assert d.z_hi - d.z_lo == 500 and d.z_lo + d.z_hi == d.lz
    # Ra = dT Lz^3 g / (nu kappa) = 1e10 at Pr = 1, Lz in length units
    nu = d.tau - 0.5
    ra = (d.t_d - d.t_u) * (r * d.lz) ** 3 * d.g / nu ** 2
    assert abs(ra / 1e10 - 1) < 1e-3


def test_campaign_options_reach_the_run(tmp_path, monkeypatch):
    """--seed, --precision and --collide-f64 change the workload and the
    lattice flags handed to the run (the run itself is replaced here: no
    GPU), and the series the run returns is written with alpha_tot."""
    from paper_1405_1253_amd import abi
    seen = {}

    def fake_run(wl, nsteps, every, ptimes, progress, flags=0):
        seen.update(wl=wl, nsteps=nsteps, flags=flags, ptimes=list(ptimes))
        t = np.arange(0, nsteps + 1, every, dtype=float)
        return {"t": t, "L_tot": 1.0 + t ** 2, "L_u": t, "L_d": t, "KE": t, "profile_steps": np.array([]),
                "profiles": np.zeros((0, 4, wl.lz)), "tau_rt": 1.0, "atwood": wl.atwood, "g": wl.g,
                "seconds": 0.0}

    monkeypatch.setattr(C, "run", fake_run)
    out = tmp_path / "run.npz"
    C.main(["--workload", "rt3_2400x6144_paper", "--precision", "f32dev", "--collide-f64", "--seed", "1406",
            "--tau-rt", "0.5", "--every", "2000", "--profiles-at", "0,0.25", "--out", str(out)])
    assert seen["wl"].precision == "f32dev" and seen["wl"].seed == 1406
    assert seen["flags"] == abi.COLLIDE_F64 and seen["nsteps"] % 2000 == 0 and seen["nsteps"] > 0
    assert seen["ptimes"][0] == 0 and all(p % 2000 == 0 for p in seen["ptimes"])
    C.main(["--workload", "rt2_2400x6144_paper", "--precision", "f64", "--tau-rt", "0.5", "--out", str(out)])
    assert seen["wl"].precision == "f64" and seen["flags"] == 0
    saved = np.load(out)
    assert np.isfinite(saved["alpha_tot"][1:-1]).all()
