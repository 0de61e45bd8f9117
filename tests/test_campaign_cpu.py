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
