"""Pins of the oracle's equilibrium: its discrete moments up to order 4 are
those of the continuous Maxwellian (Sec. III.A: the Hermite expansion must
reproduce the hydrodynamic moments), computed here by an independent
tensor-product Gauss-Hermite rule from numpy."""
import itertools

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

from oracle import lattice as L
from oracle import lbm


def maxwellian_moment(rho, ux, uz, T, p, q):
    x, w = He.hermegauss(30)
    w = w / np.sqrt(2 * np.pi)
    X = ux + np.sqrt(T) * x
    Z = uz + np.sqrt(T) * x
    return rho * np.sum(w[:, None] * w[None, :] * X[:, None] ** p * Z[None, :] ** q)


def _worst_moment_error(n=12):
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.5, 2.0, n)
    u = rng.uniform(-0.2, 0.2, (n, 2))
    T = rng.uniform(0.8, 1.2, n)
    feq = lbm.equilibrium(rho, u, T)
    _, xi, _, _ = L.lattice()
    worst = 0.0
    for s in range(n):
        for p, q in itertools.product(range(5), range(5)):
            if p + q > 4:
                continue
            got = np.sum(feq[:, s] * xi[:, 0] ** p * xi[:, 1] ** q)
            want = maxwellian_moment(rho[s], u[s, 0], u[s, 1], T[s], p, q)
            worst = max(worst, abs(got - want) / max(1.0, abs(want)))
    return worst


def test_equilibrium_moments_to_order_4():
    assert _worst_moment_error() <= 2e-14


@pytest.mark.parametrize("order", [2, 3, 4])
def test_planted_dropped_temperature_term_is_caught(monkeypatch, order):
    """Drop the (T - 1) part of one Hermite coefficient: the moment pin fails."""
    good = lbm.hermite_coefficients

    def bad(rho, u, T):
        a = list(good(rho, u, T))
        a_cold = good(rho, u, np.ones_like(T))
        a[order] = a_cold[order]
        return tuple(a)

    monkeypatch.setattr(lbm, "hermite_coefficients", bad)
    assert _worst_moment_error() > 1e-6


def test_rest_state_is_weights():
    _, _, w, _ = L.lattice()
    feq = lbm.equilibrium(np.array([1.3]), np.zeros((1, 2)), np.array([1.0]))
    assert np.allclose(feq[:, 0], 1.3 * w, rtol=1e-15, atol=0)


def test_moments_invert_equilibrium():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, (4, 5))
    u = rng.uniform(-0.1, 0.1, (4, 5, 2))
    T = rng.uniform(0.9, 1.1, (4, 5))
    r2, u2, T2 = lbm.moments(lbm.equilibrium(rho, u, T))
    assert np.allclose(r2, rho, rtol=1e-14, atol=0)
    assert np.allclose(u2, u, rtol=0, atol=1e-15)
    assert np.allclose(T2, T, rtol=1e-14, atol=0)
