"""Pins of the oracle's collision and streaming.

Collision (Sec. III.A, forcing by shifted equilibrium): with the shift
u + g tau and T + tau(1 - tau) g^2/d one collision leaves rho and T unchanged
and adds exactly rho g to the momentum; with g = 0 it conserves mass,
momentum and energy.  Streaming is checked against a brute-force loop over
sites written independently here.
"""
import numpy as np
import pytest

from oracle import lattice as L
from oracle import lbm
from paper_1405_1253_amd import workload as W


def _noneq_state(seed, shape=(6, 7)):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.7, 1.3, shape)
    u = rng.uniform(-0.1, 0.1, shape + (2,))
    T = rng.uniform(0.9, 1.1, shape)
    f = lbm.equilibrium(rho, u, T)
    return f * (1 + 0.05 * rng.standard_normal(f.shape))   # off equilibrium


@pytest.mark.parametrize("tau,g", [(0.7, 1e-3), (0.55, 0.02), (1.3, 0.05)])
def test_collide_force_identities(tau, g):
    f = _noneq_state(1)
    p = lbm.Params(6, 7, tau, g)
    rho, u, T = lbm.moments(f)
    r2, u2, T2 = lbm.moments(lbm.collide(f, p))
    assert np.allclose(r2, rho, rtol=1e-14, atol=0)
    assert np.allclose(rho[..., None] * u2, rho[..., None] * (u + np.array([0.0, -g])),
                       rtol=0, atol=1e-14)
    assert np.allclose(T2, T, rtol=1e-13, atol=0)


def test_planted_unshifted_temperature_is_caught(monkeypatch):
    """Forcing the velocity but not the temperature breaks T* = T."""
    good = lbm.shifted_state
    monkeypatch.setattr(lbm, "shifted_state", lambda u, T, p: (good(u, T, p)[0], T))
    f = _noneq_state(1)
    p = lbm.Params(6, 7, 0.7, 0.05)
    T = lbm.moments(f)[2]
    assert np.abs(lbm.moments(lbm.collide(f, p))[2] / T - 1).max() > 1e-5


def test_collide_conserves_without_gravity():
    f = _noneq_state(2)
    p = lbm.Params(6, 7, 0.8, 0.0)
    fs = lbm.collide(f, p)
    _, xi, _, _ = L.lattice()
    for weight in (np.ones(37), xi[:, 0], xi[:, 1], (xi ** 2).sum(1)):
        a = np.tensordot(weight, f, axes=(0, 0))
        b = np.tensordot(weight, fs, axes=(0, 0))
        assert np.allclose(a, b, rtol=0, atol=1e-14)


def test_collide_tau_one_gives_shifted_equilibrium():
    f = _noneq_state(3)
    g = 0.01
    fs = lbm.collide(f, lbm.Params(6, 7, 1.0, g))
    rho, u, T = lbm.moments(f)
    want = lbm.equilibrium(rho, u + np.array([0.0, -g]), T)   # tau(1-tau) = 0
    assert np.allclose(fs, want, rtol=1e-14, atol=0)


def _brute_pull(f, ghost, periodic_z):
    """out[l, x, z] = f[l, x - ex, z - ez] by explicit loops."""
    E, _, _, _ = L.lattice()
    Q, lx, lz = f.shape
    out = np.zeros_like(f)
    for l in range(Q):
        for x in range(lx):
            for z in range(lz):
                xs = (x - E[l, 0]) % lx
                zs = z - E[l, 1]
                if periodic_z:
                    out[l, x, z] = f[l, xs, zs % lz]
                elif zs < 0:
                    out[l, x, z] = ghost[0, -1 - zs, l]       # row -1 is ghost 0
                elif zs >= lz:
                    out[l, x, z] = ghost[1, zs - lz, l]       # row Lz is ghost 0
                else:
                    out[l, x, z] = f[l, xs, zs]
    return out


@pytest.mark.parametrize("lx,lz,periodic", [(5, 9, False), (7, 4, False), (6, 5, True), (4, 2, False)])
def test_pull_matches_brute_force(lx, lz, periodic):
    f = W.random_populations(11, lx, lz)
    ghost = W.random_ghost(12)
    p = lbm.Params(lx, lz, 0.7, 0.0, periodic_z=periodic, no_collide=True)
    assert np.array_equal(lbm.pull(f, ghost, p), _brute_pull(f, ghost, periodic))


def test_pull_is_permutation_and_period():
    f = W.random_populations(5, 12, 12)
    p = lbm.Params(12, 12, 0.7, 0.0, periodic_z=True, no_collide=True)
    g = lbm.pull(f, None, p)
    for l in range(37):
        assert np.array_equal(np.sort(g[l].ravel()), np.sort(f[l].ravel()))
    for _ in range(11):
        g = lbm.pull(g, None, p)
    assert np.array_equal(g, f)                 # L steps bring every population home
