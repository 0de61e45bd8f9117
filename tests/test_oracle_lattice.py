"""Pins of the oracle's velocity set, quadrature and Hermite tensors.

The quadrature must integrate every monomial up to degree 9 of the
unit-variance 2-D Gaussian exactly (reference values from numpy's
Gauss-Hermite rule, an independent library routine) and must give the
lattice constant printed in the caption of Fig. 2.
"""
import itertools

import numpy as np
from numpy.polynomial import hermite_e as He

from oracle import lattice as L
from tests._golden import paper_constants


def gaussian_moment(p):
    x, w = He.hermegauss(20)
    return float(np.sum(w * x ** p) / np.sqrt(2 * np.pi))


def test_lattice_constant_matches_paper():
    r_paper = paper_constants()["lattice_constant_r"]
    _, _, _, r = L.lattice()
    # printed to 4 decimals (Fig. 2 caption): the solved r must round down to it
    assert r_paper <= r < r_paper + 1e-4
    assert abs(r - 1.196979770393074) < 1e-13


def test_velocity_set_structure():
    E, xi, w, r = L.lattice()
    c = paper_constants()
    assert len(E) == c["n_velocities"]
    assert len({tuple(e) for e in E}) == 37
    assert np.abs(E).max() == c["halo_x"] == c["wall_rows"]
    assert tuple(E[0]) == (0, 0)
    for l in range(1, 37, 2):                      # +e then -e
        assert tuple(E[l]) == tuple(-E[l + 1])
    # closed under the square's symmetry group (needed for isotropy)
    S = {tuple(e) for e in E}
    for ex, ez in S:
        assert (ez, ex) in S and (-ex, ez) in S and (ex, -ez) in S


def test_weights_positive_and_normalised():
    _, _, w, _ = L.lattice()
    assert np.all(w > 0)
    assert abs(w.sum() - 1.0) < 1e-15
    E, shell = L.velocity_set()
    for s in range(8):
        assert np.ptp(w[shell == s]) == 0.0         # one weight per shell


def test_quadrature_exact_to_degree_9():
    _, xi, w, _ = L.lattice()
    for p, q in itertools.product(range(10), range(10)):
        if p + q > 9:
            continue
        got = np.sum(w * xi[:, 0] ** p * xi[:, 1] ** q)
        want = gaussian_moment(p) * gaussian_moment(q)
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (p, q, got, want)


def test_quadrature_not_exact_at_degree_10():
    _, xi, w, _ = L.lattice()
    got = np.sum(w * xi[:, 0] ** 10)
    assert abs(got - gaussian_moment(10)) > 10.0     # 914.99... vs 945


def test_hermite_tensors_match_library_polynomials():
    _, xi, _, _ = L.lattice()
    H = L.hermite_tensors(xi)
    for n in range(5):
        for idx in itertools.product(range(2), repeat=n):
            nx, nz = idx.count(0), idx.count(1)
            want = (He.hermeval(xi[:, 0], [0] * nx + [1])
                    * He.hermeval(xi[:, 1], [0] * nz + [1]))
            got = H[n][(slice(None),) + idx]
            assert np.allclose(got, want, rtol=0, atol=1e-12), (n, idx)
