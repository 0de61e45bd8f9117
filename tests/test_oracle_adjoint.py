"""Pins of the oracle's hand-written adjoint against complex-step derivatives
of the forward oracle (exact to rounding: J'(a) = Im J(a + i h)/h with
h = 1e-30) and by dot-product tests of each transposed piece."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import lbm as O
from paper_1405_1253_amd import workload as W

H = 1e-30


def _near_eq(seed, lx, lz):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.9, 1.1, (lx, lz))
    u = rng.uniform(-0.05, 0.05, (lx, lz, 2))
    T = rng.uniform(0.95, 1.05, (lx, lz))
    f = O.equilibrium(rho, u, T)
    return f * (1 + 0.01 * rng.standard_normal(f.shape))


@pytest.mark.parametrize("periodic", [False, True])
def test_step_vjp_dot_product(periodic):
    lx, lz = 7, 11
    p = O.Params(lx, lz, 0.65, 2e-3, periodic_z=periodic)
    f = _near_eq(1, lx, lz)
    ghost = W.random_ghost(2) * 0.01
    rng = np.random.default_rng(3)
    v = rng.standard_normal(f.shape)
    lam = rng.standard_normal(f.shape)
    jv = np.imag(O.step(f + 1j * H * v, ghost, p)) / H
    lhs = np.sum(lam * jv)
    rhs = np.sum(A.step_vjp(lam, f, ghost, p) * v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_collide_vjp_dot_product():
    """C^T alone: <lam, (d collide/dg) v> = <collide_vjp(lam, g), v>, the
    Jacobian-vector product by complex step of the forward collide."""
    lx, lz = 5, 6
    p = O.Params(lx, lz, 0.65, 2e-3)
    g = _near_eq(4, lx, lz)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(g.shape)
    lam = rng.standard_normal(g.shape)
    jv = np.imag(O.collide(g + 1j * H * v, p)) / H
    lhs = np.sum(lam * jv)
    rhs = np.sum(A.collide_vjp(lam, g, p) * v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("wall,periodic", [("dirichlet", False), ("dirichlet", True), ("diffuse", False)])
def test_pull_transpose_dot_product(wall, periodic):
    """S^T alone: <G, (d pull/df) v> = <pull_transpose(G), v> for both wall
    rules and the periodic test mode (the pull is affine in f: the table
    rows are constant, the diffuse wall's emissions linear in f)."""
    lx, lz = 7, 9
    p = O.Params(lx, lz, 0.65, 2e-3, periodic_z=periodic, wall=wall)
    f = _near_eq(6, lx, lz)
    ghost = W.random_ghost(7) * 0.01 + (0.0 if wall == "dirichlet" else 0.02)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(f.shape)
    G = rng.standard_normal(f.shape)
    jv = np.imag(O.pull(f + 1j * H * v, ghost, p)) / H
    lhs = np.sum(G * jv)
    rhs = np.sum(A.pull_transpose(G, p, ghost) * v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_objective_vjp_matches_complex_step():
    wl = W.WORKLOADS["rt3_128x384"]
    lx, lz = 12, 60
    m = W.draw_modes(5, 3)
    p = O.Params(lx, lz, 0.7, 1e-3)
    desc = O.RT3(wl.t_d, wl.t_m, wl.t_u, 4.0, m.k, m.phase)
    f0, ghost = O.init_rt3(p, desc, m.amp * 3)
    f = O.run(f0, ghost, p, 5)
    lam = A.objective_vjp(f, p, desc.t_u, desc.t_m, desc.t_d, 2.0, 0.5)
    v = np.random.default_rng(4).standard_normal(f.shape) * 1e-2
    jv = np.imag(O.objective(f + 1j * H * v, p, desc.t_u, desc.t_m, desc.t_d, 2.0, 0.5)[0]) / H
    assert abs(np.sum(lam * v) - jv) <= 1e-12 * abs(jv)


def test_rollout_gradient_matches_complex_step():
    lx, lz, steps = 16, 48, 6
    m = W.draw_modes(11, 4)
    p = O.Params(lx, lz, 0.7, 1e-3)
    desc = O.RT3(1.05, 1.0, 0.95, 3.0, m.k, m.phase)
    amp = m.amp * 2
    J, grad = A.rollout_gradient(p, desc, amp, steps)
    for fr, j in [(0, 0), (0, 3), (1, 1), (1, 2)]:
        da = np.zeros_like(amp, dtype=complex)
        da[fr, j] = 1j * H
        f0, ghost = O.init_rt3(p, desc, amp + da)
        Jc = O.objective(O.run(f0, ghost, p, steps), p, desc.t_u, desc.t_m, desc.t_d)[0]
        cs = np.imag(Jc) / H
        assert abs(np.real(Jc) - J) <= 1e-14 * abs(J)
        assert abs(grad[fr, j] - cs) <= 1e-10 * np.abs(grad).max(), (fr, j, grad[fr, j], cs)


def test_init_vjp_matches_complex_step():
    lx, lz = 10, 36
    m = W.draw_modes(12, 5)
    p = O.Params(lx, lz, 0.7, 5e-3)
    desc = O.RT3(1.05, 1.0, 0.95, 2.5, m.k, m.phase)
    lam = np.random.default_rng(6).standard_normal((37, lx, lz))
    got = A.init_vjp(lam, p, desc, m.amp)
    for fr in range(2):
        for j in range(5):
            da = np.zeros_like(m.amp, dtype=complex)
            da[fr, j] = 1j * H
            f0, _ = O.init_rt3(p, desc, m.amp + da)
            cs = np.sum(lam * np.imag(f0)) / H
            assert abs(got[fr, j] - cs) <= 1e-12 * max(1.0, abs(cs)), (fr, j)


def test_rollout_gradient_central_difference():
    """Independent of complex arithmetic: central FD with h = 1e-6."""
    lx, lz, steps = 12, 48, 4
    m = W.draw_modes(13, 3)
    p = O.Params(lx, lz, 0.7, 1e-3)
    desc = O.RT3(1.05, 1.0, 0.95, 3.0, m.k, m.phase)
    J, grad = A.rollout_gradient(p, desc, m.amp, steps)
    h = 1e-6
    for fr, j in [(0, 1), (1, 0)]:
        Js = []
        for s in (+1, -1):
            a = m.amp.copy()
            a[fr, j] += s * h
            f0, ghost = O.init_rt3(p, desc, a)
            Js.append(O.objective(O.run(f0, ghost, p, steps), p, desc.t_u, desc.t_m, desc.t_d)[0])
        fd = (Js[0] - Js[1]) / (2 * h)
        assert abs(fd - grad[fr, j]) <= 1e-6 * np.abs(grad).max()
