"""Hand-written reverse-mode derivative of the oracle's N-step rollout.

Test infrastructure (see ``oracle/__init__``).  The paper has no adjoint; this
differentiates the forward oracle (``oracle.lbm``) exactly, step by step in
reverse, so that

    dJ/d amp  for  J = wk * KE(f*_N) + wl * (L_u + L_d)(f*_N),
    f*_N = step^N(init_rt3(amp))

can be compared with the HIP adjoint.  It is pinned against complex-step
derivatives of the forward oracle and by dot-product tests (tests/).

Notation: lam_t = dJ/df*_t (adjoint of the stored post-collision state),
g_t = pull(f*_{t-1}) the pre-collision populations of step t with moments
m_t = (rho, u, T), F(m) the force-shifted equilibrium (Sec. III.A).
One step back:
    dJ/dg_t,l = (1 - omega) lam_t,l + sum_k mu_k dm_k/dg_l,
    mu_k = omega * sum_l lam_t,l dF_l/dm_k,
    dm/dg_l = (1, (xi_l - u)/rho, (|xi_l - u|^2 - D T)/(D rho)),
    lam_{t-1,l}(y) = dJ/dg_t,l(y + e_l)   where y + e_l is inside the
                                           wall-bounded rows; beyond a wall it
                                           is zero for the Dirichlet wall (a
                                           constant table) and the ghost site's
                                           summed sensitivity for the diffuse
                                           wall (see ``pull_transpose``)
"""
import numpy as np

from .lattice import D, hermite_tensors, lattice
from . import lbm


def _flat(a, n):
    return a.reshape(a.shape[0], 2 ** n) if n else a


def hermite_coefficient_derivatives(rho, v, T):
    """Partial derivatives of the Hermite coefficients a^(n)(rho, v, T).

    Returns (d_rho, d_v, d_T): lists over n = 0..4 of arrays
      d_rho[n] [S, 2^n]       = d a^(n) / d rho   (= a^(n) / rho)
      d_v[n]   [S, 2, 2^n]    = d a^(n) / d v_m   (m on axis 1)
      d_T[n]   [S, 2^n]       = d a^(n) / d T
    written out from a^(n) of ``lbm.hermite_coefficients`` term by term.
    """
    S = rho.shape[0]
    d = np.eye(D)
    th = T - 1.0
    dt = np.result_type(rho, v, T)
    a = lbm.hermite_coefficients(rho, v, T)
    d_rho = [_flat(a[n], n) / (rho[:, None] if n else rho) for n in range(5)]

    # d/dv_m --------------------------------------------------------------
    dv0 = np.zeros((S, D), dtype=dt)
    dv1 = rho[:, None, None] * np.broadcast_to(d, (S, D, D))          # [S, m, i]
    # a2_ij = rho (v_i v_j + th d_ij)
    dv2 = rho[:, None, None, None] * (np.einsum("mi,sj->smij", d, v) + np.einsum("si,mj->smij", v, d))
    # a3_ijk = rho (v_i v_j v_k + th (v_i d_jk + v_j d_ik + v_k d_ij))
    dv3 = rho[:, None, None, None, None] * (
        np.einsum("mi,sj,sk->smijk", d, v, v) + np.einsum("si,mj,sk->smijk", v, d, v)
        + np.einsum("si,sj,mk->smijk", v, v, d)
        + th[:, None, None, None, None] * (np.einsum("mi,jk->mijk", d, d)
                                           + np.einsum("mj,ik->mijk", d, d)
                                           + np.einsum("mk,ij->mijk", d, d))[None])
    # a4_ijkl = rho (v_i v_j v_k v_l + th * sum_6 (v_a v_b d_cd) + th^2 * sum_3 (d d))
    four = (np.einsum("mi,sj,sk,sl->smijkl", d, v, v, v) + np.einsum("si,mj,sk,sl->smijkl", v, d, v, v)
            + np.einsum("si,sj,mk,sl->smijkl", v, v, d, v) + np.einsum("si,sj,sk,ml->smijkl", v, v, v, d))

    def dpair(p, q, r, s_):
        # d/dv_m of v_p v_q d_rs, indices given as einsum letters
        idx = "ijkl"
        lhs = f"m{p},s{q},{r}{s_}->smijkl"
        rhs = f"s{p},m{q},{r}{s_}->smijkl"
        return np.einsum(lhs, d, v, d) + np.einsum(rhs, v, d, d)

    six = (dpair("i", "j", "k", "l") + dpair("i", "k", "j", "l") + dpair("i", "l", "j", "k")
           + dpair("j", "k", "i", "l") + dpair("j", "l", "i", "k") + dpair("k", "l", "i", "j"))
    dv4 = rho[:, None, None, None, None, None] * (four + th[:, None, None, None, None, None] * six)
    d_v = [dv0, dv1, dv2.reshape(S, D, 4), dv3.reshape(S, D, 8), dv4.reshape(S, D, 16)]

    # d/dT ------------------------------------------------------------------
    vv = np.einsum("si,sj->sij", v, v)
    dT0 = np.zeros(S, dtype=dt)
    dT1 = np.zeros((S, 2), dtype=dt)
    dT2 = rho[:, None, None] * np.broadcast_to(d, (S, D, D))
    dT3 = rho[:, None, None, None] * (np.einsum("si,jk->sijk", v, d) + np.einsum("sj,ik->sijk", v, d)
                                      + np.einsum("sk,ij->sijk", v, d))
    dd = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
          + np.einsum("il,jk->ijkl", d, d))
    dT4 = rho[:, None, None, None, None] * (
        np.einsum("sij,kl->sijkl", vv, d) + np.einsum("sik,jl->sijkl", vv, d)
        + np.einsum("sil,jk->sijkl", vv, d) + np.einsum("sjk,il->sijkl", vv, d)
        + np.einsum("sjl,ik->sijkl", vv, d) + np.einsum("skl,ij->sijkl", vv, d)
        + 2 * th[:, None, None, None, None] * dd[None])
    d_T = [dT0, dT1, dT2.reshape(S, 4), dT3.reshape(S, 8), dT4.reshape(S, 16)]
    return d_rho, d_v, d_T


def equilibrium_vjp(lam, rho, v, T):
    """(dJ/drho, dJ/dv [.., 2], dJ/dT) for lam = dJ/df^eq [37, ...] at f^eq(rho, v, T).

    With Lam^(n) = sum_l lam_l w_l H^(n)(xi_l):
        dJ/dq = sum_n (1/n!) (d a^(n)/dq) : Lam^(n)."""
    _, xi, w, _ = lattice()
    shape = np.shape(rho)
    lam_f = np.moveaxis(lam.reshape(lam.shape[0], -1), 0, 1) * w[None, :]   # [S, 37]
    H = hermite_tensors(xi)
    Lam = [lam_f @ _flat(H[n], n) if n else lam_f @ H[0] for n in range(5)]
    d_rho, d_v, d_T = hermite_coefficient_derivatives(
        np.reshape(rho, -1), np.reshape(v, (-1, D)), np.reshape(T, -1))
    fact = (1.0, 1.0, 2.0, 6.0, 24.0)
    g_rho = d_rho[0] * Lam[0]
    g_v = np.zeros_like(np.reshape(v, (-1, D)), dtype=np.result_type(lam, v))
    g_T = np.zeros_like(g_rho)
    for n in range(1, 5):
        g_rho = g_rho + np.sum(d_rho[n] * Lam[n], axis=1) / fact[n]
        g_v = g_v + np.einsum("smk,sk->sm", d_v[n], Lam[n]) / fact[n]
        g_T = g_T + np.sum(d_T[n] * Lam[n], axis=1) / fact[n]
    return g_rho.reshape(shape), g_v.reshape(shape + (D,)), g_T.reshape(shape)


def moments_vjp(f, g_rho, g_u, g_T):
    """dJ/df_l given dJ/d(rho, u, T) of moments(f): the transposed Jacobian
    dm/df_l = (1, (xi_l - u)/rho, (|xi_l - u|^2 - D T)/(D rho))."""
    _, xi, _, _ = lattice()
    rho, u, T = lbm.moments(f)
    bshape = (f.shape[0],) + (1,) * (f.ndim - 1)
    cx = xi[:, 0].reshape(bshape) - u[..., 0][None]
    cz = xi[:, 1].reshape(bshape) - u[..., 1][None]
    return (g_rho[None] + (g_u[..., 0][None] * cx + g_u[..., 1][None] * cz) / rho[None]
            + g_T[None] * (cx * cx + cz * cz - D * T[None]) / (D * rho[None]))


def pull_transpose(G, p, ghost=None):
    """Adjoint of ``lbm.pull`` with respect to its state argument:
    out_l(y) = G_l(y + e_l) where y + e_l lies inside the wall-bounded rows.

    Where y + e_l is a ghost site: zero for the Dirichlet wall (the table is
    constant); for the diffuse wall the ghost site's emitted populations are
    c_m * M with M the sum of the populations that streamed into it, so every
    one of those receives A = sum_m c_m G_m(ghost site + e_m) over the m that
    point back into the lattice (``lbm.wall_emission`` gives c from ``ghost``).
    """
    E, _, _, _ = lattice()
    out = np.empty_like(G)
    lz = G.shape[2]
    diffuse = not p.periodic_z and p.wall == "diffuse"
    if diffuse:
        c = lbm.wall_emission(ghost, lz)
        A = np.zeros((2, 3, G.shape[1]), dtype=G.dtype)
        for side in range(2):
            for i in range(3):
                k = lbm.ghost_row(side, i, lz)
                for m in range(G.shape[0]):
                    ex, ez = int(E[m, 0]), int(E[m, 1])
                    if 0 <= k + ez < lz:
                        A[side, i] += c[side, i, m] * np.roll(G[m, :, k + ez], -ex)
    for l in range(G.shape[0]):
        ex, ez = int(E[l, 0]), int(E[l, 1])
        out[l] = np.roll(G[l], shift=(-ex, -ez), axis=(0, 1))
        if p.periodic_z:
            continue
        for y in range(lz):
            k = y + ez
            if 0 <= k < lz:
                continue
            if not diffuse:
                out[l, :, y] = 0.0
            else:
                side, i = (0, -1 - k) if k < 0 else (1, k - lz)
                out[l, :, y] = np.roll(A[side, i], -ex)   # ghost site column x + e_lx
    return out


def collide_vjp(lam, g, p):
    """(d collide / d g)^T lam: dJ/dg for the pre-collision populations g of
    a step, given lam = dJ/df* of its output (eq. LBE)."""
    if p.no_collide:
        return lam
    om = 1.0 / p.tau
    rho, u, T = lbm.moments(g)
    v, Teq = lbm.shifted_state(u, T, p)
    g_rho, g_v, g_T = equilibrium_vjp(lam, rho, v, Teq)
    # v = u + tau g_vec and Teq = T + const: d/du = d/dv, d/dT = d/dTeq
    return (1.0 - om) * lam + om * moments_vjp(g, g_rho, g_v, g_T)


def step_vjp(lam, f_prev, ghost, p):
    """lam_{t-1} = (d step / d f*_{t-1})^T lam_t for the step from f_prev:
    the streaming transpose of the collision transpose."""
    g = lbm.pull(f_prev, ghost, p)
    return pull_transpose(collide_vjp(lam, g, p), p, ghost)


def objective_vjp(f, p, Tu, Tm, Td, wk=1.0, wl=1.0):
    """dJ/df*_N for J = wk KE + wl (L_u + L_d) of ``lbm.objective``.

    dJ/drho = wk |u^H|^2 / 2, dJ/du^H = wk rho u^H and
    dJ/dT^H(x, z) = (wl / Lx) [tent'(b_u)/(T_m - T_u) + tent'(b_d)/(T_d - T_m)]
    with tent' = 2 on (0, 1/2), -2 on [1/2, 1), 0 elsewhere.  u^H and T^H differ
    from the stored state's u*, T* by constants, so these are dJ/du*, dJ/dT*."""
    rho, uH, TH = lbm.hydro_fields(f, p)
    tb = lbm.tbar(TH)

    def dtent(b):
        br = np.real(b)
        return np.where((br > 0) & (br < 0.5), 2.0, np.where((br >= 0.5) & (br < 1), -2.0, 0.0))

    dtb = wl * (dtent((tb - Tu) / (Tm - Tu)) / (Tm - Tu) + dtent((tb - Tm) / (Td - Tm)) / (Td - Tm))
    g_T = np.broadcast_to(dtb[None, :] / f.shape[1], rho.shape)
    g_rho = 0.5 * wk * np.sum(uH * uH, axis=-1)
    g_u = wk * rho[..., None] * uH
    return moments_vjp(f, g_rho, g_u, g_T)


def init_vjp(lam0, p, desc, amp):
    """dJ/d amp [2, nmodes] given lam0 = dJ/df*_0 for ``lbm.init_rt3``.

    Reverses: f*_0 = f^eq(rho0, g_vec/2, T0 - g^2/8); rho0 = C exp(ln p)/T0;
    ln p = cumulative trapezoid sum of -g r (1/T(k-1) + 1/T(k))/2 from row -3;
    T0 = tanh profile of the interface heights; heights = cosine sums of amp."""
    _, _, _, r = lattice()
    lx, lz = p.lx, p.lz
    zc_all = np.arange(-3, lz + 3) + 0.5
    T_hs = lbm.layer_temperature(zc_all, *lbm.rest_heights(lz, desc), desc)
    lp_hs = lbm.hydrostatic_log_pressure(T_hs, r, p.g)
    C = 1.0 / (np.exp(lp_hs) / T_hs)[3:3 + lz].mean()
    h0, h1 = lbm.interface_heights(lx, lz, desc, amp)
    T = lbm.layer_temperature(zc_all[None, :], h0[:, None], h1[:, None], desc)   # [lx, lz+6]
    lp = lbm.hydrostatic_log_pressure(T, r, p.g)
    rho = C * np.exp(lp) / T
    Td_, rho_d = T[:, 3:3 + lz], rho[:, 3:3 + lz]

    gvec = np.array([0.0, -p.g])
    v = np.broadcast_to(0.5 * gvec, rho_d.shape + (D,))
    g_rho, _, g_Teq = equilibrium_vjp(lam0, rho_d, v, Td_ - p.g ** 2 / (4 * D))
    # rho = C exp(lp) / T on the domain rows
    g_lp = np.zeros_like(T, dtype=np.result_type(lam0, T))
    g_T = np.zeros_like(g_lp)
    g_lp[:, 3:3 + lz] = g_rho * rho_d
    g_T[:, 3:3 + lz] = g_Teq - g_rho * rho_d / Td_
    # lp[k] = sum_{m=1..k} dlp[m-1], dlp[m-1] = -g r (1/T[m] + 1/T[m-1]) / 2
    g_dlp = np.cumsum(g_lp[:, ::-1], axis=1)[:, ::-1][:, 1:]          # sum over k >= m
    dfac = 0.5 * p.g * r / T ** 2                                        # d dlp / dT (>0)
    g_T[:, 1:] += g_dlp * dfac[:, 1:]
    g_T[:, :-1] += g_dlp * dfac[:, :-1]
    # T = T_d + (T_m - T_d) s((z - h0)/w) + (T_u - T_m) s((z - h1)/w)
    sech2 = lambda y: 1.0 / np.cosh(y) ** 2
    dT_dh0 = -(desc.t_m - desc.t_d) * 0.5 * sech2((zc_all[None, :] - h0[:, None]) / desc.width) / desc.width
    dT_dh1 = -(desc.t_u - desc.t_m) * 0.5 * sech2((zc_all[None, :] - h1[:, None]) / desc.width) / desc.width
    g_h = [np.sum(g_T * dT_dh0, axis=1), np.sum(g_T * dT_dh1, axis=1)]
    xc = np.arange(lx) + 0.5
    out = np.zeros(np.shape(amp), dtype=np.result_type(lam0, float))
    for fr in range(2):
        arg = 2 * np.pi * np.outer(np.asarray(desc.k[fr], float), xc) / lx \
            + np.asarray(desc.phase[fr], float)[:, None]
        out[fr] = np.cos(arg) @ g_h[fr]
    return out


def rollout_gradient(p, desc, amp, nsteps, wk=1.0, wl=1.0):
    """(J, dJ/d amp) of the N-step rollout, storing every state (small cases)."""
    f0, ghost = lbm.init_rt3(p, desc, amp)
    states = [f0]
    for _ in range(nsteps):
        states.append(lbm.step(states[-1], ghost, p))
    J = lbm.objective(states[-1], p, desc.t_u, desc.t_m, desc.t_d, wk, wl)[0]
    lam = objective_vjp(states[-1], p, desc.t_u, desc.t_m, desc.t_d, wk, wl)
    for t in range(nsteps, 0, -1):
        lam = step_vjp(lam, states[t - 1], ghost, p)
    return J, init_vjp(lam, p, desc, amp)
