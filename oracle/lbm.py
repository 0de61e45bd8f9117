"""Forward D2Q37 thermal LBM: equilibrium, moments, streaming, walls, collide,
three-layer initial state and the mixing diagnostics.

Test infrastructure (see ``oracle/__init__``).  float64 throughout; every
function also accepts complex128 inputs so that tests can differentiate by
complex step.

Conventions (readings of the paper where it is silent):
* time step dt = 1, reference temperature T0 = 1, d = D = 2;
* gravity acts along -z: g_vec = (0, -g) with g >= 0 (Sec. II eq. NS);
* a site is one lattice step e = (1, 0) away from its neighbour, i.e. r length
  units, because the populations travel xi_l dt = r e_l per step;
* arrays of populations are laid out [37, Lx, Lz] (z fastest) and the stored
  state between steps is the post-collision population f*;
* walls: a population that would be pulled from a row outside [0, Lz) comes
  from a ghost site three rows deep past each wall; ghost[2, 3, 37] is the
  wall table, ghost[0, i] for row -1-i below the bottom wall, ghost[1, i] for
  row Lz+i above the top wall.  Two wall rules (Sec. III.B step bc, which the
  paper describes only as adjusting rows 0..2 and Lz-3..Lz-1 at rigid walls):
  "dirichlet" takes the ghost populations from the table as they stand;
  "diffuse" (mass-conserving diffuse reflection) gives each ghost site the
  distribution shape of its table row, scaled so that it returns to the
  lattice exactly the mass that streamed into it in the same step.
"""
from dataclasses import dataclass

import numpy as np

from .lattice import D, hermite_tensors, lattice


@dataclass
class Params:
    lx: int
    lz: int
    tau: float
    g: float
    periodic_z: bool = False   # test mode: no walls, z wraps like x
    no_collide: bool = False   # test mode: streaming (and walls) only
    wall: str = "dirichlet"    # "dirichlet" or "diffuse" (see module notes)


# --------------------------------------------------------------------------
# Equilibrium and moments (Sec. III.A)
# --------------------------------------------------------------------------

def _flat(a, n):
    return a.reshape(a.shape[0], 2 ** n) if n else a


def hermite_coefficients(rho, u, T):
    """Hermite coefficients a^(0..4) of the local Maxwellian at (rho, u, T).

    rho [S], u [S, 2], T [S].  Expansion about the unit-temperature Gaussian
    (reference temperature T0 = 1), with th = T - 1:
        a0 = rho
        a1_i = rho u_i
        a2_ij = rho (u_i u_j + th d_ij)
        a3_ijk = rho (u_i u_j u_k + th (u_i d_jk + u_j d_ik + u_k d_ij))
        a4_ijkl = rho (u_i u_j u_k u_l + th (sum of the 6 u u d pairings)
                       + th^2 (d_ij d_kl + d_ik d_jl + d_il d_jk))
    """
    d = np.eye(D)
    th = T - 1.0
    uu = np.einsum("si,sj->sij", u, u)
    a0 = rho
    a1 = rho[:, None] * u
    a2 = rho[:, None, None] * (uu + th[:, None, None] * d[None])
    a3 = rho[:, None, None, None] * (
        np.einsum("si,sj,sk->sijk", u, u, u)
        + th[:, None, None, None] * (np.einsum("si,jk->sijk", u, d)
                                     + np.einsum("sj,ik->sijk", u, d)
                                     + np.einsum("sk,ij->sijk", u, d)))
    dd = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
          + np.einsum("il,jk->ijkl", d, d))
    a4 = rho[:, None, None, None, None] * (
        np.einsum("si,sj,sk,sl->sijkl", u, u, u, u)
        + th[:, None, None, None, None] * (
            np.einsum("sij,kl->sijkl", uu, d) + np.einsum("sik,jl->sijkl", uu, d)
            + np.einsum("sil,jk->sijkl", uu, d) + np.einsum("sjk,il->sijkl", uu, d)
            + np.einsum("sjl,ik->sijkl", uu, d) + np.einsum("skl,ij->sijkl", uu, d))
        + (th ** 2)[:, None, None, None, None] * dd[None])
    return a0, a1, a2, a3, a4


def equilibrium(rho, u, T):
    """Discrete 4th-order Hermite equilibrium f^eq_l(rho, u, T).

    rho [...], u [..., 2], T [...]  ->  [37, ...].
    f^eq_l = w_l * sum_{n<=4} (1/n!) a^(n)(rho, u, T) : H^(n)(xi_l),
    the tensor contraction done as one matrix product per order.
    """
    _, xi, w, _ = lattice()
    shape = np.shape(rho)
    rho_f = np.reshape(rho, -1)
    u_f = np.reshape(u, (-1, D))
    T_f = np.reshape(T, -1)
    a = hermite_coefficients(rho_f, u_f, T_f)
    H = hermite_tensors(xi)
    fact = (1.0, 1.0, 2.0, 6.0, 24.0)
    acc = a[0][:, None] * H[0][None, :]
    for n in range(1, 5):
        acc = acc + (_flat(a[n], n) @ _flat(H[n], n).T) / fact[n]
    feq = acc * w[None, :]
    return np.moveaxis(feq, 1, 0).reshape((len(w),) + shape)


def moments(f):
    """(rho, u, T) of populations f [37, ...] (Sec. III.A moment definitions).

    rho = sum_l f_l,  rho u = sum_l xi_l f_l,
    d rho T = sum_l |xi_l - u|^2 f_l   (central form, as the paper writes it).
    """
    _, xi, _, _ = lattice()
    rho = f.sum(axis=0)
    j = np.tensordot(xi.T, f, axes=(1, 0))           # [2, ...]
    u = np.moveaxis(j / rho[None], 0, -1)            # [..., 2]
    bshape = (f.shape[0],) + (1,) * (f.ndim - 1)
    cx = xi[:, 0].reshape(bshape) - u[..., 0][None]
    cz = xi[:, 1].reshape(bshape) - u[..., 1][None]
    T = ((cx * cx + cz * cz) * f).sum(axis=0) / (D * rho)
    return rho, u, T


def shifted_state(u, T, p):
    """Equilibrium arguments with the body force folded in (Sec. III.A):
    u + g_vec tau and T + tau (dt - tau) g^2 / d, with dt = 1."""
    gvec = np.array([0.0, -p.g])
    return u + p.tau * gvec, T + p.tau * (1.0 - p.tau) * p.g ** 2 / D


# --------------------------------------------------------------------------
# Streaming, walls, collision (Sec. III.A eq. LBE; Sec. III.B)
# --------------------------------------------------------------------------

def ghost_row(side, i, lz):
    """Row index of ghost row i on a side (0: below the bottom wall, 1: above
    the top wall)."""
    return -1 - i if side == 0 else lz + i


def wall_masses(f, lz):
    """Mass that streams out of the lattice into each ghost site in one pull.

    M[side, i, x] for the ghost site (x, ghost_row(side, i)): the sum over l of
    f_l(x - e_lx, k - e_lz) over the l whose source row k - e_lz lies inside
    [0, Lz), i.e. every population leaving the lattice that would land there.
    """
    E, _, _, _ = lattice()
    M = np.zeros((2, 3, f.shape[1]), dtype=f.dtype)
    for side in range(2):
        for i in range(3):
            k = ghost_row(side, i, lz)
            for l in range(f.shape[0]):
                ex, ez = int(E[l, 0]), int(E[l, 1])
                if 0 <= k - ez < lz:
                    M[side, i] += np.roll(f[l, :, k - ez], ex)
    return M


def wall_emission(ghost, lz):
    """Emission shares c[side, i, l] of the diffuse wall: the table row's
    populations that point back into the lattice (k + e_lz inside [0, Lz)),
    normalised to sum to one over those l; zero for the other l."""
    E, _, _, _ = lattice()
    c = np.zeros((2, 3, E.shape[0]))
    for side in range(2):
        for i in range(3):
            k = ghost_row(side, i, lz)
            into = np.array([0 <= k + int(E[l, 1]) < lz for l in range(E.shape[0])])
            c[side, i, into] = ghost[side, i, into] / ghost[side, i, into].sum()
    return c


def pull(f, ghost, p):
    """Pull streaming: out_l(x, z) = f_l(x - e_lx mod Lx, z - e_lz).

    Sources below row 0 or above row Lz-1 are ghost sites (walls in z), unless
    ``p.periodic_z`` (then z wraps as well).  With ``p.wall == "dirichlet"`` a
    ghost site holds its table row; with ``"diffuse"`` it holds
    c_l * M, the table row's shape (``wall_emission``) times the mass M that
    streamed into that ghost site from f (``wall_masses``).
    """
    E, _, _, _ = lattice()
    out = np.empty_like(f)
    lz = f.shape[2]
    if not p.periodic_z and p.wall == "diffuse":
        M = wall_masses(f, lz)
        c = wall_emission(ghost, lz)
    elif not p.periodic_z and p.wall != "dirichlet":
        raise ValueError(f"unknown wall rule {p.wall!r}")

    def ghost_value(side, i, l, ex):
        if p.wall == "diffuse":
            # the ghost site of column x sits at x - e_lx
            return c[side, i, l] * np.roll(M[side, i], ex)
        return ghost[side, i, l]

    for l in range(f.shape[0]):
        ex, ez = int(E[l, 0]), int(E[l, 1])
        out[l] = np.roll(f[l], shift=(ex, ez), axis=(0, 1))
        if p.periodic_z:
            continue
        # rows whose source lies below the bottom wall (e_lz > 0) ...
        for z in range(0, min(ez, lz)):
            out[l, :, z] = ghost_value(0, ez - z - 1, l, ex)
        # ... or above the top wall (e_lz < 0)
        for z in range(max(lz + ez, 0), lz):
            out[l, :, z] = ghost_value(1, z - ez - lz, l, ex)
    return out


def collide(f, p):
    """BGK relaxation towards the force-shifted equilibrium (eq. LBE):
    f* = f - (f - f^eq[rho, u + g tau, T + tau (1 - tau) g^2 / d]) / tau."""
    rho, u, T = moments(f)
    ueq, Teq = shifted_state(u, T, p)
    feq = equilibrium(rho, ueq, Teq)
    return np.ascontiguousarray(f - (f - feq) / p.tau)


def step(f, ghost, p):
    """One time step in the paper's order: propagate, bc, collide."""
    g = pull(f, ghost, p)
    if p.no_collide:
        return g
    return collide(g, p)


def run(f, ghost, p, nsteps):
    for _ in range(nsteps):
        f = step(f, ghost, p)
    return f


# --------------------------------------------------------------------------
# Hydrodynamic fields and diagnostics (Sec. III.A renormalisation; Sec. IV)
# --------------------------------------------------------------------------

def hydro_fields(f, p):
    """rho, u^H [.., 2], T^H of a stored post-collision state.

    The collision leaves rho and T unchanged and adds g to u (exactly), so the
    pre-collision velocity of the same step is u* - g.  The paper's
    renormalised fields u^H = u + dt g / 2 and T^H = T + dt^2 g^2 / (4 D) are
    therefore u* - g/2 and T* + g^2/8 in terms of the stored state.
    """
    rho, ustar, Tstar = moments(f)
    gvec = np.array([0.0, -p.g])
    return rho, ustar - 0.5 * gvec, Tstar + p.g ** 2 / (4 * D)


def global_sums(f):
    """Mass, momentum (x, z) and energy sum_l |xi_l|^2 f_l / 2 over all sites."""
    _, xi, _, _ = lattice()
    Q = f.shape[0]
    fl = f.reshape(Q, -1).sum(axis=1)
    return np.array([fl.sum(), (xi[:, 0] * fl).sum(), (xi[:, 1] * fl).sum(),
                     0.5 * ((xi ** 2).sum(axis=1) * fl).sum()])


def tbar(TH):
    """Horizontal mean temperature profile  T(z) = (1/Lx) sum_x T^H(x, z)."""
    return TH.mean(axis=0)


def profiles(f, p):
    """Row profiles of Sec. IV (Figs. 8 and 9): mean and rms fluctuation
    over x of the temperature T^H and of the kinetic energy density
    E_k = rho |u^H|^2 / 2:  [<T>, sqrt(<(T - <T>)^2>), <E_k>, sqrt(<(E_k - <E_k>)^2>)],
    each [Lz]."""
    rho, uH, TH = hydro_fields(f, p)
    ek = 0.5 * rho * np.sum(uH * uH, axis=-1)
    out = []
    for X in (TH, ek):
        m = X.mean(axis=0)
        out += [m, np.sqrt(((X - m[None, :]) ** 2).mean(axis=0))]
    return np.array(out)


def tent(b):
    """Tent map of Sec. IV: 2b on (0, 1/2), 2(1 - b) on [1/2, 1), 0 outside.

    For complex inputs the branch is chosen on the real part."""
    br = np.real(b)
    out = np.where((br > 0) & (br < 0.5), 2 * b, 0 * b)
    return np.where((br >= 0.5) & (br < 1), 2 * (1 - b), out)


def mixing_lengths(tb, Tu, Tm, Td):
    """Upper and lower mixing lengths of eq. 3L, summed over rows (dz = 1 site):
    L_u = sum_z tent((T(z) - T_u)/(T_m - T_u)),
    L_d = sum_z tent((T(z) - T_m)/(T_d - T_m))."""
    Lu = tent((tb - Tu) / (Tm - Tu)).sum()
    Ld = tent((tb - Tm) / (Td - Tm)).sum()
    return Lu, Ld


def objective(f, p, Tu, Tm, Td, wk=1.0, wl=1.0):
    """J = wk * KE + wl * (L_u + L_d) at the given state.

    KE = (1/2) sum_sites rho |u^H|^2.  Returns (J, KE, L_u + L_d)."""
    rho, uH, TH = hydro_fields(f, p)
    ke = 0.5 * (rho * np.sum(uH * uH, axis=-1)).sum()
    Lu, Ld = mixing_lengths(tbar(TH), Tu, Tm, Td)
    return wk * ke + wl * (Lu + Ld), ke, Lu + Ld


# --------------------------------------------------------------------------
# Three-layer initial state (Sec. I eq. seteq and the pressure matching,
# Fig. 1 caption for the tanh smoothing)
# --------------------------------------------------------------------------

@dataclass
class RT3:
    t_d: float          # bottom layer (and bottom wall) temperature
    t_m: float          # middle layer
    t_u: float          # top layer (and top wall)
    width: float        # tanh half-width of the interfaces, in sites
    k: np.ndarray       # [2, nmodes] integer wavenumbers (front 0 lower, 1 upper)
    phase: np.ndarray   # [2, nmodes]
    z_lo: float = None  # rest height of the lower interface (sites); None: Lz/3
    z_hi: float = None  # rest height of the upper interface; None: 2 Lz/3


def rest_heights(lz, desc):
    """Rest heights of the two interfaces: the middle layer of Sec. I spans
    (z_lo, z_hi); by default the three layers are equal thirds."""
    lo = lz / 3.0 if desc.z_lo is None else float(desc.z_lo)
    hi = 2.0 * lz / 3.0 if desc.z_hi is None else float(desc.z_hi)
    return lo, hi


def interface_heights(lx, lz, desc, amp, columns=None):
    """Heights (site units, z = 0 at the bottom wall) of the two interfaces
    h_f(x) = h0_f + sum_j amp[f, j] cos(2 pi k[f, j] (x + 1/2) / Lx + phase[f, j]),
    with h0 the rest heights (lower, T_d | T_m, and upper, T_m | T_u), at every
    column or at the given column indices."""
    xc = (np.arange(lx) if columns is None else np.asarray(columns)) + 0.5
    base = rest_heights(lz, desc)
    hs = []
    for fr in range(2):
        arg = 2 * np.pi * np.outer(np.asarray(desc.k[fr], float), xc) / lx \
            + np.asarray(desc.phase[fr], float)[:, None]
        hs.append(base[fr] + (np.asarray(amp[fr])[:, None] * np.cos(arg)).sum(axis=0))
    return hs[0], hs[1]


def layer_temperature(zc, h0, h1, desc):
    """T(z) = T_d + (T_m - T_d) s((z - h0)/w) + (T_u - T_m) s((z - h1)/w),
    s(y) = (1 + tanh y)/2: three constant layers joined by tanh steps."""
    s0 = 0.5 * (1 + np.tanh((zc - h0) / desc.width))
    s1 = 0.5 * (1 + np.tanh((zc - h1) / desc.width))
    return desc.t_d + (desc.t_m - desc.t_d) * s0 + (desc.t_u - desc.t_m) * s1


def hydrostatic_log_pressure(T, r, g):
    """Column integral of d ln p / dz = -g / T (hydrostatic balance with
    p = rho T), z measured in length units so one row is r: trapezoid rule,
    ln p at the first row = 0.  T [..., nz] -> ln p [..., nz]."""
    dlp = -g * r * 0.5 * (1.0 / T[..., 1:] + 1.0 / T[..., :-1])
    lp0 = np.zeros(T.shape[:-1] + (1,), dtype=np.result_type(T, float))
    return np.concatenate([lp0, np.cumsum(dlp, axis=-1)], axis=-1)


def init_rt3(p, desc, amp, columns=None):
    """Initial post-collision state f*_0 [37, Lx, Lz] and wall table ghost.

    With ``columns`` (indices into 0..Lx-1) only those columns are built:
    f*_0 is then [37, len(columns), Lz] (columns are independent).

    Each column holds the three-layer temperature profile integrated in
    hydrostatic balance from three rows below the bottom wall; the density is
    rho = C p / T with one constant C that makes the mean density of the
    unperturbed profile equal to 1.  The state is the equilibrium at
    velocity g_vec / 2 and temperature T - g^2/8, so that its renormalised
    fields are exactly (rho, u^H = 0, T^H = T).  The ghost rows hold the same
    construction on the unperturbed profile continued 3 rows past each wall.
    """
    _, _, _, r = lattice()
    lx, lz = p.lx, p.lz
    zc_all = np.arange(-3, lz + 3) + 0.5                 # rows -3 .. Lz+2
    # unperturbed profile (also the walls)
    T_hs = layer_temperature(zc_all, *rest_heights(lz, desc), desc)
    lp_hs = hydrostatic_log_pressure(T_hs, r, p.g)
    rho_hs = np.exp(lp_hs) / T_hs
    C = 1.0 / rho_hs[3:3 + lz].mean()
    rho_hs = C * rho_hs
    # perturbed columns
    h0, h1 = interface_heights(lx, lz, desc, amp, columns)
    T = layer_temperature(zc_all[None, :], h0[:, None], h1[:, None], desc)
    lp = hydrostatic_log_pressure(T, r, p.g)
    rho = C * np.exp(lp) / T
    T, rho = T[:, 3:3 + lz], rho[:, 3:3 + lz]

    gvec = np.array([0.0, -p.g])
    ustar = np.broadcast_to(0.5 * gvec, rho.shape + (D,))
    f0 = equilibrium(rho, ustar, T - p.g ** 2 / (4 * D))

    rows = {0: [2, 1, 0], 1: [3 + lz, 4 + lz, 5 + lz]}    # indices into *_all
    ghost = np.empty((2, 3, 37), dtype=np.float64)
    for side in (0, 1):
        for i, k in enumerate(rows[side]):
            ghost[side, i] = equilibrium(np.array(rho_hs[k]),
                                         0.5 * gvec, np.array(T_hs[k] - p.g ** 2 / (4 * D)))
    return f0, ghost
