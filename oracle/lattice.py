"""D2Q37 velocity set, its quadrature weights and the Hermite tensors.

Test infrastructure (see ``oracle/__init__``).

Paper, Sec. III.A and the caption of Fig. 2: the model uses 37 discrete
velocities, and the lattice constant is r ~ 1.1969.  The figure with the
velocity diagram is not in the text, so the set is reconstructed:

* 8 shells of integer displacements e (all sign and axis-swap images of a
  representative): (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,1), with
  1+4+4+4+8+4+4+8 = 37 members, reaching at most 3 sites (the 3-column x halo
  and the 3 wall rows of Sec. III.B agree with that reach);
* velocities xi_l = r e_l;
* r and the 8 shell weights solve the 9 even-moment conditions of a degree-9
  Gauss-Hermite quadrature in 2-D:
      sum_l w_l xi_x^(2a) xi_z^(2b) = (2a-1)!! (2b-1)!!,   a + b <= 4.

The solve here is the plainest one: for trial r the 9 conditions are a linear
system in the 8 weights, which is consistent only where the determinant of the
augmented 9x9 matrix vanishes; bisection on its sign finds r, a least squares
solve of the (then consistent) system gives the weights, and a few Newton
steps on all 9 conditions together polish (w, r) to rounding level.

Population order is the one the C interface documents: rest velocity first,
then shell by shell, with each +e immediately followed by -e.
"""
import numpy as np

D = 2  # space dimension (d = D = 2 in the paper's formulas)

SHELL_REPS = ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1))

# Ordered list of the 37 integer displacements.  Within a shell the +e
# members are listed in a fixed order and each is followed by -e.
_SHELL_ORDER = {
    (0, 0): [(0, 0)],
    (1, 0): [(1, 0), (0, 1)],
    (1, 1): [(1, 1), (1, -1)],
    (2, 0): [(2, 0), (0, 2)],
    (2, 1): [(2, 1), (2, -1), (1, 2), (1, -2)],
    (2, 2): [(2, 2), (2, -2)],
    (3, 0): [(3, 0), (0, 3)],
    (3, 1): [(3, 1), (3, -1), (1, 3), (1, -3)],
}


def velocity_set():
    """Return (E, shell): E int array [37, 2] of (e_x, e_z), shell int [37]."""
    E, shell = [], []
    for s, rep in enumerate(SHELL_REPS):
        for e in _SHELL_ORDER[rep]:
            if e == (0, 0):
                E.append(e)
                shell.append(s)
            else:
                E.append(e)
                E.append((-e[0], -e[1]))
                shell += [s, s]
    return np.array(E, dtype=np.int64), np.array(shell, dtype=np.int64)


def _double_factorial(n):
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


# The 9 independent even-moment conditions (a, b), a >= b, a + b <= 4.
CONDITIONS = ((0, 0), (1, 0), (2, 0), (1, 1), (3, 0), (2, 1), (4, 0), (3, 1), (2, 2))


def _system(r):
    """Linear system A w = b for the 8 shell weights at lattice constant r."""
    E, shell = velocity_set()
    A = np.zeros((len(CONDITIONS), len(SHELL_REPS)))
    b = np.zeros(len(CONDITIONS))
    for i, (a, bb) in enumerate(CONDITIONS):
        for l in range(len(E)):
            A[i, shell[l]] += (r * E[l, 0]) ** (2 * a) * (r * E[l, 1]) ** (2 * bb)
        b[i] = _double_factorial(2 * a - 1) * _double_factorial(2 * bb - 1)
        # scale each row by r^-(2(a+b)) so the determinant stays O(1)
        A[i] /= r ** (2 * (a + bb))
        b[i] /= r ** (2 * (a + bb))
    return A, b


def _aug_det(r):
    A, b = _system(r)
    return np.linalg.det(np.column_stack([A, b]))


def solve_quadrature(lo=1.1, hi=1.3):
    """Lattice constant r and per-population weights w [37] (float64).

    Bisection on the sign of det[A(r) | b(r)] inside [lo, hi], which brackets
    the single root near the paper's r ~ 1.1969, then least squares for w.
    """
    flo, fhi = _aug_det(lo), _aug_det(hi)
    assert flo * fhi < 0, "bracket does not contain the quadrature root"
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        fm = _aug_det(mid)
        if fm == 0:
            lo = hi = mid
            break
        if (fm < 0) == (flo < 0):
            lo, flo = mid, fm
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    A, b = _system(r)
    w_shell, *_ = np.linalg.lstsq(A, b, rcond=None)
    # Newton polish of (w, r) on the unscaled conditions summed over the 37
    # velocities: the least-squares weights at a rounded r leave residuals of
    # ~1e-13 in the low-order moments, the polished ones ~1e-16.
    best = None
    for _ in range(4):
        F, J = _residual_jacobian(w_shell, r)
        err = np.abs(F).max()
        if best is None or err < best[0]:
            best = (err, w_shell.copy(), r)
        d = np.linalg.solve(J, -F)
        w_shell, r = w_shell + d[:-1], r + d[-1]
    _, w_shell, r = best
    _, shell = velocity_set()
    return r, w_shell[shell]


def _residual_jacobian(w_shell, r):
    """Residuals of the 9 conditions and their Jacobian in (w_0..w_7, r)."""
    E, shell = velocity_set()
    F = np.zeros(len(CONDITIONS))
    J = np.zeros((len(CONDITIONS), len(SHELL_REPS) + 1))
    for i, (a, b) in enumerate(CONDITIONS):
        row = np.zeros(len(SHELL_REPS))
        for l in range(len(E)):
            row[shell[l]] += (r * E[l, 0]) ** (2 * a) * (r * E[l, 1]) ** (2 * b)
        F[i] = row @ w_shell - _double_factorial(2 * a - 1) * _double_factorial(2 * b - 1)
        J[i, :-1] = row
        J[i, -1] = (row @ w_shell) * 2 * (a + b) / r
    return F, J


_CACHE = {}


def lattice():
    """Cached (E [37,2] int, xi [37,2] float, w [37] float, r)."""
    if "lat" not in _CACHE:
        E, _ = velocity_set()
        r, w = solve_quadrature()
        _CACHE["lat"] = (E, r * E.astype(np.float64), w, r)
    return _CACHE["lat"]


def hermite_tensors(xi):
    """Hermite tensors H^(n)(xi) for n = 0..4, as arrays [Q, 2, ..., 2].

    Tensor Hermite polynomials for the unit-variance Gaussian weight:
        H0 = 1
        H1_i = xi_i
        H2_ij = xi_i xi_j - d_ij
        H3_ijk = xi_i xi_j xi_k - (xi_i d_jk + xi_j d_ik + xi_k d_ij)
        H4_ijkl = xi_i xi_j xi_k xi_l
                  - (xi_i xi_j d_kl + xi_i xi_k d_jl + xi_i xi_l d_jk
                     + xi_j xi_k d_il + xi_j xi_l d_ik + xi_k xi_l d_ij)
                  + (d_ij d_kl + d_ik d_jl + d_il d_jk)
    """
    d = np.eye(D)
    x = np.asarray(xi, dtype=np.float64)
    Q = x.shape[0]
    H0 = np.ones(Q)
    H1 = x.copy()
    H2 = np.einsum("qi,qj->qij", x, x) - d[None]
    H3 = (np.einsum("qi,qj,qk->qijk", x, x, x)
          - np.einsum("qi,jk->qijk", x, d)
          - np.einsum("qj,ik->qijk", x, d)
          - np.einsum("qk,ij->qijk", x, d))
    xx = np.einsum("qi,qj->qij", x, x)
    H4 = (np.einsum("qi,qj,qk,ql->qijkl", x, x, x, x)
          - np.einsum("qij,kl->qijkl", xx, d)
          - np.einsum("qik,jl->qijkl", xx, d)
          - np.einsum("qil,jk->qijkl", xx, d)
          - np.einsum("qjk,il->qijkl", xx, d)
          - np.einsum("qjl,ik->qijkl", xx, d)
          - np.einsum("qkl,ij->qijkl", xx, d)
          + np.einsum("ij,kl->ijkl", d, d)[None]
          + np.einsum("ik,jl->ijkl", d, d)[None]
          + np.einsum("il,jk->ijkl", d, d)[None])
    return H0, H1, H2, H3, H4
