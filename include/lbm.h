/*
 * lbm.h -- C interface of the MI355X D2Q37 thermal lattice Boltzmann library.
 *
 * Method: Ripesi, Biferale, Schifano, Tripiccione, "Evolution of a
 * double-front Rayleigh-Taylor system using a GPU-based high resolution
 * thermal Lattice-Boltzmann model", Phys. Rev. E 89, 043022 (2014).
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ---------------------------------------------------------------------------
 * Lattice.  Lx x Lz sites, periodic in x, bounded by walls below row 0 and
 * above row Lz-1 (Sec. I; Sec. III.B).  Time step 1, reference temperature 1,
 * d = D = 2.  Gravity is the vector (0, -g), g >= 0 (Sec. II).
 *
 * Velocities.  37 integer displacements e_l reaching at most 3 sites; the
 * velocity used in moments and equilibrium is xi_l = r e_l with the lattice
 * constant r = 1.19697977039307... (caption of Fig. 2).  Population order:
 *    l = 0            (0,0)
 *    l = 1..4         (1,0) (-1,0) (0,1) (0,-1)
 *    l = 5..8         (1,1) (-1,-1) (1,-1) (-1,1)
 *    l = 9..12        (2,0) (-2,0) (0,2) (0,-2)
 *    l = 13..20       (2,1) (-2,-1) (2,-1) (-2,1) (1,2) (-1,-2) (1,-2) (-1,2)
 *    l = 21..24       (2,2) (-2,-2) (2,-2) (-2,2)
 *    l = 25..28       (3,0) (-3,0) (0,3) (0,-3)
 *    l = 29..36       (3,1) (-3,-1) (3,-1) (-3,1) (1,3) (-1,-3) (1,-3) (-1,3)
 * i.e. the rest velocity, then shell by shell, each +e followed by -e.
 *
 * Layout.  A population buffer (the state, and the adjoint buffers) is
 * tiled: rows are grouped in tiles of LBM_TILE = 512, and tile zt of column
 * x holds its 37 populations as 37 consecutive runs of LBM_TILE rows,
 *     element (l, x, z) at index ((zt Lx + x) 37 + l) LBM_TILE + (z - zt LBM_TILE),
 *     zt = floor(z / LBM_TILE),
 * i.e. the structure-of-arrays layout of Sec. III.B applied per tile.  A
 * buffer holds lbm_population_elems(params) = 37 Lx ceil(Lz / 512) 512
 * elements; the rows from Lz up to the next multiple of 512 are padding,
 * which no entry point reads.  lbm_pack and lbm_unpack convert from and to
 * the plain layout [37][Lx][Lz] (z fastest).  Element type by precision:
 *    LBM_F64      double, the population f_l itself;
 *    LBM_F32_DEV  float, the deviation f_l - w_l from the rest state of unit
 *                 density (w_l = quadrature weight); the step forms the
 *                 moments in double and the equilibrium and relaxation in
 *                 float (in double with LBM_COLLIDE_F64).
 * Field buffers ([4][Lx][Lz], [Lz]) are always double, in the plain layout;
 * so are the step's moments ([4][Lx][Lz]).
 *
 * State.  Buffers hold post-collision populations f*.  A step reads one
 * buffer and writes the other (the paper's prv/nxt pair, Sec. III.B).
 *
 * Wall table.  ghost [2][3][37] (element type of the state): ghost[0][i] is
 * the constant population set of the virtual row -1-i below the bottom wall,
 * ghost[1][i] that of row Lz+i above the top wall.  A pull whose source row
 * lies outside [0, Lz) reads this table (the paper's bc step on rows 0..2 and
 * Lz-3..Lz-1, Sec. III.B): as it stands (Dirichlet walls), or rescaled per
 * ghost site so that the walls conserve mass (LBM_WALL_DIFFUSE, see lbm_step).
 *
 * Memory and streams.  Pointers marked (device) are device memory, (host)
 * host memory.  All buffers are owned by the caller; the library allocates,
 * frees and synchronises nothing (device or host memory), and keeps no
 * mutable global state other than lbm_moments_noalloc's per-device scratch
 * array and the per-thread text of the last HIP error.  Every
 * call only enqueues work on `stream` (a hipStream_t; NULL = null stream) and
 * returns; results are ready when the stream reaches that point.
 *
 * Errors.  Arguments are checked before anything is enqueued; a failing call
 * enqueues nothing.  Nothing is thrown, printed or aborted.  Device pointers
 * must be 16-byte aligned.  Lx = 0 or Lz = 0 is an empty lattice: a valid
 * call that does nothing.  Lx * Lz must not exceed 2^29.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 5u
#define LBM_Q 37
#define LBM_MAX_MODES 32 /* interface modes per front accepted by lbm_init_rt3 */
#define LBM_TILE 512     /* rows per tile of a population buffer (see Layout)   */

typedef void *lbm_stream_t; /* hipStream_t */

enum lbm_status {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* bad size, tau <= 1/2, g < 0, unknown flag/precision, NULL */
    LBM_EALIAS = -2,     /* an output buffer overlaps an input buffer                  */
    LBM_EALIGN = -3,     /* a device pointer is not 16-byte aligned                    */
    LBM_EHIP = -4,       /* the HIP runtime refused a launch; see lbm_last_hip_error   */
    LBM_ESCRATCH = -5,   /* scratch buffer missing or smaller than lbm_scratch_bytes   */
    LBM_EVERSION = -6,   /* params->abi_version != LBM_ABI_VERSION                      */
    LBM_ESTATIC = -7     /* the lattice needs more than LBM_STATIC_SCRATCH_BYTES of
                            scratch (lbm_moments_noalloc only)                       */
};

enum lbm_precision { LBM_F64 = 0, LBM_F32_DEV = 1 };

enum lbm_flags {
    LBM_PERIODIC_Z = 1u, /* test mode: z wraps like x, no walls, ghost unused           */
    LBM_NO_COLLIDE = 2u, /* test mode: streaming and walls only                          */
    LBM_ADJ_F32 = 4u,    /* adjoint buffers (lam_seed, lam_in/lam_out, lam0) are float,
                            not double; the adjoint arithmetic stays double, except
                            in lbm_adjoint_step with LBM_MOM_F32 as well            */
    LBM_WALL_DIFFUSE = 8u, /* mass-conserving diffuse walls instead of Dirichlet walls
                            (lbm_step); not with LBM_PERIODIC_Z                       */
    LBM_MOM_F32 = 16u,    /* the step's moments_out and the adjoint's moments are float
                            [4][Lx][Lz] (half the memory of stored adjoint moments)   */
    LBM_COLLIDE_F64 = 32u /* LBM_F32_DEV steps: equilibrium and relaxation in double,
                            one rounding to float per stored value (ignored in FP64).
                            Near tau = 1/2 the float collision biases the interface
                            diffusion (mixing lengths +2 % after 20,000 steps at
                            tau = 0.50546); this removes it at 2-3 % of the
                            two-buffer step's time                                   */
};

typedef struct lbm_params {
    uint32_t abi_version; /* LBM_ABI_VERSION                                  */
    int32_t lx, lz;       /* lattice size                                     */
    int32_t precision;    /* enum lbm_precision                               */
    uint32_t flags;       /* enum lbm_flags, or 0                             */
    uint32_t reserved;    /* 0                                                */
    double tau;           /* BGK relaxation time, > 1/2                       */
    double g;             /* gravity magnitude along -z, >= 0                 */
} lbm_params;

/* Three-layer Rayleigh-Taylor initial state (Sec. I, eq. seteq). */
typedef struct lbm_rt3_desc {
    double t_d, t_m, t_u;  /* bottom, middle, top layer temperatures; the walls
                              are held at t_d (bottom) and t_u (top)          */
    double width;          /* tanh half-width of both interfaces, sites, > 0  */
    int32_t nmodes;        /* Fourier modes per interface, 0..LBM_MAX_MODES   */
    int32_t reserved;      /* 0                                               */
    const int32_t *k;      /* (host) [2][nmodes] integer wavenumbers          */
    const double *phase;   /* (host) [2][nmodes] phases, radians              */
    double z_lo, z_hi;     /* rest heights (sites above the bottom wall) of the
                              lower (t_d | t_m) and upper (t_m | t_u) interface;
                              a negative value selects Lz/3 and 2Lz/3         */
} lbm_rt3_desc;

/*
 * lbm_init_rt3 -- three-layer hydrostatic initial state and wall table.
 *
 * Sec. I, eq. seteq and the pressure-matching condition; the tanh smoothing
 * of the Fig. 1 caption.  Interface f (0 = lower, rest height h0_0 = z_lo;
 * 1 = upper, h0_1 = z_hi; the middle layer of width delta = z_hi - z_lo)
 * sits at height
 *     h_f(x) = h0_f + sum_j amp[f][j] cos(2 pi k[f][j] (x + 1/2) / Lx + phase[f][j])
 * (sites; site (x, z) has centre z + 1/2), the temperature is
 *     T = t_d + (t_m - t_d) s((z + 1/2 - h_0)/width) + (t_u - t_m) s((z + 1/2 - h_1)/width),
 * s(y) = (1 + tanh y)/2, and each column is in hydrostatic balance
 * d ln p/dz = -g/T (trapezoid rule, one row = r length units, integrated from
 * three rows below the bottom wall), rho = C p / T with the single constant C
 * that gives the unperturbed profile a mean density of 1.  The stored state
 * is the equilibrium at velocity (0, -g/2) and temperature T - g^2/8, so that
 * the renormalised fields (lbm_moments) are exactly (rho, 0, T).  The wall
 * table holds the same construction on the unperturbed profile 3 rows past
 * each wall.
 *
 *   amp        (device) double [2][desc->nmodes]
 *   f_out      (device) state buffer (tiled), written
 *   ghost_out  (device) wall table [2][3][37], written
 * Errors: LBM_EINVAL (sizes, nmodes, width <= 0, NULL), LBM_EALIAS (f_out and
 * ghost_out overlap), LBM_EALIGN, LBM_EVERSION, LBM_EHIP.
 */
int lbm_init_rt3(const lbm_params *params, const lbm_rt3_desc *desc, const double *amp,
                 void *f_out, void *ghost_out, lbm_stream_t stream);

/*
 * lbm_step -- one fused time step: pull streaming, walls, BGK collision.
 *
 * Sec. III.A eq. LBE with the force-shifted equilibrium (velocity u + g tau,
 * temperature T + tau (1 - tau) g^2 / d) and the moment definitions; the
 * propagate/bc/collide order of Sec. III.B.  For every site (x, z) and l:
 *     g_l(x, z) = f_in_l((x - e_lx) mod Lx, z - e_lz)   (or a ghost site)
 *     rho, u, T = moments of g
 *     f_out_l   = g_l - (g_l - f^eq_l)/tau
 * with f^eq the 4th-order Hermite expansion of the Maxwellian.
 *
 * Walls (the bc step of Sec. III.B, which only says that rows 0..2 and
 * Lz-3..Lz-1 are adjusted at rigid walls; both rules are readings of it).
 * Sources with z - e_lz outside [0, Lz) are ghost sites, row i of a side
 * being row -1-i (bottom) or Lz+i (top):
 *   Dirichlet (default): the ghost site holds its table row ghost[side][i][.].
 *   LBM_WALL_DIFFUSE: ghost site s = (x_g, k) holds ghost[side][i][l] M(s)/S,
 *     M(s) = sum over m of f_in_m(x_g - e_mx, k - e_mz) for the m whose source
 *     row lies inside [0, Lz) (the mass streaming into s), S = sum of the table
 *     row over the l with k + e_lz inside [0, Lz); the lattice's total mass is
 *     then conserved by every step.
 *
 *   ghost        (device) wall table [2][3][37]; may be NULL with LBM_PERIODIC_Z
 *   f_in         (device) state buffer, read
 *   f_out        (device) state buffer, written; must not overlap f_in
 *   moments_out  (device, nullable) double [4][Lx][Lz] (float with LBM_MOM_F32):
 *                rho, u_x, u_z, T of g (the pre-collision moments of this step,
 *                not renormalised)
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_EVERSION, LBM_EHIP.
 */
int lbm_step(const lbm_params *params, const void *ghost, const void *f_in, void *f_out,
             double *moments_out, lbm_stream_t stream);

/*
 * lbm_step_inplace -- the step of lbm_step on one population buffer.
 *
 * Same arithmetic, walls and results as lbm_step (Sec. III.A eq. LBE,
 * Sec. III.B step order), but the state lives in a single buffer instead of
 * the paper's prv/nxt pair (Sec. III.B), halving its memory.  Steps alternate
 * between two kinds; each moves the same 37 + 37 elements per site:
 *   LBM_INPLACE_FROM_STATE: f holds a post-collision state in the standard
 *     layout (as lbm_init_rt3 or lbm_step write it).  Each site pulls its
 *     populations, collides, and writes f*_l to slot -l of the site x + e_l
 *     it streams to; afterwards f holds the streamed form.
 *   LBM_INPLACE_FROM_STREAMED: f holds the streamed form; each site reads
 *     its populations from its own slots, collides and writes f*_l to slot
 *     l; afterwards f holds the post-collision state in the standard layout.
 * Streamed form: f[-l][x] is the next step's pre-collision population f_l(x)
 * for every (l, x) whose pull source x - e_l lies inside the walls; where it
 * lies beyond a wall, f[-l][x] holds the post-collision population of
 * direction -l that left x towards that wall (the walls supply f_l(x)).
 * Two steps of the two kinds equal two lbm_step calls; lbm_moments and the
 * other entry points need the standard layout (an even number of steps).
 *
 *   ghost        (device) wall table [2][3][37]; may be NULL with LBM_PERIODIC_Z
 *   f            (device) state buffer, read and written
 *   kind         LBM_INPLACE_FROM_STATE or LBM_INPLACE_FROM_STREAMED
 *   moments_out  (device, nullable) as for lbm_step
 *   scratch      (device) with LBM_WALL_DIFFUSE: at least lbm_scratch_bytes
 *                bytes, overwritten (the ghost-site masses); otherwise unused
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_ESCRATCH, LBM_EVERSION,
 * LBM_EHIP.
 */
enum lbm_inplace_kind { LBM_INPLACE_FROM_STATE = 0, LBM_INPLACE_FROM_STREAMED = 1 };
int lbm_step_inplace(const lbm_params *params, const void *ghost, void *f, int kind,
                     double *moments_out, void *scratch, size_t scratch_bytes, lbm_stream_t stream);

/*
 * lbm_population_elems -- number of elements of a population buffer (the
 * state, lam buffers) in the tiled layout: 37 Lx ceil(Lz / LBM_TILE)
 * LBM_TILE.  Returns 0 for invalid params.
 */
size_t lbm_population_elems(const lbm_params *params);

/*
 * lbm_pack, lbm_unpack -- convert a population buffer between the plain
 * layout [37][Lx][Lz] (z fastest) and the library's tiled layout.  A pure
 * permutation of elements of elt_bytes = 4 or 8 bytes (float or double
 * buffers of either precision): bit-exact both ways.  lbm_pack writes every
 * element of the tiled buffer, the padding rows as zero bits.
 *
 *   soa    (device) [37][Lx][Lz] elements
 *   tiled  (device) lbm_population_elems(params) elements
 * The two buffers must not overlap.
 * Errors: LBM_EINVAL (elt_bytes, NULL), LBM_EALIAS, LBM_EALIGN (a pointer not
 * aligned to elt_bytes), LBM_EVERSION, LBM_EHIP.
 */
int lbm_pack(const lbm_params *params, const void *soa, void *tiled, int elt_bytes, lbm_stream_t stream);
int lbm_unpack(const lbm_params *params, const void *tiled, void *soa, int elt_bytes, lbm_stream_t stream);

/*
 * lbm_scratch_bytes -- size of the scratch buffer that lbm_moments,
 * lbm_profiles, lbm_objective, lbm_init_rt3_vjp and (with diffuse walls)
 * lbm_step_inplace need (bytes).  Returns 0 for invalid params.
 */
size_t lbm_scratch_bytes(const lbm_params *params);

/*
 * lbm_moments -- renormalised fields and global diagnostics of a state.
 *
 * Sec. III.A (renormalisation u^H = u + g/2, T^H = T + g^2/(4D)) and Sec. IV
 * (mean profile T(z) = (1/Lx) sum_x T).  A stored post-collision state has
 * bare velocity u* = u + g and temperature T* = T of the step that made it,
 * so u^H = u* - g/2 and T^H = T* + g^2/8.
 *
 *   f        (device) state buffer
 *   fields   (device, nullable) double [4][Lx][Lz]: rho, u^H_x, u^H_z, T^H
 *   tbar     (device, nullable) double [Lz]: row means of T^H
 *   sums     (device, nullable) double [4]: sum over sites and l of f_l,
 *            xi_lx f_l, xi_lz f_l and |xi_l|^2 f_l / 2 (mass, momentum,
 *            energy).  Non-finite values signal a diverged state.
 *   scratch  (device) at least lbm_scratch_bytes(params) bytes, overwritten
 * All reductions use a fixed order: results are bitwise reproducible.
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_ESCRATCH, LBM_EVERSION, LBM_EHIP.
 */
int lbm_moments(const lbm_params *params, const void *f, double *fields, double *tbar,
                double *sums, void *scratch, size_t scratch_bytes, lbm_stream_t stream);

/*
 * lbm_moments_noalloc -- lbm_moments without a caller-supplied scratch buffer.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * kernels, results (bit for bit) and errors as lbm_moments, but the
 * partial sums go to a device array that the library holds, one per GPU it
 * runs on, of LBM_STATIC_SCRATCH_BYTES bytes (kept until the process ends;
 * its address is looked up on the first call on each device).  The call
 * allocates nothing, host or device.  The array needs no clearing: every
 * word a call reads was written earlier by the same call.  All calls on one
 * GPU share the array, so calls that overlap in time on one GPU (different
 * streams, or different host threads without ordering) race and give wrong
 * tbar/sums; serialise them, e.g. on one stream.
 *
 *   f, fields, tbar, sums  as for lbm_moments
 * Scratch is needed only for tbar or sums: about 8 ceil(Lx/64) Lz bytes
 * (e.g. 6.4 MB at 4096 x 12288).
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_EVERSION, LBM_EHIP,
 * LBM_ESTATIC (tbar or sums requested on a lattice whose scratch would exceed
 * LBM_STATIC_SCRATCH_BYTES).
 */
#define LBM_STATIC_SCRATCH_BYTES (16u << 20)
int lbm_moments_noalloc(const lbm_params *params, const void *f, double *fields, double *tbar,
                        double *sums, lbm_stream_t stream);

/*
 * lbm_profiles -- horizontal mean and rms fluctuation profiles of a state.
 *
 * Sec. IV (Figs. 8 and 9): for every row z, over the Lx sites of the row,
 *     prof[0][z] = <T^H>,  prof[1][z] = sqrt(<(T^H - <T^H>)^2>),
 *     prof[2][z] = <E_k>,  prof[3][z] = sqrt(<(E_k - <E_k>)^2>),
 * with E_k = rho |u^H|^2 / 2 the kinetic energy density.  The second moments
 * are accumulated about each row's value at x = 0, so small fluctuations do
 * not cancel; the order of all sums is fixed (bitwise reproducible).
 *
 *   f        (device) state buffer
 *   prof     (device) double [4][Lz], written
 *   scratch  (device) at least lbm_scratch_bytes(params) bytes
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_ESCRATCH, LBM_EVERSION, LBM_EHIP.
 */
int lbm_profiles(const lbm_params *params, const void *f, double *prof, void *scratch,
                 size_t scratch_bytes, lbm_stream_t stream);

/*
 * lbm_objective -- mixing objective of a state and (optionally) its gradient.
 *
 * Sec. IV: mean profile T(z) of T^H, tent map Theta(b) = 2b on (0, 1/2),
 * 2(1 - b) on [1/2, 1), 0 elsewhere, and the two mixing lengths of eq. 3L
 * summed over rows (one row = 1):
 *     L_u = sum_z Theta((T(z) - t_u)/(t_m - t_u)),  L_d = sum_z Theta((T(z) - t_m)/(t_d - t_m)).
 * With KE = (1/2) sum_sites rho |u^H|^2 the objective is J = wk KE + wl (L_u + L_d).
 *
 *   desc      (host) only t_d > t_m > t_u are used
 *   f         (device) state buffer
 *   j_out     (device) double [5]: J, KE, L_u + L_d, L_u, L_d
 *   lam_seed  (device, nullable) population buffer (double, or float with LBM_ADJ_F32):
 *             dJ/df_l at every site
 *             (the tent map's slope is taken as 2, -2, 0 on the three pieces)
 *   scratch   (device) at least lbm_scratch_bytes(params) bytes
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_ESCRATCH, LBM_EVERSION, LBM_EHIP.
 */
int lbm_objective(const lbm_params *params, const lbm_rt3_desc *desc, const void *f, double wk, double wl,
                  double *j_out, void *lam_seed, void *scratch, size_t scratch_bytes,
                  lbm_stream_t stream);

/*
 * lbm_adjoint_step -- transposed Jacobian of one lbm_step.
 *
 * Differentiates the step of Sec. III.A (pull, walls, force-shifted BGK
 * collision) with respect to its input state: given lam_in = dJ/df_out it
 * writes lam_out = dJ/df_in.  With m = (rho, u, T) the step's pre-collision
 * moments at site x, omega = 1/tau and mu = omega (dF/dm)^T lam_in(x),
 *     G_l(x) = (1 - omega) lam_in_l(x) + alpha + beta . xi_l + gamma |xi_l|^2,
 *     lam_out_l(y) = G_l(y + e_l)  (x periodic) where y + e_l is inside the walls,
 *     alpha = mu_rho - mu_u . u/rho + mu_T (|u|^2 - 2T)/(2 rho),
 *     beta = mu_u/rho - mu_T u/rho,  gamma = mu_T/(2 rho).
 * Where y + e_l is a ghost site s: 0 for the Dirichlet wall (the table is
 * constant and receives no derivative); with LBM_WALL_DIFFUSE
 *     lam_out_l(y) = sum_m c_m G_m(s + e_m) / sum_m c_m
 * over the m with s + e_m inside the walls, c_m = the table row of s.
 *
 *   ghost    (device) the wall table the forward step used; required with
 *            LBM_WALL_DIFFUSE, otherwise unused and may be NULL
 *   moments  (device) double [4][Lx][Lz] (float with LBM_MOM_F32): rho, u_x,
 *            u_z, T written by the forward lbm_step's moments_out (may be NULL
 *            with LBM_NO_COLLIDE)
 *   lam_in   (device) population buffer, double (float with LBM_ADJ_F32)
 *   lam_out  (device) same type and shape, must not overlap lam_in, moments
 *            or ghost
 * The adjoint arithmetic is double, except with both LBM_ADJ_F32 and
 * LBM_MOM_F32 (all inputs float): then the per-site sums of lam_in against
 * the 15 monomials xi_x^p xi_z^q (p + q <= 4) and the outputs G_l are formed
 * in float, and the moments' algebra and (alpha, beta, gamma) in double
 * (error within 32 float roundings of the largest output; about 5 on random
 * inputs).  params->precision
 * names the forward state it belongs to and the element type of ghost.
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_EVERSION, LBM_EHIP.
 */
int lbm_adjoint_step(const lbm_params *params, const void *ghost, const double *moments,
                     const void *lam_in, void *lam_out, lbm_stream_t stream);

/*
 * lbm_adjoint_collide, lbm_adjoint_gather -- the adjoint of a chain of steps
 * in gather form.
 *
 * A step is f_out = C(S f_in) with S the streaming and wall step (a pull)
 * and C the per-site collision of Sec. III.A (eq. LBE), so a chain of N
 * steps has the adjoint lam_0 = S^T C_1^T S^T C_2^T ... S^T C_N^T lam_N.
 * lbm_adjoint_step applies S^T C_t^T per call with S^T as a scatter.
 * Grouped around mu_t = C_t^T lam_t (dJ with respect to the pre-collision
 * populations g of step t), the chain is
 *     mu_N = C_N^T lam_N                       lbm_adjoint_collide (moments of step N)
 *     mu_{t-1} = C_{t-1}^T S^T mu_t            lbm_adjoint_gather (moments of step t-1)
 *     lam_0 = S^T mu_1                         lbm_adjoint_gather with LBM_NO_COLLIDE
 * and S^T becomes a gather: (S^T mu)_l(y) = mu_l(y + e_l) (x periodic) where
 * y + e_l lies inside the walls; beyond a wall it is 0 for the Dirichlet
 * wall and, with LBM_WALL_DIFFUSE, A(s) = sum_m c_m mu_m(s + e_m) / sum_m c_m
 * for the ghost site s = y + e_l (the m with s + e_m inside the walls, c_m
 * = its table row).  C^T at a site is the map of lbm_adjoint_step:
 *     out_l = (1 - omega) in_l + alpha + beta . xi_l + gamma |xi_l|^2
 * with (alpha, beta, gamma) from the site's 37 values and its moments.
 * Every output element is written by its own site (aligned writes); the
 * chain gives lbm_adjoint_step's results to rounding (the same per-site
 * arithmetic, contracted into multiply-adds as the compiler chooses).
 *
 *   moments  (device) double [4][Lx][Lz] (float with LBM_MOM_F32) of the step
 *            whose collision is transposed (NULL allowed with LBM_NO_COLLIDE)
 *   lam, mu_in  (device) population buffers, double (float with LBM_ADJ_F32)
 *   mu, mu_out  (device) same type, must not overlap the inputs
 *   ghost    (device) the forward step's wall table; required with
 *            LBM_WALL_DIFFUSE, otherwise unused
 * Arithmetic and precision as for lbm_adjoint_step.  Allocates nothing and
 * needs no scratch: with LBM_WALL_DIFFUSE the blocks at the walls form the
 * ghost sites' sums themselves.
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_EVERSION, LBM_EHIP.
 */
int lbm_adjoint_collide(const lbm_params *params, const double *moments, const void *lam, void *mu,
                        lbm_stream_t stream);
int lbm_adjoint_gather(const lbm_params *params, const void *ghost, const double *moments, const void *mu_in,
                       void *mu_out, lbm_stream_t stream);

/*
 * lbm_init_rt3_vjp -- gradient of lbm_init_rt3 with respect to the mode
 * amplitudes: d_amp[f][j] = sum over sites and l of lam0_l dF0_l/damp[f][j],
 * through the tanh profile, the column pressure integral and the
 * equilibrium (Sec. I, eq. seteq).  The wall table does not depend on amp.
 *
 *   desc, amp  as passed to lbm_init_rt3
 *   lam0       (device) population buffer (double, or float with LBM_ADJ_F32): dJ/df*_0
 *   d_amp      (device) double [2][nmodes], written
 *   scratch    (device) at least lbm_scratch_bytes(params) bytes
 * Errors: LBM_EINVAL, LBM_EALIAS, LBM_EALIGN, LBM_ESCRATCH, LBM_EVERSION, LBM_EHIP.
 */
int lbm_init_rt3_vjp(const lbm_params *params, const lbm_rt3_desc *desc, const double *amp,
                     const void *lam0, double *d_amp, void *scratch, size_t scratch_bytes,
                     lbm_stream_t stream);

/*
 * lbm_lattice -- the library's velocity set and weights (host query).
 *   r  (host, nullable) lattice constant
 *   w  (host, nullable) double [37] weights
 *   e  (host, nullable) int32 [37][2] integer displacements (e_x, e_z)
 */
int lbm_lattice(double *r, double *w, int32_t *e);

/* Static description of a status code. */
const char *lbm_strerror(int status);

/* Text of the last HIP error seen by this thread ("" if none). */
const char *lbm_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
