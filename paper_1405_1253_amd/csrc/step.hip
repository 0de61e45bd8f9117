// Fused D2Q37 time step: pull streaming + wall rows + force-shifted BGK collide.
//
// Sec. III.A eq. LBE and the shifted equilibrium; Sec. III.B step order
// (propagate, bc, collide) and the prv/nxt pair of lattice copies.
//
// Mapping.  Populations are stored in the tiled layout of common.h (tiles of
// TILE rows, a tile's 37 populations contiguous).  One thread per site; a
// block covers one tile of one column, so every population access of a
// wavefront is a contiguous 512-byte (FP64) or 256-byte (FP32) run, and
// consecutive blocks take consecutive tiles of a column.  The pull source of
// population l is column (x - e_lx) mod Lx, row z - e_lz: in an interior
// tile that is the same tile of the source column or, for the |e_lz| rows at
// the tile's edge, the tile below or above it.  Each input element is read
// by exactly one site, so the step moves 37 reads + 37 writes per site and is
// bound by HBM bandwidth; the arithmetic (~500 flops per site with the
// factored equilibrium) stays well under the FP64 ridge.  In the
// [37][Lx][Lz] layout a wavefront's 74 streams touched 74 pages a whole
// population array apart and thrashed the CU's address-translation cache;
// in tiles they lie within a few neighbouring 37 TILE-element runs.
//
// Walls.  Blocks within 3 rows of either wall (or of a ragged end) take a
// second, block-uniform code path that substitutes ghost sites for sources
// outside [0, Lz) or wraps z in the periodic test mode; all other blocks run
// the branch-free path.  The Dirichlet wall reads its ghost populations from
// the wall table.  The diffuse wall (F_WALL_DIFFUSE, mass-conserving
// reading of the bc step of Sec. III.B) gives ghost site s the table row's
// populations times M(s)/S: M(s) is the mass that streams from the lattice
// into s in this pull, S the sum of the table row over the populations that
// point back into the lattice, so s returns exactly what it received.
//
// Single-buffer form (Sec. III.B keeps two lattice copies; this halves the
// memory).  Two step kinds alternate on one buffer A, each moving the same
// 37 + 37 elements per site as the two-buffer step:
//   IN_O: thread x pulls f_l(x) = A[l][x - e_l] (the stored post-collision
//         state), collides, and writes f*_l(x) to A[-l][x + e_l];
//   IN_E: thread x reads f_l(x) = A[-l][x], collides, writes f*_l(x) to A[l][x].
// A thread writes exactly the 37 locations it read (the slots A[m][x - e_m]
// are the slots A[-l][x + e_l] with m = -l), so no two threads touch the same
// element and the update is race-free in place.  After IN_O the buffer holds
// the next step's streamed populations at the opposite slot; after IN_E it
// holds the post-collision state in the standard layout again.  A population
// leaving the lattice in IN_O is parked in its own slot A[l][x], which no one
// else reads or writes in that step (it is the slot a ghost site would fill);
// in the standard layout the same slots hold the populations that left in
// the preceding IN_E step.  So in both kinds the mass that streams into a
// ghost site s is the sum of A[m][s - e_m] over the m leaving the lattice.
// Launches of an in-place step: (diffuse walls) wall_ratio_kernel saves M/S
// of every ghost site before those slots are overwritten; step_inplace_kernel
// steps the six wall rows per column in its leading blocks and rows
// 3..Lz-4 with the interior code only in the others.  Keeping the wall rows' parking and ghost
// substitution out of the tile kernel keeps it free of spills (184-186
// VGPRs in FP64, 132-162 in FP32, instead of 256 with spills).
#include "common.h"
#include "kernels.h"

namespace lbm {

template <int PREC>
struct Elt;
template <>
struct Elt<P_F64> {
    using T = double;
};
template <>
struct Elt<P_F32_DEV> {
    using T = float;
};
template <>
struct Elt<P_F32_DEV_C64> {
    using T = float;
};

// Addressing of a step: two buffers (pull), or one of the two in-place kinds.
enum : int { M_PULL = 0, M_IN_O = 1, M_IN_E = 2 };

// Index of -e_l: the rest velocity first, then each +e followed by its -e.
__host__ __device__ constexpr int opp(int l) { return l == 0 ? 0 : ((l & 1) ? l + 1 : l - 1); }
constexpr bool opp_is_reversal() {
    for (int l = 0; l < Q; ++l)
        if (EX[opp(l)] != -EX[l] || EZ[opp(l)] != -EZ[l]) return false;
    return true;
}
static_assert(opp_is_reversal(), "population order: each +e must be followed by its -e");

// Restrict-qualified pointers only where input and output are distinct.
template <typename T, bool R>
struct Ptr {
    using type = T *;
};
template <typename T>
struct Ptr<T, true> {
    using type = T *__restrict__;
};

// Full population value of a state or table element (FP32 stores f - w).
template <int PREC, typename E>
__device__ __forceinline__ double full_value(E v, int l) {
    return PREC == P_F64 ? (double)v : (double)v + W[l];
}

// M/S of the diffuse wall for ghost site (column xg, row i of a side): M sums
// the populations f[m] at (xg - e_mx, k - e_mz) that stream into the ghost
// site from inside the walls, S the table row over the populations that
// leave the ghost site into the lattice.
template <int PREC, typename E>
__device__ __forceinline__ double ghost_ratio(const StepArgs &a, const E *f, const E *ghost, int side, int i,
                                              int xg) {
    const int k = side == 0 ? -1 - i : a.lz + i;
    const E *row = ghost + (size_t)(side * 3 + i) * Q;
    double M = 0.0, S = 0.0;
#pragma unroll
    for (int m = 0; m < Q; ++m) {
        // every load unconditional (a clamped row where the source lies beyond
        // the wall), then masked: loads under per-lane branches are issued one
        // at a time, each waiting for the previous
        const int zs = k - EZ[m];
        const int zc = zs < 0 ? 0 : (zs >= a.lz ? a.lz - 1 : zs);
        const int xs = EX[m] == 0 ? xg : wrap(xg - EX[m], a.lx);
        const double v = full_value<PREC>(f[pidx(m, xs, zc, a.lx)], m);
        M += (zs >= 0 && zs < a.lz) ? v : 0.0;
        const int zd = k + EZ[m];
        const double c = full_value<PREC>(row[m], m);
        S += (zd >= 0 && zd < a.lz) ? c : 0.0;
    }
    return M / S;
}

// Diffuse wall: the incoming population l at a site whose pull source row zs
// may lie beyond a wall.  `in` is the in-range candidate, already loaded from
// a valid row; gv[side][i][l] (LDS) holds what ghost site (x - e_lx, row i of
// the side) emits into population l, and the two are selected without a
// branch: a global load under a per-lane branch is waited for on its own.
template <int PREC, typename E>
__device__ __forceinline__ E diffuse_source(E in, const double (*gv)[3][Q], int l, int zs, int lz) {
    const bool gs = zs < 0 || zs >= lz;
    const int side = zs < 0 ? 0 : 1;
    const int i = zs < 0 ? -zs - 1 : (zs >= lz ? zs - lz : 0);
    const double f = gv[side][i][l];
    return gs ? (E)(PREC == P_F64 ? f : f - W[l]) : in;
}

// The diffuse wall's ghost values of one column x, by one wavefront: lanes
// 0..41 form M/S of the 2 x 3 x 7 ghost sites (side, row i, column x + dx),
// dx = -3..3, that the column pulls from (into ratio), then every lane forms
// gv[side][i][l] = table[side][i][l] M/S of the ghost site in column x - e_lx.
// `ratio_in`, if given, holds M/S of every ghost site ([2 x 3][Lx], formed
// beforehand) instead.  The caller synchronises the block between the two
// phases (`phase` 0 and 1).
template <int PREC, typename E>
__device__ __forceinline__ void diffuse_ghost_values(const StepArgs &a, const E *fin, const E *ghost,
                                                     const double *ratio_in, int x, int lane, int phase,
                                                     double (*ratio)[3][7], double (*gv)[3][Q]) {
    if (phase == 0) {
        if (lane >= 42) return;
        const int side = lane / 21, i = (lane % 21) / 7, dx = lane % 7 - 3;
        const int xg = wrap(x + dx, a.lx);
        ratio[side][i][dx + 3] = ratio_in ? ratio_in[(size_t)(side * 3 + i) * a.lx + xg]
                                          : ghost_ratio<PREC>(a, fin, ghost, side, i, xg);
        return;
    }
    for (int j = lane; j < 2 * 3 * Q; j += 64) {
        const int row = j / Q, l = j % Q;   // row = side * 3 + i
        gv[row / 3][row % 3][l] = full_value<PREC>(ghost[row * Q + l], l) * ratio[row / 3][row % 3][3 - EX[l]];
    }
}

// One site (x, z) of the step.  EDGE: rows within 3 of a wall may pull from
// ghost sites; lanes with z >= Lz only read (a valid row) and store nothing,
// nor do lanes with store == false.  DIFFUSE: ghost sites are the diffuse
// wall's, emitting gv (diffuse_ghost_values, for column x).  MODE: addressing
// (see the file comment); the in-place kinds read and write a.f_out.
template <int PREC, bool EDGE, bool DIFFUSE, int MODE>
__device__ __forceinline__ void step_site(const StepArgs &a, int x, int z, bool store,
                                          const double (*gv)[3][Q]) {
    using E = typename Elt<PREC>::T;
    constexpr bool two = MODE == M_PULL;
    const size_t N = (size_t)a.lx * (size_t)a.lz;   // moments_out is [4][Lx][Lz]
    typename Ptr<const E, two>::type fin = static_cast<const E *>(two ? a.f_in : a.f_out);
    typename Ptr<E, two>::type fout = static_cast<E *>(a.f_out);
    const E *__restrict__ ghost = static_cast<const E *>(a.ghost);
    const bool active = store && (!EDGE || z < a.lz);
    const int zq = (EDGE && z >= a.lz) ? a.lz - 1 : z;   // idle lanes read a valid row
    constexpr bool diffuse = EDGE && DIFFUSE;
    const bool periodic = (a.flags & F_PERIODIC_Z) != 0;

    // ---- propagate + bc: the incoming population l ------------------------
    // The two-buffer step's tile blocks (one tile per block: zt is uniform)
    // address rows relative to their tile, also in the tiles at the walls;
    // the diffuse wall blocks (one wavefront per column, rows of two tiles)
    // and the in-place kinds use the general tiled index.
    constexpr bool tile_rows = two && !DIFFUSE;
    const int zt = tile_rows ? __builtin_amdgcn_readfirstlane(z / TILE) : 0;
    const int zl = z % TILE, zlq = zq % TILE;
    const long long tstep = (long long)a.lx * (Q * TILE) - TILE;
    auto gather = [&](int l) -> E {
        // in-range value: pulled from the neighbour, or (IN_E) this site's -l slot
        const int xs = (MODE == M_IN_E || EX[l] == 0) ? x : wrap(x - EX[l], a.lx);
        const int sl = MODE == M_IN_E ? opp(l) : l;
        const int dz = MODE == M_IN_E ? 0 : EZ[l];
        if (!EDGE) return fin[pidx(sl, xs, z - dz, a.lx)];
        const int zs = zq - EZ[l];   // pull source row: beyond a wall -> ghost site
        if (diffuse) {
            // the in-range candidate only (a clamped row); the ghost values
            // are selected after all 37 loads have been issued
            const int zr = zq - dz;
            return fin[pidx(sl, xs, zr < 0 ? 0 : (zr >= a.lz ? a.lz - 1 : zr), a.lx)];
        }
        if (periodic) return fin[pidx(sl, xs, wrap(zq - dz, a.lz), a.lx)];
        if (zs < 0) return ghost[(-zs - 1) * Q + l];
        if (zs >= a.lz) return ghost[(3 + zs - a.lz) * Q + l];
        return fin[pidx(sl, xs, zq - dz, a.lx)];
    };
    // All 37 populations are held in registers from the gather to the stores;
    // in place, a pair's stores overwrite only that pair's own inputs (the
    // slots of l and -l), which are already in registers.
    constexpr bool inplace = MODE != M_PULL;
    E v[Q];
    if (inplace) {
#pragma unroll
        for (int l = 0; l < Q; ++l) v[l] = gather(l);
    } else {
#pragma unroll
        for (int l = 0; l < Q; ++l) {
            const int xs = EX[l] == 0 ? x : wrap(x - EX[l], a.lx);
            const E *tb = fin + ((size_t)zt * (size_t)a.lx + (size_t)xs) * (Q * TILE);
            if (!EDGE) {
                // row z - e_lz: this tile, or (|e_lz| rows) the one below / above
                v[l] = tb[tile_off(l, zl - EZ[l], tstep)];
            } else if (tile_rows && !periodic) {
                // a tile at a wall: in-range rows as in the interior, ghost rows from the table
                const int zs = zq - EZ[l];
                if (zs < 0)
                    v[l] = ghost[(-zs - 1) * Q + l];
                else if (zs >= a.lz)
                    v[l] = ghost[(3 + zs - a.lz) * Q + l];
                else
                    v[l] = tb[tile_off(l, zlq - EZ[l], tstep)];
            } else {
                auto src = [&](int zz) -> E { return fin[pidx(l, xs, zz, a.lx)]; };
                const int zs = zq - EZ[l];
                if (diffuse) {
                    v[l] = src(zs < 0 ? 0 : (zs >= a.lz ? a.lz - 1 : zs));   // selected below
                } else if (periodic) {
                    v[l] = src(wrap(zs, a.lz));
                } else if (zs < 0) {
                    v[l] = ghost[(-zs - 1) * Q + l];
                } else if (zs >= a.lz) {
                    v[l] = ghost[(3 + zs - a.lz) * Q + l];
                } else {
                    v[l] = src(zs);
                }
            }
        }
    }
    if (diffuse) {
        // ghost sites: one select per population once every load is in flight
        // (a select next to each load made the loads wait for each other)
#pragma unroll
        for (int l = 0; l < Q; ++l) v[l] = diffuse_source<PREC>(v[l], gv, l, zq - EZ[l], a.lz);
    }
    auto val = [&](int l) -> E { return v[l]; };

    const size_t site = (size_t)x * (size_t)a.lz + (size_t)z;
    // store f*_l of this site: own slot l (two buffers, IN_E), or slot -l of
    // the site it streams to (IN_O; parked in its own slot l when that site
    // lies beyond a wall).  The two-buffer step streams its output past the
    // caches (non-temporal); the in-place kinds store normally, so that the
    // partial cache lines of IN_O's shifted rows merge in L2 before they are
    // written back (measured 3 % faster on MI355X).
    auto put = [&](int l, E val) {
        if (MODE == M_PULL) {
            if (tile_rows)
                __builtin_nontemporal_store(
                    val, &fout[((size_t)zt * (size_t)a.lx + (size_t)x) * (Q * TILE) + (size_t)l * TILE + zl]);
            else
                __builtin_nontemporal_store(val, &fout[pidx(l, x, z, a.lx)]);
            return;
        }
        if (MODE == M_IN_E) {
            fout[pidx(l, x, z, a.lx)] = val;
            return;
        }
        const int xd = EX[l] == 0 ? x : wrap(x + EX[l], a.lx);
        const int zd = z + EZ[l];
        if (!EDGE) {
            fout[pidx(opp(l), xd, zd, a.lx)] = val;
        } else {
            if (periodic)
                fout[pidx(opp(l), xd, wrap(zd, a.lz), a.lx)] = val;
            else if (zd < 0 || zd >= a.lz)
                fout[pidx(l, x, z, a.lx)] = val;
            else
                fout[pidx(opp(l), xd, zd, a.lx)] = val;
        }
    };

    if (a.flags & F_NO_COLLIDE) {
        if (active) {
            put(0, val(0));
#pragma unroll
            for (int l = 1; l < Q; l += 2) {
                const E p = val(l), m = val(l + 1);
                put(l, p);
                put(l + 1, m);
            }
        }
        return;
    }

    // ---- moments (FP64 in both precisions) -------------------------------
    double s0 = 0.0, sx = 0.0, sz = 0.0, s2 = 0.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const double f = (double)val(l);
        s0 += f;
        if (EX[l] != 0) sx += EX[l] * f;
        if (EZ[l] != 0) sz += EZ[l] * f;
        if (SHELL[l] != 0) s2 += (EX[l] * EX[l] + EZ[l] * EZ[l]) * f;
    }
    // FP32 deviations d_l = f_l - w_l: sum w = 1, sum w xi = 0, sum w xi^2 = D
    const double rho = (PREC == P_F64) ? s0 : 1.0 + s0;
    const double inv = 1.0 / rho;
    const double ux = R * sx * inv, uz = R * sz * inv;
    const double e2 = (PREC == P_F64) ? R2 * s2 : D + R2 * s2;
    const double T = (e2 * inv - ux * ux - uz * uz) / D;

    if (a.mom && active) {
        if (a.flags & F_MOM_F32) {
            float *m = static_cast<float *>(a.mom);
            m[site] = (float)rho;
            m[N + site] = (float)ux;
            m[2 * N + site] = (float)uz;
            m[3 * N + site] = (float)T;
        } else {
            double *m = static_cast<double *>(a.mom);
            m[site] = rho;
            m[N + site] = ux;
            m[2 * N + site] = uz;
            m[3 * N + site] = T;
        }
    }

    // ---- force-shifted equilibrium and BGK relaxation --------------------
    // equilibrium arguments: v = u + tau g_vec, th = T + tau (1 - tau) g^2 / D - 1
    const double vx = ux, vz = uz - a.tau * a.g;
    const double th = T + a.tau * (1.0 - a.tau) * a.g * a.g / D - 1.0;
    const double u2 = vx * vx + vz * vz;

    if (PREC == P_F64) {
        const double om = a.omega, keep = 1.0 - a.omega;
#pragma unroll
        for (int s = 0; s < NSHELL; ++s) {
            const ShellCoef<double> c = shell_coef<double>(u2, th, XI2_SHELL[s]);
            const double wr = W_SHELL[s] * rho;
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                if (SHELL[l] != s) continue;
                if (l == 0) {
                    const double feq = wr * (1.0 + c.a0m1);
                    if (active) put(0, keep * (double)val(0) + om * feq);
                    continue;
                }
                if ((l & 1) == 0) continue;   // handled with its +e partner l-1
                double ev, od;
                pair_poly<double>(c, R * (EX[l] * vx + EZ[l] * vz), ev, od);
                const double even = wr * (1.0 + ev), odd = wr * od;
                const double vp = (double)val(l), vm = (double)val(l + 1);
                const double fp = keep * vp + om * (even + odd);
                const double fm = keep * vm + om * (even - odd);
                if (active) {
                    put(l, fp);
                    put(l + 1, fm);
                }
            }
        }
    } else if (PREC == P_F32_DEV_C64) {
        // deviation form in double arithmetic, one rounding to float per
        // stored value: d^eq_l = w_l (drho + rho (P_l - 1))
        const double om = a.omega;
#pragma unroll
        for (int s = 0; s < NSHELL; ++s) {
            const ShellCoef<double> c = shell_coef<double>(u2, th, XI2_SHELL[s]);
            const double w = W_SHELL[s];
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                if (SHELL[l] != s) continue;
                if (l == 0) {
                    const double v0 = (double)val(0);
                    if (active) put(0, (E)(v0 + om * (w * (s0 + rho * c.a0m1) - v0)));
                    continue;
                }
                if ((l & 1) == 0) continue;
                double ev, od;
                pair_poly<double>(c, R * (EX[l] * vx + EZ[l] * vz), ev, od);
                const double dp = w * (s0 + rho * (ev + od)), dm = w * (s0 + rho * (ev - od));
                const double vp = (double)val(l), vm = (double)val(l + 1);
                if (active) {
                    put(l, (E)(vp + om * (dp - vp)));
                    put(l + 1, (E)(vm + om * (dm - vm)));
                }
            }
        }
    } else {
        // deviation form: d^eq_l = w_l (rho P_l - 1) = w_l (drho + rho (P_l - 1))
        const float drho = (float)s0, rhof = (float)rho;
        const float u2f = (float)u2, thf = (float)th;
        const float vxf = (float)vx, vzf = (float)vz;
        const float om = (float)a.omega;
#pragma unroll
        for (int s = 0; s < NSHELL; ++s) {
            const ShellCoef<float> c = shell_coef<float>(u2f, thf, (float)XI2_SHELL[s]);
            const float w = (float)W_SHELL[s];
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                if (SHELL[l] != s) continue;
                if (l == 0) {
                    const float deq = w * (drho + rhof * c.a0m1);
                    const float v0 = val(0);
                    if (active) put(0, v0 + om * (deq - v0));
                    continue;
                }
                if ((l & 1) == 0) continue;
                float ev, od;
                pair_poly<float>(c, (float)R * ((float)EX[l] * vxf + (float)EZ[l] * vzf), ev, od);
                const float dp = w * (drho + rhof * (ev + od));
                const float dm = w * (drho + rhof * (ev - od));
                const float vp = val(l), vm = val(l + 1);
                const float op = vp + om * (dp - vp);
                const float omn = vm + om * (dm - vm);
                if (active) {
                    put(l, op);
                    put(l + 1, omn);
                }
            }
        }
    }
}

// Launch shape per precision: threads per block (one site each along z) and
// the number of consecutive row blocks of BS rows each block walks.  A block
// covers exactly one 512-row tile of the population layout in both
// precisions: the interior path addresses rows relative to the tile's base
// (common.h tile_off), with the tile index uniform over the block.
template <int PREC>
struct StepShape;
template <>
struct StepShape<P_F64> {
    static constexpr int BS = TILE, ZT = 1;
};
template <>
struct StepShape<P_F32_DEV> {
    static constexpr int BS = TILE, ZT = 1;
};
template <>
struct StepShape<P_F32_DEV_C64> {
    static constexpr int BS = TILE, ZT = 1;
};
static_assert(StepShape<P_F64>::BS * StepShape<P_F64>::ZT == TILE &&
                  StepShape<P_F32_DEV>::BS * StepShape<P_F32_DEV>::ZT == TILE &&
                  StepShape<P_F32_DEV_C64>::BS * StepShape<P_F32_DEV_C64>::ZT == TILE,
              "a block of the two-buffer step covers exactly one tile (the interior path's addressing)");

// Diffuse-wall rows of one column per wavefront (two-buffer step): the
// column's ghost values (diffuse_ghost_values), then lane j < min(Lz, 6)
// steps wall row j (rows 0, 1, 2, Lz-3, Lz-2, Lz-1; every row when Lz < 6).
template <int PREC, int BS>
__device__ __forceinline__ void wall_block(const StepArgs &a, uint32_t b) {
    using E = typename Elt<PREC>::T;
    constexpr int NW = BS / 64;   // columns per block
    __shared__ double ratio[NW][2][3][7];
    __shared__ double gv[NW][2][3][Q];
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    const int x = __builtin_amdgcn_readfirstlane((int)b * NW + w);
    const bool live = x < a.lx;
    const E *fin = static_cast<const E *>(a.f_in), *ghost = static_cast<const E *>(a.ghost);
    if (live) diffuse_ghost_values<PREC>(a, fin, ghost, nullptr, x, lane, 0, ratio[w], gv[w]);
    __syncthreads();
    if (live) diffuse_ghost_values<PREC>(a, fin, ghost, nullptr, x, lane, 1, ratio[w], gv[w]);
    __syncthreads();
    const int nw = a.lz < 6 ? a.lz : 6;
    if (live && lane < nw)
        step_site<PREC, true, true, M_PULL>(a, x, lane < 3 ? lane : a.lz - (nw - lane), true, gv[w]);
}

// One launch per step.  With diffuse walls the first nwall blocks step the
// wall rows (wall_block, BS/64 columns each) and the tile blocks leave rows
// 0..2 and Lz-3..Lz-1 alone; issuing the short, latency-bound wall blocks
// first lets them run under the bulk of the step.
template <int PREC>
__global__ __launch_bounds__(StepShape<PREC>::BS) void step_kernel(StepArgs a, int nzb, uint32_t nblocks,
                                                                   uint32_t nwall) {
    constexpr int BS = StepShape<PREC>::BS, ZT = StepShape<PREC>::ZT;
    if (blockIdx.x < nwall) {
        wall_block<PREC, BS>(a, blockIdx.x);
        return;
    }
    const uint32_t t = blockIdx.x - nwall;
    const int x = (int)(t / (uint32_t)nzb);
    const int zt = (int)(t % (uint32_t)nzb) * ZT;
    const bool skip_wall = nwall != 0;
    for (int k = 0; k < ZT; ++k) {
        const int z0 = (zt + k) * BS;
        if (z0 >= a.lz) break;
        const int z = z0 + (int)threadIdx.x;
        const bool edge = (z0 < 3) || (z0 + BS + 3 > a.lz);
        if (edge)
            step_site<PREC, true, false, M_PULL>(a, x, z, !skip_wall || (z >= 3 && z < a.lz - 3), nullptr);
        else
            step_site<PREC, false, false, M_PULL>(a, x, z, true, nullptr);
    }
}

// In-place kinds: the wall rows (rows 0, 1, 2, Lz-3, Lz-2, Lz-1; every row
// when Lz < 7) of BS/64 columns, one wavefront per column, with the
// Dirichlet table or the diffuse wall's M/S from a.ratio (wall_ratio_kernel).
template <int PREC, int MODE, bool DIFFUSE, int BS>
__device__ __forceinline__ void inplace_wall_block(const StepArgs &a, uint32_t b) {
    using E = typename Elt<PREC>::T;
    constexpr int NW = BS / 64;   // columns per block
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    const int x = __builtin_amdgcn_readfirstlane((int)b * NW + w);
    const bool live = x < a.lx;
    const double(*gvw)[3][Q] = nullptr;
    if constexpr (DIFFUSE) {
        __shared__ double ratio[NW][2][3][7];
        __shared__ double gv[NW][2][3][Q];
        const E *ghost = static_cast<const E *>(a.ghost);
        if (live) diffuse_ghost_values<PREC>(a, static_cast<const E *>(nullptr), ghost, a.ratio, x, lane, 0, ratio[w], gv[w]);
        __syncthreads();
        if (live) diffuse_ghost_values<PREC>(a, static_cast<const E *>(nullptr), ghost, a.ratio, x, lane, 1, ratio[w], gv[w]);
        __syncthreads();
        gvw = gv[w];
    }
    const int nw = a.lz < 7 ? a.lz : 6;
    if (live && lane < nw)
        step_site<PREC, true, DIFFUSE, MODE>(a, x, lane < 3 || a.lz < 7 ? lane : a.lz - (nw - lane), true, gvw);
}

// In-place kinds: the first nwall blocks step the wall rows
// (inplace_wall_block; WALLS = 1 Dirichlet, 2 diffuse; no wall code with
// WALLS = 0), the others rows 3 .. Lz-4 of one tile each (every source and
// destination inside the walls) with only the branch-free interior code,
// which keeps the tile path's register count at the two-buffer level; in
// tiles that reach a wall the lanes outside these rows load a valid row and
// store nothing.  Wall and tile blocks may run at the same time: every site
// reads and writes only its own 37 slots.
template <int PREC, int MODE, int WALLS>
__global__ __launch_bounds__(StepShape<PREC>::BS) void step_inplace_kernel(StepArgs a, int nzb, uint32_t nwall) {
    constexpr int BS = StepShape<PREC>::BS, ZT = StepShape<PREC>::ZT;
    if constexpr (WALLS != 0) {
        if (__builtin_expect(blockIdx.x < nwall, 0)) {
            inplace_wall_block<PREC, MODE, WALLS == 2, BS>(a, blockIdx.x);
            return;
        }
    }
    const uint32_t t = blockIdx.x - nwall;
    const int x = (int)(t / (uint32_t)nzb);
    const int zt = (int)(t % (uint32_t)nzb) * ZT;
    for (int k = 0; k < ZT; ++k) {
        const int z0 = (zt + k) * BS;
        if (z0 >= a.lz) break;
        const int z = z0 + (int)threadIdx.x;
        const bool inner = z >= 3 && z < a.lz - 3;
        const int zc = z < 3 ? 3 : (z > a.lz - 4 ? a.lz - 4 : z);
        step_site<PREC, false, false, MODE>(a, x, zc, inner, nullptr);
    }
}

// In-place kinds with diffuse walls: M/S of every ghost site into a.ratio
// ([2 x 3][Lx]) before the step overwrites the slots the masses are read from.
template <int PREC>
__global__ __launch_bounds__(256) void wall_ratio_kernel(StepArgs a) {
    using E = typename Elt<PREC>::T;
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= 6 * a.lx) return;
    const int row = t / a.lx, xg = t % a.lx;
    a.ratio[t] = ghost_ratio<PREC>(a, static_cast<const E *>(a.f_out), static_cast<const E *>(a.ghost), row / 3,
                                   row % 3, xg);
}

// One block (8 wavefronts, 2 per SIMD) per CU at a time.  The tile path
// needs 126 (FP64) / 80 (FP32) VGPRs (the kernel 160 / 112 with the diffuse
// wall rows), which would let 2 / 3 blocks share a CU; those ran 3.3 % /
// 4.5 % slower at 4096 x 12288 on MI355X (more tiles in flight at once
// contend for DRAM banks), so each launch requests this much
// dynamic LDS, which the kernel never touches, to keep a second block off
// the CU: with the kernel's static arrays of the diffuse wall (17 KB) a block
// takes more than half of the CU's 160 KB.
constexpr size_t STEP_OCCUPANCY_LDS = 80 * 1024;

template <int PREC>
static void launch_prec(const StepArgs &a, hipStream_t s) {
    constexpr int BS = StepShape<PREC>::BS, span = BS * StepShape<PREC>::ZT;
    const int nzb = (a.lz + span - 1) / span;
    const uint32_t nblocks = (uint32_t)nzb * (uint32_t)a.lx;
    const uint32_t nwall = (a.flags & F_WALL_DIFFUSE) ? (uint32_t)((a.lx + BS / 64 - 1) / (BS / 64)) : 0u;
    hipLaunchKernelGGL(step_kernel<PREC>, dim3(nwall + nblocks), dim3(BS), STEP_OCCUPANCY_LDS, s, a, nzb, nblocks,
                       nwall);
}

// One launch (wall blocks first, then tiles) removes the wall rows' own
// launch and its latency: measured on MI355X, 512 x 1536 in-place steps
// 0.071 ms against 0.085 (FP64) and 0.041 against 0.056 (FP32), 4096 x
// 12288 FP32 2.99-3.00 ms against 3.01-3.03.  Large FP64 lattices keep two
// launches: with the wall code in it the tile kernel ran 1.2-1.9 % slower at
// 2048 x 6144 and 4096 x 12288 (also when launched for the tiles alone), so
// there a kernel without wall code steps the tiles and the combined kernel,
// launched for its wall blocks only, the wall rows.
constexpr long long INPLACE_SPLIT_SITES_F64 = 1ll << 22;

template <int PREC, int MODE>
static void launch_inplace(const StepArgs &a, hipStream_t s) {
    constexpr int BS = StepShape<PREC>::BS, span = BS * StepShape<PREC>::ZT;
    const bool diffuse = (a.flags & F_WALL_DIFFUSE) != 0;
    if (diffuse)
        hipLaunchKernelGGL(wall_ratio_kernel<PREC>, dim3((uint32_t)((6 * a.lx + 255) / 256)), dim3(256), 0, s, a);
    const int nzb = (a.lz + span - 1) / span;
    const uint32_t nwall = (uint32_t)((a.lx + BS / 64 - 1) / (BS / 64));
    uint32_t ntile = a.lz >= 7 ? (uint32_t)nzb * (uint32_t)a.lx : 0u;
    if (PREC == P_F64 && ntile != 0 && (long long)a.lx * a.lz >= INPLACE_SPLIT_SITES_F64) {
        hipLaunchKernelGGL((step_inplace_kernel<PREC, MODE, 0>), dim3(ntile), dim3(BS), 0, s, a, nzb, 0u);
        ntile = 0;
    }
    if (diffuse)
        hipLaunchKernelGGL((step_inplace_kernel<PREC, MODE, 2>), dim3(nwall + ntile), dim3(BS), 0, s, a, nzb, nwall);
    else
        hipLaunchKernelGGL((step_inplace_kernel<PREC, MODE, 1>), dim3(nwall + ntile), dim3(BS), 0, s, a, nzb, nwall);
}

hipError_t launch_step(const StepArgs &a, int precision, hipStream_t s) {
    if (precision == P_F64)
        launch_prec<P_F64>(a, s);
    else if (a.flags & F_COLLIDE_F64)
        launch_prec<P_F32_DEV_C64>(a, s);
    else
        launch_prec<P_F32_DEV>(a, s);
    return hipGetLastError();
}

hipError_t launch_step_inplace(const StepArgs &a, int precision, int kind, hipStream_t s) {
    if (precision == P_F64) {
        if (kind == 0)
            launch_inplace<P_F64, M_IN_O>(a, s);
        else
            launch_inplace<P_F64, M_IN_E>(a, s);
    } else if (a.flags & F_COLLIDE_F64) {
        if (kind == 0)
            launch_inplace<P_F32_DEV_C64, M_IN_O>(a, s);
        else
            launch_inplace<P_F32_DEV_C64, M_IN_E>(a, s);
    } else {
        if (kind == 0)
            launch_inplace<P_F32_DEV, M_IN_O>(a, s);
        else
            launch_inplace<P_F32_DEV, M_IN_E>(a, s);
    }
    return hipGetLastError();
}

}  // namespace lbm
