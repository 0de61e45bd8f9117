// Fused D2Q37 time step: pull streaming + wall rows + force-shifted BGK collide.
//
// Sec. III.A eq. LBE and the shifted equilibrium; Sec. III.B step order
// (propagate, bc, collide) and the prv/nxt pair of lattice copies.
//
// Mapping.  One thread per site; a block covers BS consecutive sites of one
// column (z fastest) and walks ZT such tiles down the column, so every
// population access of a wavefront is a contiguous 512-byte (FP64) or
// 256-byte (FP32) run.  The pull source of
// population l is column (x - e_lx) mod Lx, rows z - e_lz: the column offset
// is uniform over the block (scalar), the row shift is an immediate offset.
// Each input element is read by exactly one site, so the step moves
// 37 reads + 37 writes per site and is bound by HBM bandwidth; the arithmetic
// (~500 flops per site with the factored equilibrium) stays well under the
// FP64 ridge.
//
// Walls.  Blocks within 3 rows of either wall (or of a ragged end) take a
// second, block-uniform code path that substitutes ghost sites for sources
// outside [0, Lz) or wraps z in the periodic test mode; all other blocks run
// the branch-free path.  The Dirichlet wall reads its ghost populations from
// the wall table.  The diffuse wall (F_WALL_DIFFUSE, mass-conserving
// reading of the bc step of Sec. III.B) gives ghost site s the table row's
// populations times M(s)/S: M(s) is the mass that streams from the lattice
// into s in this pull, S the sum of the table row over the populations that
// point back into the lattice, so s returns exactly what it received.  The
// block first evaluates M/S for the 2 x 3 x 7 ghost sites its column can
// pull from (columns x-3..x+3) into LDS.
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

// Full population value of a state or table element (FP32 stores f - w).
template <int PREC, typename E>
__device__ __forceinline__ double full_value(E v, int l) {
    return PREC == P_F64 ? (double)v : (double)v + W[l];
}

// M/S of the diffuse wall for the ghost sites (side, row i, column x + dx),
// dx = -3..3, one lane each (lanes 0..41 of a wavefront).
template <int PREC, typename E>
__device__ __forceinline__ void diffuse_wall_ratios(const StepArgs &a, const E *fin, const E *ghost, int x,
                                                    int lane, double (*ratio)[3][7]) {
    if (lane >= 42) return;
    const size_t N = (size_t)a.lx * (size_t)a.lz;
    const int side = lane / 21, i = (lane % 21) / 7, dx = lane % 7 - 3;
    const int k = side == 0 ? -1 - i : a.lz + i;
    const int xg = wrap(x + dx, a.lx);
    const E *row = ghost + (size_t)(side * 3 + i) * Q;
    double M = 0.0, S = 0.0;
#pragma unroll
    for (int m = 0; m < Q; ++m) {
        const int zs = k - EZ[m];   // population m streams from (xg - e_mx, zs) into the ghost site
        if (zs >= 0 && zs < a.lz) {
            const int xs = EX[m] == 0 ? xg : wrap(xg - EX[m], a.lx);
            M += full_value<PREC>(fin[(size_t)m * N + (size_t)xs * (size_t)a.lz + (size_t)zs], m);
        }
        const int zd = k + EZ[m];   // population m leaves the ghost site towards row zd
        if (zd >= 0 && zd < a.lz) S += full_value<PREC>(row[m], m);
    }
    ratio[side][i][dx + 3] = M / S;
}

// One site (x, z) of the step.  EDGE: rows within 3 of a wall may pull from
// ghost sites; lanes with z >= Lz only read (a valid row) and store nothing,
// nor do lanes with store == false.  DIFFUSE: ghost sites are the diffuse
// wall's, with M/S from ratio (columns x-3..x+3).
template <int PREC, bool EDGE, bool DIFFUSE>
__device__ __forceinline__ void step_site(const StepArgs &a, int x, int z, bool store,
                                          const double (*ratio)[3][7]) {
    using E = typename Elt<PREC>::T;
    const size_t N = (size_t)a.lx * (size_t)a.lz;
    const E *__restrict__ fin = static_cast<const E *>(a.f_in);
    E *__restrict__ fout = static_cast<E *>(a.f_out);
    const E *__restrict__ ghost = static_cast<const E *>(a.ghost);
    const bool active = store && (!EDGE || z < a.lz);
    const int zq = (EDGE && z >= a.lz) ? a.lz - 1 : z;   // idle lanes read a valid row
    constexpr bool diffuse = EDGE && DIFFUSE;

    // ---- propagate + bc: gather the 37 incoming populations -------------
    E v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const int xs = EX[l] == 0 ? x : wrap(x - EX[l], a.lx);
        const E *src = fin + (size_t)l * N + (size_t)xs * (size_t)a.lz;
        if (!EDGE) {
            v[l] = src[z - EZ[l]];
        } else {
            const int zs = zq - EZ[l];
            if (diffuse) {
                if (zs < 0 || zs >= a.lz) {   // ghost site (x - e_lx, zs)
                    const int side = zs < 0 ? 0 : 1, i = zs < 0 ? -zs - 1 : zs - a.lz;
                    const double f = full_value<PREC>(ghost[(side * 3 + i) * Q + l], l) *
                                     ratio[side][i][3 - EX[l]];
                    v[l] = (E)(PREC == P_F64 ? f : f - W[l]);
                } else {
                    v[l] = src[zs];
                }
            } else if (a.flags & F_PERIODIC_Z) {
                v[l] = src[wrap(zs, a.lz)];
            } else if (zs < 0) {
                v[l] = ghost[(-zs - 1) * Q + l];
            } else if (zs >= a.lz) {
                v[l] = ghost[(3 + zs - a.lz) * Q + l];
            } else {
                v[l] = src[zs];
            }
        }
    }

    const size_t site = (size_t)x * (size_t)a.lz + (size_t)z;
    if (a.flags & F_NO_COLLIDE) {
        if (active) {
#pragma unroll
            for (int l = 0; l < Q; ++l) fout[(size_t)l * N + site] = v[l];
        }
        return;
    }

    // ---- moments (FP64 in both precisions) -------------------------------
    double s0 = 0.0, sx = 0.0, sz = 0.0, s2 = 0.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const double f = (double)v[l];
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
        a.mom[site] = rho;
        a.mom[N + site] = ux;
        a.mom[2 * N + site] = uz;
        a.mom[3 * N + site] = T;
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
                    if (active) __builtin_nontemporal_store(keep * (double)v[0] + om * feq, &fout[site]);
                    continue;
                }
                if ((l & 1) == 0) continue;   // handled with its +e partner l-1
                double ev, od;
                pair_poly<double>(c, R * (EX[l] * vx + EZ[l] * vz), ev, od);
                const double even = wr * (1.0 + ev), odd = wr * od;
                const double fp = keep * (double)v[l] + om * (even + odd);
                const double fm = keep * (double)v[l + 1] + om * (even - odd);
                if (active) {
                    __builtin_nontemporal_store(fp, &fout[(size_t)l * N + site]);
                    __builtin_nontemporal_store(fm, &fout[(size_t)(l + 1) * N + site]);
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
                    if (active) __builtin_nontemporal_store(v[0] + om * (deq - v[0]), &fout[site]);
                    continue;
                }
                if ((l & 1) == 0) continue;
                float ev, od;
                pair_poly<float>(c, (float)R * ((float)EX[l] * vxf + (float)EZ[l] * vzf), ev, od);
                const float dp = w * (drho + rhof * (ev + od));
                const float dm = w * (drho + rhof * (ev - od));
                const float op = v[l] + om * (dp - v[l]);
                const float omn = v[l + 1] + om * (dm - v[l + 1]);
                if (active) {
                    __builtin_nontemporal_store(op, &fout[(size_t)l * N + site]);
                    __builtin_nontemporal_store(omn, &fout[(size_t)(l + 1) * N + site]);
                }
            }
        }
    }
}

// Launch shape per precision: threads per block (one site each along z) and
// the number of consecutive tiles of BS rows each block walks.  Walking
// several tiles of one column lets the cache lines that neighbouring tiles
// share (pull sources shifted by up to 3 rows) be re-read from this block's
// L2 instead of being fetched again by a block on another XCD.  Chosen by
// measurement on MI355X at 4096 x 12288 (FP64 512 x 2, FP32 256 x 2).
template <int PREC>
struct StepShape;
template <>
struct StepShape<P_F64> {
    static constexpr int BS = 512, ZT = 2;
};
template <>
struct StepShape<P_F32_DEV> {
    static constexpr int BS = 256, ZT = 2;
};

// Diffuse-wall rows of one column per wavefront.  Lanes 0..41 evaluate M/S
// of the 2 x 3 x 7 ghost sites the column pulls from, then lane j < min(Lz, 6)
// steps wall row j (rows 0, 1, 2, Lz-3, Lz-2, Lz-1; every row when Lz < 6).
template <int PREC, int BS>
__device__ __forceinline__ void wall_block(const StepArgs &a, uint32_t b) {
    using E = typename Elt<PREC>::T;
    constexpr int NW = BS / 64;   // columns per block
    __shared__ double ratio[NW][2][3][7];
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    const int x = __builtin_amdgcn_readfirstlane((int)b * NW + w);
    const bool live = x < a.lx;
    if (live)
        diffuse_wall_ratios<PREC>(a, static_cast<const E *>(a.f_in), static_cast<const E *>(a.ghost), x, lane,
                                  ratio[w]);
    __syncthreads();
    const int nw = a.lz < 6 ? a.lz : 6;
    if (live && lane < nw)
        step_site<PREC, true, true>(a, x, lane < 3 ? lane : a.lz - (nw - lane), true, ratio[w]);
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
    const uint32_t t = xcd_tile(blockIdx.x - nwall, nblocks);
    const int x = (int)(t / (uint32_t)nzb);
    const int zt = (int)(t % (uint32_t)nzb) * ZT;
    const bool skip_wall = nwall != 0;
    for (int k = 0; k < ZT; ++k) {
        const int z0 = (zt + k) * BS;
        if (z0 >= a.lz) break;
        const int z = z0 + (int)threadIdx.x;
        const bool edge = (z0 < 3) || (z0 + BS + 3 > a.lz);
        if (edge)
            step_site<PREC, true, false>(a, x, z, !skip_wall || (z >= 3 && z < a.lz - 3), nullptr);
        else
            step_site<PREC, false, false>(a, x, z, true, nullptr);
    }
}

template <int PREC>
static void launch_prec(const StepArgs &a, hipStream_t s) {
    constexpr int BS = StepShape<PREC>::BS, span = BS * StepShape<PREC>::ZT;
    const int nzb = (a.lz + span - 1) / span;
    const uint32_t nblocks = (uint32_t)nzb * (uint32_t)a.lx;
    const uint32_t nwall = (a.flags & F_WALL_DIFFUSE) ? (uint32_t)((a.lx + BS / 64 - 1) / (BS / 64)) : 0u;
    hipLaunchKernelGGL(step_kernel<PREC>, dim3(nwall + nblocks), dim3(BS), 0, s, a, nzb, nblocks, nwall);
}

hipError_t launch_step(const StepArgs &a, int precision, hipStream_t s) {
    if (precision == P_F64)
        launch_prec<P_F64>(a, s);
    else
        launch_prec<P_F32_DEV>(a, s);
    return hipGetLastError();
}

}  // namespace lbm
