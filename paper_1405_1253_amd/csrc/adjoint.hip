// Reverse mode of the fused step, of the mixing objective and of the
// three-layer initial state.
//
// The paper has no adjoint; these kernels differentiate the forward kernels'
// arithmetic exactly (Sec. III.A step; Sec. IV mixing lengths; Sec. I init).
//
// Adjoint step (push form).  With lam_t = dJ/df*_t and m = (rho, u, T) the
// pre-collision moments of step t at site x,
//     G_l(x) = (1 - omega) lam_l(x) + alpha(x) + beta(x) . xi_l + gamma(x) |xi_l|^2
// where mu = omega (dF/dm)^T lam(x) and
//     alpha = mu_rho - mu_u . u / rho + mu_T (|u|^2 - D T) / (D rho)
//     beta  = mu_u / rho - 2 mu_T u / (D rho),   gamma = mu_T / (D rho),
// and lam_{t-1,l}(y) = G_l(y + e_l).  Each site computes its own G from its
// own 37 lam values and 4 moments and writes G_l to site x - e_l: every
// output element has exactly one writer (a permutation), so the kernel moves
// 37 + 4 reads and 37 writes per site.  The lam buffers use the tiled layout
// of the state (common.h); the moments are [4][Lx][Lz].  Rows y whose source y + e_l lies
// beyond a wall receive an explicit zero with the Dirichlet wall (those pulls
// read the constant wall table, which carries no derivative).
//
// Diffuse wall.  The forward ghost site s = y + e_l emits c_m M(s) with
// M(s) = sum of the populations streaming into it, so every such population
// receives A(s) = sum_m c_m G_m(s + e_m) over the m pointing back into the
// lattice (c_m = table row / its sum over those m).  The step kernel parks
// G_{-l}(y) in the slot (l, y) that A(y + e_l) will fill (the slots of one
// ghost site are exactly the slots its sum reads, by the e -> -e pairing),
// and a second kernel with one thread per ghost site reads its slots, forms
// A and writes it back into the same slots: no other thread touches them.
//
// Equilibrium derivatives.  With P(x) = A0 + A1 x + A2 x^2 + x^3/6 + x^4/24
// (common.h), x = xi . v, u2 = |v|^2, th = T_eq - 1:
//     dP/dv  = (A1 + 2 A2 x + x^2/2 + x^3/6) xi + 2 v dP/du2
//     dP/du2 = dA0/du2 - x/2 - x^2/4,  dA0/du2 = -1/2 + u2/4 + th (4 - xi2)/4
//     dP/dth = dA0/dth + x (xi2 - 4)/2 + x^2 (xi2 - 6)/4,
//     dA0/dth = (xi2 - 2)/2 + u2 (4 - xi2)/4 + th (xi2^2 - 8 xi2 + 8)/4
// and F_l = w_l rho P_l, so dF/drho = w P, dF/dv = w rho dP/dv, dF/dT = w rho dP/dth.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace lbm {

// sum_l lam_l w_l {P_l, dP_l/dx xi_l, dP_l/du2, dP_l/dth} at (v, th).
//
// P is a polynomial of degree 4 in xi (through x = xi . v and xi2 = |xi|^2),
// so every sum is a fixed polynomial in (v, u2, th) contracted with the 15
// raw moments m_pq = sum_l lam_l w_l xi_x^p xi_z^q, p + q <= 4.  With
//   A0 = a0 + a1 xi2 + a2 xi2^2, A1 = b0 + b1 xi2, A2 = c0 + c1 xi2,
//   a0 = 1 - u2/2 - th + u2^2/8 + th u2 + th^2, a1 = th/2 - th u2/4 - th^2,
//   a2 = th^2/8, b0 = 1 - u2/2 - 2 th, b1 = th/2, c0 = 1/2 - u2/4 - 3 th/2,
//   c1 = th/4,
// and the shorthand M_f = sum_l lam_l w_l f(xi_l):
//   sum P        = a0 M_1 + a1 M_xi2 + a2 M_xi2^2 + b0 M_x + b1 M_xi2x + c0 M_x^2
//                  + c1 M_xi2x^2 + M_x^3/6 + M_x^4/24
//   sum P' xi_i  = b0 M_i + b1 M_xi2 i + 2 c0 M_x i + 2 c1 M_xi2 x i + M_x^2 i/2 + M_x^3 i/6
//   sum dP/du2   = (u2/4 + th - 1/2) M_1 - th/4 M_xi2 - M_x/2 - M_x^2/4
//   sum dP/dth   = (u2 + 2 th - 1) M_1 + (1/2 - u2/4 - 2 th) M_xi2 + th/4 M_xi2^2
//                  + M_xi2x/2 - 2 M_x + M_xi2x^2/4 - 3/2 M_x^2.
// The moments are a constant linear map of the 37 inputs (15 accumulators),
// which keeps the register footprint small.  In the all-float mode (float
// adjoint buffers and float stored moments) the 15 sums and the outputs G
// are formed in float: about 40 % fewer operations than in double, and the
// inputs already carry float rounding.
struct EqVjp {
    double sp, sxx, sxz, su2, sth;
};

// The +-e pairs (l, l + 1) share their weight and have opposite velocities,
// so a monomial of even degree sees lam_l + lam_{l+1} and one of odd degree
// lam_l - lam_{l+1}: 18 pairs instead of 37 terms per sum.
__host__ __device__ constexpr bool pairs_share_weight() {
    for (int l = 1; l < Q; l += 2)
        if (W[l] != W[l + 1] || EX[l + 1] != -EX[l] || EZ[l + 1] != -EZ[l]) return false;
    return true;
}
static_assert(pairs_share_weight(), "population l + 1 must be -e_l with the weight of l, l odd");

// A: accumulator type of the 15 sums (double; float in the all-float mode)
template <typename A, typename LT>
__device__ __forceinline__ EqVjp eq_vjp_sums(const LT lam[Q], double vx, double vz, double th) {
    // q[p][q]: p powers of xi_x, q of xi_z
    A q00 = (A)lam[0] * (A)W[0], q10 = 0, q01 = 0, q20 = 0, q11 = 0, q02 = 0, q30 = 0, q21 = 0, q12 = 0,
      q03 = 0, q40 = 0, q31 = 0, q22 = 0, q13 = 0, q04 = 0;
#pragma unroll
    for (int l = 1; l < Q; l += 2) {
        const A s = ((A)lam[l] + (A)lam[l + 1]) * (A)W[l];   // even degrees
        const A d = ((A)lam[l] - (A)lam[l + 1]) * (A)W[l];   // odd degrees
        const double a = R * EX[l], b = R * EZ[l];
        q00 += s;
        if (EX[l] != 0) {
            q10 += d * (A)a;
            q20 += s * (A)(a * a);
            q30 += d * (A)(a * a * a);
            q40 += s * (A)(a * a * a * a);
        }
        if (EZ[l] != 0) {
            q01 += d * (A)b;
            q02 += s * (A)(b * b);
            q03 += d * (A)(b * b * b);
            q04 += s * (A)(b * b * b * b);
        }
        if (EX[l] != 0 && EZ[l] != 0) {
            q11 += s * (A)(a * b);
            q21 += d * (A)(a * a * b);
            q12 += d * (A)(a * b * b);
            q31 += s * (A)(a * a * a * b);
            q22 += s * (A)(a * a * b * b);
            q13 += s * (A)(a * b * b * b);
        }
    }
    const double m00 = q00, m10 = q10, m01 = q01, m20 = q20, m11 = q11, m02 = q02, m30 = q30, m21 = q21,
                 m12 = q12, m03 = q03, m40 = q40, m31 = q31, m22 = q22, m13 = q13, m04 = q04;
    const double u2 = vx * vx + vz * vz;
    const double vxx = vx * vx, vxz = vx * vz, vzz = vz * vz;
    // contracted moments
    const double Ms = m20 + m02, Mss = m40 + 2.0 * m22 + m04;
    const double Mx = vx * m10 + vz * m01;
    const double Msx = vx * (m30 + m12) + vz * (m21 + m03);
    const double Mxx = vxx * m20 + 2.0 * vxz * m11 + vzz * m02;
    const double Msxx = vxx * (m40 + m22) + 2.0 * vxz * (m31 + m13) + vzz * (m22 + m04);
    const double Mx3 = vx * vxx * m30 + 3.0 * vxx * vz * m21 + 3.0 * vx * vzz * m12 + vz * vzz * m03;
    const double Mx4 = vxx * vxx * m40 + 4.0 * vxx * vxz * m31 + 6.0 * vxx * vzz * m22 +
                       4.0 * vxz * vzz * m13 + vzz * vzz * m04;
    const double a0 = 1.0 - 0.5 * u2 - th + 0.125 * u2 * u2 + th * u2 + th * th;
    const double a1 = 0.5 * th - 0.25 * th * u2 - th * th, a2 = 0.125 * th * th;
    const double b0 = 1.0 - 0.5 * u2 - 2.0 * th, b1 = 0.5 * th;
    const double c0 = 0.5 - 0.25 * u2 - 1.5 * th, c1 = 0.25 * th;
    EqVjp r;
    r.sp = a0 * m00 + a1 * Ms + a2 * Mss + b0 * Mx + b1 * Msx + c0 * Mxx + c1 * Msxx + Mx3 * (1.0 / 6.0) +
           Mx4 * (1.0 / 24.0);
    // x-component: M_i = m10, M_xi2 i = m30 + m12, M_x i = vx m20 + vz m11, ...
    r.sxx = b0 * m10 + b1 * (m30 + m12) + 2.0 * c0 * (vx * m20 + vz * m11) +
            2.0 * c1 * (vx * (m40 + m22) + vz * (m31 + m13)) +
            0.5 * (vxx * m30 + 2.0 * vxz * m21 + vzz * m12) +
            (vx * vxx * m40 + 3.0 * vxx * vz * m31 + 3.0 * vx * vzz * m22 + vz * vzz * m13) * (1.0 / 6.0);
    r.sxz = b0 * m01 + b1 * (m21 + m03) + 2.0 * c0 * (vx * m11 + vz * m02) +
            2.0 * c1 * (vx * (m31 + m13) + vz * (m22 + m04)) +
            0.5 * (vxx * m21 + 2.0 * vxz * m12 + vzz * m03) +
            (vx * vxx * m31 + 3.0 * vxx * vz * m22 + 3.0 * vx * vzz * m13 + vz * vzz * m04) * (1.0 / 6.0);
    r.su2 = (0.25 * u2 + th - 0.5) * m00 - 0.25 * th * Ms - 0.5 * Mx - 0.25 * Mxx;
    r.sth = (u2 + 2.0 * th - 1.0) * m00 + (0.5 - 0.25 * u2 - 2.0 * th) * Ms + 0.25 * th * Mss + 0.5 * Msx -
            2.0 * Mx + 0.25 * Msxx - 1.5 * Mxx;
    return r;
}

// ---------------------------------------------------------------------------
// adjoint step
// ---------------------------------------------------------------------------
// Accumulator type: float in the all-float mode (float buffers and float
// moments: the 15 sums and the outputs G, whose inputs already carry float
// rounding); double otherwise.  The moments' algebra and (alpha, beta,
// gamma) are double in every mode.
template <typename L, typename MT>
using AdjAcc = typename std::conditional<std::is_same<L, float>::value && std::is_same<MT, float>::value, float,
                                         double>::type;

// Collision adjoint of one site: G_l = keep lam_l + alpha + beta . xi_l +
// gamma |xi_l|^2 from the site's 37 lam values and pre-collision moments
// (NO_COLLIDE: G = lam).
template <typename A>
struct AdjSite {
    A gk, ga, gbx, gbz, gg;
};

// The stored pre-collision moments of site (x, z) (none with F_NO_COLLIDE,
// where a.mom may be null).
struct SiteMoments {
    double rho, ux, uz, T;
};
template <typename MT>
__device__ __forceinline__ SiteMoments load_moments(const AdjointArgs &a, int x, int z) {
    SiteMoments m{1.0, 0.0, 0.0, 1.0};
    if (!(a.flags & F_NO_COLLIDE)) {
        // moments [4][Lx][Lz]: uniform column base + 32-bit per-lane byte offset
        const size_t N = (size_t)a.lx * (size_t)a.lz;
        const MT *mcol = static_cast<const MT *>(a.mom) + (size_t)x * (size_t)a.lz;
        const uint32_t moff = (uint32_t)z * (uint32_t)sizeof(MT);
        m.rho = ldg_off(mcol, moff);
        m.ux = ldg_off(mcol + N, moff);
        m.uz = ldg_off(mcol + 2 * N, moff);
        m.T = ldg_off(mcol + 3 * N, moff);
    }
    return m;
}

template <typename A, typename L>
__device__ __forceinline__ AdjSite<A> adj_site(const AdjointArgs &a, const L lam[Q], const SiteMoments &m) {
    double keep = 1.0, alpha = 0.0, bx = 0.0, bz = 0.0, gamma = 0.0;
    if (!(a.flags & F_NO_COLLIDE)) {
        const double rho = m.rho, ux = m.ux, uz = m.uz, T = m.T;
        const double vx = ux, vz = uz - a.tau * a.g;
        const double th = T + a.tau * (1.0 - a.tau) * a.g * a.g / D - 1.0;
        const EqVjp s = eq_vjp_sums<A>(lam, vx, vz, th);
        const double om = a.omega;
        const double mu_rho = om * s.sp;
        const double mux = om * rho * (s.sxx + 2.0 * vx * s.su2);
        const double muz = om * rho * (s.sxz + 2.0 * vz * s.su2);
        const double mu_t = om * rho * s.sth;
        const double inv = 1.0 / rho, idr = 1.0 / (D * rho);
        alpha = mu_rho - (mux * ux + muz * uz) * inv + mu_t * (ux * ux + uz * uz - D * T) * idr;
        bx = R * (mux * inv - 2.0 * mu_t * ux * idr);
        bz = R * (muz * inv - 2.0 * mu_t * uz * idr);
        gamma = mu_t * idr;
        keep = 1.0 - om;
    }
    return AdjSite<A>{(A)keep, (A)alpha, (A)bx, (A)bz, (A)gamma};
}

// G_l of a site; G_l and G_{l+1} (= -e_l) share alpha + gamma |xi|^2 and +-beta . xi_l
template <typename A, typename L>
__device__ __forceinline__ A adj_g(const AdjSite<A> &c, const L lam[Q], int l) {
    if (l == 0) return c.gk * (A)lam[0] + c.ga;
    const int p = (l & 1) ? l : l - 1;
    const A cc = c.ga + c.gg * (A)XI2_SHELL[SHELL[p]];
    A bxi;
    if (EX[p] != 0 && EZ[p] != 0)
        bxi = (A)EX[p] * c.gbx + (A)EZ[p] * c.gbz;
    else if (EX[p] != 0)
        bxi = (A)EX[p] * c.gbx;
    else
        bxi = (A)EZ[p] * c.gbz;
    const A k = c.gk * (A)lam[l] + cc;
    return (l & 1) ? k + bxi : k - bxi;
}

template <bool EDGE, typename L, typename MT>
__device__ __forceinline__ void adjoint_tile(const AdjointArgs &a, int x, int z0) {
    using A = AdjAcc<L, MT>;
    const L *__restrict__ lam_in = static_cast<const L *>(a.lam_in);
    L *__restrict__ lam_out = static_cast<L *>(a.lam_out);
    const int z = z0 + (int)threadIdx.x;
    if (EDGE && z >= a.lz) return;
    // lam buffers are tiled (common.h); the block's rows lie in one tile zt
    const int zt = z0 / TILE, zl = z % TILE;
    const long long tstep = (long long)a.lx * (Q * TILE) - TILE;
    const size_t own = ((size_t)zt * (size_t)a.lx + (size_t)x) * (Q * TILE) + (size_t)zl;   // (0, x, z)
    L lam[Q];   // held in the buffer's type (float buffers: half the registers)
#pragma unroll
    for (int l = 0; l < Q; ++l) lam[l] = lam_in[own + (size_t)l * TILE];
    const AdjSite<A> c = adj_site<A, L>(a, lam, load_moments<MT>(a, x, z));
    auto gval = [&](int l) -> A { return adj_g<A, L>(c, lam, l); };
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const L G = (L)gval(l);
        const int xd = EX[l] == 0 ? x : wrap(x - EX[l], a.lx);
        const int zd = z - EZ[l];
        if (!EDGE) {
            // row z - e_lz of column x - e_lx: this tile or the one below / above
            L *tb = lam_out + ((size_t)zt * (size_t)a.lx + (size_t)xd) * (Q * TILE);
            tb[tile_off(l, zl - EZ[l], tstep)] = G;
        } else if (a.flags & F_PERIODIC_Z) {
            lam_out[pidx(l, xd, wrap(zd, a.lz), a.lx)] = G;
        } else {
            if (zd >= 0 && zd < a.lz) lam_out[pidx(l, xd, zd, a.lx)] = G;
            // lam_out_l(z) = G_l(z + e_lz) has no writer when row z + e_lz lies
            // beyond a wall: zero for the Dirichlet wall (that pull read the
            // constant table); the diffuse wall parks G_{-l} of this site there
            const int zsrc = z + EZ[l];
            if (zsrc < 0 || zsrc >= a.lz) {
                L park = L(0);
                if (a.flags & F_WALL_DIFFUSE) {
                    const int o = l == 0 ? 0 : ((l & 1) ? l + 1 : l - 1);   // -e_l
                    park = (L)gval(o);
                }
                lam_out[own + (size_t)l * TILE] = park;
            }
        }
    }
}

#ifndef LBM_ADJ_BS
#define LBM_ADJ_BS 256
#endif
#ifndef LBM_ADJ_ZT
#define LBM_ADJ_ZT 1
#endif
constexpr int ADJ_BS = LBM_ADJ_BS, ADJ_ZT = LBM_ADJ_ZT;
static_assert(TILE % ADJ_BS == 0, "an adjoint block's rows must lie in one tile of the lam buffers");

// L: element type of the adjoint buffers; MT: of the stored moments
// Occupancy target: 3 wavefronts per SIMD with float buffers and float
// moments (140 VGPRs, no spills), 2 otherwise (165-209 VGPRs);
// measured fastest on MI355X for the 2048 x 6144 float rollout and the
// 512 x 1536 double rollout respectively.
template <typename L, typename MT>
struct AdjWaves {
    static constexpr int value = (sizeof(L) == 4 && sizeof(MT) == 4) ? 3 : 2;
};

template <typename L, typename MT>
__global__ __launch_bounds__(ADJ_BS) __attribute__((amdgpu_waves_per_eu(AdjWaves<L, MT>::value)))
void adjoint_step_kernel(AdjointArgs a, int nzb) {
    const int x = (int)(blockIdx.x / (uint32_t)nzb);
    if (ADJ_ZT == 1) {
        const int z0 = (int)(blockIdx.x % (uint32_t)nzb) * ADJ_BS;
        if ((z0 < 3) || (z0 + ADJ_BS + 3 > a.lz))
            adjoint_tile<true, L, MT>(a, x, z0);
        else
            adjoint_tile<false, L, MT>(a, x, z0);
        return;
    }
    const int zt = (int)(blockIdx.x % (uint32_t)nzb) * ADJ_ZT;
    for (int k = 0; k < ADJ_ZT; ++k) {
        const int z0 = (zt + k) * ADJ_BS;
        if (z0 >= a.lz) break;
        if ((z0 < 3) || (z0 + ADJ_BS + 3 > a.lz))
            adjoint_tile<true, L, MT>(a, x, z0);
        else
            adjoint_tile<false, L, MT>(a, x, z0);
    }
}

// Diffuse wall, second pass: one thread per ghost site (x_g, row k), reading
// the parked G values of the sites it emits to and writing A into the slots
// of the populations that stream into it (the same slots).
template <typename L, typename GT>
__global__ __launch_bounds__(BLOCK) void adjoint_wall_kernel(AdjointArgs a) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= 6 * a.lx) return;
    L *__restrict__ lam = static_cast<L *>(a.lam_out);
    const int xg = t % a.lx, row = t / a.lx;      // row = side * 3 + i
    const int k = row < 3 ? -1 - row : a.lz + (row - 3);
    const GT *gh = static_cast<const GT *>(a.ghost) + (size_t)row * Q;
    constexpr bool dev = std::is_same<GT, float>::value;   // FP32 table stores f - w
    double S = 0.0, A = 0.0;
#pragma unroll
    for (int m = 1; m < Q; ++m) {
        // the ghost site emits population m to (xg + e_mx, zd); loads from a
        // clamped row, masked, so that they are all in flight at once
        const int zd = k + EZ[m];
        const bool in = zd >= 0 && zd < a.lz;
        const double c = (double)gh[m] + (dev ? W[m] : 0.0);
        const int o = (m & 1) ? m + 1 : m - 1;
        const int xd = EX[m] == 0 ? xg : wrap(xg + EX[m], a.lx);
        const double v = (double)lam[pidx(o, xd, zd < 0 ? 0 : (zd >= a.lz ? a.lz - 1 : zd), a.lx)];
        S += in ? c : 0.0;
        A += in ? c * v : 0.0;
    }
    const L out = (L)(A / S);
#pragma unroll
    for (int m = 1; m < Q; ++m) {
        const int zs = k - EZ[m];   // population m streams into the ghost site from (xg - e_mx, zs)
        if (zs < 0 || zs >= a.lz) continue;
        const int xs = EX[m] == 0 ? xg : wrap(xg - EX[m], a.lx);
        lam[pidx(m, xs, zs, a.lx)] = out;
    }
}

hipError_t launch_adjoint_step(const AdjointArgs &a, hipStream_t s) {
    const int nzb = (a.lz + ADJ_BS * ADJ_ZT - 1) / (ADJ_BS * ADJ_ZT);
    const dim3 grid((uint32_t)nzb * (uint32_t)a.lx);
    const bool f32 = (a.flags & F_ADJ_F32) != 0;
    const bool m32 = (a.flags & F_MOM_F32) != 0;
    if (f32 && m32)
        hipLaunchKernelGGL((adjoint_step_kernel<float, float>), grid, dim3(ADJ_BS), 0, s, a, nzb);
    else if (f32)
        hipLaunchKernelGGL((adjoint_step_kernel<float, double>), grid, dim3(ADJ_BS), 0, s, a, nzb);
    else if (m32)
        hipLaunchKernelGGL((adjoint_step_kernel<double, float>), grid, dim3(ADJ_BS), 0, s, a, nzb);
    else
        hipLaunchKernelGGL((adjoint_step_kernel<double, double>), grid, dim3(ADJ_BS), 0, s, a, nzb);
    if (a.flags & F_WALL_DIFFUSE) {
        const dim3 wgrid((uint32_t)((6 * a.lx + BLOCK - 1) / BLOCK));
        const bool gf = a.precision == P_F32_DEV;
        if (f32 && gf)
            hipLaunchKernelGGL((adjoint_wall_kernel<float, float>), wgrid, dim3(BLOCK), 0, s, a);
        else if (f32)
            hipLaunchKernelGGL((adjoint_wall_kernel<float, double>), wgrid, dim3(BLOCK), 0, s, a);
        else if (gf)
            hipLaunchKernelGGL((adjoint_wall_kernel<double, float>), wgrid, dim3(BLOCK), 0, s, a);
        else
            hipLaunchKernelGGL((adjoint_wall_kernel<double, double>), wgrid, dim3(BLOCK), 0, s, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjoint step, gather form
// ---------------------------------------------------------------------------
// The step is f_out = C(S f_in): S streams (pull, walls), C collides per
// site.  Its transpose S^T C^T is applied above in push form.  Regrouping a
// chain of steps, lam_0 = S^T C_1^T S^T C_2^T ... S^T C_N^T lam_N, around
// mu_t = C_t^T lam_t (the derivative with respect to the pre-collision
// populations of step t) gives mu_{t-1} = C_{t-1}^T S^T mu_t: the streaming
// transpose becomes a gather, (S^T mu)_l(y) = mu_l(y + e_l), and the
// collision adjoint then runs on the gathered values of one site, stored in
// place (aligned writes).  A backward sweep is C_N^T once (shift = false),
// then N - 1 gather steps, then S^T alone (F_NO_COLLIDE): every output
// element is written by its own site, and the shifted accesses are reads,
// which measured faster than shifted writes on this chip (the Sec. III.B
// pull/push comparison).
//
// Walls: where y + e_l lies beyond a wall, (S^T mu)_l(y) is 0 for the
// Dirichlet wall and, for the diffuse wall, the sum A(s) of the ghost site
// s = y + e_l, formed by the blocks at the walls themselves.
constexpr int GATHER_BS = 256;   // rows per gather block (launch shapes measured below)
static_assert(TILE % GATHER_BS == 0, "a gather block's rows must lie in one tile");

// Diffuse wall: the ghost site s = (xg, row k) emits c_m M(s) into
// population m, so (S^T mu) at every population that streamed into s is
// A(s) = sum_m c_m mu_m(s + e_m) / sum_m c_m over the m pointing back into
// the lattice (c_m = its table row; row = side * 3 + i).  Every load is
// issued from a clamped row and masked, so that they are in flight together.

template <typename L, typename GT>
__device__ __forceinline__ double ghost_site_sum(const AdjointArgs &a, const L *mu, int row, int xg) {
    const int k = row < 3 ? -1 - row : a.lz + (row - 3);
    const GT *gh = static_cast<const GT *>(a.ghost) + (size_t)row * Q;
    constexpr bool dev = std::is_same<GT, float>::value;   // FP32 table stores f - w
    double S = 0.0, A = 0.0;
#pragma unroll
    for (int m = 1; m < Q; ++m) {
        const int zd = k + EZ[m];   // s emits population m to (xg + e_mx, zd)
        const bool in = zd >= 0 && zd < a.lz;
        const double c = (double)gh[m] + (dev ? W[m] : 0.0);
        const int xd = EX[m] == 0 ? xg : wrap(xg + EX[m], a.lx);
        const double v = (double)mu[pidx(m, xd, zd < 0 ? 0 : (zd >= a.lz ? a.lz - 1 : zd), a.lx)];
        S += in ? c : 0.0;
        A += in ? c * v : 0.0;
    }
    return A / S;
}

// WALL (tiles at a wall or the lattice end only): 0 Dirichlet walls, 1
// diffuse walls with a double wall table, 3 with a float (deviation) table,
// 2 periodic in z, fixed at compile time so that the gather's loads sit in
// no branch.  With diffuse walls the block first forms the sums A(s) of the
// 2 x 3 x 7 ghost sites its column gathers from (ghost_site_sum), one lane
// each, into LDS.
template <bool EDGE, bool SHIFT, typename L, typename MT, int WALL = 0>
__device__ __forceinline__ void adjoint_gather_tile(const AdjointArgs &a, int x, int z0) {
    using A = AdjAcc<L, MT>;
    const L *__restrict__ in = static_cast<const L *>(a.lam_in);
    L *__restrict__ out = static_cast<L *>(a.lam_out);
    const int z = z0 + (int)threadIdx.x;
    constexpr bool diffuse = WALL == 1 || WALL == 3;
    __shared__ double gsum[6][7];   // [side * 3 + i][dx + 3]: A of ghost site (x + dx, row i of side)
    if (diffuse) {
        const int t = (int)threadIdx.x, row = t / 7;
        if (t < 42 && (row < 3 ? z0 < 3 : z0 + GATHER_BS + 3 > a.lz)) {   // the walls this block reaches
            const int xg = wrap(x + t % 7 - 3, a.lx);
            gsum[row][t % 7] = WALL == 3 ? ghost_site_sum<L, float>(a, in, row, xg)
                                         : ghost_site_sum<L, double>(a, in, row, xg);
        }
        __syncthreads();   // every lane of the block reaches this (the return below comes after)
    }
    if (EDGE && z >= a.lz) return;
    const int zt = z0 / TILE, zl = z % TILE;
    const long long tstep = (long long)a.lx * (Q * TILE) - TILE;
    const size_t own = ((size_t)zt * (size_t)a.lx + (size_t)x) * (Q * TILE) + (size_t)zl;   // (0, x, z)
    // the moments first: their loads overlap the 37 gathers (measured 2 %
    // faster than after them, with 4 wavefronts per SIMD)
    const SiteMoments m = load_moments<MT>(a, x, z);
    L lam[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        if (!SHIFT) {
            lam[l] = in[own + (size_t)l * TILE];
            continue;
        }
        const int xs = EX[l] == 0 ? x : wrap(x + EX[l], a.lx);
        if (!EDGE) {
            // row z + e_lz of column x + e_lx: this tile or the one below / above
            const L *tb = in + ((size_t)zt * (size_t)a.lx + (size_t)xs) * (Q * TILE);
            lam[l] = tb[tile_off(l, zl + EZ[l], tstep)];
            continue;
        }
        const int zs = z + EZ[l];
        if (WALL == 2) {
            lam[l] = in[pidx(l, xs, wrap(zs, a.lz), a.lx)];
            continue;
        }
        // Loads without per-lane branches (loads under such branches are
        // issued one at a time): the in-range candidate from a clamped row
        // (within 3 rows of z, so tile_off still applies), the diffuse ghost
        // site's sum for a clamped ghost row, then a select.
        const int zc = zs < 0 ? 0 : (zs >= a.lz ? a.lz - 1 : zs);
        const L *tb = in + ((size_t)zt * (size_t)a.lx + (size_t)xs) * (Q * TILE);
        const L inval = tb[tile_off(l, zl + (zc - z), tstep)];
        L ghostval = L(0);
        if (diffuse) {   // ghost site (x + e_lx, zs)
            const int row = zs < 0 ? -zs - 1 : (zs >= a.lz ? 3 + zs - a.lz : 0);
            ghostval = (L)gsum[row][EX[l] + 3];
        }
        lam[l] = (zs >= 0 && zs < a.lz) ? inval : ghostval;
    }
    const AdjSite<A> c = adj_site<A, L>(a, lam, m);
#pragma unroll
    for (int l = 0; l < Q; ++l) __builtin_nontemporal_store((L)adj_g<A, L>(c, lam, l), &out[own + (size_t)l * TILE]);
}

// Launch shape of the gather form: 256 rows per block (a tile holds two
// such blocks); 4 wavefronts per SIMD with float buffers and float moments
// (128 VGPRs, no spills in the interior tiles), 2 otherwise.  Measured on
// MI355X, 2048 x 6144
// all-float: 0.704 ms, against 0.718 with 512-row blocks at 3 wavefronts
// per SIMD, 0.726 with 256 rows and the moments loaded after the gathers,
// 0.737 with non-temporal gathers and 0.724 with XCD-contiguous tile order;
// 512 x 1536 double: 0.110 ms with 256 rows vs 0.145 with 512.  With the
// wall tiles' loads free of per-lane branches (above): 0.693 ms and
// 0.082 ms.
template <typename L, typename MT>
struct GatherWaves {
    static constexpr int value = (sizeof(L) == 4 && sizeof(MT) == 4) ? 4 : 2;
};
template <typename L, typename MT, bool SHIFT>
__global__ __launch_bounds__(GATHER_BS) __attribute__((amdgpu_waves_per_eu(GatherWaves<L, MT>::value)))
void adjoint_gather_kernel(AdjointArgs a, int nzb) {
    constexpr int BS = GATHER_BS;
    const int x = (int)(blockIdx.x / (uint32_t)nzb);
    const int z0 = (int)(blockIdx.x % (uint32_t)nzb) * BS;
    const bool edge = SHIFT ? (z0 < 3) || (z0 + BS + 3 > a.lz) : (z0 + BS > a.lz);
    // the interior tiles are the hot path: marked as such, register allocation
    // places the spills that 128 VGPRs force (all-float) in the wall tiles
    if (__builtin_expect(!edge, 1))
        adjoint_gather_tile<false, SHIFT, L, MT>(a, x, z0);
    else if (!SHIFT)
        adjoint_gather_tile<true, false, L, MT>(a, x, z0);
    else if (a.flags & F_PERIODIC_Z)
        adjoint_gather_tile<true, true, L, MT, 2>(a, x, z0);
    else if ((a.flags & F_WALL_DIFFUSE) && a.precision == P_F32_DEV)
        adjoint_gather_tile<true, true, L, MT, 3>(a, x, z0);
    else if (a.flags & F_WALL_DIFFUSE)
        adjoint_gather_tile<true, true, L, MT, 1>(a, x, z0);
    else
        adjoint_gather_tile<true, true, L, MT, 0>(a, x, z0);
}

template <typename L, typename MT>
static void launch_gather_t(const AdjointArgs &a, bool shift, hipStream_t s) {
    constexpr int BS = GATHER_BS;
    const int nzb = (a.lz + BS - 1) / BS;
    const dim3 grid((uint32_t)nzb * (uint32_t)a.lx);
    if (shift)
        hipLaunchKernelGGL((adjoint_gather_kernel<L, MT, true>), grid, dim3(BS), 0, s, a, nzb);
    else
        hipLaunchKernelGGL((adjoint_gather_kernel<L, MT, false>), grid, dim3(BS), 0, s, a, nzb);
}

hipError_t launch_adjoint_gather(const AdjointArgs &a, bool shift, hipStream_t s) {
    const bool f32 = (a.flags & F_ADJ_F32) != 0;
    const bool m32 = (a.flags & F_MOM_F32) != 0;
    if (f32 && m32)
        launch_gather_t<float, float>(a, shift, s);
    else if (f32)
        launch_gather_t<float, double>(a, shift, s);
    else if (m32)
        launch_gather_t<double, float>(a, shift, s);
    else
        launch_gather_t<double, double>(a, shift, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// objective J = wk KE + wl (L_u + L_d) and its seed dJ/df*
// ---------------------------------------------------------------------------
constexpr int OXC = 64;   // columns per strip

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

struct ObjLayout {
    int nxc, nzb, nb;
    size_t tpart, kpart, dtbar, misc, total;   // byte offsets
};

static ObjLayout obj_layout(int lx, int lz) {
    ObjLayout L;
    L.nxc = (lx + OXC - 1) / OXC;
    L.nzb = (lz + BLOCK - 1) / BLOCK;
    L.nb = L.nxc * L.nzb;
    L.tpart = 0;
    L.kpart = al256((size_t)L.nxc * lz * sizeof(double));
    L.dtbar = L.kpart + al256((size_t)L.nb * sizeof(double));
    L.misc = L.dtbar + al256((size_t)lz * sizeof(double));
    L.total = L.misc + 256;
    return L;
}

size_t objective_scratch_bytes(int lx, int lz) { return obj_layout(lx, lz).total; }

template <int PREC>
__device__ __forceinline__ void site_moments(const void *fp, int lx, int x, int z, double &rho, double &ux,
                                             double &uz, double &T) {
    using E = typename std::conditional<PREC == P_F64, double, float>::type;
    const E *f = static_cast<const E *>(fp) + pidx(0, x, z, lx);
    double s0 = 0.0, sx = 0.0, sz = 0.0, s2 = 0.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const double v = (double)f[(size_t)l * TILE];
        s0 += v;
        if (EX[l] != 0) sx += EX[l] * v;
        if (EZ[l] != 0) sz += EZ[l] * v;
        if (SHELL[l] != 0) s2 += (EX[l] * EX[l] + EZ[l] * EZ[l]) * v;
    }
    rho = (PREC == P_F64) ? s0 : 1.0 + s0;
    const double e2 = (PREC == P_F64) ? R2 * s2 : D + R2 * s2;
    const double inv = 1.0 / rho;
    ux = R * sx * inv;
    uz = R * sz * inv;
    T = (e2 * inv - ux * ux - uz * uz) / D;
}

template <int PREC>
__global__ __launch_bounds__(BLOCK) void objective_pass1(ObjectiveArgs a, ObjLayout L) {
    __shared__ double red[BLOCK];
    char *sc = static_cast<char *>(a.scratch);
    double *tpart = reinterpret_cast<double *>(sc + L.tpart);
    double *kpart = reinterpret_cast<double *>(sc + L.kpart);
    const int zb = blockIdx.x % L.nzb, xc = blockIdx.x / L.nzb;
    const int tid = threadIdx.x, z = zb * BLOCK + tid;
    double tacc = 0.0, ke = 0.0;
    if (z < a.lz) {
        const int x1 = min(xc * OXC + OXC, a.lx);
        for (int x = xc * OXC; x < x1; ++x) {
            double rho, ux, uz, T;
            site_moments<PREC>(a.f, a.lx, x, z, rho, ux, uz, T);
            const double uhz = uz + 0.5 * a.g;                 // u^H = u* - g_vec/2
            tacc += T + a.g * a.g / (4.0 * D);                  // T^H
            ke += 0.5 * rho * (ux * ux + uhz * uhz);
        }
        tpart[(size_t)xc * a.lz + z] = tacc;
    }
    red[tid] = ke;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) kpart[blockIdx.x] = red[0];
}

__device__ __forceinline__ double tent(double b) {
    return (b > 0.0 && b < 0.5) ? 2.0 * b : ((b >= 0.5 && b < 1.0) ? 2.0 * (1.0 - b) : 0.0);
}
__device__ __forceinline__ double tent_slope(double b) {
    return (b > 0.0 && b < 0.5) ? 2.0 : ((b >= 0.5 && b < 1.0) ? -2.0 : 0.0);
}

// One block: T(z), the tent sums, dJ/dT(z) and J.
__global__ __launch_bounds__(BLOCK) void objective_pass2(ObjectiveArgs a, ObjLayout L) {
    __shared__ double red[3][BLOCK];
    char *sc = static_cast<char *>(a.scratch);
    const double *tpart = reinterpret_cast<const double *>(sc + L.tpart);
    const double *kpart = reinterpret_cast<const double *>(sc + L.kpart);
    double *dtbar = reinterpret_cast<double *>(sc + L.dtbar);
    const int tid = threadIdx.x;
    double lu = 0.0, ld = 0.0, ke = 0.0;
    for (int z = tid; z < a.lz; z += BLOCK) {
        double s = 0.0;
        for (int c = 0; c < L.nxc; ++c) s += tpart[(size_t)c * a.lz + z];
        const double tb = s / (double)a.lx;
        const double bu = (tb - a.t_u) / (a.t_m - a.t_u), bd = (tb - a.t_m) / (a.t_d - a.t_m);
        lu += tent(bu);
        ld += tent(bd);
        dtbar[z] = a.wl * (tent_slope(bu) / (a.t_m - a.t_u) + tent_slope(bd) / (a.t_d - a.t_m));
    }
    for (int b = tid; b < L.nb; b += BLOCK) ke += kpart[b];
    red[0][tid] = lu;
    red[1][tid] = ld;
    red[2][tid] = ke;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < 3; ++k) red[k][tid] += red[k][tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        const double L_ = red[0][0] + red[1][0];
        a.j_out[0] = a.wk * red[2][0] + a.wl * L_;
        a.j_out[1] = red[2][0];
        a.j_out[2] = L_;
        a.j_out[3] = red[0][0];
        a.j_out[4] = red[1][0];
    }
}

// Seed lam_N = dJ/df*: dJ/drho = wk |u^H|^2/2, dJ/du* = wk rho u^H,
// dJ/dT* = dJ/dT(z) / Lx, chained through the moment Jacobian.
template <int PREC, typename LT>
__global__ __launch_bounds__(BLOCK) void objective_seed(ObjectiveArgs a, ObjLayout L) {
    LT *lam_seed = static_cast<LT *>(a.lam_seed);
    const double *dtbar = reinterpret_cast<const double *>(static_cast<char *>(a.scratch) + L.dtbar);
    const int x = blockIdx.x / L.nzb, z = (blockIdx.x % L.nzb) * BLOCK + threadIdx.x;
    if (z >= a.lz) return;
    const size_t base = pidx(0, x, z, a.lx);
    double rho, ux, uz, T;
    site_moments<PREC>(a.f, a.lx, x, z, rho, ux, uz, T);
    const double uhz = uz + 0.5 * a.g;
    const double g_rho = 0.5 * a.wk * (ux * ux + uhz * uhz);
    const double gux = a.wk * rho * ux, guz = a.wk * rho * uhz;
    const double g_t = dtbar[z] / (double)a.lx;
    const double inv = 1.0 / rho, idr = 1.0 / (D * rho);
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const double cx = R * EX[l] - ux, cz = R * EZ[l] - uz;
        lam_seed[base + (size_t)l * TILE] =
            (LT)(g_rho + (gux * cx + guz * cz) * inv + g_t * (cx * cx + cz * cz - D * T) * idr);
    }
}

hipError_t launch_objective(const ObjectiveArgs &a, int precision, hipStream_t s) {
    const ObjLayout L = obj_layout(a.lx, a.lz);
    if (precision == P_F64)
        hipLaunchKernelGGL(objective_pass1<P_F64>, dim3(L.nb), dim3(BLOCK), 0, s, a, L);
    else
        hipLaunchKernelGGL(objective_pass1<P_F32_DEV>, dim3(L.nb), dim3(BLOCK), 0, s, a, L);
    hipLaunchKernelGGL(objective_pass2, dim3(1), dim3(BLOCK), 0, s, a, L);
    if (a.lam_seed) {
        const dim3 g((uint32_t)L.nzb * (uint32_t)a.lx);
        if (precision == P_F64 && !a.lam_f32)
            hipLaunchKernelGGL((objective_seed<P_F64, double>), g, dim3(BLOCK), 0, s, a, L);
        else if (precision == P_F64)
            hipLaunchKernelGGL((objective_seed<P_F64, float>), g, dim3(BLOCK), 0, s, a, L);
        else if (!a.lam_f32)
            hipLaunchKernelGGL((objective_seed<P_F32_DEV, double>), g, dim3(BLOCK), 0, s, a, L);
        else
            hipLaunchKernelGGL((objective_seed<P_F32_DEV, float>), g, dim3(BLOCK), 0, s, a, L);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initial-state VJP: dJ/d amp from lam_0 = dJ/df*_0
// ---------------------------------------------------------------------------
// Per column (one block), rows i = 0 .. Lz+2 stand for rows k = i - 3.
// Forward: T_i (tanh profile of the heights), dlp_i = -g r (1/T_{i-1} + 1/T_i)/2,
// lp_i = sum_{m<=i} dlp_m, rho_i = C exp(lp_i)/T_i, f*_0 = f^eq(rho, g_vec/2, T - g^2/8).
// Reverse: g_lp_i = g_rho_i rho_i; rc_i = sum_{m>=i} g_lp_m = total - prefix_{i-1};
// g_T_i = g_Teq_i - g_rho_i rho_i / T_i + dfac_i (rc_i [i>=1] + rc_{i+1} [i<=n-2]),
// dfac_i = g r / (2 T_i^2);  dJ/dh_f = sum_i g_T_i dT_i/dh_f.
__device__ __forceinline__ double vjp_layer_t(const InitVjpArgs &a, double zc, double h0, double h1) {
    const double s0 = 0.5 * (1.0 + tanh((zc - h0) / a.width));
    const double s1 = 0.5 * (1.0 + tanh((zc - h1) / a.width));
    return a.t_d + (a.t_m - a.t_d) * s0 + (a.t_u - a.t_m) * s1;
}

__device__ __forceinline__ double block_scan_incl(double v, double *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int off = 1; off < BLOCK; off <<= 1) {
        const double add = tid >= off ? red[tid - off] : 0.0;
        __syncthreads();
        red[tid] += add;
        __syncthreads();
    }
    const double out = red[tid];
    __syncthreads();
    return out;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    const double out = red[0];
    __syncthreads();
    return out;
}

template <typename LT>
__global__ __launch_bounds__(BLOCK) void init_vjp_columns(InitVjpArgs a) {
    const LT *lam0 = static_cast<const LT *>(a.lam0);
    __shared__ double red[BLOCK];
    __shared__ double heights[2];
    const int x = blockIdx.x, tid = threadIdx.x;
    if (tid < 2) {
        double h = tid == 0 ? a.z_lo : a.z_hi;
        for (int j = 0; j < a.nmodes; ++j)
            h += a.amp[tid * a.nmodes + j] *
                 cos(2.0 * M_PI * (double)a.k[tid][j] * ((double)x + 0.5) / (double)a.lx + a.phase[tid][j]);
        heights[tid] = h;
    }
    __syncthreads();
    const double h0 = heights[0], h1 = heights[1];
    const int n = a.lz + 3;

    double total_glp = 0.0;
    for (int sweep = 0; sweep < 2; ++sweep) {
        double carry_lp = 0.0, carry_glp = 0.0, gh0 = 0.0, gh1 = 0.0;
        for (int c0 = 0; c0 < n; c0 += BLOCK) {
            const int i = c0 + tid;
            const bool in = i < n;
            const double zc = (double)(i - 3) + 0.5;
            double T = 1.0, d = 0.0;
            if (in) {
                T = vjp_layer_t(a, zc, h0, h1);
                if (i > 0) d = -a.g * R * 0.5 * (1.0 / vjp_layer_t(a, zc - 1.0, h0, h1) + 1.0 / T);
            }
            const double lp = carry_lp + block_scan_incl(d, red);
            // the chunk's last prefix carries into the next chunk
            if (tid == BLOCK - 1) red[0] = lp;
            __syncthreads();
            carry_lp = red[0];
            __syncthreads();

            double g_lp = 0.0, g_tdir = 0.0;
            if (in && i >= 3) {
                const size_t base = pidx(0, x, i - 3, a.lx);
                const double rho = a.norm * exp(lp) / T;
                double lam[Q];
#pragma unroll
                for (int l = 0; l < Q; ++l) lam[l] = (double)lam0[base + (size_t)l * TILE];
                const double th = T - a.g * a.g / (4.0 * D) - 1.0;
                const EqVjp s = eq_vjp_sums<double>(lam, 0.0, -0.5 * a.g, th);
                const double g_rho = s.sp, g_teq = rho * s.sth;
                g_lp = g_rho * rho;
                g_tdir = g_teq - g_rho * rho / T;
            }
            if (sweep == 0) {
                total_glp += block_sum(g_lp, red);
                continue;
            }
            // suffix sums rc_i = total - (prefix through i-1)
            const double pre_incl = carry_glp + block_scan_incl(g_lp, red);
            const double rc_i = total_glp - (pre_incl - g_lp);
            const double rc_next = total_glp - pre_incl;
            if (tid == BLOCK - 1) red[0] = pre_incl;
            __syncthreads();
            carry_glp = red[0];
            __syncthreads();
            double g_t = 0.0;
            if (in) {
                const double dfac = 0.5 * a.g * R / (T * T);
                g_t = g_tdir + dfac * ((i >= 1 ? rc_i : 0.0) + (i <= n - 2 ? rc_next : 0.0));
            }
            const double y0 = (zc - h0) / a.width, y1 = (zc - h1) / a.width;
            const double ch0 = cosh(y0), ch1 = cosh(y1);
            const double dt_dh0 = -(a.t_m - a.t_d) * 0.5 / (ch0 * ch0) / a.width;
            const double dt_dh1 = -(a.t_u - a.t_m) * 0.5 / (ch1 * ch1) / a.width;
            gh0 += in ? g_t * dt_dh0 : 0.0;
            gh1 += in ? g_t * dt_dh1 : 0.0;
        }
        if (sweep == 1) {
            const double s0 = block_sum(gh0, red);
            const double s1 = block_sum(gh1, red);
            if (tid == 0) {
                a.dh[x] = s0;
                a.dh[a.lx + x] = s1;
            }
        }
    }
}

// d amp[f][j] = sum_x dh[f][x] cos(2 pi k (x + 1/2)/Lx + phase); one block per (f, j)
__global__ __launch_bounds__(BLOCK) void init_vjp_modes(InitVjpArgs a) {
    __shared__ double red[BLOCK];
    const int f = blockIdx.x / a.nmodes, j = blockIdx.x % a.nmodes;
    double s = 0.0;
    for (int x = threadIdx.x; x < a.lx; x += BLOCK)
        s += a.dh[(size_t)f * a.lx + x] *
             cos(2.0 * M_PI * (double)a.k[f][j] * ((double)x + 0.5) / (double)a.lx + a.phase[f][j]);
    s = block_sum(s, red);
    if (threadIdx.x == 0) a.d_amp[f * a.nmodes + j] = s;
}

hipError_t launch_init_vjp(const InitVjpArgs &a, hipStream_t s) {
    if (a.lam_f32)
        hipLaunchKernelGGL(init_vjp_columns<float>, dim3(a.lx), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(init_vjp_columns<double>, dim3(a.lx), dim3(BLOCK), 0, s, a);
    if (a.nmodes > 0) hipLaunchKernelGGL(init_vjp_modes, dim3(2 * a.nmodes), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace lbm
