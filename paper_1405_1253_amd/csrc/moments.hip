// Diagnostics of a stored state: renormalised fields, mean temperature
// profile and global conservation sums.
//
// Sec. III.A renormalisation (u^H = u + g/2, T^H = T + g^2/(4D)) and the
// profile T(z) = (1/Lx) sum_x T of Sec. IV.  Pass 1: a block owns 256 rows of
// a strip of XC columns; each thread walks its row across the strip in x
// order and keeps the partial row sum of T^H, and the block reduces its
// sites' mass, momentum and energy in a fixed tree.  Pass 2 adds the strip
// partials in strip order.  No atomics: results are bitwise reproducible.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace lbm {

constexpr int XC = 64;   // columns per strip

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t moments_scratch_bytes(int lx, int lz) {
    const size_t nxc = (size_t)(lx + XC - 1) / XC, nzb = (size_t)(lz + BLOCK - 1) / BLOCK;
    return align256(nxc * (size_t)lz * sizeof(double)) + align256(nxc * nzb * 4 * sizeof(double));
}

template <int PREC>
__global__ __launch_bounds__(BLOCK) void moments_pass1(MomentArgs a, int nzb, double *tpart,
                                                        double *spart) {
    using E = typename std::conditional<PREC == P_F64, double, float>::type;
    __shared__ double red[4][BLOCK];
    const int zb = blockIdx.x % nzb, xc = blockIdx.x / nzb;
    const int tid = threadIdx.x;
    const int z = zb * BLOCK + tid;
    const bool active = z < a.lz;
    const size_t N = (size_t)a.lx * (size_t)a.lz;
    const E *__restrict__ f = static_cast<const E *>(a.f);
    const int x0 = xc * XC, x1 = min(x0 + XC, a.lx);

    double tacc = 0.0, m0 = 0.0, mx = 0.0, mz = 0.0, me = 0.0;
    if (active) {
        for (int x = x0; x < x1; ++x) {
            const size_t site = (size_t)x * (size_t)a.lz + (size_t)z;   // fields: [4][Lx][Lz]
            const size_t base = pidx(0, x, z, a.lx);                     // state: tiled
            double s0 = 0.0, sx = 0.0, sz = 0.0, s2 = 0.0;
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                const double v = (double)f[base + (size_t)l * TILE];
                s0 += v;
                if (EX[l] != 0) sx += EX[l] * v;
                if (EZ[l] != 0) sz += EZ[l] * v;
                if (SHELL[l] != 0) s2 += (EX[l] * EX[l] + EZ[l] * EZ[l]) * v;
            }
            const double rho = (PREC == P_F64) ? s0 : 1.0 + s0;
            const double e2 = (PREC == P_F64) ? R2 * s2 : D + R2 * s2;
            const double inv = 1.0 / rho;
            const double ux = R * sx * inv, uz = R * sz * inv;
            const double T = (e2 * inv - ux * ux - uz * uz) / D;
            // stored state: u* = u + g_vec, so u^H = u* - g_vec/2 = u* + (0, g/2)
            const double uhz = uz + 0.5 * a.g;
            const double th = T + a.g * a.g / (4.0 * D);
            if (a.fields) {
                a.fields[site] = rho;
                a.fields[N + site] = ux;
                a.fields[2 * N + site] = uhz;
                a.fields[3 * N + site] = th;
            }
            tacc += th;
            m0 += rho;
            mx += R * sx;
            mz += R * sz;
            me += 0.5 * e2;
        }
    }
    if (tpart && active) tpart[(size_t)xc * (size_t)a.lz + (size_t)z] = tacc;
    if (!spart) return;
    red[0][tid] = m0;
    red[1][tid] = mx;
    red[2][tid] = mz;
    red[3][tid] = me;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + off];
        __syncthreads();
    }
    if (tid < 4) spart[(size_t)blockIdx.x * 4 + tid] = red[tid][0];
}

// Blocks 0..ntb-1: tbar rows; block ntb: global sums.
__global__ __launch_bounds__(BLOCK) void moments_pass2(MomentArgs a, int nxc, int nb, int ntb,
                                                       const double *tpart, const double *spart) {
    __shared__ double red[4][BLOCK];
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < ntb) {
        const int z = blockIdx.x * BLOCK + tid;
        if (z >= a.lz) return;
        double s = 0.0;
        for (int c = 0; c < nxc; ++c) s += tpart[(size_t)c * (size_t)a.lz + (size_t)z];
        a.tbar[z] = s / (double)a.lx;
        return;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = tid; b < nb; b += BLOCK)
        for (int k = 0; k < 4; ++k) acc[k] += spart[(size_t)b * 4 + k];
    for (int k = 0; k < 4; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + off];
        __syncthreads();
    }
    if (tid < 4) a.sums[tid] = red[tid][0];
}

hipError_t launch_moments(const MomentArgs &a, int precision, hipStream_t s) {
    const int nxc = (a.lx + XC - 1) / XC, nzb = (a.lz + BLOCK - 1) / BLOCK;
    const int nb = nxc * nzb;
    double *tpart = a.tbar ? static_cast<double *>(a.scratch) : nullptr;
    double *spart = a.sums ? reinterpret_cast<double *>(static_cast<char *>(a.scratch) +
                                                        align256((size_t)nxc * a.lz * sizeof(double)))
                           : nullptr;
    if (precision == P_F64)
        hipLaunchKernelGGL(moments_pass1<P_F64>, dim3(nb), dim3(BLOCK), 0, s, a, nzb, tpart, spart);
    else
        hipLaunchKernelGGL(moments_pass1<P_F32_DEV>, dim3(nb), dim3(BLOCK), 0, s, a, nzb, tpart, spart);
    if (a.tbar || a.sums) {
        const int ntb = a.tbar ? nzb : 0;
        const int grid = ntb + (a.sums ? 1 : 0);
        // block index ntb is the sums block; with no tbar it is block 0
        hipLaunchKernelGGL(moments_pass2, dim3(grid), dim3(BLOCK), 0, s, a, nxc, nb, ntb, tpart, spart);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// row profiles: mean and rms fluctuation of T^H and E_k = rho |u^H|^2 / 2
// ---------------------------------------------------------------------------
template <int PREC>
__device__ __forceinline__ void site_th_ek(const void *fp, int lx, int x, int z, double g, double &th,
                                           double &ek) {
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
    const double rho = (PREC == P_F64) ? s0 : 1.0 + s0;
    const double e2 = (PREC == P_F64) ? R2 * s2 : D + R2 * s2;
    const double inv = 1.0 / rho;
    const double ux = R * sx * inv, uz = R * sz * inv;
    th = (e2 * inv - ux * ux - uz * uz) / D + g * g / (4.0 * D);
    const double uhz = uz + 0.5 * g;
    ek = 0.5 * rho * (ux * ux + uhz * uhz);
}

size_t profiles_scratch_bytes(int lx, int lz) {
    const size_t nxc = (size_t)(lx + XC - 1) / XC;
    return align256(4 * nxc * (size_t)lz * sizeof(double));
}

// pass 1: strip partials of (T - T0), (T - T0)^2, (E - E0), (E - E0)^2 with
// T0, E0 the row's values at x = 0
template <int PREC>
__global__ __launch_bounds__(BLOCK) void profiles_pass1(ProfileArgs a, int nzb, int nxc) {
    const int zb = blockIdx.x % nzb, xc = blockIdx.x / nzb;
    const int z = zb * BLOCK + threadIdx.x;
    if (z >= a.lz) return;
    double t0, e0;
    site_th_ek<PREC>(a.f, a.lx, 0, z, a.g, t0, e0);
    double st = 0.0, stt = 0.0, se = 0.0, see = 0.0;
    const int x1 = min(xc * XC + XC, a.lx);
    for (int x = xc * XC; x < x1; ++x) {
        double th, ek;
        site_th_ek<PREC>(a.f, a.lx, x, z, a.g, th, ek);
        const double dt = th - t0, de = ek - e0;
        st += dt;
        stt += dt * dt;
        se += de;
        see += de * de;
    }
    double *part = static_cast<double *>(a.scratch);
    const size_t stride = (size_t)nxc * a.lz, o = (size_t)xc * a.lz + z;
    part[o] = st;
    part[stride + o] = stt;
    part[2 * stride + o] = se;
    part[3 * stride + o] = see;
}

template <int PREC>
__global__ __launch_bounds__(BLOCK) void profiles_pass2(ProfileArgs a, int nxc) {
    const int z = blockIdx.x * BLOCK + threadIdx.x;
    if (z >= a.lz) return;
    const double *part = static_cast<const double *>(a.scratch);
    const size_t stride = (size_t)nxc * a.lz;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < nxc; ++c)
        for (int k = 0; k < 4; ++k) m[k] += part[k * stride + (size_t)c * a.lz + z];
    double t0, e0;
    site_th_ek<PREC>(a.f, a.lx, 0, z, a.g, t0, e0);
    const double inv = 1.0 / (double)a.lx;
    const double mt = m[0] * inv, me = m[2] * inv;
    a.prof[z] = t0 + mt;
    a.prof[a.lz + z] = sqrt(fmax(m[1] * inv - mt * mt, 0.0));
    a.prof[2 * a.lz + z] = e0 + me;
    a.prof[3 * a.lz + z] = sqrt(fmax(m[3] * inv - me * me, 0.0));
}

hipError_t launch_profiles(const ProfileArgs &a, int precision, hipStream_t s) {
    const int nxc = (a.lx + XC - 1) / XC, nzb = (a.lz + BLOCK - 1) / BLOCK;
    if (precision == P_F64) {
        hipLaunchKernelGGL(profiles_pass1<P_F64>, dim3(nzb * nxc), dim3(BLOCK), 0, s, a, nzb, nxc);
        hipLaunchKernelGGL(profiles_pass2<P_F64>, dim3(nzb), dim3(BLOCK), 0, s, a, nxc);
    } else {
        hipLaunchKernelGGL(profiles_pass1<P_F32_DEV>, dim3(nzb * nxc), dim3(BLOCK), 0, s, a, nzb, nxc);
        hipLaunchKernelGGL(profiles_pass2<P_F32_DEV>, dim3(nzb), dim3(BLOCK), 0, s, a, nxc);
    }
    return hipGetLastError();
}

}  // namespace lbm
