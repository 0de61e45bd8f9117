// Three-layer hydrostatic initial state and the wall table.
//
// Sec. I, eq. seteq and the pressure-matching condition; tanh smoothing of
// the interfaces (Fig. 1 caption).  One block per column: each thread
// evaluates the temperature of one row, the block scans the trapezoid
// increments of d ln p / dz = -g / T up the column (fixed order, so the state
// is bitwise reproducible), and each thread writes the 37 equilibrium
// populations of its site.
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace lbm {

__device__ __forceinline__ double layer_t(const InitArgs &a, double zc, double h0, double h1) {
    const double s0 = 0.5 * (1.0 + tanh((zc - h0) / a.width));
    const double s1 = 0.5 * (1.0 + tanh((zc - h1) / a.width));
    return a.t_d + (a.t_m - a.t_d) * s0 + (a.t_u - a.t_m) * s1;
}

// The 37 populations of one site: element l at index base + l * stride
// (tiled state: stride TILE; wall table: stride 1).
template <int PREC>
__device__ __forceinline__ void store_state(void *f, size_t base, size_t stride, const double feq[Q]) {
    if (PREC == P_F64) {
        double *o = static_cast<double *>(f);
#pragma unroll
        for (int l = 0; l < Q; ++l) o[base + (size_t)l * stride] = feq[l];
    } else {
        float *o = static_cast<float *>(f);
#pragma unroll
        for (int l = 0; l < Q; ++l) o[base + (size_t)l * stride] = (float)(feq[l] - W[l]);
    }
}

template <int PREC>
__global__ __launch_bounds__(BLOCK) void init_columns(InitArgs a) {
    __shared__ double red[BLOCK];
    __shared__ double heights[2];
    const int x = blockIdx.x;
    const int tid = threadIdx.x;

    if (tid < 2) {
        double h = tid == 0 ? a.z_lo : a.z_hi;
        for (int j = 0; j < a.nmodes; ++j)
            h += a.amp[tid * a.nmodes + j] *
                 cos(2.0 * M_PI * (double)a.k[tid][j] * ((double)x + 0.5) / (double)a.lx +
                     a.phase[tid][j]);
        heights[tid] = h;
    }
    __syncthreads();
    const double h0 = heights[0], h1 = heights[1];

    // rows k = -3 .. Lz-1 are entries i = k + 3 of the column; ln p(-3) = 0
    const int nrows = a.lz + 3;
    double carry = 0.0;
    for (int c0 = 0; c0 < nrows; c0 += BLOCK) {
        const int i = c0 + tid;
        double T = 1.0, d = 0.0;
        if (i < nrows) {
            const double zc = (double)(i - 3) + 0.5;
            T = layer_t(a, zc, h0, h1);
            if (i > 0) d = -a.g * R * 0.5 * (1.0 / layer_t(a, zc - 1.0, h0, h1) + 1.0 / T);
        }
        // inclusive scan of d over the block (Hillis-Steele)
        red[tid] = d;
        __syncthreads();
        for (int off = 1; off < BLOCK; off <<= 1) {
            const double add = tid >= off ? red[tid - off] : 0.0;
            __syncthreads();
            red[tid] += add;
            __syncthreads();
        }
        const double lnp = carry + red[tid];
        carry += red[BLOCK - 1];
        __syncthreads();
        if (i >= 3 && i < nrows) {
            const double rho = a.norm * exp(lnp) / T;
            double feq[Q];
            equilibrium_f64(rho, 0.0, -0.5 * a.g, T - a.g * a.g / (4.0 * D), feq);
            store_state<PREC>(a.f_out, pidx(0, x, i - 3, a.lx), TILE, feq);
        }
    }
}

// Wall table: rows -1, -2, -3 below and Lz, Lz+1, Lz+2 above, from the
// unperturbed hydrostatic profile (density and temperature given by the host).
template <int PREC>
__global__ void init_ghost(InitArgs a) {
    const int i = threadIdx.x;
    if (i >= 6) return;
    double feq[Q];
    equilibrium_f64(a.ghost_rho[i], 0.0, -0.5 * a.g, a.ghost_t[i] - a.g * a.g / (4.0 * D), feq);
    store_state<PREC>(a.ghost_out, (size_t)i * Q, 1, feq);   // element (i, l) at i*37 + l
}

hipError_t launch_init(const InitArgs &a, int precision, hipStream_t s) {
    if (precision == P_F64) {
        hipLaunchKernelGGL(init_columns<P_F64>, dim3(a.lx), dim3(BLOCK), 0, s, a);
        hipLaunchKernelGGL(init_ghost<P_F64>, dim3(1), dim3(64), 0, s, a);
    } else {
        hipLaunchKernelGGL(init_columns<P_F32_DEV>, dim3(a.lx), dim3(BLOCK), 0, s, a);
        hipLaunchKernelGGL(init_ghost<P_F32_DEV>, dim3(1), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace lbm
