// Device-side building blocks shared by the D2Q37 kernels.
//
// Equilibrium (Sec. III.A): the 4th-order Hermite expansion of the Maxwellian
// about the unit-temperature Gaussian, f^eq_l = w_l rho P(x_l), with
// x_l = xi_l . v, u2 = |v|^2, th = T - 1 and xi2 = |xi_l|^2.  Collecting the
// expansion in powers of x gives, for every velocity of one shell,
//     P(+-x) = (A0 + A2 x^2 + x^4/24) +- x (A1 + x^2/6)
//     A2 = 1/2 - u2/4 + th (xi2 - 6)/4
//     A1 = 1 - u2/2 + th (xi2 - 4)/2
//     A0 = 1 - u2/2 + th (xi2 - 2)/2 + u2^2/8 + th u2 (4 - xi2)/4
//          + th^2 (xi2^2 - 8 xi2 + 8)/8
// so the three shell coefficients are computed once per shell and each +-e
// pair costs one even and one odd polynomial.  The kernels evaluate this
// factored form; the equivalent tensor contraction costs ~10x more flops and
// would make the FP64 step compute-bound on this chip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice_constants.h"

namespace lbm {

#ifndef LBM_BLOCK
#define LBM_BLOCK 256
#endif
constexpr int BLOCK = LBM_BLOCK;   // threads per block, one site each along z
constexpr double D = 2.0;    // space dimension

// Shell coefficients of the factored equilibrium.  A0m1 = A0 - 1 so that the
// FP32 deviation form never forms 1 + small.
template <typename R>
struct ShellCoef {
    R a0m1, a1, a2;
};

template <typename R>
__device__ __forceinline__ ShellCoef<R> shell_coef(R u2, R th, R xi2) {
    ShellCoef<R> c;
    c.a2 = R(0.5) - R(0.25) * u2 + R(0.25) * th * (xi2 - R(6));
    c.a1 = R(1) - R(0.5) * u2 + R(0.5) * th * (xi2 - R(4));
    c.a0m1 = -R(0.5) * u2 + R(0.5) * th * (xi2 - R(2)) + R(0.125) * u2 * u2
             + R(0.25) * th * u2 * (R(4) - xi2)
             + R(0.125) * th * th * (xi2 * xi2 - R(8) * xi2 + R(8));
    return c;
}

// Even and odd parts of P - 1 at projection x for one shell.
template <typename R>
__device__ __forceinline__ void pair_poly(const ShellCoef<R> &c, R x, R &even_m1, R &odd) {
    const R x2 = x * x;
    even_m1 = c.a0m1 + x2 * (c.a2 + x2 * R(1.0 / 24.0));
    odd = x * (c.a1 + x2 * R(1.0 / 6.0));
}

// Full FP64 equilibrium f^eq_l(rho, v, T) for all 37 populations (used by
// the initial state and the wall table, not by the step's hot loop).
__device__ __forceinline__ void equilibrium_f64(double rho, double vx, double vz, double T,
                                                double feq[Q]) {
    const double u2 = vx * vx + vz * vz, th = T - 1.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const ShellCoef<double> c = shell_coef<double>(u2, th, XI2_SHELL[SHELL[l]]);
        double ev, od;
        pair_poly<double>(c, R * (EX[l] * vx + EZ[l] * vz), ev, od);
        feq[l] = W[l] * rho * (1.0 + ev + od);
    }
}

// Access at a wave-uniform base plus a 32-bit per-lane byte offset: lets the
// compiler use the scalar-base form of global loads/stores (one shared
// offset register instead of a 64-bit address per access).
template <typename T>
__device__ __forceinline__ T ldg_off(const T *base, uint32_t byte_off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void stg_off(T *base, uint32_t byte_off, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}
template <typename T>
__device__ __forceinline__ void stg_off_nt(T *base, uint32_t byte_off, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off));
}

// Tiled layout of population buffers (the state and the adjoint buffers).
// Rows are grouped in tiles of TILE; tile zt of column x holds its 37
// populations as 37 consecutive runs of TILE elements:
//     element (l, x, z) at ((zt Lx + x) 37 + l) TILE + (z - zt TILE),  zt = z / TILE,
// for z in [0, Lz); the rows of the last tile from Lz up are padding.  A
// wavefront's 37 + 37 memory streams then lie within a few contiguous
// 37 TILE-element tiles instead of 37 + 37 arrays a whole lattice apart,
// which keeps the per-CU address-translation cache from thrashing.
constexpr int TILE = 512;
static_assert((TILE & (TILE - 1)) == 0, "TILE is a power of two");

__host__ __device__ __forceinline__ int tile_count(int lz) { return (lz + TILE - 1) / TILE; }

// Index of element (l, x, z), 0 <= z < Lz.
__host__ __device__ __forceinline__ size_t pidx(int l, int x, int z, int lx) {
    const unsigned uz = (unsigned)z;
    return (((size_t)(uz / TILE) * (size_t)lx + (size_t)x) * Q + (size_t)l) * TILE + (size_t)(uz % TILE);
}

// Index of element (l, x, z0 + r) for a block whose rows [z0, z0 + n) lie in
// one tile (z0 / TILE block-uniform) and -TILE <= r - (z0 % TILE) < 2 TILE:
// the row may sit in the tile below or above (pulls and pushes shifted by
// up to 3 rows).  `base` is the index of (0, x, zt TILE), `step` the index
// distance between tiles zt and zt + 1 of one column less TILE.
__device__ __forceinline__ long long tile_off(int l, int rl, long long step) {
    // rl = row within tile zt, possibly -3 .. TILE + 2
    long long off = (long long)l * TILE + rl;
    if (rl < 0) off -= step;
    if (rl >= TILE) off += step;
    return off;
}

// Wrap an index into [0, n) for any integer (periodic directions).
__device__ __forceinline__ int wrap(int i, int n) {
    int m = i % n;
    return m < 0 ? m + n : m;
}

}  // namespace lbm
