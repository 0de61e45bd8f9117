// Conversion between the library's tiled population layout (common.h) and
// the plain structure-of-arrays layout [37][Lx][Lz] (z fastest).  A pure
// permutation of elements of 4 or 8 bytes: bit-exact both ways.  Packing
// also zeroes the padding rows of the last tile, so a packed buffer is
// fully defined.
#include "common.h"
#include "kernels.h"

namespace lbm {

// One thread per (l, x, row of the padded column); blocks of BLOCK rows.
template <typename T, bool PACK>
__global__ __launch_bounds__(BLOCK) void layout_kernel(LayoutArgs a, int nzb) {
    const int zb = (int)(blockIdx.x % (uint32_t)nzb);
    const int lx_ = (int)(blockIdx.x / (uint32_t)nzb);   // l * Lx + x
    const int l = lx_ / a.lx, x = lx_ % a.lx;
    const int z = zb * BLOCK + (int)threadIdx.x;
    if (z >= tile_count(a.lz) * TILE) return;
    const size_t t = pidx(l, x, z, a.lx);
    const size_t s = ((size_t)l * (size_t)a.lx + (size_t)x) * (size_t)a.lz + (size_t)z;
    const T *src = static_cast<const T *>(a.src);
    T *dst = static_cast<T *>(a.dst);
    if (PACK)
        dst[t] = z < a.lz ? src[s] : T(0);
    else if (z < a.lz)
        dst[s] = src[t];
}

hipError_t launch_layout(const LayoutArgs &a, bool pack, hipStream_t s) {
    const int nzb = (tile_count(a.lz) * TILE + BLOCK - 1) / BLOCK;
    const dim3 grid((uint32_t)nzb * (uint32_t)Q * (uint32_t)a.lx);
    if (a.elt == 8) {
        if (pack)
            hipLaunchKernelGGL((layout_kernel<uint64_t, true>), grid, dim3(BLOCK), 0, s, a, nzb);
        else
            hipLaunchKernelGGL((layout_kernel<uint64_t, false>), grid, dim3(BLOCK), 0, s, a, nzb);
    } else {
        if (pack)
            hipLaunchKernelGGL((layout_kernel<uint32_t, true>), grid, dim3(BLOCK), 0, s, a, nzb);
        else
            hipLaunchKernelGGL((layout_kernel<uint32_t, false>), grid, dim3(BLOCK), 0, s, a, nzb);
    }
    return hipGetLastError();
}

}  // namespace lbm
