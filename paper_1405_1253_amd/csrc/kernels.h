// Internal launch interface between the C ABI layer (api.hip) and the kernels.
// Arguments have been validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

enum : uint32_t { F_PERIODIC_Z = 1u, F_NO_COLLIDE = 2u };
enum : int { P_F64 = 0, P_F32_DEV = 1 };

struct StepArgs {
    const void *f_in;
    void *f_out;
    const void *ghost;   // [2][3][37] elements, unused with F_PERIODIC_Z
    double *mom;         // nullable [4][lx][lz]
    int lx, lz;
    double tau, omega, g;
    uint32_t flags;
};
hipError_t launch_step(const StepArgs &a, int precision, hipStream_t s);

struct MomentArgs {
    const void *f;
    double *fields;      // nullable [4][lx][lz]
    double *tbar;        // nullable [lz]
    double *sums;        // nullable [4]
    void *scratch;
    int lx, lz;
    double g;
};
size_t moments_scratch_bytes(int lx, int lz);
hipError_t launch_moments(const MomentArgs &a, int precision, hipStream_t s);

constexpr int MAX_MODES = 32;
struct InitArgs {
    void *f_out;
    void *ghost_out;
    const double *amp;   // device [2][nmodes]
    int lx, lz, nmodes;
    double g, t_d, t_m, t_u, width;
    double norm;         // C: density = C p / T
    double ghost_rho[6], ghost_t[6];   // rows -1,-2,-3 then Lz, Lz+1, Lz+2
    int k[2][MAX_MODES];
    double phase[2][MAX_MODES];
};
hipError_t launch_init(const InitArgs &a, int precision, hipStream_t s);

}  // namespace lbm
