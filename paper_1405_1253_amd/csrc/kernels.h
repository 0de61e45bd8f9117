// Internal launch interface between the C ABI layer (api.hip) and the kernels.
// Arguments have been validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

enum : uint32_t {
    F_PERIODIC_Z = 1u, F_NO_COLLIDE = 2u, F_ADJ_F32 = 4u, F_WALL_DIFFUSE = 8u, F_MOM_F32 = 16u, F_COLLIDE_F64 = 32u
};
// P_F32_DEV_C64: float deviation storage as P_F32_DEV, collision arithmetic in
// double (F_COLLIDE_F64); a kernel template value only, never a params value.
enum : int { P_F64 = 0, P_F32_DEV = 1, P_F32_DEV_C64 = 2 };

struct StepArgs {
    const void *f_in;    // two-buffer step: input state (unused in place)
    void *f_out;         // two-buffer step: output state; in place: the buffer
    const void *ghost;   // [2][3][37] elements, unused with F_PERIODIC_Z
    void *mom;           // nullable [4][lx][lz], double (float with F_MOM_F32)
    double *ratio;       // in place with F_WALL_DIFFUSE: scratch [2 x 3][lx]
    int lx, lz;
    double tau, omega, g;
    uint32_t flags;
};
hipError_t launch_step(const StepArgs &a, int precision, hipStream_t s);
// kind 0: the buffer holds the post-collision state, 1: the streamed form
hipError_t launch_step_inplace(const StepArgs &a, int precision, int kind, hipStream_t s);

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

struct ProfileArgs {
    const void *f;
    double *prof;        // [4][lz]
    void *scratch;
    int lx, lz;
    double g;
};
size_t profiles_scratch_bytes(int lx, int lz);
hipError_t launch_profiles(const ProfileArgs &a, int precision, hipStream_t s);

constexpr int MAX_MODES = 32;
struct InitArgs {
    void *f_out;
    void *ghost_out;
    const double *amp;   // device [2][nmodes]
    int lx, lz, nmodes;
    double g, t_d, t_m, t_u, width;
    double z_lo, z_hi;   // rest heights of the two interfaces (sites)
    double norm;         // C: density = C p / T
    double ghost_rho[6], ghost_t[6];   // rows -1,-2,-3 then Lz, Lz+1, Lz+2
    int k[2][MAX_MODES];
    double phase[2][MAX_MODES];
};
hipError_t launch_init(const InitArgs &a, int precision, hipStream_t s);

struct AdjointArgs {
    const void *mom;       // [4][lx][lz] pre-collision moments of the step (double, or float with F_MOM_F32)
    const void *lam_in;    // population buffer (tiled) dJ/df*_t (double, or float with F_ADJ_F32)
    void *lam_out;         // population buffer (tiled) dJ/df*_{t-1}
    const void *ghost;     // [2][3][37] wall table of the forward step (F_WALL_DIFFUSE)
    int precision;         // element type of ghost (P_F64 / P_F32_DEV)
    int lx, lz;
    double tau, omega, g;
    uint32_t flags;
};
hipError_t launch_adjoint_step(const AdjointArgs &a, hipStream_t s);
// Gather form: shift = false: lam_out = C^T lam_in (the collision alone, per
// site); shift = true: lam_out = C^T S^T lam_in (S^T alone with F_NO_COLLIDE).
hipError_t launch_adjoint_gather(const AdjointArgs &a, bool shift, hipStream_t s);

struct ObjectiveArgs {
    const void *f;
    void *scratch;
    double *j_out;         // [5]: J, KE, L_u + L_d, L_u, L_d
    void *lam_seed;        // nullable population buffer (tiled), double or float
    int lx, lz;
    bool lam_f32;
    double g, t_d, t_m, t_u, wk, wl;
};
size_t objective_scratch_bytes(int lx, int lz);
hipError_t launch_objective(const ObjectiveArgs &a, int precision, hipStream_t s);

struct InitVjpArgs {
    const void *lam0;      // population buffer (tiled), double or float
    bool lam_f32;
    const double *amp;     // [2][nmodes]
    double *d_amp;         // [2][nmodes]
    double *dh;            // scratch [2][lx]
    int lx, lz, nmodes;
    double g, t_d, t_m, t_u, width, norm;
    double z_lo, z_hi;
    int k[2][MAX_MODES];
    double phase[2][MAX_MODES];
};
hipError_t launch_init_vjp(const InitVjpArgs &a, hipStream_t s);

struct LayoutArgs {
    const void *src;
    void *dst;
    int lx, lz;
    int elt;               // element size in bytes, 4 or 8
};
// pack: [37][Lx][Lz] -> tiled (padding rows zeroed); unpack: tiled -> [37][Lx][Lz]
hipError_t launch_layout(const LayoutArgs &a, bool pack, hipStream_t s);

}  // namespace lbm
