// C ABI of the D2Q37 library: argument validation, host-side set-up and
// dispatch to the kernels.  No allocation (device or host), no
// synchronisation, no global mutable state except the per-thread text of
// the last HIP error (a fixed buffer).
#include <math.h>
#include <string.h>

#include <atomic>

#include "../../include/lbm.h"
#include "common.h"
#include "kernels.h"

static_assert(lbm::F_PERIODIC_Z == LBM_PERIODIC_Z && lbm::F_NO_COLLIDE == LBM_NO_COLLIDE &&
                  lbm::F_ADJ_F32 == LBM_ADJ_F32 && lbm::F_WALL_DIFFUSE == LBM_WALL_DIFFUSE &&
                  lbm::F_MOM_F32 == LBM_MOM_F32 && lbm::F_COLLIDE_F64 == LBM_COLLIDE_F64,
              "the kernels read params->flags as given");

// Scratch of the allocation-free diagnostics entry point (lbm_moments_noalloc).
static __device__ __align__(256) unsigned char scratch[LBM_STATIC_SCRATCH_BYTES];

namespace {

thread_local char g_last_hip_error[256];

int hip_status(hipError_t e) {
    if (e == hipSuccess) return LBM_OK;
    const char *msg = hipGetErrorString(e);
    strncpy(g_last_hip_error, msg ? msg : "unknown HIP error", sizeof(g_last_hip_error) - 1);
    g_last_hip_error[sizeof(g_last_hip_error) - 1] = '\0';
    return LBM_EHIP;
}

constexpr long long MAX_SITES = 1LL << 29;

int elt_size(int precision) { return precision == LBM_F64 ? 8 : 4; }

// Common parameter checks.  Sets *empty when the lattice has no sites.
int check_params(const lbm_params *p, bool *empty) {
    if (!p) return LBM_EINVAL;
    if (p->abi_version != LBM_ABI_VERSION) return LBM_EVERSION;
    if (p->lx < 0 || p->lz < 0) return LBM_EINVAL;
    if ((long long)p->lx * (long long)p->lz > MAX_SITES) return LBM_EINVAL;
    if (p->precision != LBM_F64 && p->precision != LBM_F32_DEV) return LBM_EINVAL;
    if (p->flags & ~(uint32_t)(LBM_PERIODIC_Z | LBM_NO_COLLIDE | LBM_ADJ_F32 | LBM_WALL_DIFFUSE | LBM_MOM_F32 |
                            LBM_COLLIDE_F64))
        return LBM_EINVAL;
    if ((p->flags & LBM_PERIODIC_Z) && (p->flags & LBM_WALL_DIFFUSE)) return LBM_EINVAL;
    if (p->reserved != 0) return LBM_EINVAL;
    if (!(p->tau > 0.5) || !isfinite(p->tau)) return LBM_EINVAL;
    if (!(p->g >= 0.0) || !isfinite(p->g)) return LBM_EINVAL;
    *empty = (p->lx == 0 || p->lz == 0);
    return LBM_OK;
}

bool aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// elements of a population buffer (state or adjoint) in the tiled layout
size_t pop_elems(const lbm_params *p) {
    return (size_t)LBM_Q * (size_t)p->lx * (size_t)lbm::tile_count(p->lz) * (size_t)lbm::TILE;
}
size_t state_bytes(const lbm_params *p) { return pop_elems(p) * (size_t)elt_size(p->precision); }
size_t ghost_bytes(const lbm_params *p) { return (size_t)2 * 3 * LBM_Q * elt_size(p->precision); }
size_t field_bytes(const lbm_params *p) { return (size_t)4 * p->lx * p->lz * sizeof(double); }
// the step's moments output / the adjoint's moments input: double, or float with LBM_MOM_F32
size_t mom_bytes(const lbm_params *p) {
    return (size_t)4 * p->lx * p->lz * ((p->flags & LBM_MOM_F32) ? sizeof(float) : sizeof(double));
}
// diffuse-wall M/S of every ghost site for the in-place step: [2 x 3][Lx] double
size_t wall_ratio_bytes(int lx) { return (size_t)6 * (size_t)lx * sizeof(double); }

// Unperturbed column, rows -3 .. Lz+2, on the host: the density
// normalisation C and the wall rows.  Same construction as the device
// columns: trapezoid rule for d ln p/dz = -g/T, one row = r length units.
// Rest heights of the interfaces; a negative entry selects Lz/3 or 2Lz/3.
void rest_heights(const lbm_params *p, const lbm_rt3_desc *d, double *lo, double *hi) {
    *lo = d->z_lo < 0.0 ? p->lz / 3.0 : d->z_lo;
    *hi = d->z_hi < 0.0 ? 2.0 * p->lz / 3.0 : d->z_hi;
}

void host_profile(const lbm_params *p, const lbm_rt3_desc *d, double *norm, double ghost_rho[6],
                  double ghost_t[6]) {
    // one pass over rows -3 .. Lz+2 (index i = row + 3), no buffers: the
    // log-pressure recursion needs only the previous row's temperature
    const int lz = p->lz, n = lz + 6;
    double z_lo, z_hi;
    rest_heights(p, d, &z_lo, &z_hi);
    auto temp = [&](int i) {
        const double zc = (double)(i - 3) + 0.5;
        const double s0 = 0.5 * (1.0 + tanh((zc - z_lo) / d->width));
        const double s1 = 0.5 * (1.0 + tanh((zc - z_hi) / d->width));
        return d->t_d + (d->t_m - d->t_d) * s0 + (d->t_u - d->t_m) * s1;
    };
    const int rows[6] = {2, 1, 0, 3 + lz, 4 + lz, 5 + lz};   // -1,-2,-3, Lz,Lz+1,Lz+2
    double ghost_lnp[6] = {0, 0, 0, 0, 0, 0};
    double mean = 0.0, lnp = 0.0, t_prev = 0.0;
    for (int i = 0; i < n; ++i) {
        const double T = temp(i);
        if (i > 0) lnp = lnp - p->g * lbm::R * 0.5 * (1.0 / t_prev + 1.0 / T);
        if (i >= 3 && i < 3 + lz) mean += exp(lnp) / T;
        for (int k = 0; k < 6; ++k)
            if (rows[k] == i) {
                ghost_lnp[k] = lnp;
                ghost_t[k] = T;
            }
        t_prev = T;
    }
    mean /= (double)lz;
    *norm = 1.0 / mean;
    for (int k = 0; k < 6; ++k) ghost_rho[k] = *norm * exp(ghost_lnp[k]) / ghost_t[k];
}

// Checks shared by the entry points that take an lbm_rt3_desc.
int check_desc(const lbm_rt3_desc *d, const double *amp) {
    if (!d) return LBM_EINVAL;
    if (d->nmodes < 0 || d->nmodes > LBM_MAX_MODES || d->reserved != 0) return LBM_EINVAL;
    if (d->nmodes > 0 && (!d->k || !d->phase || !amp)) return LBM_EINVAL;
    if (!(d->width > 0.0) || !isfinite(d->width)) return LBM_EINVAL;
    if (!(d->t_d > 0.0) || !(d->t_m > 0.0) || !(d->t_u > 0.0) || !isfinite(d->t_d) ||
        !isfinite(d->t_m) || !isfinite(d->t_u))
        return LBM_EINVAL;
    for (int i = 0; i < 2 * d->nmodes; ++i)
        if (!isfinite(d->phase[i])) return LBM_EINVAL;
    if (!isfinite(d->z_lo) || !isfinite(d->z_hi)) return LBM_EINVAL;
    return LBM_OK;
}

// The allocation-free diagnostics entry point's scratch: one array per device
// (each GPU the library runs on holds its own copy until the process ends).
// Host code never uses the array's name as an address: its device address is
// looked up once per device and kept in g_static_scratch.
constexpr int MAX_DEVICES = 64;
std::atomic<void *> g_static_scratch[MAX_DEVICES];

// Device address of the current device's array (looked up on the first call
// on that device; concurrent first calls store the same address).
int static_scratch(void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= MAX_DEVICES) return LBM_EINVAL;
    void *p = g_static_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        if (!p) return LBM_EHIP;
        g_static_scratch[dev].store(p, std::memory_order_release);
    }
    *ptr = p;
    return LBM_OK;
}

size_t lam_bytes(const lbm_params *p) {
    return pop_elems(p) * ((p->flags & LBM_ADJ_F32) ? sizeof(float) : sizeof(double));
}
size_t vjp_scratch_bytes(int lx) { return ((size_t)2 * lx * sizeof(double) + 255) & ~size_t(255); }

}  // namespace

extern "C" {

const char *lbm_strerror(int status) {
    switch (status) {
        case LBM_OK: return "success";
        case LBM_EINVAL: return "invalid argument";
        case LBM_EALIAS: return "output buffer overlaps an input buffer";
        case LBM_EALIGN: return "device pointer is not suitably aligned";
        case LBM_EHIP: return "HIP runtime error";
        case LBM_ESCRATCH: return "scratch buffer missing or too small";
        case LBM_EVERSION: return "lbm_params.abi_version does not match the library";
        case LBM_ESTATIC: return "lattice too large for the library's static scratch array";
        default: return "unknown status";
    }
}

const char *lbm_last_hip_error(void) { return g_last_hip_error; }

int lbm_lattice(double *r, double *w, int32_t *e) {
    if (r) *r = lbm::R;
    for (int l = 0; l < LBM_Q; ++l) {
        if (w) w[l] = lbm::W[l];
        if (e) {
            e[2 * l] = lbm::EX[l];
            e[2 * l + 1] = lbm::EZ[l];
        }
    }
    return LBM_OK;
}

size_t lbm_population_elems(const lbm_params *p) {
    bool empty = false;
    if (check_params(p, &empty) != LBM_OK) return 0;
    return pop_elems(p);
}

static int layout_call(const lbm_params *p, const void *src, void *dst, int elt, bool pack, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!src || !dst || (elt != 4 && elt != 8)) return LBM_EINVAL;
    if (!aligned(src, (size_t)elt) || !aligned(dst, (size_t)elt)) return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t soa = (size_t)LBM_Q * (size_t)p->lx * (size_t)p->lz * (size_t)elt;
    const size_t tiled = pop_elems(p) * (size_t)elt;
    if (overlap(src, pack ? soa : tiled, dst, pack ? tiled : soa)) return LBM_EALIAS;
    lbm::LayoutArgs a;
    a.src = src;
    a.dst = dst;
    a.lx = p->lx;
    a.lz = p->lz;
    a.elt = elt;
    return hip_status(lbm::launch_layout(a, pack, (hipStream_t)stream));
}

int lbm_pack(const lbm_params *p, const void *soa, void *tiled, int elt_bytes, lbm_stream_t stream) {
    return layout_call(p, soa, tiled, elt_bytes, true, stream);
}

int lbm_unpack(const lbm_params *p, const void *tiled, void *soa, int elt_bytes, lbm_stream_t stream) {
    return layout_call(p, tiled, soa, elt_bytes, false, stream);
}

size_t lbm_scratch_bytes(const lbm_params *p) {
    bool empty = false;
    if (check_params(p, &empty) != LBM_OK || empty) return 0;
    size_t b = lbm::moments_scratch_bytes(p->lx, p->lz);
    if (lbm::objective_scratch_bytes(p->lx, p->lz) > b) b = lbm::objective_scratch_bytes(p->lx, p->lz);
    if (vjp_scratch_bytes(p->lx) > b) b = vjp_scratch_bytes(p->lx);
    if (lbm::profiles_scratch_bytes(p->lx, p->lz) > b) b = lbm::profiles_scratch_bytes(p->lx, p->lz);
    if (wall_ratio_bytes(p->lx) > b) b = wall_ratio_bytes(p->lx);
    return b;
}

int lbm_profiles(const lbm_params *p, const void *f, double *prof, void *scratch, size_t scratch_bytes,
                 lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!f || !prof) return LBM_EINVAL;
    if (!aligned(f, 16) || !aligned(prof, 8) || !aligned(scratch, 256)) return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t need = lbm::profiles_scratch_bytes(p->lx, p->lz);
    if (!scratch || scratch_bytes < need) return LBM_ESCRATCH;
    const size_t sb = state_bytes(p), pb = (size_t)4 * p->lz * sizeof(double);
    if (overlap(prof, pb, f, sb) || overlap(scratch, need, f, sb) || overlap(scratch, need, prof, pb))
        return LBM_EALIAS;
    lbm::ProfileArgs a;
    a.f = f;
    a.prof = prof;
    a.scratch = scratch;
    a.lx = p->lx;
    a.lz = p->lz;
    a.g = p->g;
    return hip_status(lbm::launch_profiles(a, p->precision, (hipStream_t)stream));
}

int lbm_step(const lbm_params *p, const void *ghost, const void *f_in, void *f_out,
             double *moments_out, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!f_in || !f_out) return LBM_EINVAL;
    if (!ghost && !(p->flags & LBM_PERIODIC_Z)) return LBM_EINVAL;
    if (!aligned(f_in, 16) || !aligned(f_out, 16) || !aligned(ghost, 8) || !aligned(moments_out, 8))
        return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t sb = state_bytes(p);
    if (overlap(f_in, sb, f_out, sb) || overlap(ghost, ghost_bytes(p), f_out, sb) ||
        overlap(moments_out, mom_bytes(p), f_in, sb) ||
        overlap(moments_out, mom_bytes(p), f_out, sb) ||
        overlap(moments_out, mom_bytes(p), ghost, ghost_bytes(p)))
        return LBM_EALIAS;
    lbm::StepArgs a;
    a.f_in = f_in;
    a.f_out = f_out;
    a.ghost = ghost;
    a.mom = moments_out;
    a.lx = p->lx;
    a.lz = p->lz;
    a.tau = p->tau;
    a.omega = 1.0 / p->tau;
    a.g = p->g;
    a.flags = p->flags;
    a.ratio = nullptr;
    return hip_status(lbm::launch_step(a, p->precision, (hipStream_t)stream));
}

int lbm_step_inplace(const lbm_params *p, const void *ghost, void *f, int kind, double *moments_out,
                     void *scratch, size_t scratch_bytes, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!f || (kind != LBM_INPLACE_FROM_STATE && kind != LBM_INPLACE_FROM_STREAMED)) return LBM_EINVAL;
    if (!ghost && !(p->flags & LBM_PERIODIC_Z)) return LBM_EINVAL;
    const bool diffuse = (p->flags & LBM_WALL_DIFFUSE) != 0;
    if (!aligned(f, 16) || !aligned(ghost, 8) || !aligned(moments_out, 8) || !aligned(scratch, 8))
        return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t rb = wall_ratio_bytes(p->lx);
    if (diffuse && (!scratch || scratch_bytes < rb)) return LBM_ESCRATCH;
    const size_t sb = state_bytes(p), gb = ghost_bytes(p), fb = mom_bytes(p);
    if (overlap(ghost, gb, f, sb) || overlap(moments_out, fb, f, sb) || overlap(moments_out, fb, ghost, gb) ||
        (diffuse && (overlap(scratch, rb, f, sb) || overlap(scratch, rb, ghost, gb) ||
                     overlap(scratch, rb, moments_out, fb))))
        return LBM_EALIAS;
    lbm::StepArgs a;
    a.f_in = nullptr;
    a.f_out = f;
    a.ghost = ghost;
    a.mom = moments_out;
    a.ratio = diffuse ? static_cast<double *>(scratch) : nullptr;
    a.lx = p->lx;
    a.lz = p->lz;
    a.tau = p->tau;
    a.omega = 1.0 / p->tau;
    a.g = p->g;
    a.flags = p->flags;
    return hip_status(lbm::launch_step_inplace(a, p->precision, kind, (hipStream_t)stream));
}

int lbm_moments(const lbm_params *p, const void *f, double *fields, double *tbar, double *sums,
                void *scratch, size_t scratch_bytes, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!f) return LBM_EINVAL;
    if (!aligned(f, 16) || !aligned(fields, 8) || !aligned(tbar, 8) || !aligned(sums, 8) ||
        !aligned(scratch, 256))
        return LBM_EALIGN;
    if (empty) return LBM_OK;
    const bool need_scratch = tbar || sums;
    if (need_scratch && (!scratch || scratch_bytes < lbm::moments_scratch_bytes(p->lx, p->lz)))
        return LBM_ESCRATCH;
    const size_t sb = state_bytes(p), fb = field_bytes(p);
    const size_t tb = (size_t)p->lz * sizeof(double), scb = need_scratch ? scratch_bytes : 0;
    if (overlap(fields, fb, f, sb) || overlap(tbar, tb, f, sb) || overlap(sums, 32, f, sb) ||
        overlap(scratch, scb, f, sb) || overlap(fields, fb, tbar, tb) || overlap(fields, fb, sums, 32) ||
        overlap(tbar, tb, sums, 32) || overlap(scratch, scb, fields, fb) ||
        overlap(scratch, scb, tbar, tb) || overlap(scratch, scb, sums, 32))
        return LBM_EALIAS;
    if (!fields && !tbar && !sums) return LBM_OK;
    lbm::MomentArgs a;
    a.f = f;
    a.fields = fields;
    a.tbar = tbar;
    a.sums = sums;
    a.scratch = scratch;
    a.lx = p->lx;
    a.lz = p->lz;
    a.g = p->g;
    return hip_status(lbm::launch_moments(a, p->precision, (hipStream_t)stream));
}

int lbm_moments_noalloc(const lbm_params *p, const void *f, double *fields, double *tbar, double *sums,
                        lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!f) return LBM_EINVAL;
    if (!aligned(f, 16) || !aligned(fields, 8) || !aligned(tbar, 8) || !aligned(sums, 8)) return LBM_EALIGN;
    if (empty) return LBM_OK;
    const bool need_scratch = tbar || sums;
    const size_t need = need_scratch ? lbm::moments_scratch_bytes(p->lx, p->lz) : 0;
    if (need > (size_t)LBM_STATIC_SCRATCH_BYTES) return LBM_ESTATIC;
    const size_t sb = state_bytes(p), fb = field_bytes(p), tb = (size_t)p->lz * sizeof(double);
    if (overlap(fields, fb, f, sb) || overlap(tbar, tb, f, sb) || overlap(sums, 32, f, sb) ||
        overlap(fields, fb, tbar, tb) || overlap(fields, fb, sums, 32) || overlap(tbar, tb, sums, 32))
        return LBM_EALIAS;
    if (!fields && !tbar && !sums) return LBM_OK;
    void *scr = nullptr;
    if (need_scratch && (st = static_scratch(&scr)) != LBM_OK) return st;
    lbm::MomentArgs a;
    a.f = f;
    a.fields = fields;
    a.tbar = tbar;
    a.sums = sums;
    a.scratch = scr;
    a.lx = p->lx;
    a.lz = p->lz;
    a.g = p->g;
    return hip_status(lbm::launch_moments(a, p->precision, (hipStream_t)stream));
}

int lbm_init_rt3(const lbm_params *p, const lbm_rt3_desc *d, const double *amp, void *f_out,
                 void *ghost_out, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!f_out || !ghost_out) return LBM_EINVAL;
    if ((st = check_desc(d, amp)) != LBM_OK) return st;
    if (!aligned(f_out, 16) || !aligned(ghost_out, 8) || !aligned(amp, 8)) return LBM_EALIGN;
    if (overlap(f_out, state_bytes(p), ghost_out, ghost_bytes(p))) return LBM_EALIAS;
    if (empty) return LBM_OK;

    lbm::InitArgs a;
    memset(&a, 0, sizeof(a));
    a.f_out = f_out;
    a.ghost_out = ghost_out;
    a.amp = amp;
    a.lx = p->lx;
    a.lz = p->lz;
    a.nmodes = d->nmodes;
    a.g = p->g;
    a.t_d = d->t_d;
    a.t_m = d->t_m;
    a.t_u = d->t_u;
    a.width = d->width;
    rest_heights(p, d, &a.z_lo, &a.z_hi);
    for (int f = 0; f < 2; ++f)
        for (int j = 0; j < d->nmodes; ++j) {
            a.k[f][j] = d->k[f * d->nmodes + j];
            a.phase[f][j] = d->phase[f * d->nmodes + j];
        }

    host_profile(p, d, &a.norm, a.ghost_rho, a.ghost_t);
    return hip_status(lbm::launch_init(a, p->precision, (hipStream_t)stream));
}

int lbm_objective(const lbm_params *p, const lbm_rt3_desc *d, const void *f, double wk, double wl,
                  double *j_out, void *lam_seed, void *scratch, size_t scratch_bytes,
                  lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!d || !f || !j_out) return LBM_EINVAL;
    if (!(d->t_d > d->t_m) || !(d->t_m > d->t_u) || !isfinite(d->t_d) || !isfinite(d->t_u))
        return LBM_EINVAL;
    if (!isfinite(wk) || !isfinite(wl)) return LBM_EINVAL;
    if (!aligned(f, 16) || !aligned(j_out, 8) || !aligned(lam_seed, 16) || !aligned(scratch, 256))
        return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t need = lbm::objective_scratch_bytes(p->lx, p->lz);
    if (!scratch || scratch_bytes < need) return LBM_ESCRATCH;
    const size_t sb = state_bytes(p), lb = lam_bytes(p);
    if (overlap(j_out, 40, f, sb) || overlap(lam_seed, lb, f, sb) || overlap(scratch, need, f, sb) ||
        overlap(j_out, 40, lam_seed, lb) || overlap(j_out, 40, scratch, need) ||
        overlap(lam_seed, lb, scratch, need))
        return LBM_EALIAS;
    lbm::ObjectiveArgs a;
    a.f = f;
    a.scratch = scratch;
    a.j_out = j_out;
    a.lam_seed = lam_seed;
    a.lam_f32 = (p->flags & LBM_ADJ_F32) != 0;
    a.lx = p->lx;
    a.lz = p->lz;
    a.g = p->g;
    a.t_d = d->t_d;
    a.t_m = d->t_m;
    a.t_u = d->t_u;
    a.wk = wk;
    a.wl = wl;
    return hip_status(lbm::launch_objective(a, p->precision, (hipStream_t)stream));
}

int lbm_adjoint_step(const lbm_params *p, const void *ghost, const double *moments, const void *lam_in,
                     void *lam_out, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!lam_in || !lam_out || (!moments && !(p->flags & LBM_NO_COLLIDE))) return LBM_EINVAL;
    if (!ghost && (p->flags & LBM_WALL_DIFFUSE)) return LBM_EINVAL;
    if (!aligned(lam_in, 16) || !aligned(lam_out, 16) || !aligned(moments, 16) || !aligned(ghost, 8))
        return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t lb = lam_bytes(p), mb = mom_bytes(p);
    if (overlap(lam_in, lb, lam_out, lb) || overlap(moments, mb, lam_out, lb) ||
        overlap(ghost, ghost_bytes(p), lam_out, lb))
        return LBM_EALIAS;
    lbm::AdjointArgs a;
    a.mom = moments;
    a.lam_in = lam_in;
    a.lam_out = lam_out;
    a.ghost = ghost;
    a.precision = p->precision;
    a.lx = p->lx;
    a.lz = p->lz;
    a.tau = p->tau;
    a.omega = 1.0 / p->tau;
    a.g = p->g;
    a.flags = p->flags;
    return hip_status(lbm::launch_adjoint_step(a, (hipStream_t)stream));
}

int lbm_adjoint_collide(const lbm_params *p, const double *moments, const void *lam, void *mu,
                        lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!lam || !mu || (!moments && !(p->flags & LBM_NO_COLLIDE))) return LBM_EINVAL;
    if (!aligned(lam, 16) || !aligned(mu, 16) || !aligned(moments, 16)) return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t lb = lam_bytes(p), mb = mom_bytes(p);
    if (overlap(lam, lb, mu, lb) || overlap(moments, mb, mu, lb)) return LBM_EALIAS;
    lbm::AdjointArgs a;
    a.mom = moments;
    a.lam_in = lam;
    a.lam_out = mu;
    a.ghost = nullptr;
    a.precision = p->precision;
    a.lx = p->lx;
    a.lz = p->lz;
    a.tau = p->tau;
    a.omega = 1.0 / p->tau;
    a.g = p->g;
    a.flags = p->flags;
    return hip_status(lbm::launch_adjoint_gather(a, false, (hipStream_t)stream));
}

int lbm_adjoint_gather(const lbm_params *p, const void *ghost, const double *moments, const void *mu_in,
                       void *mu_out, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!mu_in || !mu_out || (!moments && !(p->flags & LBM_NO_COLLIDE))) return LBM_EINVAL;
    if (!ghost && (p->flags & LBM_WALL_DIFFUSE)) return LBM_EINVAL;
    if (!aligned(mu_in, 16) || !aligned(mu_out, 16) || !aligned(moments, 16) || !aligned(ghost, 8))
        return LBM_EALIGN;
    if (empty) return LBM_OK;
    const size_t lb = lam_bytes(p), mb = mom_bytes(p), gb = ghost_bytes(p);
    if (overlap(mu_in, lb, mu_out, lb) || overlap(moments, mb, mu_out, lb) || overlap(ghost, gb, mu_out, lb))
        return LBM_EALIAS;
    lbm::AdjointArgs a;
    a.mom = moments;
    a.lam_in = mu_in;
    a.lam_out = mu_out;
    a.ghost = ghost;
    a.precision = p->precision;
    a.lx = p->lx;
    a.lz = p->lz;
    a.tau = p->tau;
    a.omega = 1.0 / p->tau;
    a.g = p->g;
    a.flags = p->flags;
    return hip_status(lbm::launch_adjoint_gather(a, true, (hipStream_t)stream));
}

int lbm_init_rt3_vjp(const lbm_params *p, const lbm_rt3_desc *d, const double *amp, const void *lam0,
                     double *d_amp, void *scratch, size_t scratch_bytes, lbm_stream_t stream) {
    bool empty = false;
    int st = check_params(p, &empty);
    if (st != LBM_OK) return st;
    if (!lam0 || (!d_amp && d && d->nmodes > 0)) return LBM_EINVAL;
    if ((st = check_desc(d, amp)) != LBM_OK) return st;
    if (!aligned(lam0, 16) || !aligned(d_amp, 8) || !aligned(amp, 8) || !aligned(scratch, 256))
        return LBM_EALIGN;
    if (empty || d->nmodes == 0) return LBM_OK;
    const size_t need = vjp_scratch_bytes(p->lx);
    if (!scratch || scratch_bytes < need) return LBM_ESCRATCH;
    const size_t ab = (size_t)2 * d->nmodes * sizeof(double), lb = lam_bytes(p);
    if (overlap(d_amp, ab, lam0, lb) || overlap(d_amp, ab, amp, ab) || overlap(d_amp, ab, scratch, need) ||
        overlap(scratch, need, lam0, lb) || overlap(scratch, need, amp, ab))
        return LBM_EALIAS;
    lbm::InitVjpArgs a;
    memset(&a, 0, sizeof(a));
    a.lam0 = lam0;
    a.lam_f32 = (p->flags & LBM_ADJ_F32) != 0;
    a.amp = amp;
    a.d_amp = d_amp;
    a.dh = static_cast<double *>(scratch);
    a.lx = p->lx;
    a.lz = p->lz;
    a.nmodes = d->nmodes;
    a.g = p->g;
    a.t_d = d->t_d;
    a.t_m = d->t_m;
    a.t_u = d->t_u;
    a.width = d->width;
    rest_heights(p, d, &a.z_lo, &a.z_hi);
    for (int f = 0; f < 2; ++f)
        for (int j = 0; j < d->nmodes; ++j) {
            a.k[f][j] = d->k[f * d->nmodes + j];
            a.phase[f][j] = d->phase[f * d->nmodes + j];
        }
    double gr[6], gt[6];
    host_profile(p, d, &a.norm, gr, gt);
    return hip_status(lbm::launch_init_vjp(a, (hipStream_t)stream));
}

}  // extern "C"
