"""ctypes binding of liblbm.so: the C entry points under the same names.

Argument marshalling only -- every step of the method runs in the library's
HIP kernels.  Population buffers (the state, adjoint buffers) are in the
library's tiled layout (include/lbm.h); to_tiled / to_soa convert to and from
the plain [37, Lx, Lz] layout through the library's pack/unpack kernels.
Before a call, each tensor's element type and size are checked against what
the parameters imply (the C entry points see only addresses), so a
mismatched buffer raises ValueError instead of being overrun.  Buffers are
torch tensors (device memory) or raw integer addresses (passed unchecked);
streams default to torch's current stream.  A failing call raises LbmError
with the library's status text.  Loading fails loudly when the library has
not been built: there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

ABI_VERSION = 5
Q = 37
MAX_MODES = 32
TILE = 512   # rows per tile of a population buffer (tiled layout, include/lbm.h)
F64, F32_DEV = 0, 1
PERIODIC_Z, NO_COLLIDE, ADJ_F32, WALL_DIFFUSE, MOM_F32, COLLIDE_F64 = 1, 2, 4, 8, 16, 32
INPLACE_FROM_STATE, INPLACE_FROM_STREAMED = 0, 1

STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_EALIAS", -3: "LBM_EALIGN",
          -4: "LBM_EHIP", -5: "LBM_ESCRATCH", -6: "LBM_EVERSION", -7: "LBM_ESTATIC"}
STATIC_SCRATCH_BYTES = 16 << 20


class LbmError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        text = lib.lbm_strerror(status).decode()
        hip = lib.lbm_last_hip_error().decode() if status == -4 else ""
        super().__init__(f"{where}: {STATUS.get(status, status)} ({text}){' ' + hip if hip else ''}")
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("lx", ctypes.c_int32), ("lz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("tau", ctypes.c_double), ("g", ctypes.c_double)]


class lbm_rt3_desc(ctypes.Structure):
    _fields_ = [("t_d", ctypes.c_double), ("t_m", ctypes.c_double), ("t_u", ctypes.c_double),
                ("width", ctypes.c_double), ("nmodes", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("k", ctypes.POINTER(ctypes.c_int32)),
                ("phase", ctypes.POINTER(ctypes.c_double)), ("z_lo", ctypes.c_double),
                ("z_hi", ctypes.c_double)]


_LIB = None
_VP = ctypes.c_void_p


def load():
    """Load liblbm.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # torch ships its own HIP runtime; loading it first makes liblbm.so
        # bind to that same runtime (one runtime per process shares the
        # device, the streams and the memory torch allocates)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1405_1253_amd.build` (no CPU fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        lib.lbm_init_rt3.argtypes = [P(lbm_params), P(lbm_rt3_desc), _VP, _VP, _VP, _VP]
        lib.lbm_step.argtypes = [P(lbm_params), _VP, _VP, _VP, _VP, _VP]
        lib.lbm_step_inplace.argtypes = [P(lbm_params), _VP, _VP, ctypes.c_int, _VP, _VP, ctypes.c_size_t,
                                         _VP]
        lib.lbm_moments.argtypes = [P(lbm_params), _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]
        lib.lbm_moments_noalloc.argtypes = [P(lbm_params), _VP, _VP, _VP, _VP, _VP]
        lib.lbm_population_elems.argtypes = [P(lbm_params)]
        lib.lbm_population_elems.restype = ctypes.c_size_t
        lib.lbm_pack.argtypes = [P(lbm_params), _VP, _VP, ctypes.c_int, _VP]
        lib.lbm_unpack.argtypes = [P(lbm_params), _VP, _VP, ctypes.c_int, _VP]
        lib.lbm_scratch_bytes.argtypes = [P(lbm_params)]
        lib.lbm_scratch_bytes.restype = ctypes.c_size_t
        lib.lbm_lattice.argtypes = [P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_int32)]
        lib.lbm_strerror.argtypes = [ctypes.c_int]
        lib.lbm_strerror.restype = ctypes.c_char_p
        lib.lbm_last_hip_error.argtypes = []
        lib.lbm_last_hip_error.restype = ctypes.c_char_p
        lib.lbm_objective.argtypes = [P(lbm_params), P(lbm_rt3_desc), _VP, ctypes.c_double,
                                      ctypes.c_double, _VP, _VP, _VP, ctypes.c_size_t, _VP]
        lib.lbm_adjoint_step.argtypes = [P(lbm_params), _VP, _VP, _VP, _VP, _VP]
        lib.lbm_adjoint_collide.argtypes = [P(lbm_params), _VP, _VP, _VP, _VP]
        lib.lbm_adjoint_gather.argtypes = [P(lbm_params), _VP, _VP, _VP, _VP, _VP]
        lib.lbm_init_rt3_vjp.argtypes = [P(lbm_params), P(lbm_rt3_desc), _VP, _VP, _VP, _VP,
                                         ctypes.c_size_t, _VP]
        lib.lbm_profiles.argtypes = [P(lbm_params), _VP, _VP, _VP, ctypes.c_size_t, _VP]
        for name in ("lbm_init_rt3", "lbm_step", "lbm_step_inplace", "lbm_moments", "lbm_moments_noalloc",
                     "lbm_lattice", "lbm_objective", "lbm_pack", "lbm_unpack",
                     "lbm_adjoint_step", "lbm_adjoint_collide", "lbm_adjoint_gather", "lbm_init_rt3_vjp",
                     "lbm_profiles"):
            getattr(lib, name).restype = ctypes.c_int
        _LIB = lib
    return _LIB


def wall_flag(wall):
    """Flag bits of a wall rule name: "dirichlet" (the default) or "diffuse"."""
    if wall not in ("dirichlet", "diffuse"):
        raise ValueError(f"unknown wall rule {wall!r}")
    return WALL_DIFFUSE if wall == "diffuse" else 0


def make_params(lx, lz, tau, g, precision=F64, flags=0):
    return lbm_params(ABI_VERSION, lx, lz, precision, flags, 0, tau, g)


def _ptr(x):
    """Device address of a contiguous GPU tensor (or a raw integer address)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError("liblbm buffers must be GPU tensors")
    if not x.is_contiguous():
        raise ValueError("liblbm buffers must be contiguous (the layouts of include/lbm.h)")
    return x.data_ptr()


def _sites(params):
    return int(params.lx) * int(params.lz)


def population_elems(params):
    """Elements of a population buffer (state or adjoint) in the tiled
    layout: 37 Lx ceil(Lz / TILE) TILE (the same as lbm_population_elems)."""
    return Q * int(params.lx) * (-(-int(params.lz) // TILE)) * TILE


def _state_dtype(params):
    import torch
    return torch.float64 if params.precision == F64 else torch.float32


def _lam_dtype(params):
    import torch
    return torch.float32 if params.flags & ADJ_F32 else torch.float64


def _mom_dtype(params):
    import torch
    return torch.float32 if params.flags & MOM_F32 else torch.float64


def _need(name, x, dtype, numel):
    """Host-side check of one buffer against what the parameters imply.

    The C entry points see only addresses, so a tensor of the wrong element
    type or too few elements would be read or written past its end on the
    device; this raises ValueError before anything is launched.  Raw integer
    addresses are passed through unchecked (the caller vouches for them)."""
    if x is None or isinstance(x, int):
        return
    if x.dtype != dtype:
        raise ValueError(f"{name}: dtype {x.dtype}, expected {dtype} for these parameters")
    if x.numel() < numel:
        raise ValueError(f"{name}: {x.numel()} elements, expected at least {numel} for these parameters")


def _f64():
    import torch
    return torch.float64


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status, where):
    if status != 0:
        raise LbmError(status, where)


class RT3Desc:
    """Host-side lbm_rt3_desc with the arrays it points to kept alive."""

    def __init__(self, t_d, t_m, t_u, width, k=None, phase=None, z_lo=None, z_hi=None):
        self.k = np.ascontiguousarray(np.zeros((2, 0)) if k is None else k, dtype=np.int32)
        self.phase = np.ascontiguousarray(np.zeros((2, 0)) if phase is None else phase,
                                          dtype=np.float64)
        nmodes = self.k.shape[1] if self.k.ndim == 2 else 0
        self.c = lbm_rt3_desc(t_d, t_m, t_u, width, nmodes, 0,
                              self.k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              self.phase.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              -1.0 if z_lo is None else z_lo, -1.0 if z_hi is None else z_hi)

    @property
    def nmodes(self):
        return self.c.nmodes


def lbm_init_rt3(params, desc, amp, f_out, ghost_out, stream=None):
    """Three-layer hydrostatic initial state (see include/lbm.h).

    desc: RT3Desc (host k, phase [2, nmodes]); amp: device float64 [2, nmodes]."""
    _need("amp", amp, _f64(), 2 * desc.nmodes)
    _need("f_out", f_out, _state_dtype(params), population_elems(params))
    _need("ghost_out", ghost_out, _state_dtype(params), 2 * 3 * Q)
    st = load().lbm_init_rt3(ctypes.byref(params), ctypes.byref(desc.c), _ptr(amp), _ptr(f_out),
                             _ptr(ghost_out), _stream(stream))
    _check(st, "lbm_init_rt3")


def lbm_step(params, ghost, f_in, f_out, moments_out=None, stream=None):
    """One fused propagate + bc + collide step (see include/lbm.h)."""
    _need("ghost", ghost, _state_dtype(params), 2 * 3 * Q)
    _need("f_in", f_in, _state_dtype(params), population_elems(params))
    _need("f_out", f_out, _state_dtype(params), population_elems(params))
    _need("moments_out", moments_out, _mom_dtype(params), 4 * _sites(params))
    st = load().lbm_step(ctypes.byref(params), _ptr(ghost), _ptr(f_in), _ptr(f_out),
                         _ptr(moments_out), _stream(stream))
    _check(st, "lbm_step")


def lbm_step_inplace(params, ghost, f, kind, moments_out=None, scratch=None, stream=None):
    """One step on a single buffer, kind INPLACE_FROM_STATE or
    INPLACE_FROM_STREAMED (see include/lbm.h)."""
    _need("ghost", ghost, _state_dtype(params), 2 * 3 * Q)
    _need("f", f, _state_dtype(params), population_elems(params))
    _need("moments_out", moments_out, _mom_dtype(params), 4 * _sites(params))
    st = load().lbm_step_inplace(ctypes.byref(params), _ptr(ghost), _ptr(f), int(kind), _ptr(moments_out),
                                 _ptr(scratch), _nbytes(scratch), _stream(stream))
    _check(st, "lbm_step_inplace")


def lbm_scratch_bytes(params):
    return int(load().lbm_scratch_bytes(ctypes.byref(params)))


def lbm_moments(params, f, fields=None, tbar=None, sums=None, scratch=None, stream=None):
    """Renormalised fields, mean profile and global sums (see include/lbm.h)."""
    _need("f", f, _state_dtype(params), population_elems(params))
    _need("fields", fields, _f64(), 4 * _sites(params))
    _need("tbar", tbar, _f64(), int(params.lz))
    _need("sums", sums, _f64(), 4)
    nbytes = 0 if scratch is None else scratch.numel() * scratch.element_size()
    st = load().lbm_moments(ctypes.byref(params), _ptr(f), _ptr(fields), _ptr(tbar), _ptr(sums),
                            _ptr(scratch), nbytes, _stream(stream))
    _check(st, "lbm_moments")


def lbm_moments_noalloc(params, f, fields=None, tbar=None, sums=None, stream=None):
    """lbm_moments with the library's own static scratch: no allocation
    (see include/lbm.h; calls overlapping on one GPU race)."""
    _need("f", f, _state_dtype(params), population_elems(params))
    _need("fields", fields, _f64(), 4 * _sites(params))
    _need("tbar", tbar, _f64(), int(params.lz))
    _need("sums", sums, _f64(), 4)
    st = load().lbm_moments_noalloc(ctypes.byref(params), _ptr(f), _ptr(fields), _ptr(tbar), _ptr(sums),
                                    _stream(stream))
    _check(st, "lbm_moments_noalloc")


def _elt(x):
    return x.element_size() if not isinstance(x, int) else None


def lbm_pack(params, soa, tiled, elt_bytes=None, stream=None):
    """Plain [37][Lx][Lz] buffer -> tiled population buffer (see include/lbm.h)."""
    elt = elt_bytes or _elt(soa)
    for name, t, n in (("soa", soa, Q * _sites(params)), ("tiled", tiled, population_elems(params))):
        if not isinstance(t, int):
            if t.element_size() != elt:
                raise ValueError(f"{name}: element size {t.element_size()}, expected {elt}")
            if t.numel() < n:
                raise ValueError(f"{name}: {t.numel()} elements, expected at least {n}")
    st = load().lbm_pack(ctypes.byref(params), _ptr(soa), _ptr(tiled), int(elt), _stream(stream))
    _check(st, "lbm_pack")


def lbm_unpack(params, tiled, soa, elt_bytes=None, stream=None):
    """Tiled population buffer -> plain [37][Lx][Lz] buffer (see include/lbm.h)."""
    elt = elt_bytes or _elt(tiled)
    for name, t, n in (("tiled", tiled, population_elems(params)), ("soa", soa, Q * _sites(params))):
        if not isinstance(t, int):
            if t.element_size() != elt:
                raise ValueError(f"{name}: element size {t.element_size()}, expected {elt}")
            if t.numel() < n:
                raise ValueError(f"{name}: {t.numel()} elements, expected at least {n}")
    st = load().lbm_unpack(ctypes.byref(params), _ptr(tiled), _ptr(soa), int(elt), _stream(stream))
    _check(st, "lbm_unpack")


def empty_populations(params, dtype, device="cuda"):
    """An uninitialised population buffer (tiled layout) of element type dtype."""
    import torch
    return torch.empty(population_elems(params), dtype=dtype, device=device)


def to_tiled(params, soa, device="cuda"):
    """A new tiled buffer holding the plain-layout populations `soa` ([37, Lx,
    Lz] numpy array or tensor; the element type is kept)."""
    import torch
    src = torch.as_tensor(soa).to(device).contiguous()
    out = empty_populations(params, src.dtype, device)
    lbm_pack(params, src, out)
    return out


def to_soa(params, tiled):
    """A new [37, Lx, Lz] tensor (same device and element type) holding the
    populations of the tiled buffer."""
    import torch
    out = torch.empty((Q, int(params.lx), int(params.lz)), dtype=tiled.dtype, device=tiled.device)
    lbm_unpack(params, tiled, out)
    return out


def tiled_view(params, t):
    """A [ceil(Lz / TILE), Lx, 37, TILE] view of a tiled population buffer."""
    return t.view(-(-int(params.lz) // TILE), int(params.lx), Q, TILE)


def column(params, t, x):
    """The populations of column x of a tiled buffer as a new [37, Lz] tensor."""
    v = tiled_view(params, t)[:, x]                       # [tiles, 37, TILE]
    return v.permute(1, 0, 2).reshape(Q, -1)[:, :int(params.lz)].contiguous()


def lbm_lattice():
    """(r, w [37], e [37, 2]) as compiled into the library."""
    r = ctypes.c_double()
    w = (ctypes.c_double * Q)()
    e = (ctypes.c_int32 * (2 * Q))()
    _check(load().lbm_lattice(ctypes.byref(r), w, e), "lbm_lattice")
    return r.value, np.array(w[:]), np.array(e[:], dtype=np.int64).reshape(Q, 2)


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def lbm_objective(params, desc, f, wk, wl, j_out, lam_seed=None, scratch=None, stream=None):
    """J = wk KE + wl (L_u + L_d) into j_out[5] = (J, KE, L_u + L_d, L_u, L_d) and
    optionally dJ/df (see include/lbm.h)."""
    _need("f", f, _state_dtype(params), population_elems(params))
    _need("j_out", j_out, _f64(), 5)
    _need("lam_seed", lam_seed, _lam_dtype(params), population_elems(params))
    st = load().lbm_objective(ctypes.byref(params), ctypes.byref(desc.c), _ptr(f), wk, wl,
                              _ptr(j_out), _ptr(lam_seed), _ptr(scratch), _nbytes(scratch),
                              _stream(stream))
    _check(st, "lbm_objective")


def lbm_adjoint_step(params, ghost, moments, lam_in, lam_out, stream=None):
    """lam_out = (d step / d f_in)^T lam_in (see include/lbm.h).  ``ghost`` is
    the forward step's wall table (needed with WALL_DIFFUSE, else may be None)."""
    _need("ghost", ghost, _state_dtype(params), 2 * 3 * Q)
    _need("moments", moments, _mom_dtype(params), 4 * _sites(params))
    _need("lam_in", lam_in, _lam_dtype(params), population_elems(params))
    _need("lam_out", lam_out, _lam_dtype(params), population_elems(params))
    st = load().lbm_adjoint_step(ctypes.byref(params), _ptr(ghost), _ptr(moments), _ptr(lam_in),
                                 _ptr(lam_out), _stream(stream))
    _check(st, "lbm_adjoint_step")


def lbm_adjoint_collide(params, moments, lam, mu, stream=None):
    """mu = C^T lam, the collision adjoint of one step alone (see include/lbm.h)."""
    _need("moments", moments, _mom_dtype(params), 4 * _sites(params))
    _need("lam", lam, _lam_dtype(params), population_elems(params))
    _need("mu", mu, _lam_dtype(params), population_elems(params))
    st = load().lbm_adjoint_collide(ctypes.byref(params), _ptr(moments), _ptr(lam), _ptr(mu), _stream(stream))
    _check(st, "lbm_adjoint_collide")


def lbm_adjoint_gather(params, ghost, moments, mu_in, mu_out, stream=None):
    """mu_out = C^T S^T mu_in (S^T alone with NO_COLLIDE), the gather form of
    the adjoint step (see include/lbm.h)."""
    _need("ghost", ghost, _state_dtype(params), 2 * 3 * Q)
    _need("moments", moments, _mom_dtype(params), 4 * _sites(params))
    _need("mu_in", mu_in, _lam_dtype(params), population_elems(params))
    _need("mu_out", mu_out, _lam_dtype(params), population_elems(params))
    st = load().lbm_adjoint_gather(ctypes.byref(params), _ptr(ghost), _ptr(moments), _ptr(mu_in), _ptr(mu_out),
                                   _stream(stream))
    _check(st, "lbm_adjoint_gather")


def lbm_init_rt3_vjp(params, desc, amp, lam0, d_amp, scratch, stream=None):
    """d_amp = (d init / d amp)^T lam0 (see include/lbm.h)."""
    _need("amp", amp, _f64(), 2 * desc.nmodes)
    _need("lam0", lam0, _lam_dtype(params), population_elems(params))
    _need("d_amp", d_amp, _f64(), 2 * desc.nmodes)
    st = load().lbm_init_rt3_vjp(ctypes.byref(params), ctypes.byref(desc.c), _ptr(amp), _ptr(lam0),
                                 _ptr(d_amp), _ptr(scratch), _nbytes(scratch), _stream(stream))
    _check(st, "lbm_init_rt3_vjp")


def lbm_profiles(params, f, prof, scratch, stream=None):
    """Row means and rms fluctuations of T^H and E_k into prof [4, Lz] (see include/lbm.h)."""
    _need("f", f, _state_dtype(params), population_elems(params))
    _need("prof", prof, _f64(), 4 * int(params.lz))
    st = load().lbm_profiles(ctypes.byref(params), _ptr(f), _ptr(prof), _ptr(scratch),
                             _nbytes(scratch), _stream(stream))
    _check(st, "lbm_profiles")
