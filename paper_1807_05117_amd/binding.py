"""Thin ctypes binding of libbl_lddmm.so with the names of the C interface (bl_lddmm.h).

Argument marshalling only: every step of the computation runs in the library's HIP
kernels.  Host mode takes NumPy arrays; device mode (`device=True`) takes torch CUDA
tensors and a torch stream, whose raw pointers are handed to the library.

Arrays: images are float32 of shape ([Nz,] Ny, Nx); band vectors are complex64 of shape
(dim, [Kz,] Ky, Kx) in centred order (index j stands for frequency j - K/2), with a leading
time-node axis (nt + 1, ...) for a non-stationary velocity.  complex64
memory is the interleaved (re, im) float32 layout of the interface.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbl_lddmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "bl_lddmm.h")

BL_OK, BL_E_INVALID, BL_E_UNSUPPORTED, BL_E_NOMEM, BL_E_DEVICE, BL_E_NONFINITE = 0, -1, -2, -3, -4, -5
BL_PENDING, BL_E_CANCELLED = 1, -6
BL_FP32, BL_MIXED = 0, 1
BL_DEVICE_PTRS = 1
BL_NEWTON = 2
BL_NONSTATIONARY = 4
BL_DEFORMATION = 8
BL_CONVERGED, BL_MAXITER, BL_STALLED = 0, 1, 2
BL_MAX_GN = 64
FIELDS = {"velocity": 0, "div": 1, "X": 2, "Y": 3, "a": 4, "state": 5}


class BLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bl_lddmm error {code}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("k", C.c_int32 * 3),
                ("nt", C.c_int32), ("alpha", C.c_double), ("s", C.c_int32),
                ("sigma", C.c_double), ("gamma", C.c_int32), ("precision", C.c_int32),
                ("flags", C.c_int32), ("stream", C.c_void_p)]


class SolverOpts(C.Structure):
    _fields_ = [("max_gn", C.c_int32), ("max_pcg", C.c_int32), ("gtol", C.c_double),
                ("c1", C.c_double), ("max_halvings", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("gn_iters", C.c_int32), ("hessvecs", C.c_int32),
                ("gradients", C.c_int32), ("evaluations", C.c_int32), ("pcg_total", C.c_int32),
                ("E", C.c_double * (BL_MAX_GN + 1)), ("mse_rel", C.c_double * (BL_MAX_GN + 1)),
                ("ginf_rel", C.c_double * (BL_MAX_GN + 1)), ("pcg_iters", C.c_int32 * BL_MAX_GN),
                ("ls_trials", C.c_int32 * BL_MAX_GN), ("eps", C.c_double * BL_MAX_GN),
                ("seconds", C.c_double)]

    def to_dict(self):
        k = self.gn_iters
        nit = k + (1 if self.status == BL_STALLED else 0)
        return {"status": self.status, "gn_iters": k, "hessvecs": self.hessvecs,
                "gradients": self.gradients, "evaluations": self.evaluations,
                "pcg_total": self.pcg_total, "E": list(self.E[:k + 1]),
                "mse_rel": list(self.mse_rel[:k + 1]), "ginf_rel": list(self.ginf_rel[:k + 1]),
                "pcg_iters": list(self.pcg_iters[:nit]), "ls_trials": list(self.ls_trials[:nit]),
                "eps": list(self.eps[:nit]), "seconds": self.seconds}


class RequestTimes(C.Structure):
    _fields_ = [("submitted", C.c_double), ("admitted", C.c_double), ("finished", C.c_double),
                ("slot", C.c_int32)]


class ServerInfo(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("peak_bytes", C.c_uint64),
                ("max_slots", C.c_int32), ("peak_resident", C.c_int32),
                ("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("cancelled", C.c_int64)]


_lib = None
_P = C.c_void_p


def load():
    """Load the library (fails loudly when it has not been built).

    torch wheels ship their own HIP runtime under the same soname as /opt/rocm's.  Two
    runtimes in one process cannot share the GPU, so torch is imported first: the library's
    libamdhip64.so.7 dependency then resolves to the runtime torch already loaded and device
    pointers, streams and events are shared.
    """
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1807_05117_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    PP = C.POINTER(Problem)
    sig = {
        "bl_lddmm_gradient": (C.c_int, [PP, _P, _P, _P, _P, C.POINTER(C.c_double)]),
        "bl_lddmm_hessvec": (C.c_int, [PP, _P, _P, _P, _P, _P]),
        "bl_lddmm_hessvec_noalloc": (C.c_int, [PP, _P, _P, _P, _P, _P]),
        "bl_lddmm_noalloc_limit": (C.c_uint64, []),
        "bl_lddmm_register": (C.c_int, [PP, C.POINTER(SolverOpts), _P, _P, _P, _P, C.POINTER(Stats)]),
        "bl_lddmm_warp": (C.c_int, [PP, _P, _P, _P]),
        "bl_band_to_grid": (C.c_int, [PP, C.c_int32, _P, _P]),
        "bl_grid_to_band": (C.c_int, [PP, C.c_int32, _P, _P]),
        "bl_lddmm_ctx_create": (C.c_int, [PP, _P, _P, C.POINTER(C.c_void_p)]),
        "bl_lddmm_ctx_set_velocity": (C.c_int, [_P, _P, C.POINTER(C.c_double), _P]),
        "bl_lddmm_ctx_hessvec": (C.c_int, [_P, _P, _P]),
        "bl_lddmm_ctx_get_field": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
        "bl_lddmm_ctx_destroy": (None, [_P]),
        "bl_lddmm_footprint": (C.c_uint64, [PP]),
        "bl_lddmm_release_cached": (None, []),
        "bl_lddmm_tune_reload": (None, []),
        "bl_lddmm_last_error": (C.c_char_p, []),
        "bl_lddmm_device_count": (C.c_int, []),
        "bl_lddmm_default_opts": (None, [C.POINTER(SolverOpts)]),
        "bl_kernel_timing_enable": (C.c_int, [_P, C.c_int32]),
        "bl_kernel_timing_read": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
        "bl_lddmm_ctx_launch_shapes": (C.c_int, [_P, C.POINTER(C.c_int32)]),
        "bl_server_create": (C.c_int, [C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
        "bl_server_create_batched": (C.c_int, [C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
        "bl_server_submit": (C.c_int, [_P, PP, C.POINTER(SolverOpts), _P, _P, _P,
                                       C.POINTER(C.c_uint64)]),
        "bl_server_wait": (C.c_int, [_P, C.c_uint64, C.c_double, _P, _P, C.POINTER(Stats),
                                     C.POINTER(RequestTimes)]),
        "bl_server_cancel": (C.c_int, [_P, C.c_uint64]),
        "bl_server_info_get": (C.c_int, [_P, C.POINTER(ServerInfo)]),
        "bl_server_destroy": (None, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def header_functions():
    """Names of the functions declared in include/bl_lddmm.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int|void|uint64_t)\s+\**\s*(bl_\w+)\s*\(",
                                 txt, flags=re.M)))


def device_available() -> bool:
    return load().bl_lddmm_device_count() > 0


def _check(rc):
    if rc != BL_OK:
        raise BLError(rc, load().bl_lddmm_last_error().decode())


def make_problem(dim, n, k, nt, alpha=1e-3, s=2, sigma=1.0, gamma=0, precision=BL_FP32,
                 device=False, stream=None, newton=False, nonstationary=False,
                 deformation=False) -> Problem:
    p = Problem()
    p.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    kk = list(k) + [1] * (3 - len(k))
    for j in range(3):
        p.n[j] = int(nn[j])
        p.k[j] = int(kk[j])
    p.nt, p.alpha, p.s, p.sigma = int(nt), float(alpha), int(s), float(sigma)
    p.gamma, p.precision = int(gamma), int(precision)
    p.flags = ((BL_DEVICE_PTRS if device else 0) | (BL_NEWTON if newton else 0)
               | (BL_NONSTATIONARY if nonstationary else 0)
               | (BL_DEFORMATION if deformation else 0))
    p.stream = C.c_void_p(stream) if stream else None
    return p


def grid_shape(p: Problem):
    return tuple(int(p.n[j]) for j in reversed(range(p.dim)))


def band_shape(p: Problem):
    """(dim, band...) of a velocity; (nt + 1, dim, band...) for a non-stationary one"""
    shape = (p.dim,) + tuple(int(p.k[j]) for j in reversed(range(p.dim)))
    return ((int(p.nt) + 1,) + shape) if (p.flags & BL_NONSTATIONARY) else shape


def _f32(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _c64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex64)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


def _tptr(t):
    return C.c_void_p(t.data_ptr())


def opts_struct(max_gn=10, max_pcg=10, gtol=1e-3, c1=1e-4, max_halvings=10) -> SolverOpts:
    o = SolverOpts()
    o.max_gn, o.max_pcg, o.gtol, o.c1, o.max_halvings = max_gn, max_pcg, gtol, c1, max_halvings
    return o


# ----------------------------------------------------------------------------- host calls
def bl_lddmm_gradient(p, I0, I1, v_hat):
    lib = load()
    I0 = _f32(I0, grid_shape(p))
    I1 = _f32(I1, grid_shape(p))
    v = _c64(v_hat, band_shape(p))
    g = np.empty(band_shape(p), np.complex64)
    E = C.c_double()
    _check(lib.bl_lddmm_gradient(C.byref(p), _ptr(I0), _ptr(I1), _ptr(v), _ptr(g), C.byref(E)))
    return g, E.value


def bl_lddmm_hessvec(p, I0, I1, v_hat, dv_hat):
    lib = load()
    I0 = _f32(I0, grid_shape(p))
    I1 = _f32(I1, grid_shape(p))
    v = _c64(v_hat, band_shape(p))
    d = _c64(dv_hat, band_shape(p))
    h = np.empty(band_shape(p), np.complex64)
    _check(lib.bl_lddmm_hessvec(C.byref(p), _ptr(I0), _ptr(I1), _ptr(v), _ptr(d), _ptr(h)))
    return h


def bl_lddmm_hessvec_noalloc(p, I0, I1, v_hat, dv_hat):
    """bl_lddmm_hessvec in the library's fixed device scratch array (allocates nothing)"""
    lib = load()
    I0 = _f32(I0, grid_shape(p))
    I1 = _f32(I1, grid_shape(p))
    v = _c64(v_hat, band_shape(p))
    d = _c64(dv_hat, band_shape(p))
    h = np.empty(band_shape(p), np.complex64)
    _check(lib.bl_lddmm_hessvec_noalloc(C.byref(p), _ptr(I0), _ptr(I1), _ptr(v), _ptr(d),
                                        _ptr(h)))
    return h


def bl_lddmm_noalloc_limit():
    return int(load().bl_lddmm_noalloc_limit())


def bl_lddmm_register(p, I0, I1, v0, opts=None):
    lib = load()
    I0 = _f32(I0, grid_shape(p))
    I1 = _f32(I1, grid_shape(p))
    v = _c64(v0, band_shape(p)).copy()
    w = np.empty(grid_shape(p), np.float32)
    st = Stats()
    o = opts if opts is not None else opts_struct()
    _check(lib.bl_lddmm_register(C.byref(p), C.byref(o), _ptr(I0), _ptr(I1), _ptr(v), _ptr(w),
                                 C.byref(st)))
    return v, w, st.to_dict()


def bl_lddmm_register_device(p, I0, I1, v, warped=None, opts=None):
    """bl_lddmm_register on device memory (p made with device=True): I0, I1, warped are torch
    float32 tensors of the grid shape, v a complex64 tensor of the band shape, updated in
    place; stream-ordered on p.stream, and the call returns after its work is complete."""
    lib = load()
    for t in (I0, I1, v) + ((warped,) if warped is not None else ()):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("device tensors must be contiguous GPU tensors")
    st = Stats()
    o = opts if opts is not None else opts_struct()
    _check(lib.bl_lddmm_register(C.byref(p), C.byref(o), _tptr(I0), _tptr(I1), _tptr(v),
                                 _tptr(warped) if warped is not None else None, C.byref(st)))
    return st.to_dict()


def bl_lddmm_release_cached():
    load().bl_lddmm_release_cached()


def bl_lddmm_warp(p, I0, v_hat):
    lib = load()
    I0 = _f32(I0, grid_shape(p))
    v = _c64(v_hat, band_shape(p))
    w = np.empty(grid_shape(p), np.float32)
    _check(lib.bl_lddmm_warp(C.byref(p), _ptr(I0), _ptr(v), _ptr(w)))
    return w


def bl_band_to_grid(p, band):
    lib = load()
    band = np.ascontiguousarray(band, dtype=np.complex64)
    nc = band.shape[0]
    if band.shape[1:] != band_shape(p)[-p.dim:]:
        raise ValueError("band shape mismatch")
    out = np.empty((nc,) + grid_shape(p), np.float32)
    _check(lib.bl_band_to_grid(C.byref(p), nc, _ptr(band), _ptr(out)))
    return out


def bl_grid_to_band(p, grid):
    lib = load()
    grid = np.ascontiguousarray(grid, dtype=np.float32)
    nc = grid.shape[0]
    if grid.shape[1:] != grid_shape(p):
        raise ValueError("grid shape mismatch")
    out = np.empty((nc,) + band_shape(p)[-p.dim:], np.complex64)
    _check(lib.bl_grid_to_band(C.byref(p), nc, _ptr(grid), _ptr(out)))
    return out


def bl_lddmm_footprint(p) -> int:
    return int(load().bl_lddmm_footprint(C.byref(p)))


# ----------------------------------------------------------------------------- contexts
class Ctx:
    """A device context (bl_lddmm_ctx_*).  Host mode: NumPy in/out.  Device mode: torch
    tensors on the GPU, work ordered on the problem's stream."""

    def __init__(self, p: Problem, I0, I1):
        self.lib = load()
        self.p = p
        self.device = bool(p.flags & BL_DEVICE_PTRS)
        h = C.c_void_p()
        if self.device:
            self._keep = (I0, I1)
            _check(self.lib.bl_lddmm_ctx_create(C.byref(p), _tptr(I0), _tptr(I1), C.byref(h)))
        else:
            I0 = _f32(I0, grid_shape(p))
            I1 = _f32(I1, grid_shape(p))
            _check(self.lib.bl_lddmm_ctx_create(C.byref(p), _ptr(I0), _ptr(I1), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.bl_lddmm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bl_lddmm_ctx_set_velocity(self, v_hat, want_gradient=True):
        E = C.c_double()
        if self.device:
            import torch
            g = torch.empty_like(v_hat) if want_gradient else None
            _check(self.lib.bl_lddmm_ctx_set_velocity(self.h, _tptr(v_hat), C.byref(E),
                                                      _tptr(g) if g is not None else None))
            return E.value, g
        v = _c64(v_hat, band_shape(self.p))
        g = np.empty(band_shape(self.p), np.complex64) if want_gradient else None
        _check(self.lib.bl_lddmm_ctx_set_velocity(self.h, _ptr(v), C.byref(E),
                                                  _ptr(g) if g is not None else None))
        return E.value, g

    def bl_lddmm_ctx_hessvec(self, dv_hat, out=None):
        if self.device:
            import torch
            out = torch.empty_like(dv_hat) if out is None else out
            _check(self.lib.bl_lddmm_ctx_hessvec(self.h, _tptr(dv_hat), _tptr(out)))
            return out
        d = _c64(dv_hat, band_shape(self.p))
        out = np.empty(band_shape(self.p), np.complex64)
        _check(self.lib.bl_lddmm_ctx_hessvec(self.h, _ptr(d), _ptr(out)))
        return out

    def bl_lddmm_ctx_get_field(self, which, index=0):
        w = FIELDS[which] if isinstance(which, str) else int(which)
        if self.device:
            import torch
            out = torch.empty(grid_shape(self.p), dtype=torch.float32, device="cuda")
            _check(self.lib.bl_lddmm_ctx_get_field(self.h, w, index, _tptr(out)))
            return out
        out = np.empty(grid_shape(self.p), np.float32)
        _check(self.lib.bl_lddmm_ctx_get_field(self.h, w, index, _ptr(out)))
        return out

    def bl_kernel_timing_enable(self, on=True):
        _check(self.lib.bl_kernel_timing_enable(self.h, 1 if on else 0))

    def bl_kernel_timing_read(self, kclass):
        n = C.c_int64()
        ms = C.c_double()
        _check(self.lib.bl_kernel_timing_read(self.h, kclass, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def bl_lddmm_ctx_launch_shapes(self):
        """voxels per thread along z of the transport launches: state, incremental, adjoint,
        body force"""
        out = (C.c_int32 * 4)()
        _check(self.lib.bl_lddmm_ctx_launch_shapes(self.h, out))
        return tuple(out)


# ----------------------------------------------------------------------------- serving
class Server:
    """The registration request loop (bl_server_*): submit returns a ticket immediately;
    wait returns (rc, v_hat, warped, stats, times).  batched=True: the cohort engine
    (bl_server_create_batched, max_slots = pairs per cohort)."""

    def __init__(self, budget_bytes=0, max_slots=4, batched=False):
        self.lib = load()
        h = C.c_void_p()
        create = self.lib.bl_server_create_batched if batched else self.lib.bl_server_create
        _check(create(int(budget_bytes), int(max_slots), C.byref(h)))
        self.h = h
        self._shapes = {}

    def submit(self, p, I0, I1, v0=None, opts=None):
        I0 = _f32(I0, grid_shape(p))
        I1 = _f32(I1, grid_shape(p))
        v = _c64(v0, band_shape(p)) if v0 is not None else None
        t = C.c_uint64()
        o = C.byref(opts) if opts is not None else None
        _check(self.lib.bl_server_submit(self.h, C.byref(p), o, _ptr(I0), _ptr(I1),
                                         _ptr(v) if v is not None else None, C.byref(t)))
        self._shapes[t.value] = (grid_shape(p), band_shape(p))
        return t.value

    def wait(self, ticket, timeout=-1.0):
        gs, bs = self._shapes[ticket]
        v = np.empty(bs, np.complex64)
        w = np.empty(gs, np.float32)
        st = Stats()
        tm = RequestTimes()
        rc = self.lib.bl_server_wait(self.h, ticket, float(timeout), _ptr(v), _ptr(w),
                                     C.byref(st), C.byref(tm))
        if rc == BL_PENDING:
            return rc, None, None, None, None
        self._shapes.pop(ticket, None)
        times = {"submitted": tm.submitted, "admitted": tm.admitted, "finished": tm.finished,
                 "slot": tm.slot}
        if rc != BL_OK:
            return rc, None, None, None, times
        return rc, v, w, st.to_dict(), times

    def cancel(self, ticket):
        return self.lib.bl_server_cancel(self.h, ticket)

    def info(self):
        i = ServerInfo()
        _check(self.lib.bl_server_info_get(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.bl_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
