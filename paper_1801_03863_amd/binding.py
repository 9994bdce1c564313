"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the method runs in the HIP library ``liblbm.so``; this module
only converts arguments.  torch is imported before the library is loaded so
that both use the one HIP runtime torch already holds; torch provides device
memory (workspaces) and streams.

If the library is not built, importing this module raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime first; see module doc)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("liblbm.so is not built; run __graft_entry__.build() (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

# Enumerations of lbm.h.
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ENODEV = 0, -1, -2, -3, -4
LBM_D1Q3, LBM_D2Q9 = 1, 2
LBM_MINXENT4, LBM_MINXENT2, LBM_SRT, LBM_TRT, LBM_MRT = 0, 1, 2, 3, 4
LBM_BC_PERIODIC, LBM_BC_TUBE, LBM_BC_CAVITY, LBM_BC_BOX = 0, 1, 2, 3
LBM_FP64, LBM_FP32_NEWTON64, LBM_FP32, LBM_FP16DEV = 0, 1, 2, 3
STATUS_UNSTABLE, STATUS_GUARDED = 1, 2

_NAMES = {
    "lattice": {"d1q3": LBM_D1Q3, "d2q9": LBM_D2Q9},
    "collision": {"minxent4": LBM_MINXENT4, "minxent2": LBM_MINXENT2, "srt": LBM_SRT, "trt": LBM_TRT,
                  "mrt": LBM_MRT},
    "bc": {"periodic": LBM_BC_PERIODIC, "tube": LBM_BC_TUBE, "cavity": LBM_BC_CAVITY, "box": LBM_BC_BOX},
    "precision": {"fp64": LBM_FP64, "fp32_newton64": LBM_FP32_NEWTON64, "fp32": LBM_FP32,
                  "fp16dev": LBM_FP16DEV},
}


class lbm_params_t(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("fp16_exp", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("tau2", ctypes.c_double),
        ("u_lid", ctypes.c_double),
        ("rho0", ctypes.c_double),
    ]


class lbm_status_t(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
        ("first_step", ctypes.c_int64),
        ("first_node", ctypes.c_int64),
        ("guarded", ctypes.c_int64),
    ]


_P = ctypes.POINTER(lbm_params_t)
_D = ctypes.POINTER(ctypes.c_double)
_V = ctypes.c_void_p
_I64 = ctypes.c_int64


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_sig("lbm_workspace_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)])
_sig("lbm_workspace_bytes_batch", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)])
_sig("lbm_init", ctypes.c_int, [_P, _D, _D, _D, _V, ctypes.c_size_t, _V, ctypes.POINTER(_V)])
_sig("lbm_init_batch", ctypes.c_int, [_P, ctypes.c_int32, _D, _D, _D, _V, ctypes.c_size_t, _V, ctypes.POINTER(_V)])
_sig("lbm_step", ctypes.c_int, [_V, _I64])
_sig("lbm_set_graph_chunk", ctypes.c_int, [_V, ctypes.c_int32])
_sig("lbm_autotune", ctypes.c_int, [_V, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)])
_sig("lbm_set_variant", ctypes.c_int, [_V, ctypes.c_int32])
_sig("lbm_variant_count", ctypes.c_int, [_V])
_sig("lbm_variant_name", ctypes.c_char_p, [_V, ctypes.c_int32])
_sig("lbm_variant_steps", ctypes.c_int, [_V, ctypes.c_int32])
_sig("lbm_set_plane_pad", ctypes.c_int, [_V, ctypes.c_int32])
_sig("lbm_set_batch_steps", ctypes.c_int, [_V, ctypes.POINTER(_I64), ctypes.c_int32])
_sig("lbm_get_layout", ctypes.c_int, [_V, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int32)])
_sig("lbm_moments", ctypes.c_int, [_V, _D, _D, _D])
_sig("lbm_get_populations", ctypes.c_int, [_V, _D])
_sig("lbm_set_populations", ctypes.c_int, [_V, _D])
_sig("lbm_status", ctypes.c_int, [_V, ctypes.POINTER(lbm_status_t)])
_sig("lbm_status_batch", ctypes.c_int, [_V, ctypes.POINTER(lbm_status_t), ctypes.c_int32])
_sig("lbm_reset_status", ctypes.c_int, [_V])
_sig("lbm_info", ctypes.c_int, [_V, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)])
_sig("lbm_free", None, [_V])
_sig("lbm_copy_kernel", ctypes.c_int, [_V, _V, ctypes.c_size_t, _V])
_sig("lbm_run_noalloc", ctypes.c_int, [_P, _V, _V, _V, _I64, _V, _V, _V, ctypes.POINTER(lbm_status_t), _V])
_sig("lbm_last_error", ctypes.c_char_p, [])
_sig("lbm_strerror", ctypes.c_char_p, [ctypes.c_int])


class LbmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.lbm_last_error().decode(errors="replace")
        super().__init__("%s failed: %s (%s)" % (where, _lib.lbm_strerror(code).decode(), msg))


def _check(rc, where):
    if rc != LBM_OK:
        raise LbmError(rc, where)


def _enum(kind, v):
    return _NAMES[kind][v] if isinstance(v, str) else int(v)


def make_params(lattice="d2q9", collision="minxent4", bc="cavity", precision="fp64", nx=16, ny=None, tau=0.6,
                tau2=0.0, u_lid=0.0, rho0=1.0, fp16_exp=0):
    lat = _enum("lattice", lattice)
    if ny is None:
        ny = 1 if lat == LBM_D1Q3 else nx
    return lbm_params_t(lat, _enum("collision", collision), _enum("bc", bc), _enum("precision", precision),
                        int(nx), int(ny), int(fp16_exp), 0, float(tau), float(tau2), float(u_lid), float(rho0))


def _ptr_or_none(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _f64(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def lbm_workspace_bytes(params):
    out = ctypes.c_size_t(0)
    _check(_lib.lbm_workspace_bytes(ctypes.byref(params), ctypes.byref(out)), "lbm_workspace_bytes")
    return out.value


def lbm_workspace_bytes_batch(params_list):
    arr = (lbm_params_t * len(params_list))(*params_list)
    out = ctypes.c_size_t(0)
    _check(_lib.lbm_workspace_bytes_batch(arr, len(params_list), ctypes.byref(out)), "lbm_workspace_bytes_batch")
    return out.value


def lbm_init(params, rho, ux, uy=None, workspace=None, stream=None):
    """Returns an opaque context handle.  workspace: a torch uint8 CUDA tensor
    (kept alive by the caller) or None; stream: torch stream, raw handle or
    None (torch's current stream)."""
    n = params.nx * params.ny
    r, u = _f64(rho, n), _f64(ux, n)
    v = _f64(uy, n) if uy is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    ctx = _V()
    rc = _lib.lbm_init(ctypes.byref(params), r.ctypes.data_as(_D), u.ctypes.data_as(_D),
                       v.ctypes.data_as(_D) if v is not None else None, _ptr_or_none(workspace), ws_bytes,
                       _stream_handle(stream), ctypes.byref(ctx))
    _check(rc, "lbm_init")
    return ctx


def lbm_init_batch(params_list, rho, ux, uy=None, workspace=None, stream=None):
    n = sum(p.nx * p.ny for p in params_list)
    arr = (lbm_params_t * len(params_list))(*params_list)
    r, u = _f64(rho, n), _f64(ux, n)
    v = _f64(uy, n) if uy is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    ctx = _V()
    rc = _lib.lbm_init_batch(arr, len(params_list), r.ctypes.data_as(_D), u.ctypes.data_as(_D),
                             v.ctypes.data_as(_D) if v is not None else None, _ptr_or_none(workspace), ws_bytes,
                             _stream_handle(stream), ctypes.byref(ctx))
    _check(rc, "lbm_init_batch")
    return ctx


def lbm_step(ctx, nsteps):
    _check(_lib.lbm_step(ctx, int(nsteps)), "lbm_step")


def lbm_set_graph_chunk(ctx, chunk):
    _check(_lib.lbm_set_graph_chunk(ctx, int(chunk)), "lbm_set_graph_chunk")


def lbm_autotune(ctx, cache_path=None):
    ch = ctypes.c_int32(-1)
    _check(_lib.lbm_autotune(ctx, cache_path.encode() if cache_path else None, ctypes.byref(ch)), "lbm_autotune")
    return ch.value


def lbm_set_variant(ctx, v):
    _check(_lib.lbm_set_variant(ctx, int(v)), "lbm_set_variant")


def lbm_variant_count(ctx):
    return _lib.lbm_variant_count(ctx)


def lbm_set_batch_steps(ctx, stop_steps):
    """Per-instance step limits of a batch (None removes them)."""
    if stop_steps is None:
        _check(_lib.lbm_set_batch_steps(ctx, None, 0), "lbm_set_batch_steps")
        return
    a = np.ascontiguousarray(np.asarray(stop_steps, dtype=np.int64))
    _check(_lib.lbm_set_batch_steps(ctx, a.ctypes.data_as(ctypes.POINTER(_I64)), len(a)), "lbm_set_batch_steps")


def lbm_set_plane_pad(ctx, pad_bytes):
    _check(_lib.lbm_set_plane_pad(ctx, int(pad_bytes)), "lbm_set_plane_pad")


def lbm_get_layout(ctx):
    """(plane stride in elements, plane pad in bytes or -1) of instance 0."""
    stride, pad = _I64(0), ctypes.c_int32(0)
    _check(_lib.lbm_get_layout(ctx, ctypes.byref(stride), ctypes.byref(pad)), "lbm_get_layout")
    return stride.value, pad.value


def lbm_variant_name(ctx, v):
    return _lib.lbm_variant_name(ctx, int(v)).decode()


def lbm_variant_steps(ctx, v):
    """Steps one launch of shape v takes at most (1; 2 for the temporally
    blocked D2Q9 shapes; up to 256 for the D1Q3 shapes that keep segments on
    chip)."""
    return _lib.lbm_variant_steps(ctx, int(v))


def lbm_info(ctx):
    s, n, b = _I64(), _I64(), _I64()
    _check(_lib.lbm_info(ctx, ctypes.byref(s), ctypes.byref(n), ctypes.byref(b)), "lbm_info")
    return {"steps_done": s.value, "nodes": n.value, "bytes_per_step": b.value}


def lbm_moments(ctx):
    """(rho, ux, uy) as flat float64 arrays over all nodes."""
    n = lbm_info(ctx)["nodes"]
    r, u, v = np.empty(n), np.empty(n), np.empty(n)
    _check(_lib.lbm_moments(ctx, r.ctypes.data_as(_D), u.ctypes.data_as(_D), v.ctypes.data_as(_D)), "lbm_moments")
    return r, u, v


def lbm_get_populations(ctx, b):
    n = lbm_info(ctx)["nodes"]
    f = np.empty(b * n)
    _check(_lib.lbm_get_populations(ctx, f.ctypes.data_as(_D)), "lbm_get_populations")
    return f


def lbm_set_populations(ctx, f):
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
    _check(_lib.lbm_set_populations(ctx, f.ctypes.data_as(_D)), "lbm_set_populations")


def _status_dict(s):
    return {"flags": s.flags, "unstable": bool(s.flags & STATUS_UNSTABLE), "guarded": s.guarded,
            "first_step": s.first_step, "first_node": s.first_node}


def lbm_status(ctx):
    s = lbm_status_t()
    _check(_lib.lbm_status(ctx, ctypes.byref(s)), "lbm_status")
    return _status_dict(s)


def lbm_status_batch(ctx, n):
    arr = (lbm_status_t * n)()
    _check(_lib.lbm_status_batch(ctx, arr, n), "lbm_status_batch")
    return [_status_dict(s) for s in arr]


def lbm_reset_status(ctx):
    _check(_lib.lbm_reset_status(ctx), "lbm_reset_status")


def lbm_free(ctx):
    _lib.lbm_free(ctx)


def lbm_copy_kernel(dst, src, nbytes, stream=None):
    _check(_lib.lbm_copy_kernel(_ptr_or_none(dst), _ptr_or_none(src), int(nbytes), _stream_handle(stream)),
           "lbm_copy_kernel")


NOALLOC_SCRATCH_BYTES = 64 << 20


def lbm_run_noalloc(params, rho, ux, uy, nsteps, rho_out, ux_out, uy_out, want_status=True, stream=None):
    """One single-lattice run with no allocation: fields in and out are torch
    float64 CUDA tensors of nx*ny values (uy / uy_out may be None for D1Q3).
    Returns the status dict (waits for the stream) or None."""
    st = lbm_status_t() if want_status else None
    rc = _lib.lbm_run_noalloc(ctypes.byref(params), _ptr_or_none(rho), _ptr_or_none(ux), _ptr_or_none(uy),
                              int(nsteps), _ptr_or_none(rho_out), _ptr_or_none(ux_out), _ptr_or_none(uy_out),
                              ctypes.byref(st) if st is not None else None, _stream_handle(stream))
    _check(rc, "lbm_run_noalloc")
    return _status_dict(st) if st is not None else None


def library_path():
    return LIB_PATH
