"""Python access to the FP64 reference of MinxEnt-LBM in ``lbm_oracle.c``.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark import this module; the product library
never does.  It shares nothing with the HIP library: the C source is compiled
here with gcc into ``oracle/liboracle.so``.

Every function is a thin ctypes shim over the C routine of the same name
without the ``orc_`` prefix; the paper passage each one follows is cited in
the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Enumerations of lbm_oracle.c.
D1Q3, D2Q9 = 1, 2
MINXENT4, MINXENT2, SRT, TRT, MRT, CONVERGED4 = 0, 1, 2, 3, 4, 5
BC_PERIODIC, BC_TUBE, BC_CAVITY, BC_BOX = 0, 1, 2, 3

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (single-threaded, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *GCC_FLAGS, "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("tau2", ctypes.c_double),
        ("u_lid", ctypes.c_double),
        ("rho0", ctypes.c_double),
    ]


class Status(ctypes.Structure):
    _fields_ = [
        ("unstable", ctypes.c_int32),
        ("first_step", ctypes.c_int32),
        ("guarded", ctypes.c_int64),
        ("first_node", ctypes.c_int64),
        ("min_post", ctypes.c_double),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(LIB)
        lib.orc_constants.argtypes = [_D, _D, _D, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        lib.orc_feq_d2q9.argtypes = [ctypes.c_double] * 3 + [_D]
        lib.orc_feq_d1q3.argtypes = [ctypes.c_double] * 2 + [_D]
        lib.orc_kld_d2q9.argtypes = [_D]
        lib.orc_kld_d2q9.restype = ctypes.c_double
        lib.orc_collide_minxent.argtypes = [_D, ctypes.c_double, ctypes.c_double, ctypes.c_int, _D]
        lib.orc_collide_minxent.restype = ctypes.c_int
        lib.orc_minxent_start.argtypes = [_D, ctypes.c_double, ctypes.c_double, ctypes.c_int, _D]
        lib.orc_converged_minxent.argtypes = [_D, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_double, _D]
        lib.orc_converged_minxent.restype = ctypes.c_int
        lib.orc_collide_srt_d2q9.argtypes = [_D, ctypes.c_double, _D]
        lib.orc_collide_mrt_d2q9.argtypes = [_D, _D, _D]
        lib.orc_collide_srt_d1q3.argtypes = [_D, ctypes.c_double, _D]
        lib.orc_collide_moment_d1q3.argtypes = [_D, ctypes.c_double, _D]
        lib.orc_collide_node.argtypes = [ctypes.POINTER(Params), _D, _D]
        lib.orc_collide_node.restype = ctypes.c_int
        lib.orc_run_window.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _D, _D, _D, ctypes.c_int64, _D, _D, _D, _D,
                                       ctypes.POINTER(Status)]
        lib.orc_run_window.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    assert a.shape == (n,), a.shape
    return a


def constants():
    """(T, T^{-1}, W, vx, vy) with populations in T's column order."""
    lib = _load()
    t = np.zeros(81)
    ti = np.zeros(81)
    w = np.zeros(9)
    vx = (ctypes.c_int * 9)()
    vy = (ctypes.c_int * 9)()
    lib.orc_constants(_ptr(t), _ptr(ti), _ptr(w), vx, vy)
    return t.reshape(9, 9), ti.reshape(9, 9), w, np.array(list(vx)), np.array(list(vy))


def feq_d2q9(rho, ux, uy):
    out = np.zeros(9)
    _load().orc_feq_d2q9(rho, ux, uy, _ptr(out))
    return out


def feq_d1q3(rho, ux):
    out = np.zeros(3)
    _load().orc_feq_d1q3(rho, ux, _ptr(out))
    return out


def kld(p):
    return _load().orc_kld_d2q9(_ptr(_vec(p, 9)))


def collide_minxent(f, tau, tau2=0.0, variant=4):
    """Single-step MinxEnt collision; returns (f_post, guarded)."""
    out = np.zeros(9)
    g = _load().orc_collide_minxent(_ptr(_vec(f, 9)), tau, tau2, variant, _ptr(out))
    return out, bool(g)


def minxent_start(f, tau, tau2=0.0, variant=4):
    out = np.zeros(9)
    _load().orc_minxent_start(_ptr(_vec(f, 9)), tau, tau2, variant, _ptr(out))
    return out


def converged_minxent(f, tau, tau2=0.0, variant=4, maxit=200, tol=1e-16):
    """Converged constrained minimiser (long double damped Newton)."""
    out = np.zeros(9)
    it = _load().orc_converged_minxent(_ptr(_vec(f, 9)), tau, tau2, variant, maxit, tol, _ptr(out))
    if it < 0:
        raise RuntimeError("converged minimiser did not converge")
    return out, it


def collide_srt_d2q9(f, tau):
    out = np.zeros(9)
    _load().orc_collide_srt_d2q9(_ptr(_vec(f, 9)), tau, _ptr(out))
    return out


def collide_mrt_d2q9(f, b):
    out = np.zeros(9)
    _load().orc_collide_mrt_d2q9(_ptr(_vec(f, 9)), _ptr(_vec(b, 9)), _ptr(out))
    return out


def collide_srt_d1q3(f, tau):
    out = np.zeros(3)
    _load().orc_collide_srt_d1q3(_ptr(_vec(f, 3)), tau, _ptr(out))
    return out


def collide_moment_d1q3(f, tau):
    out = np.zeros(3)
    _load().orc_collide_moment_d1q3(_ptr(_vec(f, 3)), tau, _ptr(out))
    return out


def collide_node(collision, f, tau, tau2=0.0, lattice=D2Q9):
    """The fluid collision a whole run applies at one node (rule, tau, tau2);
    returns (f_post, guarded)."""
    b = 3 if lattice == D1Q3 else 9
    P = Params(lattice, collision, BC_PERIODIC, 0, 3, 1 if lattice == D1Q3 else 3, tau, tau2, 0.0, 1.0)
    out = np.zeros(b)
    g = _load().orc_collide_node(ctypes.byref(P), _ptr(_vec(f, b)), _ptr(out))
    return out, bool(g)


def run(lattice, collision, bc, nx, ny, tau, rho, ux, uy=None, steps=1, tau2=0.0, u_lid=0.0,
        rho0=1.0, window=None, want_f=False):
    """Run a whole lattice (or a window (x0, y0, wx, wy) of it) for `steps`
    steps from the equilibrium of (rho, ux, uy).  Input arrays cover the
    window, shape (wy, wx) (or (wx,) for D1Q3).  Returns a dict with rho, ux,
    uy, status fields and optionally f (b, wy, wx)."""
    lib = _load()
    if lattice == D1Q3:
        ny = 1
    if window is None:
        window = (0, 0, nx, ny)
    x0, y0, wx, wy = window
    n = wx * wy
    r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(n))
    u = np.ascontiguousarray(np.asarray(ux, dtype=np.float64).reshape(n))
    v = np.ascontiguousarray(np.zeros(n) if uy is None else np.asarray(uy, dtype=np.float64).reshape(n))
    P = Params(lattice, collision, bc, 0, nx, ny, tau, tau2, u_lid, rho0)
    b = 3 if lattice == D1Q3 else 9
    ro, uo, vo = np.zeros(n), np.zeros(n), np.zeros(n)
    fo = np.zeros(b * n) if want_f else None
    st = Status()
    rc = lib.orc_run_window(ctypes.byref(P), x0, y0, wx, wy, _ptr(r), _ptr(u), _ptr(v), int(steps),
                            _ptr(ro), _ptr(uo), _ptr(vo), _ptr(fo), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle run rejected its parameters")
    shape = (wx,) if lattice == D1Q3 else (wy, wx)
    out = {"rho": ro.reshape(shape), "ux": uo.reshape(shape), "uy": vo.reshape(shape),
           "unstable": bool(st.unstable), "first_step": st.first_step, "first_node": st.first_node,
           "guarded": st.guarded, "min_post": st.min_post}
    if want_f:
        out["f"] = fo.reshape((b,) + shape)
    return out
