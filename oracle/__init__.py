"""FP64 CPU oracle for the ghost-gluon Dyson-Schwinger system (arXiv:1206.1779).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the HIP
library is checked against.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
does, and the two share no code.

The numerics live in ``dse_ref.c`` (plain C, double precision, compensated sums
in a fixed order).  This module compiles it with gcc and wraps it with ctypes;
every wrapper only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dse_ref.c")
_LIB = os.path.join(_HERE, "libdse_ref.so")
_LIB_NATIVE = os.path.join(_HERE, "libdse_ref_native.so")


_NATIVE_FLAGS = ["-O3", "-march=native", "-ffp-contract=off"]
_native = False


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle into ``oracle/libdse_ref.so`` (gcc, -O2, OpenMP).

    No -ffast-math (it would undo the compensated sums) and no -march=native
    (the library is built here and may run on another host).  native: a second
    library, ``oracle/libdse_ref_native.so``, for the host it is built on
    (-O3 -march=native, FMA contraction off so that the arithmetic stays that
    of the -O2 build); the CPU baseline is timed with it."""
    out = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        flags = _NATIVE_FLAGS if native else ["-O2"]
        cmd = ["gcc"] + flags + ["-std=c11", "-fPIC", "-shared", "-fopenmp",
                                 "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


def use_native_build() -> str:
    """Build the host-tuned library and load it instead of the portable one
    (before any other call of this module in the process); returns the
    compiler flags in use."""
    global _native
    if _lib is not None:
        raise RuntimeError("the oracle library is loaded already")
    build(force=True, native=True)
    _native = True
    return " ".join(["gcc"] + _NATIVE_FLAGS + ["-fopenmp"])


class Params(C.Structure):
    _fields_ = [
        ("n_z", C.c_int32), ("n_g", C.c_int32), ("n_rad", C.c_int32),
        ("n_ir", C.c_int32), ("n_ang", C.c_int32), ("quad", C.c_int32),
        ("eps2", C.c_double), ("lambda2", C.c_double), ("ir_efolds", C.c_double),
        ("alpha_mu", C.c_double), ("n_c", C.c_double), ("g0_inv", C.c_double),
        ("z_lambda_inv", C.c_double), ("kappa", C.c_double), ("delta", C.c_double),
        ("gamma", C.c_double),
    ]


class NewtonOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("extra_iters", C.c_int32),
                ("max_halvings", C.c_int32), ("pad_", C.c_int32), ("step_tol", C.c_double)]


class NewtonReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("fnorm", C.c_double),
                ("fnorm2", C.c_double), ("fnorm_hist", C.c_double * 128),
                ("relax_hist", C.c_double * 128)]


_lib = None
_D = C.POINTER(C.c_double)


def load():
    global _lib
    if _lib is None:
        path = _LIB_NATIVE if _native else _LIB
        if not os.path.exists(path):
            build(force=False, native=_native)
        lib = C.CDLL(path)
        P = C.POINTER(Params)
        sig = {
            "dse_ref_gauss_legendre": (C.c_int, [C.c_int, _D, _D]),
            "dse_ref_gl_node": (C.c_int, [C.c_int, C.c_int, _D, _D]),
            "dse_ref_renorm_scale": (C.c_int, [P, _D, C.c_int, _D]),
            "dse_ref_schwinger_nodes": (C.c_int, [C.c_int, C.c_double, _D, _D]),
            "dse_ref_schwinger": (C.c_int, [P, _D, C.c_int, C.c_double, _D, C.c_int, _D]),
            "dse_ref_cheb": (None, [C.c_double, C.c_int, _D]),
            "dse_ref_map": (C.c_double, [P, C.c_double]),
            "dse_ref_lnZ": (C.c_double, [P, _D, C.c_double]),
            "dse_ref_lnG": (C.c_double, [P, _D, C.c_double]),
            "dse_ref_kernel_Q_printed": (C.c_double, [C.c_double] * 3),
            "dse_ref_kernel_Q": (C.c_double, [C.c_double] * 3),
            "dse_ref_kernel_M_printed": (C.c_double, [C.c_double] * 3),
            "dse_ref_kernel_M": (C.c_double, [C.c_double] * 3),
            "dse_ref_momentum_z": (C.c_double, [C.c_double] * 3),
            "dse_ref_grid_sizes": (C.c_int, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "dse_ref_grid": (C.c_int, [P, _D, _D, _D, _D, _D, _D]),
            "dse_ref_row_grid": (C.c_int, [P, C.c_double, _D, _D]),
            "dse_ref_pi_gluon": (C.c_double, [P, _D, C.c_double, C.c_int, _D, _D, C.c_int, _D, _D]),
            "dse_ref_pi_ghost": (C.c_double, [P, _D, C.c_double, C.c_int, _D, _D, C.c_int, _D, _D]),
            "dse_ref_residual": (C.c_int, [P, _D, _D]),
            "dse_ref_residual_scale": (C.c_int, [P, _D, _D]),
            "dse_ref_jacobian": (C.c_int, [P, _D, _D, _D, C.c_int, C.POINTER(C.c_int32)]),
            "dse_ref_jacobian_fd": (C.c_int, [P, _D, C.c_double, _D]),
            "dse_ref_dF_dtheta": (C.c_int, [P, _D, _D]),
            "dse_ref_lu_solve": (C.c_int, [C.c_int, _D, _D, _D, C.c_int]),
            "dse_ref_start_guess": (C.c_int, [P, _D]),
            "dse_ref_newton": (C.c_int, [P, _D, C.POINTER(NewtonOpts), C.POINTER(NewtonReport)]),
            "dse_ref_set_order": (None, [C.c_int]),
            "dse_ref_set_jitter": (None, [C.c_double]),
            "dse_ref_set_threads": (None, [C.c_int]),
            "dse_ref_get_threads": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


# --------------------------------------------------------------------------- #
# parameters

#: (93 - sqrt(1201)) / 98, the IR exponent quoted as 0.595353 in Sec. 2
KAPPA = (93.0 - 1201.0 ** 0.5) / 98.0
DELTA = -9.0 / 44.0   # Sec. 2, ghost anomalous dimension
GAMMA = -13.0 / 22.0  # Sec. 2, gluon anomalous dimension

#: quadrature bits: tanh-sinh angular rule, radial split at x (Sec. 2, Sec. 3)
QUAD_TANH_SINH = 1
QUAD_SPLIT = 2

_DEFAULTS = dict(n_z=16, n_g=16, n_rad=64, n_ir=16, n_ang=16, quad=0, eps2=1e-6, lambda2=1e6,
                 ir_efolds=40.0, alpha_mu=1.0, n_c=3.0, g0_inv=0.0, z_lambda_inv=1.0,
                 kappa=KAPPA, delta=DELTA, gamma=GAMMA)


def params(**kw) -> Params:
    d = dict(_DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError("unknown parameter(s): %s" % sorted(unknown))
    d.update(kw)
    p = Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def n_unknowns(p: Params) -> int:
    return p.n_z + p.n_g


# --------------------------------------------------------------------------- #
# building blocks

def gauss_legendre(n: int):
    x = np.zeros(n); w = np.zeros(n)
    st = load().dse_ref_gauss_legendre(n, _arr(x)[1], _arr(w)[1])
    if st:
        raise ValueError("bad n")
    return x, w


def gl_node(n: int, i: int):
    """Node i (ascending) of the n-point rule and its weight, computed alone."""
    x = C.c_double(); w = C.c_double()
    if load().dse_ref_gl_node(n, i, C.byref(x), C.byref(w)):
        raise ValueError("bad n or i")
    return x.value, w.value


def cheb(s: float, n: int) -> np.ndarray:
    out = np.zeros(n)
    load().dse_ref_cheb(float(s), n, out.ctypes.data_as(_D))
    return out


def mapping(p: Params, u: float) -> float:
    return load().dse_ref_map(C.byref(p), float(u))


def lnZ(p: Params, a, u: float) -> float:
    a, pa = _arr(a)
    return load().dse_ref_lnZ(C.byref(p), pa, float(u))


def lnG(p: Params, b, u: float) -> float:
    b, pb = _arr(b)
    return load().dse_ref_lnG(C.byref(p), pb, float(u))


def running_coupling(p: Params, c, u: float) -> float:
    """alpha(u) = alpha(mu^2) G(u)^2 Z(u) (Sec. 2 running coupling), from the
    dressings lnG, lnZ above (series plus IR / UV extension)."""
    c = np.asarray(c, dtype=np.float64)
    return p.alpha_mu * math.exp(2.0 * lnG(p, c[p.n_z:], u) + lnZ(p, c[:p.n_z], u))


def renorm_scale(p: Params, c, scan: int = 4096) -> float:
    """mu^2 with G^2(mu^2) Z(mu^2) = 1 (Sec. 2.1 footnote), the largest root in
    [eps2, lambda2]; NaN when there is none."""
    c, pc = _arr(c)
    mu2 = C.c_double()
    load().dse_ref_renorm_scale(C.byref(p), pc, int(scan), C.byref(mu2))
    return mu2.value


def schwinger_nodes(n: int, p_max: float):
    """The mapped rule of the Schwinger function: p_i = p_max ((1 + x_i)/2)^2
    and weights W_i over the n Gauss-Legendre nodes x_i."""
    pn = np.zeros(n); W = np.zeros(n)
    _check(load().dse_ref_schwinger_nodes(n, float(p_max), pn.ctypes.data_as(_D), W.ctypes.data_as(_D)),
           "schwinger_nodes")
    return pn, W


def schwinger(p: Params, c, t, n: int = 1 << 17, p_max: float = 1e3) -> np.ndarray:
    """Delta(t) = (1/pi) int_0^p_max dp cos(t p) Z(p^2)/p^2 (Sec. 2.2) at each t."""
    c, pc = _arr(c)
    t, pt = _arr(np.atleast_1d(t))
    out = np.zeros(len(t))
    _check(load().dse_ref_schwinger(C.byref(p), pc, int(n), float(p_max), pt, len(t), out.ctypes.data_as(_D)),
           "schwinger")
    return out


def kernel_Q(x, y, theta):
    return load().dse_ref_kernel_Q(float(x), float(y), float(theta))


def kernel_Q_printed(x, y, z):
    return load().dse_ref_kernel_Q_printed(float(x), float(y), float(z))


def kernel_M(x, y, theta):
    return load().dse_ref_kernel_M(float(x), float(y), float(theta))


def kernel_M_printed(x, y, z):
    return load().dse_ref_kernel_M_printed(float(x), float(y), float(z))


def momentum_z(x, y, theta):
    return load().dse_ref_momentum_z(float(x), float(y), float(theta))


@dataclass
class Grid:
    y: np.ndarray
    W: np.ndarray
    theta: np.ndarray
    v: np.ndarray
    x_z: np.ndarray
    x_g: np.ndarray


def grid(p: Params) -> Grid:
    nq = C.c_int32(); nk = C.c_int32()
    load().dse_ref_grid_sizes(C.byref(p), C.byref(nq), C.byref(nk))
    g = Grid(np.zeros(nq.value), np.zeros(nq.value), np.zeros(nk.value), np.zeros(nk.value),
             np.zeros(p.n_z), np.zeros(p.n_g))
    st = load().dse_ref_grid(C.byref(p), *[a.ctypes.data_as(_D) for a in
                                           (g.y, g.W, g.theta, g.v, g.x_z, g.x_g)])
    if st:
        raise ValueError("invalid parameters")
    return g


def row_grid(p: Params, x: float):
    """Radial nodes and weights of the row at x with the split at x (Sec. 3)."""
    m = p.n_ir + 2 * p.n_rad
    y = np.zeros(m); W = np.zeros(m)
    k = load().dse_ref_row_grid(C.byref(p), float(x), y.ctypes.data_as(_D), W.ctypes.data_as(_D))
    if k < 0:
        raise ValueError("invalid parameters")
    return y[:k], W[:k]


def pi_gluon(p: Params, c, x, y, W, theta, v) -> float:
    c, pc = _arr(c); y, py = _arr(y); W, pW = _arr(W); t, pt = _arr(theta); v, pv = _arr(v)
    return load().dse_ref_pi_gluon(C.byref(p), pc, float(x), len(y), py, pW, len(t), pt, pv)


def pi_ghost(p: Params, c, x, y, W, theta, v) -> float:
    c, pc = _arr(c); y, py = _arr(y); W, pW = _arr(W); t, pt = _arr(theta); v, pv = _arr(v)
    return load().dse_ref_pi_ghost(C.byref(p), pc, float(x), len(y), py, pW, len(t), pt, pv)


# --------------------------------------------------------------------------- #
# the method

class OracleError(RuntimeError):
    pass


def _check(st, what):
    if st:
        raise OracleError("%s failed with status %d" % (what, st))


def residual(p: Params, c) -> np.ndarray:
    c, pc = _arr(c)
    F = np.zeros(n_unknowns(p))
    _check(load().dse_ref_residual(C.byref(p), pc, F.ctypes.data_as(_D)), "residual")
    return F


def residual_scale(p: Params, c) -> np.ndarray:
    c, pc = _arr(c)
    S = np.zeros(n_unknowns(p))
    _check(load().dse_ref_residual_scale(C.byref(p), pc, S.ctypes.data_as(_D)), "residual_scale")
    return S


def jacobian(p: Params, c, rows=None, with_F: bool = False):
    c, pc = _arr(c)
    n = n_unknowns(p)
    J = np.full((n, n), np.nan) if rows is not None else np.zeros((n, n))
    F = np.zeros(n) if with_F else None
    if rows is not None:
        r = np.ascontiguousarray(rows, dtype=np.int32)
        rp, nr = r.ctypes.data_as(C.POINTER(C.c_int32)), len(r)
    else:
        r, rp, nr = None, None, 0
    st = load().dse_ref_jacobian(C.byref(p), pc, J.ctypes.data_as(_D),
                                 F.ctypes.data_as(_D) if with_F else None, nr, rp)
    _check(st, "jacobian")
    return (J, F) if with_F else J


def jacobian_fd(p: Params, c, h_rel: float = 1e-5) -> np.ndarray:
    c, pc = _arr(c)
    n = n_unknowns(p)
    J = np.zeros((n, n))
    _check(load().dse_ref_jacobian_fd(C.byref(p), pc, float(h_rel), J.ctypes.data_as(_D)),
           "jacobian_fd")
    return J


def dF_dtheta(p: Params, c) -> np.ndarray:
    """n x 3: derivatives of F with respect to (alpha_mu, g0_inv, z_lambda_inv)."""
    c, pc = _arr(c)
    out = np.zeros((n_unknowns(p), 3))
    _check(load().dse_ref_dF_dtheta(C.byref(p), pc, out.ctypes.data_as(_D)), "dF_dtheta")
    return out


def lu_solve(A, b, trans: bool = False) -> np.ndarray:
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    b = np.array(b, dtype=np.float64, copy=True)
    x = np.zeros_like(b)
    st = load().dse_ref_lu_solve(len(b), A.ctypes.data_as(_D), b.ctypes.data_as(_D),
                                 x.ctypes.data_as(_D), 1 if trans else 0)
    if st:
        raise OracleError("singular matrix")
    return x


def start_guess(p: Params) -> np.ndarray:
    c = np.zeros(n_unknowns(p))
    _check(load().dse_ref_start_guess(C.byref(p), c.ctypes.data_as(_D)), "start_guess")
    return c


def newton(p: Params, c0=None, tol=1e-10, max_iter=60, extra_iters=2, max_halvings=30,
           step_tol=1e-14):
    """Newton solve from c0 (default: the asymptotic start guess)."""
    if c0 is None:
        c0 = start_guess(p)
    c = np.array(c0, dtype=np.float64, copy=True)
    o = NewtonOpts(tol=tol, max_iter=max_iter, extra_iters=extra_iters,
                   max_halvings=max_halvings, step_tol=step_tol)
    rep = NewtonReport()
    load().dse_ref_newton(C.byref(p), c.ctypes.data_as(_D), C.byref(o), C.byref(rep))
    hist = list(rep.fnorm_hist[: rep.iters + 1])
    relax = list(rep.relax_hist[: rep.iters])
    return c, dict(iters=rep.iters, status=rep.status, fnorm=rep.fnorm, fnorm2=rep.fnorm2,
                   fnorm_hist=hist, relax_hist=relax)


def set_order(reversed_: bool):
    load().dse_ref_set_order(1 if reversed_ else 0)


def set_jitter(rel: float):
    load().dse_ref_set_jitter(float(rel))


def set_threads(n: int):
    load().dse_ref_set_threads(int(n))


def get_threads() -> int:
    return load().dse_ref_get_threads()
