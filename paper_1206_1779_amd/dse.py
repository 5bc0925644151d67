"""Python binding of the C ABI in ``include/dse.h``.

Argument marshalling only: PyTorch provides device memory (the workspace and
the vectors) and the HIP stream; every computation runs in ``libdse.so``.  The
binding refuses to run without the HIP library and a GPU -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch  # loads the HIP runtime that libdse.so binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdse.so")

ABI_VERSION = 2
MAX_N = 128
QUAD_TANH_SINH = 1  # dse_params.quad bits (include/dse.h)
QUAD_SPLIT = 2

STATUS = {0: "ok", 1: "invalid argument", 2: "HIP device error", 3: "workspace too small",
          4: "singular Newton matrix", 5: "no convergence", 6: "non-finite"}

EXPORTS = [
    "dse_params_default", "dse_workspace_bytes", "dse_init", "dse_destroy", "dse_start_guess",
    "dse_residual", "dse_jacobian", "dse_jacobian_fd", "dse_running_coupling", "dse_dressing_vjp", "dse_newton_solve", "dse_lu_solve", "dse_status_string",
    "dse_last_error", "dse_sizes", "dse_set_timing", "dse_read_timings", "dse_vjp",
    "dse_set_physics", "dse_newton_step", "dse_set_graphs",
    "dse_batch_workspace_bytes", "dse_batch_init", "dse_batch_destroy", "dse_batch_last_error",
    "dse_batch_offsets", "dse_batch_start_guess", "dse_batch_jacobian", "dse_batch_newton_solve",
    "dse_batch_autotune", "dse_batch_set_launch", "dse_batch_get_launch",
    "dse_batch_set_launch_ex", "dse_batch_get_launch_ex", "dse_lu_solve_noalloc",
    "dse_renorm_scale", "dse_gauss_legendre_workspace_bytes", "dse_gauss_legendre",
    "dse_schwinger_workspace_bytes", "dse_schwinger",
]


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("n_z", C.c_int32), ("n_g", C.c_int32),
        ("n_rad", C.c_int32), ("n_ir", C.c_int32), ("n_ang", C.c_int32),
        ("precision", C.c_int32), ("quad", C.c_int32),
        ("eps2", C.c_double), ("lambda2", C.c_double), ("ir_efolds", C.c_double),
        ("alpha_mu", C.c_double), ("n_c", C.c_double), ("g0_inv", C.c_double),
        ("z_lambda_inv", C.c_double), ("kappa", C.c_double), ("delta", C.c_double),
        ("gamma", C.c_double),
    ]


class NewtonOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("extra_iters", C.c_int32),
                ("max_halvings", C.c_int32), ("reserved_", C.c_int32), ("step_tol", C.c_double)]


class NewtonReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("fnorm", C.c_double),
                ("fnorm2", C.c_double), ("fnorm_hist", C.c_double * 128),
                ("relax_hist", C.c_double * 128), ("n_jacobians", C.c_int32),
                ("n_residuals", C.c_int32), ("t_total_ms", C.c_double),
                ("n_jacobians_mixed", C.c_int32), ("reserved2_", C.c_int32),
                ("t_assembly_ms", C.c_double), ("t_lu_ms", C.c_double)]


class BatchTuning(C.Structure):
    _fields_ = [("slices", C.c_int32), ("persistent_blocks", C.c_int32), ("order", C.c_int32),
                ("n_candidates", C.c_int32), ("best_ms", C.c_double),
                ("cand_slices", C.c_int32 * 32), ("cand_blocks", C.c_int32 * 32),
                ("cand_order", C.c_int32 * 32), ("cand_ms", C.c_double * 32),
                ("tiles_per_item", C.c_int32), ("fused", C.c_int32),
                ("cand_tiles", C.c_int32 * 32), ("cand_fused", C.c_int32 * 32)]


class DSEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


_lib = None


def load():
    """Loads libdse.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdse.so not built: run `python -m paper_1206_1779_amd.build`")
        lib = C.CDLL(LIB_PATH)
        vp, P = C.c_void_p, C.POINTER(Params)
        sig = {
            "dse_params_default": (C.c_int, [P]),
            "dse_workspace_bytes": (C.c_size_t, [P]),
            "dse_init": (C.c_int, [P, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "dse_destroy": (C.c_int, [vp]),
            "dse_start_guess": (C.c_int, [vp, vp]),
            "dse_residual": (C.c_int, [vp, vp, vp, vp]),
            "dse_jacobian": (C.c_int, [vp, vp, vp, vp]),
            "dse_jacobian_fd": (C.c_int, [vp, vp, vp, C.c_double]),
            "dse_running_coupling": (C.c_int, [vp, vp, vp, C.c_int32, vp, vp, vp]),
            "dse_dressing_vjp": (C.c_int, [vp, vp, C.c_int32, vp, vp, vp]),
            "dse_newton_solve": (C.c_int, [vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonReport)]),
            "dse_lu_solve": (C.c_int, [vp, vp, vp, vp, C.c_int32]),
            "dse_lu_solve_noalloc": (C.c_int, [C.c_int32, vp, vp, vp, C.c_int32, vp, vp]),
            "dse_renorm_scale": (C.c_int, [vp, vp, vp]),
            "dse_gauss_legendre_workspace_bytes": (C.c_size_t, [C.c_int32]),
            "dse_gauss_legendre": (C.c_int, [C.c_int32, vp, vp, vp, C.c_size_t, vp]),
            "dse_schwinger_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
            "dse_schwinger": (C.c_int, [vp, vp, C.c_int32, C.c_double, vp, C.c_int32, vp, vp, C.c_size_t]),
            "dse_status_string": (C.c_char_p, [C.c_int]),
            "dse_last_error": (C.c_char_p, [vp]),
            "dse_sizes": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
            "dse_set_timing": (C.c_int, [vp, C.c_int32]),
            "dse_read_timings": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
            "dse_vjp": (C.c_int, [vp, vp, vp, vp, vp]),
            "dse_set_physics": (C.c_int, [vp, C.c_double, C.c_double, C.c_double]),
            "dse_newton_step": (C.c_int, [vp, vp, C.c_double, vp, vp, vp, C.c_int32]),
            "dse_set_graphs": (C.c_int, [vp, C.c_int32]),
            "dse_batch_workspace_bytes": (C.c_size_t, [P, C.c_int32]),
            "dse_batch_init": (C.c_int, [P, C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "dse_batch_destroy": (C.c_int, [vp]),
            "dse_batch_last_error": (C.c_char_p, [vp]),
            "dse_batch_offsets": (C.c_int, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
            "dse_batch_start_guess": (C.c_int, [vp, vp]),
            "dse_batch_jacobian": (C.c_int, [vp, vp, vp, vp]),
            "dse_batch_newton_solve": (C.c_int, [vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonReport)]),
            "dse_batch_autotune": (C.c_int, [vp, vp, C.POINTER(BatchTuning)]),
            "dse_batch_set_launch": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32]),
            "dse_batch_set_launch_ex": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
            "dse_batch_get_launch_ex": (C.c_int, [vp] + [C.POINTER(C.c_int32)] * 5),
            "dse_batch_get_launch": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                               C.POINTER(C.c_int32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def params(**kw) -> Params:
    """dse_params_default() overridden by keyword arguments."""
    p = Params()
    load().dse_params_default(C.byref(p))
    names = {f[0] for f in Params._fields_}
    for k, v in kw.items():
        if k not in names:
            raise KeyError("unknown parameter %r" % k)
        setattr(p, k, v)
    return p


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def lu_solve_noalloc(J: torch.Tensor, b: torch.Tensor, x: torch.Tensor, trans: bool = False,
                     info: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None) -> None:
    """dse_lu_solve_noalloc: x = J^{-1} b (or J^{-T} b) into the caller's x,
    enqueued on `stream` (default: the current stream of x's device) without
    any allocation; `info` (int32 device scalar, optional) receives the pivot
    status.  All tensors float64, contiguous, on one device."""
    lib = load()
    n = int(b.numel())
    for t in (J, b, x):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("J, b and x must be contiguous float64 device tensors")
    if J.shape != (n, n) or x.numel() != n:
        raise ValueError("J must be n x n for vectors of length n")
    if info is not None and (info.dtype != torch.int32 or info.device != x.device):
        raise ValueError("info must be an int32 tensor on the same device")
    with torch.cuda.device(x.device):
        st = stream if stream is not None else torch.cuda.current_stream(x.device)
        s = lib.dse_lu_solve_noalloc(n, _ptr(J), _ptr(b), _ptr(x), 1 if trans else 0, _ptr(info),
                                     C.c_void_p(st.cuda_stream))
    if s:
        raise DSEError(s, lib.dse_last_error(None).decode())


def gauss_legendre(n: int, device="cuda", stream: torch.cuda.Stream | None = None):
    """dse_gauss_legendre: the n-node Gauss-Legendre rule (nodes ascending,
    weights) computed on the device; returns two float64 tensors."""
    lib = load()
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    nb = lib.dse_gauss_legendre_workspace_bytes(int(n))
    if nb == 0:
        raise DSEError(1, "n = %d out of range" % n)
    with torch.cuda.device(dev):
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        x = torch.empty(n, dtype=torch.float64, device=dev)
        w = torch.empty(n, dtype=torch.float64, device=dev)
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        wp = (ws.data_ptr() + 255) // 256 * 256
        s = lib.dse_gauss_legendre(int(n), _ptr(x), _ptr(w), C.c_void_p(wp), nb, C.c_void_p(st.cuda_stream))
    if s:
        raise DSEError(s, lib.dse_last_error(None).decode())
    return x, w


@dataclass
class NewtonResult:
    c: torch.Tensor
    status: int
    iters: int
    fnorm: float
    fnorm2: float
    fnorm_hist: list = field(default_factory=list)
    relax_hist: list = field(default_factory=list)
    n_jacobians: int = 0
    n_residuals: int = 0
    t_total_ms: float = 0.0
    n_jacobians_mixed: int = 0
    t_assembly_ms: float = 0.0
    t_lu_ms: float = 0.0


class Solver:
    """One context of the HIP solver on one device and stream.

    Buffers are torch tensors (float64, on the context's device); the
    workspace is allocated here once, as a uint8 tensor."""

    def __init__(self, device="cuda", stream: torch.cuda.Stream | None = None, **kw):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU")
        self.lib = load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.p = params(**kw)
        nbytes = self.lib.dse_workspace_bytes(C.byref(self.p))
        if nbytes == 0:
            h = C.c_void_p()
            st = self.lib.dse_init(C.byref(self.p), None, 0, None, C.byref(h))
            raise DSEError(st, self.lib.dse_last_error(None).decode())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            h = C.c_void_p()
            st = self.lib.dse_init(C.byref(self.p), C.c_void_p(self._ws_ptr), nbytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st:
            raise DSEError(st, self.lib.dse_last_error(None).decode())
        self.h = h
        self.n = self.p.n_z + self.p.n_g

    # ---------------------------------------------------------------- helpers
    def _check(self, st):
        if st:
            raise DSEError(st, self.lib.dse_last_error(self.h).decode())

    def _vec(self, x=None):
        if x is None:
            return torch.empty(self.n, dtype=torch.float64, device=self.device)
        x = torch.as_tensor(x, dtype=torch.float64)
        if x.device != self.device:
            x = x.to(self.device)
        if x.shape != (self.n,):
            raise ValueError("expected a vector of length %d" % self.n)
        return x.contiguous()

    def close(self):
        if getattr(self, "h", None):
            self.lib.dse_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------- API
    def start_guess(self) -> torch.Tensor:
        c = self._vec()
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_start_guess(self.h, _ptr(c)))
        return c

    def residual(self, c, with_scale: bool = False):
        c = self._vec(c)
        F = self._vec()
        S = self._vec() if with_scale else None
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_residual(self.h, _ptr(c), _ptr(F), _ptr(S)))
        return (F, S) if with_scale else F

    def jacobian(self, c, with_F: bool = True):
        c = self._vec(c)
        J = torch.empty(self.n, self.n, dtype=torch.float64, device=self.device)
        F = self._vec() if with_F else None
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_jacobian(self.h, _ptr(c), _ptr(J), _ptr(F)))
        return (J, F) if with_F else J

    def jacobian_fd(self, c, h_rel: float = 1e-5) -> torch.Tensor:
        """Newton matrix by central differences of the residual (dse_jacobian_fd)."""
        c = self._vec(c)
        J = torch.empty(self.n, self.n, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_jacobian_fd(self.h, _ptr(c), _ptr(J), float(h_rel)))
        return J

    def running_coupling(self, c, u):
        """alpha(u), ln Z(u), ln G(u) at the momenta u (dse_running_coupling)."""
        c = self._vec(c)
        u = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        out = [torch.empty_like(u) for _ in range(3)]
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_running_coupling(self.h, _ptr(c), _ptr(u), int(u.numel()),
                                                       _ptr(out[0]), _ptr(out[1]), _ptr(out[2])))
        return tuple(out)

    def dressing_vjp(self, u, wZ=None, wG=None) -> torch.Tensor:
        """dL/dc for weights wZ = dL/d ln Z(u), wG = dL/d ln G(u) at the momenta
        u (dse_dressing_vjp); either weight may be None."""
        u = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        m = int(u.numel())

        def w(x):
            if x is None:
                return None
            x = torch.as_tensor(x, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
            if x.numel() != m:
                raise ValueError("weights must have one entry per momentum")
            return x
        wZ, wG = w(wZ), w(wG)
        g = self._vec()
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_dressing_vjp(self.h, _ptr(u), m, _ptr(wZ), _ptr(wG), _ptr(g)))
        return g

    def renorm_scale(self, c) -> float:
        """mu^2 with G^2(mu^2) Z(mu^2) = 1 (dse_renorm_scale); NaN if none."""
        c = self._vec(c)
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_renorm_scale(self.h, _ptr(c), _ptr(out)))
        return float(out.item())

    def schwinger(self, c, t, n: int = 1 << 17, p_max: float = 1e3, ws: torch.Tensor | None = None):
        """Delta(t) of the gluon propagator (dse_schwinger) with the n-node
        mapped rule on [0, p_max]; `ws` (uint8 device tensor, optional) is the
        workspace, reused across calls when given."""
        c = self._vec(c)
        t = torch.as_tensor(t, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        m = int(t.numel())
        nb = self.lib.dse_schwinger_workspace_bytes(int(n), m)
        if nb == 0:
            raise DSEError(1, "n = %d or m = %d out of range" % (n, m))
        if ws is None or ws.numel() < nb + 256:
            ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        wp = (ws.data_ptr() + 255) // 256 * 256
        out = torch.empty(m, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_schwinger(self.h, _ptr(c), int(n), float(p_max), _ptr(t), m, _ptr(out),
                                               C.c_void_p(wp), nb))
        return out

    def lu_solve(self, J, b, trans: bool = False) -> torch.Tensor:
        J = torch.as_tensor(J, dtype=torch.float64).to(self.device).contiguous()
        b = self._vec(b)
        x = self._vec()
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_lu_solve(self.h, _ptr(J), _ptr(b), _ptr(x), 1 if trans else 0))
        return x

    def newton(self, c0=None, tol=1e-10, max_iter=60, extra_iters=0, max_halvings=30,
               step_tol=1e-14, raise_on_error: bool = True) -> NewtonResult:
        c = self.start_guess() if c0 is None else self._vec(c0).clone()
        o = NewtonOpts(tol=tol, max_iter=max_iter, extra_iters=extra_iters,
                       max_halvings=max_halvings, step_tol=step_tol)
        rep = NewtonReport()
        with torch.cuda.device(self.device):
            st = self.lib.dse_newton_solve(self.h, _ptr(c), C.byref(o), C.byref(rep))
        if st and raise_on_error:
            self._check(st)
        return NewtonResult(c=c, status=rep.status, iters=rep.iters, fnorm=rep.fnorm,
                            fnorm2=rep.fnorm2, fnorm_hist=list(rep.fnorm_hist[: rep.iters + 1]),
                            relax_hist=list(rep.relax_hist[: rep.iters]),
                            n_jacobians=rep.n_jacobians, n_residuals=rep.n_residuals,
                            t_total_ms=rep.t_total_ms, n_jacobians_mixed=rep.n_jacobians_mixed,
                            t_assembly_ms=rep.t_assembly_ms, t_lu_ms=rep.t_lu_ms)

    def newton_step(self, c, rho: float = 1.0, out=None, check: bool = False):
        """One Newton iteration: returns (c_new, F(c_new), S(c_new)).  `out`
        (optional) is a tuple of three preallocated vectors; with graph replay
        switched on (set_graphs) reusing the same ones lets the library replay
        its recorded graph."""
        c = self._vec(c)
        cn, F, S = out if out is not None else (self._vec(), self._vec(), self._vec())
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_newton_step(self.h, _ptr(c), float(rho), _ptr(cn), _ptr(F), _ptr(S),
                                                 1 if check else 0))
        return cn, F, S

    def set_graphs(self, on: bool = True):
        """Graph replay of newton_step (off by default: kernel by kernel is faster)."""
        self._check(self.lib.dse_set_graphs(self.h, 1 if on else 0))

    def vjp(self, c, u, with_c: bool = True):
        """u^T dF/dc (or None) and u^T dF/d(alpha_mu, g0_inv, z_lambda_inv)."""
        c = self._vec(c)
        u = self._vec(u)
        uJ = self._vec() if with_c else None
        ut = torch.empty(3, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_vjp(self.h, _ptr(c), _ptr(u), _ptr(uJ), _ptr(ut)))
        return uJ, ut

    def set_physics(self, alpha_mu=None, g0_inv=None, z_lambda_inv=None):
        a = self.p.alpha_mu if alpha_mu is None else float(alpha_mu)
        g = self.p.g0_inv if g0_inv is None else float(g0_inv)
        z = self.p.z_lambda_inv if z_lambda_inv is None else float(z_lambda_inv)
        self._check(self.lib.dse_set_physics(self.h, a, g, z))
        self.p.alpha_mu, self.p.g0_inv, self.p.z_lambda_inv = a, g, z

    def set_timing(self, on: bool = True):
        self._check(self.lib.dse_set_timing(self.h, 1 if on else 0))

    def read_timings(self):
        """Average device ms per dse_jacobian since set_timing(True):
        dressing, gluon points, ghost points, contraction, assembly; and the count."""
        out = (C.c_double * 5)()
        cnt = C.c_int32()
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_read_timings(self.h, out, C.byref(cnt)))
        return list(out), cnt.value

    def sizes(self):
        n, nr, na = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.dse_sizes(self.h, C.byref(n), C.byref(nr), C.byref(na)))
        return n.value, nr.value, na.value


def _report(rep: NewtonReport, c) -> NewtonResult:
    return NewtonResult(c=c, status=rep.status, iters=rep.iters, fnorm=rep.fnorm, fnorm2=rep.fnorm2,
                        fnorm_hist=list(rep.fnorm_hist[: rep.iters + 1]),
                        relax_hist=list(rep.relax_hist[: rep.iters]), n_jacobians=rep.n_jacobians,
                        n_residuals=rep.n_residuals, t_total_ms=rep.t_total_ms)


class Batch:
    """A family of independent problems assembled and solved together.

    ``problems`` is a list of keyword dicts (each as for Solver).  Unknowns of
    all problems live in one packed float64 vector (problem b at
    ``off_c[b]:off_c[b+1]``), Newton matrices in one packed array
    (``off_J[b]:off_J[b+1]``, row-major n_b x n_b)."""

    def __init__(self, problems, device="cuda", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU")
        self.lib = load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.count = len(problems)
        arr = (Params * self.count)()
        for i, kw in enumerate(problems):
            arr[i] = params(**kw)
        self.params = arr
        nbytes = self.lib.dse_batch_workspace_bytes(arr, self.count)
        if nbytes == 0:
            h = C.c_void_p()
            st = self.lib.dse_batch_init(arr, self.count, None, 0, None, C.byref(h))
            raise DSEError(st, self.lib.dse_batch_last_error(None).decode())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.ws.data_ptr() + 255) // 256 * 256
            h = C.c_void_p()
            st = self.lib.dse_batch_init(arr, self.count, C.c_void_p(ptr), nbytes,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st:
            raise DSEError(st, self.lib.dse_batch_last_error(None).decode())
        self.h = h
        oc = (C.c_int64 * (self.count + 1))()
        oj = (C.c_int64 * (self.count + 1))()
        self._check(self.lib.dse_batch_offsets(self.h, oc, oj))
        self.off_c = list(oc)
        self.off_J = list(oj)

    def _check(self, st):
        if st:
            raise DSEError(st, self.lib.dse_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dse_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _packed(self, c=None):
        n = self.off_c[-1]
        if c is None:
            return torch.empty(n, dtype=torch.float64, device=self.device)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        if c.shape != (n,):
            raise ValueError("expected a packed vector of length %d" % n)
        return c

    def split(self, packed):
        """Per-problem views of a packed vector."""
        return [packed[self.off_c[b]: self.off_c[b + 1]] for b in range(self.count)]

    def split_J(self, packed):
        out = []
        for b in range(self.count):
            n = self.off_c[b + 1] - self.off_c[b]
            out.append(packed[self.off_J[b]: self.off_J[b + 1]].view(n, n))
        return out

    def start_guess(self):
        c = self._packed()
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_batch_start_guess(self.h, _ptr(c)))
        return c

    def jacobian(self, c):
        c = self._packed(c)
        J = torch.empty(self.off_J[-1], dtype=torch.float64, device=self.device)
        F = self._packed()
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_batch_jacobian(self.h, _ptr(c), _ptr(J), _ptr(F)))
        return J, F

    def newton(self, c0=None, tol=1e-10, max_iter=60, extra_iters=0, max_halvings=30,
               step_tol=1e-14, raise_on_error: bool = True):
        c = self.start_guess() if c0 is None else self._packed(c0).clone()
        o = NewtonOpts(tol=tol, max_iter=max_iter, extra_iters=extra_iters,
                       max_halvings=max_halvings, step_tol=step_tol)
        reps = (NewtonReport * self.count)()
        with torch.cuda.device(self.device):
            st = self.lib.dse_batch_newton_solve(self.h, _ptr(c), C.byref(o), reps)
        if st and raise_on_error:
            self._check(st)
        cs = self.split(c)
        return c, [_report(reps[b], cs[b]) for b in range(self.count)]

    def autotune(self, c):
        c = self._packed(c)
        r = BatchTuning()
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_batch_autotune(self.h, _ptr(c), C.byref(r)))
        cands = [dict(slices=r.cand_slices[i], persistent_blocks=r.cand_blocks[i],
                      order=r.cand_order[i], tiles_per_item=r.cand_tiles[i], fused=r.cand_fused[i],
                      ms=r.cand_ms[i]) for i in range(r.n_candidates)]
        return dict(slices=r.slices, persistent_blocks=r.persistent_blocks, order=r.order,
                    tiles_per_item=r.tiles_per_item, fused=r.fused, best_ms=r.best_ms, candidates=cands)

    def set_launch(self, slices=1, persistent_blocks=0, order=1, tiles_per_item=1, fused=0):
        with torch.cuda.device(self.device):
            self._check(self.lib.dse_batch_set_launch_ex(self.h, slices, persistent_blocks, order,
                                                         tiles_per_item, fused))

    def get_launch(self, full: bool = False):
        a, b, c, d, e = (C.c_int32() for _ in range(5))
        self._check(self.lib.dse_batch_get_launch_ex(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d),
                                                     C.byref(e)))
        out = dict(slices=a.value, persistent_blocks=b.value, order=c.value)
        if full:
            out.update(tiles_per_item=d.value, fused=e.value)
        return out
