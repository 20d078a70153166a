"""Python binding of libqrctm.so (ctypes; argument marshalling only).

Every computation runs in the HIP library; this module only passes device
pointers (from torch tensors), sizes and the current HIP stream, and turns
status codes into exceptions.  The library must be built in-tree first
(``python -m paper_2505_00494_amd.build``); nothing falls back to the CPU.
"""
from __future__ import annotations

import ctypes
import os
import re
import warnings
from ctypes import POINTER, byref, c_double, c_int, c_longlong, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqrctm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "qrctm.h")

CTM_OK, CTM_NOTCONV = 0, 1
CTM_EINVAL, CTM_EWORKSPACE, CTM_EHIP, CTM_ENONFINITE, CTM_ESINGULAR, CTM_ESTATE = (
    -1, -2, -3, -4, -5, -6)
PREC_FP64, PREC_FP32_MFMA, PREC_BF16X6_MFMA = 0, 1, 2
GRAD_CHECKPOINT, GRAD_FIXED_POINT = 0, 1
QR_AUTO, QR_HOUSEHOLDER = 0, 1


class CTMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class CtmOpts(ctypes.Structure):
    _fields_ = [("precision", c_int), ("n_warmup", c_int), ("k_tracked", c_int),
                ("qr_sing_tol", c_double), ("mixed_tol", c_double), ("edge_split", c_int),
                ("grad_mode", c_int), ("fp_tol", c_double), ("fp_max_iter", c_int),
                ("grad_keep_yz", c_int), ("qr_reg_eps", c_double), ("qr_method", c_int)]


class CtmStats(ctypes.Structure):
    _fields_ = [("chi", c_int), ("chi_cur", c_int), ("Dab", c_int), ("steps", c_longlong),
                ("last_delta", c_double), ("flops_per_step", c_double),
                ("r_diag_ratio", c_double), ("timed_steps", c_longlong),
                ("ms_phase", c_double * 8), ("grad_steps", c_longlong),
                ("fp_residual", c_double), ("qr_fallbacks", c_longlong),
                ("edge_3b_form", c_int)]

EDGE_3B_FORMS = {0: "double-layer GEMM, FP64", 1: "double-layer GEMM, FP32 matrix cores",
                 2: "double-layer GEMM as six bf16 products of split planes (FP32 accumulation)",
                 3: "fused ket/bra split, FP64", 4: "fused ket/bra split, FP32 matrix cores"}

PHASES = ("reduced_corner", "qr", "edge_3a", "edge_3b", "edge_3c", "corner", "sym_norm",
          "spectrum")


_lib = None


def header_functions():
    """Names of the functions declared in include/qrctm.h."""
    with open(HEADER) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ctm_[a-z0-9_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2505_00494_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, cp, dp, ip = c_void_p, POINTER(c_void_p), POINTER(c_double), POINTER(c_int)
    sig = {
        "ctm_default_opts": (None, [POINTER(CtmOpts)]),
        "ctm_workspace_bytes": (c_size_t, [c_int, c_int, c_int, POINTER(CtmOpts)]),
        "ctm_workspace_bytes_dl": (c_size_t, [c_int, c_int, POINTER(CtmOpts)]),
        "ctm_init": (c_int, [cp, vp, c_int, c_int, c_int, POINTER(CtmOpts), vp, c_size_t, vp]),
        "ctm_init_dl": (c_int, [cp, vp, vp, c_int, c_int, POINTER(CtmOpts), vp, c_size_t, vp]),
        "ctm_set_tensor": (c_int, [vp, vp]),
        "ctm_step": (c_int, [vp, c_int, dp]),
        "ctm_converge": (c_int, [vp, c_double, c_int, ip, dp]),
        "ctm_get_env": (c_int, [vp, vp, vp, ip]),
        "ctm_set_env": (c_int, [vp, vp, vp, c_int]),
        "ctm_spectrum": (c_int, [vp, dp]),
        "ctm_energy": (c_int, [vp, dp, dp, c_double, dp]),
        "ctm_energy_grad": (c_int, [vp, dp, dp, c_double, dp, vp]),
        "ctm_lnz_per_site": (c_int, [vp, dp]),
        "ctm_expect_site": (c_int, [vp, vp, dp]),
        "ctm_stats": (c_int, [vp, POINTER(CtmStats)]),
        "ctm_set_timing": (c_int, [vp, c_int]),
        "ctm_last_error": (ctypes.c_char_p, [vp]),
        "ctm_destroy": (None, [vp]),
        "ctm_qr_workspace_bytes": (c_size_t, [c_int, c_int]),
        "ctm_qr": (c_int, [vp, vp, vp, c_int, c_int, c_int, vp, c_size_t, vp, ip]),
        "ctm_qr_noalloc_max_bytes": (c_size_t, []),
        "ctm_qr_noalloc": (c_int, [vp, vp, vp, c_int, c_int, c_int, vp, ip]),
        "ctm_gemm_workspace_bytes": (c_size_t, [c_int, c_int, c_int]),
        "ctm_gemm": (c_int, [c_int, c_int, c_int, c_int, c_int, c_double, vp, c_int, vp, c_int,
                             c_double, vp, c_int, vp, c_size_t, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the QR-CTMRG library runs on the GPU only")
    return torch


def _stream(dev):
    return c_void_p(_torch().cuda.current_stream(dev).cuda_stream)


def _check(rc: int, ctx=None):
    if rc < 0:
        msg = lib().ctm_last_error(ctx)
        raise CTMError(rc, msg.decode() if msg else "")
    return rc


def _dev_f64(x, dev):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64, device=dev)
    return t.contiguous()


class ConvergenceWarning(UserWarning):
    """The environment (or the fixed-point series) stopped before its tolerance."""


def default_opts(precision=PREC_FP64, n_warmup=-1, k_tracked=None, qr_sing_tol=1e-14,
                 mixed_tol=None, edge_split=None, grad_mode=None, fp_tol=None,
                 fp_max_iter=None, grad_keep_yz=None, qr_reg_eps=None, qr_method=None) -> CtmOpts:
    """ctm_opts with the library's defaults, overridden where an argument is given
    (k_tracked None or -1: the per-D default)."""
    o = CtmOpts()
    lib().ctm_default_opts(byref(o))
    o.precision, o.n_warmup, o.qr_sing_tol = precision, n_warmup, qr_sing_tol
    if k_tracked is not None:
        o.k_tracked = int(k_tracked)
    if mixed_tol is not None:
        o.mixed_tol = mixed_tol
    if edge_split is not None:
        o.edge_split = int(edge_split)
    if grad_mode is not None:
        o.grad_mode = int(grad_mode)
    if fp_tol is not None:
        o.fp_tol = float(fp_tol)
    if fp_max_iter is not None:
        o.fp_max_iter = int(fp_max_iter)
    if grad_keep_yz is not None:
        o.grad_keep_yz = int(grad_keep_yz)
    if qr_reg_eps is not None:
        o.qr_reg_eps = float(qr_reg_eps)
    if qr_method is not None:
        o.qr_method = int(qr_method)
    return o


class Context:
    """One CTMRG environment on one GPU (wraps ctm_ctx)."""

    def __init__(self, A=None, chi: int = 16, *, a=None, bvec=None, device="cuda:0",
                 n_warmup: int = -1, precision: int = PREC_FP64, k_tracked=None,
                 qr_sing_tol: float = 1e-14, mixed_tol=None, edge_split=None,
                 grad_mode=None, fp_tol=None, fp_max_iter=None, grad_keep_yz=None,
                 qr_reg_eps=None, qr_method=None):
        torch = _torch()
        self.device = torch.device(device)
        self.opts = default_opts(precision, n_warmup, k_tracked, qr_sing_tol, mixed_tol,
                                 edge_split, grad_mode, fp_tol, fp_max_iter, grad_keep_yz,
                                 qr_reg_eps, qr_method)
        self.chi = chi
        L = lib()
        ctx = c_void_p()
        st = _stream(self.device)
        if A is not None:
            A = _dev_f64(A, self.device)
            self.d, self.D = int(A.shape[0]), int(A.shape[1])
            self.Dab = self.D * self.D
            nb = L.ctm_workspace_bytes(self.d, self.D, chi, byref(self.opts))
            if nb == 0:
                raise CTMError(CTM_EINVAL, "invalid sizes")
            self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            rc = L.ctm_init(byref(ctx), c_void_p(A.data_ptr()), self.d, self.D, chi,
                            byref(self.opts), c_void_p(self.ws.data_ptr()), nb, st)
        else:
            a = _dev_f64(a, self.device)
            bvec = _dev_f64(bvec, self.device)
            self.d, self.D = 0, 0
            self.Dab = int(a.shape[0])
            nb = L.ctm_workspace_bytes_dl(self.Dab, chi, byref(self.opts))
            if nb == 0:
                raise CTMError(CTM_EINVAL, "invalid sizes")
            self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            rc = L.ctm_init_dl(byref(ctx), c_void_p(a.data_ptr()), c_void_p(bvec.data_ptr()),
                               self.Dab, chi, byref(self.opts), c_void_p(self.ws.data_ptr()), nb,
                               st)
        _check(rc, None)
        self._ctx = ctx
        self.ws_bytes = nb

    # -- lifetime --------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().ctm_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, rc):
        return _check(rc, self._ctx)

    # -- the path --------------------------------------------------------------
    def set_tensor(self, A):
        A = _dev_f64(A, self.device)
        self._c(lib().ctm_set_tensor(self._ctx, c_void_p(A.data_ptr())))

    def step(self, n: int = 1) -> float:
        dl = c_double()
        self._c(lib().ctm_step(self._ctx, n, byref(dl)))
        return dl.value

    def converge(self, tol: float, max_steps: int):
        steps, dl = c_int(), c_double()
        rc = self._c(lib().ctm_converge(self._ctx, tol, max_steps, byref(steps), byref(dl)))
        return rc == CTM_OK, steps.value, dl.value

    def get_env(self):
        torch = _torch()
        chi = self.chi
        C = torch.empty(chi * chi, dtype=torch.float64, device=self.device)
        T = torch.empty(chi * chi * self.Dab, dtype=torch.float64, device=self.device)
        cc = c_int()
        self._c(lib().ctm_get_env(self._ctx, c_void_p(C.data_ptr()), c_void_p(T.data_ptr()),
                                  byref(cc)))
        n = cc.value
        return (C[: n * n].reshape(n, n).clone(), T[: n * n * self.Dab].reshape(n, self.Dab, n).clone())

    def set_env(self, C, T):
        C = _dev_f64(C, self.device)
        T = _dev_f64(T, self.device)
        n = int(C.shape[0])
        self._c(lib().ctm_set_env(self._ctx, c_void_p(C.data_ptr()), c_void_p(T.data_ptr()), n))

    def spectrum(self) -> np.ndarray:
        st = self.stats()
        s = np.zeros(st["chi_cur"])
        self._c(lib().ctm_spectrum(self._ctx, s.ctypes.data_as(POINTER(c_double))))
        return s

    def energy(self, h_nn, h_nnn=None, J2: float = 0.0) -> float:
        h1 = np.ascontiguousarray(h_nn, dtype=np.float64)
        h2 = None if h_nnn is None else np.ascontiguousarray(h_nnn, dtype=np.float64)
        E = c_double()
        self._c(lib().ctm_energy(self._ctx, h1.ctypes.data_as(POINTER(c_double)),
                                 None if h2 is None else h2.ctypes.data_as(POINTER(c_double)),
                                 J2, byref(E)))
        return E.value

    def energy_grad(self, h_nn, h_nnn=None, J2: float = 0.0):
        torch = _torch()
        h1 = np.ascontiguousarray(h_nn, dtype=np.float64)
        h2 = None if h_nnn is None else np.ascontiguousarray(h_nnn, dtype=np.float64)
        dA = torch.empty((self.d, self.D, self.D, self.D, self.D), dtype=torch.float64,
                         device=self.device)
        E = c_double()
        rc = self._c(lib().ctm_energy_grad(self._ctx, h1.ctypes.data_as(POINTER(c_double)),
                                           None if h2 is None else h2.ctypes.data_as(POINTER(c_double)),
                                           J2, byref(E), c_void_p(dA.data_ptr())))
        # fixed-point scheme: False when the series stopped at opts.fp_max_iter
        self.grad_converged = rc == CTM_OK
        return E.value, dA

    def lnz_per_site(self) -> float:
        v = c_double()
        self._c(lib().ctm_lnz_per_site(self._ctx, byref(v)))
        return v.value

    def expect_site(self, imp) -> float:
        imp = _dev_f64(imp, self.device)
        v = c_double()
        self._c(lib().ctm_expect_site(self._ctx, c_void_p(imp.data_ptr()), byref(v)))
        return v.value

    def stats(self) -> dict:
        s = CtmStats()
        self._c(lib().ctm_stats(self._ctx, byref(s)))
        out = {k: getattr(s, k) for k, _ in CtmStats._fields_ if k != "ms_phase"}
        out["ms_phase"] = {name: s.ms_phase[i] for i, name in enumerate(PHASES)}
        out["edge_3b_kernel"] = EDGE_3B_FORMS.get(s.edge_3b_form, "unknown")
        return out

    def set_timing(self, on: bool = True):
        self._c(lib().ctm_set_timing(self._ctx, int(on)))


_ENERGY_FN = None


def _energy_function():
    """torch.autograd.Function for E(A) with the library's hand-written adjoint.

    forward: ctm_set_tensor (the context keeps its environment as the starting
    point, as the AD paragraph reuses the previous environment), ctm_converge,
    then ctm_energy_grad, whose dE/dA is saved; backward returns gE * dE/dA.
    An environment that stopped before tol (CTM_NOTCONV), or a fixed-point
    series that stopped before fp_tol, is reported as the caller asks
    (on_notconv: "warn", "raise" or "ignore") and recorded on the context
    (ctx.last_converged, ctx.last_delta, ctx.last_steps, ctx.grad_converged).
    """
    global _ENERGY_FN
    if _ENERGY_FN is None:
        torch = _torch()

        class QRCTMEnergy(torch.autograd.Function):
            @staticmethod
            def forward(fctx, A, ctx, h_nn, h_nnn, J2, tol, max_steps, on_notconv):
                ctx.set_tensor(A.detach())
                ok, steps, dl = ctx.converge(tol, max_steps)
                ctx.last_converged, ctx.last_steps, ctx.last_delta = ok, steps, dl
                if not ok:
                    _report(on_notconv, CTM_NOTCONV,
                            f"environment not converged: delta {dl:.3e} >= tol {tol:.1e} "
                            f"after {steps} steps; E and dE/dA come from this environment")
                e, dA = ctx.energy_grad(h_nn, h_nnn, J2)
                if not ctx.grad_converged:
                    _report(on_notconv, CTM_NOTCONV,
                            "fixed-point series stopped before fp_tol; dE/dA is truncated")
                fctx.save_for_backward(dA.to(A.dtype))
                return torch.tensor(e, dtype=A.dtype, device=A.device)

            @staticmethod
            def backward(fctx, gE):
                (dA,) = fctx.saved_tensors
                return gE * dA, None, None, None, None, None, None, None

        _ENERGY_FN = QRCTMEnergy
    return _ENERGY_FN


def _report(policy: str, code: int, msg: str):
    if policy == "raise":
        raise CTMError(code, msg)
    if policy == "warn":
        warnings.warn(msg, ConvergenceWarning, stacklevel=4)
    elif policy != "ignore":
        raise ValueError(f"on_notconv must be 'warn', 'raise' or 'ignore', not {policy!r}")


def energy(A, ctx: "Context", h_nn, h_nnn=None, J2: float = 0.0, tol: float = 1e-10,
           max_steps: int = 200, on_notconv: str = "warn"):
    """Differentiable energy per site E(A) (a torch scalar on A's device).

    The environment of ctx is converged for A (to tol, at most max_steps
    steps), then E and dE/dA come from ctm_energy_grad: dE/dA is the derivative
    of E_k(P(A); C*, T*), k = the context's tracked steps (or, with the
    fixed-point scheme, of the converged energy).  on_notconv decides what an
    unconverged environment or series does: "warn" (default), "raise" or
    "ignore"; either way ctx.last_converged and ctx.grad_converged record it.
    """
    return _energy_function().apply(A, ctx, h_nn, h_nnn, J2, tol, max_steps, on_notconv)


def qr(M, method: int = QR_AUTO, return_used=False):
    """Thin QR with diag(R) >= 0 of a device matrix (m x n, m >= n) via ctm_qr.

    return_used: also return whether the Householder factorisation ran."""
    torch = _torch()
    M = M.to(torch.float64).contiguous()
    m, n = M.shape
    Q = torch.empty((m, n), dtype=torch.float64, device=M.device)
    R = torch.empty((n, n), dtype=torch.float64, device=M.device)
    nb = lib().ctm_qr_workspace_bytes(m, n)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=M.device)
    used = c_int()
    _check(lib().ctm_qr(c_void_p(M.data_ptr()), c_void_p(Q.data_ptr()), c_void_p(R.data_ptr()), m,
                        n, int(method), c_void_p(ws.data_ptr()), nb, _stream(M.device), byref(used)))
    return (Q, R, bool(used.value)) if return_used else (Q, R)


def qr_noalloc(M, Q=None, R=None, method: int = QR_AUTO, return_used=False):
    """ctm_qr_noalloc: the same thin QR with the library's fixed scratch (no
    allocation inside the call; Q and R may be passed in preallocated)."""
    torch = _torch()
    if M.dtype != torch.float64 or not M.is_contiguous():
        raise ValueError("M must be a contiguous float64 device tensor")
    m, n = M.shape
    if Q is None:
        Q = torch.empty((m, n), dtype=torch.float64, device=M.device)
    if R is None:
        R = torch.empty((n, n), dtype=torch.float64, device=M.device)
    used = c_int()
    _check(lib().ctm_qr_noalloc(c_void_p(M.data_ptr()), c_void_p(Q.data_ptr()), c_void_p(R.data_ptr()),
                                m, n, int(method), _stream(M.device), byref(used)))
    return (Q, R, bool(used.value)) if return_used else (Q, R)


def gemm(A, B, C=None, *, trans_a=False, trans_b=False, alpha=1.0, beta=0.0):
    """C = alpha op(A) op(B) + beta C on the FP64 matrix cores via ctm_gemm."""
    torch = _torch()
    A = A.contiguous()
    B = B.contiguous()
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[0] if trans_b else B.shape[1]
    if C is None:
        C = torch.zeros((M, N), dtype=torch.float64, device=A.device)
    nb = lib().ctm_gemm_workspace_bytes(M, N, K)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=A.device)
    _check(lib().ctm_gemm(int(trans_a), int(trans_b), M, N, K, alpha, c_void_p(A.data_ptr()),
                          A.shape[1], c_void_p(B.data_ptr()), B.shape[1], beta,
                          c_void_p(C.data_ptr()), C.shape[1], c_void_p(ws.data_ptr()), nb,
                          _stream(A.device)))
    return C
