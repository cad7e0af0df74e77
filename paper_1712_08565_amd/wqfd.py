"""Thin torch binding of the C ABI (include/wqfd.h): same names as the C entry
points, argument marshalling only.  Device memory (vectors, fields and the
library workspaces) is owned by torch tensors; work is enqueued on the current
torch stream (a HIP stream on ROCm).  Every computation runs in libwqfd.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from ._lib import (WQ_BF16, WQ_F32, WQ_F64, WQ_FD_NOALLOC_BYTES, WQ_K_IDENTITY, WQ_K_SCALAR, WQ_K_SYM6, WQError,
                   check, lib)

__all__ = ["WqOp", "FdPc", "wq_setup", "wq_dims", "wq_quad_points", "wq_detj", "wq_set_coef", "wq_apply",
           "wq_apply_T", "wq_apply_acc", "wq_set_alpha", "wq_apply_mass", "wq_rhs", "wq_grad_K", "wq_grad_f", "wq_grad_Kf",
           "wq_grad_alpha", "wq_alpha_mean", "fd_setup", "fd_apply", "fd_apply_noalloc", "fd_set_shift", "fd_factors",
           "krylov_solve", "ir_solve", "ir_fallback_count", "krylov_restart_count", "WqEval", "wq_eval_setup", "wq_eval_slab", "WQ_F64", "WQ_F32", "WQ_BF16", "WQ_K_IDENTITY", "WQ_K_SCALAR",
           "WQ_K_SYM6", "WQError"]

_DT = {WQ_F64: torch.float64, WQ_F32: torch.float32, WQ_BF16: torch.float32}


def _stream(stream=None):
    """The stream a call is enqueued on: torch's current stream by default.  A
    torch stream other than the current one first waits for the work already
    queued on the current stream (where the tensors passed in were produced)."""
    cur = torch.cuda.current_stream()
    if stream is None:
        return C.c_void_p(cur.cuda_stream)
    if isinstance(stream, torch.cuda.Stream) and stream != cur:
        stream.wait_stream(cur)
    return C.c_void_p(stream.cuda_stream)


def _keep_for(t: torch.Tensor, stream):
    """A tensor allocated here and used on another stream: its memory is not
    reused before that stream's queued work (a solve may return with work of its
    own still queued) has finished."""
    if isinstance(stream, torch.cuda.Stream):
        t.record_stream(stream)


def _p(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _knots(knots: Sequence[np.ndarray]):
    ks = [np.ascontiguousarray(k, dtype=np.float64) for k in knots]
    nk = (C.c_int32 * 3)(*[len(k) for k in ks])
    kp = (C.c_void_p * 3)(*[k.ctypes.data for k in ks])
    return ks, nk, kp


def _need(t: torch.Tensor, dtype, numel: int, name: str):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name}: need a contiguous {dtype} device tensor with {numel} entries")


def _ws_bytes(ws: torch.Tensor, nbytes: int, name: str) -> int:
    """Byte size of a caller-supplied workspace, checked to be device memory of at least nbytes."""
    if not ws.is_cuda or not ws.is_contiguous() or ws.numel() * ws.element_size() < nbytes:
        raise ValueError(f"{name}: need a contiguous device tensor of at least {nbytes} bytes")
    return ws.numel() * ws.element_size()


# planes of N_q doubles that K_q holds for each k_kind (layout in wq_set_coef)
_K_PLANES = {WQ_K_IDENTITY: 0, WQ_K_SCALAR: 1, WQ_K_SYM6: 6}


class WqOp:
    """MF-WQ operator handle (stiffness, plus the reaction term once set); owns its device workspace tensor."""

    def __init__(self, handle, ws, p, prec_mask, k_kind, device):
        self.handle, self.ws, self.p, self.prec_mask, self.k_kind, self.device = \
            handle, ws, p, prec_mask, k_kind, device
        self._destroy = lib().wq_destroy
        n = (C.c_int32 * 3)()
        nq = (C.c_int32 * 3)()
        check(lib().wq_dims(handle, n, nq), "wq_dims")
        self.n, self.nq = tuple(n), tuple(nq)
        self.N = int(np.prod(self.n))
        self.Nq = int(np.prod(self.nq))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._destroy(h)
            self.handle = None


class FdPc:
    """Fast Diagonalization preconditioner handle; owns its workspace tensor."""

    def __init__(self, handle, ws, n, prec_mask, device):
        self.handle, self.ws, self.n, self.prec_mask, self.device = handle, ws, n, prec_mask, device
        self.N = int(np.prod(n))
        self._destroy = lib().fd_destroy

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._destroy(h)
            self.handle = None


class WqEval:
    """Gauss-point evaluator of discrete solutions (wq_eval_setup); owns its workspace tensor."""

    def __init__(self, handle, ws, p, ng, device):
        self.handle, self.ws, self.p, self.ng, self.device = handle, ws, p, ng, device
        self._destroy = lib().wq_eval_destroy
        ne = (C.c_int32 * 3)()
        nq = (C.c_int32 * 3)()
        check(lib().wq_eval_dims(handle, ne, nq), "wq_eval_dims")
        self.ne, self.nq = tuple(ne), tuple(nq)
        self.N = int(np.prod([e + p - 2 for e in self.ne]))   # interior B-splines (simple interior knots)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._destroy(h)
            self.handle = None


def wq_eval_setup(p: int, knots: Sequence[np.ndarray], ctrl: np.ndarray, ng: int,
                  weights: Optional[np.ndarray] = None, device="cuda", stream=None) -> WqEval:
    """Evaluator at ng Gauss points per element and direction on the map (ctrl, weights) of wq_setup."""
    ks, nk, kp = _knots(knots)
    ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
    m = [len(k) - p - 1 for k in ks]
    if p >= 1 and min(m) > 0 and ctrl.size != 3 * m[0] * m[1] * m[2]:
        raise ValueError(f"ctrl: need {m[2]} x {m[1]} x {m[0]} control points of 3 coordinates, got {ctrl.size} values")
    wp = C.c_void_p(0)
    if weights is not None:
        weights = np.ascontiguousarray(weights, dtype=np.float64)
        if weights.size != m[0] * m[1] * m[2]:
            raise ValueError(f"weights: need {m[2]} x {m[1]} x {m[0]} values, got {weights.size}")
        wp = C.c_void_p(weights.ctypes.data)
    L = lib()
    need = C.c_size_t(0)
    h = C.c_void_p(0)
    check(L.wq_eval_setup(p, nk, kp, C.c_void_p(ctrl.ctypes.data), wp, ng, None, 0, C.byref(need), _stream(stream),
                          C.byref(h)), "wq_eval_setup(size)")
    ws = torch.empty(need.value, dtype=torch.uint8, device=device)
    check(L.wq_eval_setup(p, nk, kp, C.c_void_p(ctrl.ctypes.data), wp, ng, _p(ws), need.value, None,
                          _stream(stream), C.byref(h)), "wq_eval_setup")
    return WqEval(h, ws, p, ng, device)


def wq_eval_slab(E: WqEval, u: torch.Tensor, e3_begin: int, e3_end: int, out=None, stream=None):
    """(X [3, n], wdet [n], uh [n], grad [3, n]) at the Gauss points of elements [e3_begin, e3_end) along z."""
    n = E.nq[0] * E.nq[1] * (e3_end - e3_begin) * E.ng
    if out is None:
        out = tuple(torch.empty(k * n, dtype=torch.float64, device=E.device) for k in (3, 1, 1, 3))
    X, wdet, uh, grad = out
    for t, k, name in ((X, 3, "X"), (wdet, 1, "wdet"), (uh, 1, "uh"), (grad, 3, "grad")):
        _need(t, torch.float64, k * n, name)
    _need(u, torch.float64, E.N, "u")
    if not (0 <= e3_begin <= e3_end <= E.ne[2]):
        raise ValueError(f"element range [{e3_begin}, {e3_end}) outside [0, {E.ne[2]}]")
    check(lib().wq_eval_slab(E.handle, _p(u), e3_begin, e3_end, _p(X), _p(wdet), _p(uh), _p(grad),
                             _stream(stream)), "wq_eval_slab")
    return X.view(3, n), wdet, uh, grad.view(3, n)


def wq_setup(p: int, knots: Sequence[np.ndarray], ctrl: np.ndarray, k_kind: int = WQ_K_IDENTITY,
             K_q: Optional[torch.Tensor] = None, prec_mask: int = WQ_F64, device="cuda", stream=None,
             rule: str = "wq", weights: Optional[np.ndarray] = None) -> WqOp:
    """rule "wq": weighted quadrature (wq_setup, or wq_setup_nurbs with control weights); "gauss": p + 1 Gauss
    points per element (wq_setup_gauss).

    ctrl holds the control points [m3][m2][m1][3] (m_l = len(knots[l]) - p - 1), weights (optional) the
    positive control weights [m3][m2][m1] of a rational map; a conductivity K_q is installed with wq_set_coef
    once the operator exists, so that its size is checked against N_q."""
    ks, nk, kp = _knots(knots)
    ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
    m = [len(k) - p - 1 for k in ks]
    if p >= 1 and min(m) > 0 and ctrl.size != 3 * m[0] * m[1] * m[2]:
        raise ValueError(f"ctrl: need {m[2]} x {m[1]} x {m[0]} control points of 3 coordinates, got {ctrl.size} values")
    if k_kind not in _K_PLANES:
        raise ValueError(f"unknown k_kind {k_kind}")
    if k_kind != WQ_K_IDENTITY and K_q is None:
        raise ValueError("K_q is required for this k_kind")
    L = lib()
    if weights is not None:
        if rule != "wq":
            raise ValueError("control weights are supported with rule 'wq'")
        weights = np.ascontiguousarray(weights, dtype=np.float64)
        if p >= 1 and min(m) > 0 and weights.size != m[0] * m[1] * m[2]:
            raise ValueError(f"weights: need {m[2]} x {m[1]} x {m[0]} values, got {weights.size}")
        wp = C.c_void_p(weights.ctypes.data)
        name = "wq_setup_nurbs"

        def fn(p_, nk_, kp_, c_, *rest):
            return L.wq_setup_nurbs(p_, nk_, kp_, c_, wp, *rest)
    else:
        fn, name = {"wq": (L.wq_setup, "wq_setup"), "gauss": (L.wq_setup_gauss, "wq_setup_gauss")}[rule]
    need = C.c_size_t(0)
    h = C.c_void_p(0)
    check(fn(p, nk, kp, C.c_void_p(ctrl.ctypes.data), WQ_K_IDENTITY, C.c_void_p(0), prec_mask, None, 0,
             C.byref(need), _stream(stream), C.byref(h)), name + "(size)")
    ws = torch.empty(need.value, dtype=torch.uint8, device=device)
    check(fn(p, nk, kp, C.c_void_p(ctrl.ctypes.data), WQ_K_IDENTITY, C.c_void_p(0), prec_mask, _p(ws), need.value,
             None, _stream(stream), C.byref(h)), name)
    op = WqOp(h, ws, p, prec_mask, WQ_K_IDENTITY, device)
    if k_kind != WQ_K_IDENTITY:
        wq_set_coef(op, k_kind, K_q, stream)
    return op


def wq_dims(op: WqOp) -> Tuple[Tuple[int, int, int], Tuple[int, int, int]]:
    return op.n, op.nq


def wq_quad_points(op: WqOp, stream=None):
    """(xq: three numpy arrays of parametric points, Fq: device tensor [3, N_q])."""
    xq = np.empty(sum(op.nq))
    Fq = torch.empty(3, op.Nq, dtype=torch.float64, device=op.device)
    check(lib().wq_quad_points(op.handle, C.c_void_p(xq.ctypes.data), _p(Fq), _stream(stream)), "wq_quad_points")
    o = np.cumsum((0,) + op.nq)
    return [xq[o[i]:o[i + 1]] for i in range(3)], Fq


def wq_detj(op: WqOp, stream=None) -> torch.Tensor:
    d = torch.empty(op.Nq, dtype=torch.float64, device=op.device)
    check(lib().wq_detj(op.handle, _p(d), _stream(stream)), "wq_detj")
    return d


def wq_set_coef(op: WqOp, k_kind: int, K_q: Optional[torch.Tensor] = None, stream=None):
    """Conductivity at the quadrature points: None for K = I, [N_q] for WQ_K_SCALAR, [6][N_q] for WQ_K_SYM6."""
    if k_kind not in _K_PLANES:
        raise ValueError(f"unknown k_kind {k_kind}")
    if k_kind != WQ_K_IDENTITY:
        if K_q is None:
            raise ValueError("K_q is required for this k_kind")
        K_q = K_q.contiguous()
        _need(K_q, torch.float64, _K_PLANES[k_kind] * op.Nq, "K_q")
    else:
        K_q = None
    check(lib().wq_set_coef(op.handle, k_kind, _p(K_q), _stream(stream)), "wq_set_coef")
    op.k_kind = k_kind


def wq_set_alpha(op: WqOp, alpha_q: Optional[torch.Tensor], stream=None):
    """Reaction coefficient alpha at the quadrature points ([N_q] FP64), or None to remove it."""
    if alpha_q is not None:
        alpha_q = alpha_q.contiguous()
        _need(alpha_q, torch.float64, op.Nq, "alpha_q")
    check(lib().wq_set_alpha(op.handle, _p(alpha_q), _stream(stream)), "wq_set_alpha")


def _apply(fn, name, op, v, w, prec, stream):
    prec = prec or (WQ_F64 if v.dtype == torch.float64 else WQ_F32)
    _need(v, _DT[prec], op.N, "v")
    if w is None:
        w = torch.empty_like(v)
    _need(w, _DT[prec], op.N, "w")
    check(fn(op.handle, prec, _p(v), _p(w), _stream(stream)), name)
    return w


def wq_apply(op: WqOp, v: torch.Tensor, w: Optional[torch.Tensor] = None, prec: Optional[int] = None,
             stream=None) -> torch.Tensor:
    return _apply(lib().wq_apply, "wq_apply", op, v, w, prec, stream)


def wq_apply_T(op: WqOp, v: torch.Tensor, w: Optional[torch.Tensor] = None, prec: Optional[int] = None,
               stream=None) -> torch.Tensor:
    return _apply(lib().wq_apply_T, "wq_apply_T", op, v, w, prec, stream)


def wq_apply_acc(op: WqOp, v: torch.Tensor, w: torch.Tensor, prec: Optional[int] = None, stream=None) -> torch.Tensor:
    """w += K~ v in place (fused operators, p <= 7)."""
    return _apply(lib().wq_apply_acc, "wq_apply_acc", op, v, w, prec, stream)


def wq_alpha_mean(op: WqOp, stream=None) -> float:
    """Mean of the reaction diagonal alpha det J over the quadrature points (the
    FD shift of the reaction term), computed by the library."""
    m = C.c_double(0.0)
    check(lib().wq_alpha_mean(op.handle, C.byref(m), _stream(stream)), "wq_alpha_mean")
    return m.value


def wq_apply_mass(op: WqOp, v: torch.Tensor, w: Optional[torch.Tensor] = None, prec: Optional[int] = None,
                  stream=None) -> torch.Tensor:
    """w = M~ v (Algorithm 1) for the reaction coefficient set by wq_set_alpha."""
    return _apply(lib().wq_apply_mass, "wq_apply_mass", op, v, w, prec, stream)


def wq_rhs(op: WqOp, f_q: torch.Tensor, b: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    _need(f_q, torch.float64, op.Nq, "f_q")
    b = torch.empty(op.N, dtype=torch.float64, device=op.device) if b is None else b
    _need(b, torch.float64, op.N, "b")
    check(lib().wq_rhs(op.handle, _p(f_q), _p(b), _stream(stream)), "wq_rhs")
    return b


def wq_grad_K(op: WqOp, lam: torch.Tensor, u: torch.Tensor, gK: Optional[torch.Tensor] = None,
              stream=None) -> torch.Tensor:
    _need(lam, torch.float64, op.N, "lam")
    _need(u, torch.float64, op.N, "u")
    planes = {WQ_K_IDENTITY: 6, WQ_K_SCALAR: 1, WQ_K_SYM6: 6}[op.k_kind]
    gK = torch.empty(planes * op.Nq, dtype=torch.float64, device=op.device) if gK is None else gK
    _need(gK, torch.float64, planes * op.Nq, "gK")
    check(lib().wq_grad_K(op.handle, _p(lam), _p(u), _p(gK), _stream(stream)), "wq_grad_K")
    return gK


def wq_grad_f(op: WqOp, lam: torch.Tensor, gf: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    _need(lam, torch.float64, op.N, "lam")
    gf = torch.empty(op.Nq, dtype=torch.float64, device=op.device) if gf is None else gf
    _need(gf, torch.float64, op.Nq, "gf")
    check(lib().wq_grad_f(op.handle, _p(lam), _p(gf), _stream(stream)), "wq_grad_f")
    return gf


def wq_grad_Kf(op: WqOp, lam: torch.Tensor, u: torch.Tensor, gK: Optional[torch.Tensor] = None,
               gf: Optional[torch.Tensor] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """(dJ/dK, dJ/df) in one pass (wq_grad_Kf)."""
    _need(lam, torch.float64, op.N, "lam")
    _need(u, torch.float64, op.N, "u")
    planes = {WQ_K_IDENTITY: 6, WQ_K_SCALAR: 1, WQ_K_SYM6: 6}[op.k_kind]
    gK = torch.empty(planes * op.Nq, dtype=torch.float64, device=op.device) if gK is None else gK
    gf = torch.empty(op.Nq, dtype=torch.float64, device=op.device) if gf is None else gf
    _need(gK, torch.float64, planes * op.Nq, "gK")
    _need(gf, torch.float64, op.Nq, "gf")
    check(lib().wq_grad_Kf(op.handle, _p(lam), _p(u), _p(gK), _p(gf), _stream(stream)), "wq_grad_Kf")
    return gK, gf


def wq_grad_alpha(op: WqOp, lam: torch.Tensor, u: torch.Tensor, g: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    _need(lam, torch.float64, op.N, "lam")
    _need(u, torch.float64, op.N, "u")
    g = torch.empty(op.Nq, dtype=torch.float64, device=op.device) if g is None else g
    _need(g, torch.float64, op.Nq, "g")
    check(lib().wq_grad_alpha(op.handle, _p(lam), _p(u), _p(g), _stream(stream)), "wq_grad_alpha")
    return g


def fd_setup(p: int, knots: Sequence[np.ndarray], prec_mask: int = WQ_F64, device="cuda", stream=None) -> FdPc:
    ks, nk, kp = _knots(knots)
    need = C.c_size_t(0)
    h = C.c_void_p(0)
    L = lib()
    check(L.fd_setup(p, nk, kp, prec_mask, None, 0, C.byref(need), _stream(stream), C.byref(h)), "fd_setup(size)")
    ws = torch.empty(need.value, dtype=torch.uint8, device=device)
    check(L.fd_setup(p, nk, kp, prec_mask, _p(ws), need.value, None, _stream(stream), C.byref(h)), "fd_setup")
    n = tuple(len(k) - p - 3 for k in ks)
    return FdPc(h, ws, n, prec_mask, device)


def fd_apply(P: FdPc, r: torch.Tensor, z: Optional[torch.Tensor] = None, prec: Optional[int] = None,
             stream=None) -> torch.Tensor:
    prec = prec or (WQ_F64 if r.dtype == torch.float64 else WQ_F32)
    _need(r, _DT[prec], P.N, "r")
    z = torch.empty_like(r) if z is None else z
    _need(z, _DT[prec], P.N, "z")
    check(lib().fd_apply(P.handle, prec, _p(r), _p(z), _stream(stream)), "fd_apply")
    return z


def fd_apply_noalloc(P: FdPc, r: torch.Tensor, z: torch.Tensor, prec: Optional[int] = None, stream=None) -> torch.Tensor:
    """z = P^{-1} r with the library's static scratch instead of the
    preconditioner's workspace (the C call allocates nothing; z must be given)."""
    prec = prec or (WQ_F64 if r.dtype == torch.float64 else WQ_F32)
    _need(r, _DT[prec], P.N, "r")
    _need(z, _DT[prec], P.N, "z")
    check(lib().fd_apply_noalloc(P.handle, prec, _p(r), _p(z), _stream(stream)), "fd_apply_noalloc")
    return z


def fd_set_shift(P: FdPc, sigma: float, stream=None):
    """Add sigma M3 x M2 x M1 to the FD operator (reaction term); 0 removes it."""
    check(lib().fd_set_shift(P.handle, float(sigma), _stream(stream)), "fd_set_shift")


def fd_factors(P: FdPc, l: int):
    n = P.n[l]
    lam = np.empty(n)
    U = np.empty((n, n))
    check(lib().fd_factors(P.handle, l, C.c_void_p(lam.ctypes.data), C.c_void_p(U.ctypes.data)), "fd_factors")
    return lam, U


def krylov_solve(A: WqOp, P: FdPc, b: torch.Tensor, x: Optional[torch.Tensor] = None, transpose: bool = False,
                 rtol: float = 1e-10, maxit: int = 2000, ws: Optional[torch.Tensor] = None, stream=None,
                 raise_on_noconv: bool = True):
    """Right-preconditioned BiCGStab in FP64.  Returns (x, iterations, relres)."""
    _need(b, torch.float64, A.N, "b")
    x = torch.zeros_like(b) if x is None else x
    _need(x, torch.float64, A.N, "x")
    nb = lib().krylov_ws_bytes(A.handle)
    if ws is None:
        ws = torch.empty(nb, dtype=torch.uint8, device=A.device)
        _keep_for(ws, stream)
    wsb = _ws_bytes(ws, nb, "ws")
    it, rel = C.c_int(0), C.c_double(0)
    rc = lib().krylov_solve(A.handle, P.handle, int(transpose), _p(b), _p(x), rtol, maxit, _p(ws), wsb,
                            C.byref(it), C.byref(rel), _stream(stream))
    if rc != 0 and (raise_on_noconv or rc != -6):
        check(rc, "krylov_solve")
    return x, it.value, rel.value


def ir_solve(A: WqOp, P: FdPc, b: torch.Tensor, x: Optional[torch.Tensor] = None, fd_prec: int = WQ_BF16,
             rtol: float = 1e-10, tau_inner: float = 1e-3, max_outer: int = 30, maxit_inner: int = 500,
             ws: Optional[torch.Tensor] = None, stream=None):
    """Mixed-precision iterative refinement.  Returns (x, outer, inner_total, relres)."""
    _need(b, torch.float64, A.N, "b")
    x = torch.zeros_like(b) if x is None else x
    _need(x, torch.float64, A.N, "x")
    nb = lib().ir_ws_bytes(A.handle)
    if ws is None:
        ws = torch.empty(nb, dtype=torch.uint8, device=A.device)
        _keep_for(ws, stream)
    wsb = _ws_bytes(ws, nb, "ws")
    outer, inner, rel = C.c_int(0), C.c_int(0), C.c_double(0)
    check(lib().ir_solve(A.handle, P.handle, fd_prec, _p(b), _p(x), rtol, tau_inner, max_outer, maxit_inner, _p(ws),
                         wsb, C.byref(outer), C.byref(inner), C.byref(rel), _stream(stream)), "ir_solve")
    return x, outer.value, inner.value, rel.value


def krylov_restart_count() -> int:
    """Number of BiCGStab restarts from the true residual (a converged recurrence
    residual whose true residual missed the tolerance) in this thread's solves."""
    return int(lib().krylov_restart_count())


def ir_fallback_count() -> int:
    """Number of ir_solve calls of this thread that switched to FP64 inner
    solves after a stagnating outer step."""
    return int(lib().ir_fallback_count())
