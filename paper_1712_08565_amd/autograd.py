"""Differentiable MF-WQ solve: u = K~(K)^{-1} b(f) as a torch autograd function.

Forward: the coefficient planes are recomputed from K_q (eq. C), the load
vector is the weighted-quadrature mass rule of det J f (Section 3.1), and
K~ u = b is solved by the library's right-preconditioned BiCGStab with the FD
preconditioner.  Backward (the adjoint of the factorisation of Section 3.2):
for an upstream gradient g = dL/du,

    lam = K~^{-T} g                              (transposed solve, same preconditioner)
    dL/dC_ab(q) = -(W^(ab)T lam)_q (B^(b) u)_q   chained through eq. C to K_q
    dL/df_q     = det J(q) (W^(00)T lam)_q

Every step runs in libwqfd.so (wq_set_coef, wq_rhs, krylov_solve, wq_grad_K,
wq_grad_f); this module only marshals tensors.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import wqfd
from .wqfd import WQ_K_IDENTITY


class _WqSolve(torch.autograd.Function):

    @staticmethod
    def forward(ctx, K_q, f_q, A, P, rtol, maxit):
        if A.k_kind != WQ_K_IDENTITY:
            if K_q is None:
                raise ValueError("K_q is required for a scalar or six-component coefficient field")
            wqfd.wq_set_coef(A, A.k_kind, K_q.detach())
        b = wqfd.wq_rhs(A, f_q.detach().contiguous())
        u, iters, relres = wqfd.krylov_solve(A, P, b, rtol=rtol, maxit=maxit)
        ctx.A, ctx.P, ctx.rtol, ctx.maxit = A, P, rtol, maxit
        ctx.has_K = K_q is not None
        ctx.save_for_backward(K_q.detach() if K_q is not None else None, u)
        return u

    @staticmethod
    def backward(ctx, gu):
        K_q, u = ctx.saved_tensors
        A, P = ctx.A, ctx.P
        need_K, need_f = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_K or need_f):
            return None, None, None, None, None, None
        if A.k_kind != WQ_K_IDENTITY:          # the handle may have been re-used since the forward
            wqfd.wq_set_coef(A, A.k_kind, K_q)
        lam, _, _ = wqfd.krylov_solve(A, P, gu.contiguous(), transpose=True, rtol=ctx.rtol, maxit=ctx.maxit)
        gK = wqfd.wq_grad_K(A, lam, u) if (need_K and ctx.has_K) else None
        if gK is not None:
            gK = gK.view_as(K_q)
        gf = wqfd.wq_grad_f(A, lam) if need_f else None
        return gK, gf, None, None, None, None


def solve(A: wqfd.WqOp, P: wqfd.FdPc, K_q: Optional[torch.Tensor], f_q: torch.Tensor,
          rtol: float = 1e-12, maxit: int = 2000) -> torch.Tensor:
    """u with K~(K_q) u = b(f_q), differentiable in K_q and f_q.

    K_q: FP64 device tensor in the layout of A's coefficient kind
    (WQ_K_SCALAR: [N_q]; WQ_K_SYM6: [6 * N_q], planes K11, K22, K33, K12, K13,
    K23), or None for WQ_K_IDENTITY.  f_q: FP64 [N_q] source samples at the
    quadrature points.  Returns u, FP64 [N] (x fastest).
    """
    return _WqSolve.apply(K_q, f_q, A, P, rtol, maxit)
