"""Differentiable MF-WQ solve: u = (K~(K) + M~(alpha))^{-1} b(f) as a torch
autograd function (M~: the reaction term, Section 3.1, when alpha is given).

Forward: the coefficient planes are recomputed from K_q (eq. C), the load
vector is the weighted-quadrature mass rule of det J f (Section 3.1), and
K~ u = b is solved by the library's right-preconditioned BiCGStab with the FD
preconditioner.  Backward (the adjoint of the factorisation of Section 3.2):
for an upstream gradient g = dL/du,

    lam = K~^{-T} g                              (transposed solve, same preconditioner)
    dL/dC_ab(q) = -(W^(ab)T lam)_q (B^(b) u)_q   chained through eq. C to K_q
    dL/df_q     = det J(q) (W^(00)T lam)_q
    dL/dalpha_q = -det J(q) (W^(00)T lam)_q (B u)_q

Every step runs in libwqfd.so (wq_set_coef, wq_set_alpha, wq_rhs, krylov_solve,
wq_grad_K, wq_grad_f, wq_grad_Kf, wq_grad_alpha); this module only marshals tensors.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import wqfd
from .wqfd import WQ_K_IDENTITY


class _WqSolve(torch.autograd.Function):

    @staticmethod
    def forward(ctx, K_q, f_q, alpha_q, A, P, rtol, maxit):
        if A.k_kind != WQ_K_IDENTITY:
            if K_q is None:
                raise ValueError("K_q is required for a scalar or six-component coefficient field")
            wqfd.wq_set_coef(A, A.k_kind, K_q.detach())
        wqfd.wq_set_alpha(A, alpha_q.detach().contiguous() if alpha_q is not None else None)
        b = wqfd.wq_rhs(A, f_q.detach().contiguous())
        u, iters, relres = wqfd.krylov_solve(A, P, b, rtol=rtol, maxit=maxit)
        ctx.A, ctx.P, ctx.rtol, ctx.maxit = A, P, rtol, maxit
        ctx.has_K, ctx.has_alpha = K_q is not None, alpha_q is not None
        ctx.save_for_backward(K_q.detach() if K_q is not None else None,
                              alpha_q.detach().contiguous() if alpha_q is not None else None, u)
        return u

    @staticmethod
    def backward(ctx, gu):
        K_q, alpha_q, u = ctx.saved_tensors
        A, P = ctx.A, ctx.P
        need_K, need_f, need_a = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        if not (need_K or need_f or need_a):
            return None, None, None, None, None, None, None
        # the handle may have been re-used since the forward: restore its coefficients
        if A.k_kind != WQ_K_IDENTITY:
            wqfd.wq_set_coef(A, A.k_kind, K_q)
        wqfd.wq_set_alpha(A, alpha_q)
        lam, _, _ = wqfd.krylov_solve(A, P, gu.contiguous(), transpose=True, rtol=ctx.rtol, maxit=ctx.maxit)
        want_K = need_K and ctx.has_K
        if want_K and need_f:
            gK, gf = wqfd.wq_grad_Kf(A, lam, u)          # one pass for both
        else:
            gK = wqfd.wq_grad_K(A, lam, u) if want_K else None
            gf = wqfd.wq_grad_f(A, lam) if need_f else None
        if gK is not None:
            gK = gK.view_as(K_q)
        ga = wqfd.wq_grad_alpha(A, lam, u) if (need_a and ctx.has_alpha) else None
        return gK, gf, ga, None, None, None, None


def solve(A: wqfd.WqOp, P: wqfd.FdPc, K_q: Optional[torch.Tensor], f_q: torch.Tensor,
          rtol: float = 1e-12, maxit: int = 2000, alpha_q: Optional[torch.Tensor] = None) -> torch.Tensor:
    """u with (K~(K_q) + M~(alpha_q)) u = b(f_q), differentiable in K_q, f_q and alpha_q.

    K_q: FP64 device tensor in the layout of A's coefficient kind
    (WQ_K_SCALAR: [N_q]; WQ_K_SYM6: [6 * N_q], planes K11, K22, K33, K12, K13,
    K23), or None for WQ_K_IDENTITY.  f_q: FP64 [N_q] source samples at the
    quadrature points.  alpha_q: FP64 [N_q] reaction coefficient at the
    quadrature points, or None for none (the operator's reaction term is set
    from it; the preconditioner P is used as given).  Returns u, FP64 [N].
    """
    return _WqSolve.apply(K_q, f_q, alpha_q, A, P, rtol, maxit)
