"""Build device handles for a synthetic workload (``synth.Workload``): the MF-WQ
operator, the coefficient field K at the quadrature points, the load vector and
the FD preconditioner.  Every computation runs in libwqfd.so; the coefficient
and source fields are evaluated with torch on the device at the physical
quadrature points the library reports."""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import wqfd
from .wqfd import WQ_BF16, WQ_F32, WQ_F64, WQ_K_IDENTITY, WQ_K_SCALAR, WQ_K_SYM6


@dataclasses.dataclass
class DeviceProblem:
    A: wqfd.WqOp
    P: wqfd.FdPc
    b: torch.Tensor
    K_q: Optional[torch.Tensor]
    f_q: torch.Tensor
    Fq: torch.Tensor
    k_kind: int


def K_at(wl, Fq: torch.Tensor):
    """(k_kind, K_q) of the workload at physical points Fq [3, N_q]."""
    fn = wl.K_field()
    if fn is None:
        return WQ_K_IDENTITY, None
    X = Fq.t().contiguous()
    K = fn(X)
    if wl.k_kind == "scalar":
        return WQ_K_SCALAR, K.contiguous()
    return WQ_K_SYM6, K.t().contiguous().reshape(-1)


def build(wl, prec_mask: int = WQ_F64, fd_prec_mask: int = WQ_F64, device="cuda", rule: str = "wq") -> DeviceProblem:
    knots = wl.knots()
    A = wqfd.wq_setup(wl.p, knots, wl.ctrl(), WQ_K_IDENTITY, None, prec_mask, device, rule=rule,
                      weights=wl.weights())
    _, Fq = wqfd.wq_quad_points(A)
    kind, K_q = K_at(wl, Fq)
    if kind != WQ_K_IDENTITY:
        wqfd.wq_set_coef(A, kind, K_q)
    f_q = wl.f()(Fq.t()).contiguous()
    b = wqfd.wq_rhs(A, f_q)
    P = wqfd.fd_setup(wl.p, knots, fd_prec_mask, device)
    return DeviceProblem(A, P, b, K_q, f_q, Fq, kind)


def set_reaction(dp: DeviceProblem, alpha_fn, stream=None) -> tuple:
    """Reaction term alpha u of the model problem: alpha_fn evaluated at the
    physical quadrature points goes to the operator (wq_set_alpha), and the FD
    preconditioner gets the shift mean(alpha det J) (wq_alpha_mean, fd_set_shift).  Returns
    (alpha_q, sigma); alpha_fn = None removes both."""
    if alpha_fn is None:
        wqfd.wq_set_alpha(dp.A, None, stream)
        wqfd.fd_set_shift(dp.P, 0.0, stream)
        return None, 0.0
    alpha_q = alpha_fn(dp.Fq.t()).contiguous()
    wqfd.wq_set_alpha(dp.A, alpha_q, stream)
    sigma = wqfd.wq_alpha_mean(dp.A, stream)
    wqfd.fd_set_shift(dp.P, sigma, stream)
    return alpha_q, sigma
