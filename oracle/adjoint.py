"""Gradients of J(u) = 1/2 |u - u_obs|_2^2, where K~(K) u = b(f), with respect to
the conductivity at the quadrature points and to the source samples f_q.
CPU oracle, test infrastructure only.

K~ = sum_{ab} W^(ab) diag(C_ab) B^(b) is linear in each C_ab(x_q), with
d K~ / d C_ab(x_q) = W^(ab)[:, q] B^(b)[q, :] (a rank-one matrix).  With the
adjoint lambda = K~^{-T} (u - u_obs):

    dJ/dC_ab(q) = -(W^(ab)^T lambda)_q (B^(b) u)_q
    dJ/df_q     =  det J(q) (W^(00)^T lambda)_q            (b = W^(00)(det J f), reading R6)
    dJ/dalpha_q = -det J(q) (W^(00)^T lambda)_q (B u)_q    (reaction term M~ = W^(00) diag(alpha det J) B)

and, through C = det J J^{-1} K J^{-T} (reading R5),
    K = kappa I :  dJ/dkappa_q = sum_ab dJ/dC_ab(q) G_ab(q),  G = det J J^{-1} J^{-T}
    K stored as (K11, K22, K33, K12, K13, K23):  H = det J J^{-T} g J^{-1},
                   dJ/dK_aa = H_aa,  dJ/dK_ab = H_ab + H_ba (a != b).
"""
from __future__ import annotations

import numpy as np

from .geometry import SYM_PAIRS
from .operator import mode


def grad_C_full(prob, lam, u):
    """g[a, b] (3, 3, nq3, nq2, nq1): dJ/dC_ab for the nine (unsymmetrised) pairs."""
    g_u = prob.grad_at_quad(u)
    Y = prob._shape(lam)
    g = np.empty((3, 3) + g_u[0].shape)
    for al in range(3):
        for be in range(3):
            g[al, be] = -prob.test_contract_T(al, be, Y) * g_u[be]
    return g


def grad_kappa(prob, lam, u):
    g = grad_C_full(prob, lam, u)
    Ji = np.linalg.inv(prob.J)
    G = prob.detJ[..., None, None] * (Ji @ np.swapaxes(Ji, -1, -2))
    return np.einsum("abxyz,xyzab->xyz", g, G)


def grad_sym6(prob, lam, u):
    g = grad_C_full(prob, lam, u)
    gm = np.moveaxis(np.moveaxis(g, 0, -1), 0, -1)   # (..., a, b)
    Ji = np.linalg.inv(prob.J)
    H = prob.detJ[..., None, None] * (np.swapaxes(Ji, -1, -2) @ gm @ Ji)
    out = np.empty((6,) + prob.detJ.shape)
    for c, (a, b) in enumerate(SYM_PAIRS):
        out[c] = H[..., a, b] if a == b else H[..., a, b] + H[..., b, a]
    return out


def grad_f(prob, lam):
    S = prob.spaces
    Y = prob._shape(lam)
    Wt = mode(S[2].W[(0, 0)].T, mode(S[1].W[(0, 0)].T, mode(S[0].W[(0, 0)].T, Y, 2), 1), 0)
    return prob.detJ * Wt


def grad_alpha(prob, lam, u):
    """dJ/dalpha at the quadrature points: M~ is linear in alpha_q with
    d M~ / d alpha_q = det J(q) W^(00)[:, q] B[q, :]."""
    return -prob.detJ * prob.W00_T(prob._shape(lam)) * prob.values_at_quad(u)
