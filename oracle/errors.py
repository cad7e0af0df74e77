"""H1-seminorm and L2 errors of a discrete solution against an exact one,
integrated by Gauss quadrature with p+3 points per element in physical
coordinates (the error measure of Section 4, Table 1).  CPU oracle, test
infrastructure only."""
from __future__ import annotations

import numpy as np

from .bspline import basis_matrix, gauss_points
from .geometry import map_from_bases, tensor_apply


def gauss_point_values(knots3, p, ctrl, u_coef, ng, weights=None):
    """At the tensor Gauss points (ng per element and direction, ascending, x
    fastest): F (k3, k2, k1, 3), w |det J| (k3, k2, k1), u_h and its physical
    gradient J^{-T} grad_xi u_h (k3, k2, k1, 3), for u_h = sum_j u_j b_j with the
    interior coefficients u_coef."""
    pts, wts, B, D = [], [], [], []
    for k in knots3:
        x, w = gauss_points(k, ng)
        pts.append(x)
        wts.append(w)
        B.append(basis_matrix(k, p, x, 0))
        D.append(basis_matrix(k, p, x, 1))
    F, J = map_from_bases(B, D, ctrl, weights)
    n = [b.shape[1] - 2 for b in B]
    U = np.zeros((n[2] + 2, n[1] + 2, n[0] + 2))
    U[1:-1, 1:-1, 1:-1] = np.asarray(u_coef).reshape(n[2], n[1], n[0])
    uh = tensor_apply(B[2], B[1], B[0], U)
    gxi = []
    for b in range(3):
        M = [D[l] if l == b else B[l] for l in range(3)]
        gxi.append(tensor_apply(M[2], M[1], M[0], U))
    gxi = np.stack(gxi, -1)
    detJ = np.linalg.det(J)
    gx = np.einsum("...ba,...b->...a", np.linalg.inv(J), gxi)   # J^{-T} grad_xi
    wq = np.einsum("k,j,i->kji", wts[2], wts[1], wts[0]) * np.abs(detJ)
    return F, wq, uh, gx


def errors(knots3, p, ctrl, u_coef, u_fn, grad_fn, weights=None):
    """Relative (L2, H1-seminorm) errors of u_h = sum_j u_j b_j o F^{-1} (interior
    coefficients, x fastest) against u_fn and its gradient grad_fn (callables on
    (..., 3) physical points; grad_fn returns (..., 3)).  The exact gradient is
    required: a difference quotient would put a floor of about 1e-10 under the
    H1 figure, above the finest errors of Table 1.  ``weights``: control weights
    of a rational map (the discrete space stays the B-spline space)."""
    F, wq, uh, gx = gauss_point_values(knots3, p, ctrl, u_coef, p + 3, weights)
    ue = u_fn(F)
    ge = grad_fn(F)
    l2 = np.sqrt(np.sum(wq * (uh - ue) ** 2) / np.sum(wq * ue ** 2))
    h1 = np.sqrt(np.sum(wq[..., None] * (gx - ge) ** 2) / np.sum(wq[..., None] * ge ** 2))
    return l2, h1
