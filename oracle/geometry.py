"""Spline geometry map, Jacobian and coefficient tensor (Section 2.1, eq. C).
CPU oracle, test infrastructure only.

F(xi) = sum_k P_k b_k(xi) over all m1 m2 m3 tensor B-splines (single patch,
polynomial spline), or for a rational (NURBS) map with control weights w_k,
F = sum_k w_k P_k b_k / sum_k w_k b_k (Section 2.1 states that the method
carries over to NURBS, and Section 4 computes on the NURBS ring): numerator and
denominator are polynomial splines and J follows from the quotient rule.  The
discrete space stays the B-spline space.  J_{ab} = dF_a / dxi_b.  Physical gradients satisfy
grad_x b = J^{-T} grad_xi b-hat, so the stiffness integrand in parametric
coordinates carries

    C = det(J) J^{-1} K J^{-T}                                      (reading R5)

(the paper's eq. C writes the same tensor with the transposed-Jacobian
convention).  Component order of the six stored planes:
(C11, C22, C33, C12, C13, C23); index 1 is the x direction (fastest).
"""
from __future__ import annotations

import numpy as np

SYM_PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def tensor_apply(A3, A2, A1, X):
    """(A3 (x) A2 (x) A1) applied to a 3D array X[k3, k2, k1]."""
    return np.einsum("ck,bj,ai,kji->cba", A3, A2, A1, X, optimize=True)


def map_from_bases(B, D, ctrl, weights=None):
    """F (k3, k2, k1, 3) and J (k3, k2, k1, 3, 3) at the tensor grid of points whose
    basis values are B[l] (points x functions) and first derivatives D[l],
    l = 0, 1, 2 for x, y, z; ``weights`` [k3, k2, k1] for a rational map."""
    comps = [ctrl[..., a] for a in range(3)]
    if weights is not None:
        comps = [weights * c for c in comps] + [weights]
    val = [tensor_apply(B[2], B[1], B[0], c) for c in comps]
    der = []
    for c in comps:
        row = []
        for b in range(3):
            M = [D[l] if l == b else B[l] for l in range(3)]
            row.append(tensor_apply(M[2], M[1], M[0], c))
        der.append(row)
    J = np.empty(val[0].shape + (3, 3))
    if weights is None:
        F = np.stack(val, -1)
        for a in range(3):
            for b in range(3):
                J[..., a, b] = der[a][b]
        return F, J
    W = val[3]
    F = np.stack([val[a] / W for a in range(3)], -1)
    for a in range(3):
        for b in range(3):
            J[..., a, b] = (der[a][b] - F[..., a] * der[3][b]) / W
    return F, J


def map_and_jacobian(spaces, ctrl, weights=None):
    """F (nq3, nq2, nq1, 3) and J (nq3, nq2, nq1, 3, 3) at the quadrature points.
    ``spaces`` = (S1, S2, S3) oracle.wq.Space1D objects, ``ctrl`` = P[k3, k2, k1, :],
    ``weights`` = w[k3, k2, k1] for a rational map (None: polynomial)."""
    return map_from_bases([S.Bfull[0] for S in spaces], [S.Bfull[1] for S in spaces], ctrl, weights)


def coefficient_tensor(J, K=None):
    """C = det(J) J^{-1} K J^{-T} at every point; K is None (identity), an array of
    scalars kappa (K = kappa I) or an array (..., 6) of stored components."""
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0):
        raise ValueError("geometry map is not orientation preserving (det J <= 0)")
    Ji = np.linalg.inv(J)
    if K is None:
        Km = np.broadcast_to(np.eye(3), J.shape)
    elif np.ndim(K) == J.ndim - 2:
        Km = K[..., None, None] * np.eye(3)
    else:
        Km = np.empty(J.shape)
        for c, (a, b) in enumerate(SYM_PAIRS):
            Km[..., a, b] = K[..., c]
            Km[..., b, a] = K[..., c]
    C = detJ[..., None, None] * (Ji @ Km @ np.swapaxes(Ji, -1, -2))
    return C, detJ


def coefficient_planes(C):
    """Six stored planes (C11, C22, C33, C12, C13, C23), each (nq3, nq2, nq1)."""
    return np.stack([C[..., a, b] for a, b in SYM_PAIRS], 0)
