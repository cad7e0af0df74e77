"""Weighted-quadrature points and weights (Section 2.2).  CPU oracle, test
infrastructure only.

Readings of the paper used here (the library implements the same readings with
its own code):

R1 (quadrature points; the paper gives "midpoints and endpoints of each knot
   span, with a few more points in the first and last span"): all breakpoints,
   the midpoint of every element except the first and the last, and p+1
   equispaced interior points t_0 + k h/(p+2), k = 1..p+1, in the first element
   (mirrored in the last).  n_q = 2 n_el + 2 p + 1.
R2 (the local exactness systems are underdetermined and, for derivative trial
   functions, rank deficient): the minimum-2-norm solution, via an SVD
   pseudo-inverse with relative rank cut-off 1e-12.  Rows are first scaled to
   unit 2-norm: that leaves the solution set of the (consistent) system, hence
   its minimum-norm element, unchanged and makes the solve far better
   conditioned (trial functions that barely overlap supp(b_i) give tiny rows).
   On strongly graded knots the systems still reach condition numbers of 1e6
   and more, and the SVD solution then leaks into the null space of A (it is no
   longer the minimum-norm element to FP64 accuracy).  It is refined once on
   the two conditions that define the minimum-norm solution, w = A^T z (row
   space) and A w = r, with both residuals formed with exact products and one
   rounding; the correction is computed by the same pseudo-inverse.
R3 (exactness trial set): exactness is imposed for every trial B-spline b_j,
   j = 0..m-1 (boundary ones included), not only the interior ones; functions
   with |j - i| > p vanish with their first derivative on supp(b_i) for p >= 2,
   so the local system only carries |j - i| <= p.

Weights depend on (a, b) = (test derivative order, trial derivative order):
    sum_q W^{ab}_{i q} b_j^{(b)}(x_q) = int b_i^{(a)} b_j^{(b)}     (eqs. exactness1d, exactness_K)
    W^{ab}_{i q} = 0 if x_q outside supp(b_i)                         (eq. weights-support)
for interior test functions i = 1..m-2 (0-based), giving W^{ab} in R^{n x n_q}.
"""
from __future__ import annotations

import math

import numpy as np

from .bspline import basis_matrix, breakpoints, galerkin_1d, gauss_points, n_basis

RANK_RTOL = 1e-12


def quad_points(knots, p: int) -> np.ndarray:
    """Reading R1 of the point placement (Section 2.2)."""
    br = breakpoints(knots)
    n_el = len(br) - 1
    if n_el < 2:
        raise ValueError("need at least two elements")
    pts = list(br)
    for e in range(1, n_el - 1):
        pts.append(0.5 * (br[e] + br[e + 1]))
    for e in (0, n_el - 1):
        h = br[e + 1] - br[e]
        pts.extend(br[e] + k * h / (p + 2) for k in range(1, p + 2))
    return np.array(sorted(pts))


def interior_B(knots, p: int, xq, deriv: int) -> np.ndarray:
    """B_l (deriv 0) or B-dot_l (deriv 1): [n_q, n] values of the interior
    B-splines j = 1..m-2 at the quadrature points (eq. Bl and its derivative)."""
    m = n_basis(knots, p)
    return basis_matrix(knots, p, xq, deriv)[:, 1:m - 1]


def local_system(knots, p, xq, i, a, b, Bfull=None, G=None):
    """Unknown set S_i, equation set T_i, matrix A (|T_i| x |S_i|) and right-hand
    side of the exactness conditions for test function i and derivative pair (a,b)."""
    t = np.asarray(knots, dtype=np.float64)
    m = n_basis(t, p)
    if Bfull is None:
        Bfull = basis_matrix(t, p, xq, b)
    if G is None:
        G = galerkin_1d(t, p, a, b)
    lo, hi = t[i], t[i + p + 1]
    S = np.nonzero((xq >= lo) & (xq <= hi))[0]
    T = np.array([j for j in range(m) if abs(j - i) <= p])
    A = Bfull[np.ix_(S, T)].T
    rhs = G[i, T]
    return S, T, A, rhs


def _split(x):
    """Veltkamp splitting x = hi + lo, each half with at most 26 significant
    bits, so products of halves are exact in FP64."""
    c = 134217729.0 * x                      # 2^27 + 1
    hi = c - (c - x)
    return hi, x - hi


def exact_residual(A, w, r):
    """r - A w for each row, with every product A_ts w_s formed exactly (as the
    sum of four products of split halves) and the whole sum rounded once
    (math.fsum)."""
    ah, al = _split(np.asarray(A, dtype=np.float64))
    wh, wl = _split(np.asarray(w, dtype=np.float64))
    parts = [ah * wh, ah * wl, al * wh, al * wl]
    return np.array([math.fsum([float(r[t])] + [-float(x) for P in parts for x in P[t]])
                     for t in range(A.shape[0])])


def min_norm_solve(A, rhs):
    """Minimum-norm solution of the consistent system A w = rhs (reading R2):
    rows equilibrated, SVD pseudo-inverse with relative cut-off RANK_RTOL, then
    one refinement step of the pair of conditions w - A^T z = 0, A w = r:
    with f = A^T z - w and g = r - A w (exactly rounded), the correction
    dw = f + pinv(A) (g - A f) restores both."""
    d = 1.0 / np.linalg.norm(A, axis=1)
    As, rs = d[:, None] * A, d * rhs
    w, _, _, _ = np.linalg.lstsq(As, rs, rcond=RANK_RTOL)
    z, _, _, _ = np.linalg.lstsq(As.T, w, rcond=RANK_RTOL)
    f = -exact_residual(As.T, z, w)
    g = exact_residual(As, w, rs)
    dv, _, _, _ = np.linalg.lstsq(As, g - As @ f, rcond=RANK_RTOL)
    return w + (f + dv)


def weights(knots, p: int, xq=None):
    """All four 1D weight matrices {(a, b): W^{ab}} (each n x n_q)."""
    t = np.asarray(knots, dtype=np.float64)
    if xq is None:
        xq = quad_points(t, p)
    m = n_basis(t, p)
    nq = len(xq)
    Bf = {b: basis_matrix(t, p, xq, b) for b in (0, 1)}
    out = {}
    for a in (0, 1):
        for b in (0, 1):
            G = galerkin_1d(t, p, a, b)
            W = np.zeros((m - 2, nq))
            for i in range(1, m - 1):
                S, T, A, rhs = local_system(t, p, xq, i, a, b, Bf[b], G)
                W[i - 1, S] = min_norm_solve(A, rhs)
            out[(a, b)] = W
    return out


def gauss_weights(knots, p: int, xq, wq):
    """Standard Gauss quadrature written as test factors (the remark after
    rem:memory, eq. WDBgaussian): W^{ab}_{iq} = w_q b_i^{(a)}(x_q) for the
    interior i, the same for both trial orders b."""
    out = {}
    for a in (0, 1):
        Wa = (interior_B(knots, p, xq, a) * np.asarray(wq)[:, None]).T
        out[(a, 0)] = Wa
        out[(a, 1)] = Wa.copy()
    return out


class Space1D:
    """Everything one direction contributes: knots, points, B, B-dot, W^{ab}.
    rule "wq": weighted quadrature (Section 2.2); "gauss": p + 1 Gauss points per
    element with the weights as test factors (the remark after rem:memory)."""

    def __init__(self, knots, p: int, rule: str = "wq"):
        self.knots = np.asarray(knots, dtype=np.float64)
        self.p = p
        self.rule = rule
        self.m = n_basis(self.knots, p)
        self.n = self.m - 2
        if rule == "gauss":
            self.xq, self.wq = gauss_points(self.knots, p + 1)
        else:
            self.xq = quad_points(self.knots, p)
        self.nq = len(self.xq)
        self.B = {b: interior_B(self.knots, p, self.xq, b) for b in (0, 1)}
        self.Bfull = {b: basis_matrix(self.knots, p, self.xq, b) for b in (0, 1)}
        if rule == "gauss":
            self.W = gauss_weights(self.knots, p, self.xq, self.wq)
        else:
            self.W = weights(self.knots, p, self.xq)
        # interior 1D Galerkin mass and stiffness (used by FD and by pins)
        self.M = galerkin_1d(self.knots, p, 0, 0)[1:-1, 1:-1]
        self.K = galerkin_1d(self.knots, p, 1, 1)[1:-1, 1:-1]
