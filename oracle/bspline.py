"""Univariate B-splines by the Cox-de Boor recursion and exact 1D Galerkin
integrals (Section 2.1).  Part of the CPU oracle (test infrastructure only).

Definitions (Section 2.1): open knot vector Xi = (xi_0 .. xi_{m+p}), 0-based,
with p+1 repeated end knots; B-splines b_0 .. b_{m-1} of degree p.

    N_{i,0}(x) = 1 if xi_i <= x < xi_{i+1} else 0
    N_{i,k}(x) = (x - xi_i)/(xi_{i+k} - xi_i) N_{i,k-1}(x)
               + (xi_{i+k+1} - x)/(xi_{i+k+1} - xi_{i+1}) N_{i+1,k-1}(x)      (0/0 := 0)
    N'_{i,p}(x) = p/(xi_{i+p} - xi_i) N_{i,p-1}(x) - p/(xi_{i+p+1} - xi_{i+1}) N_{i+1,p-1}(x)

Reading R4: the right end x = 1 is evaluated as the left limit (the last
non-empty knot span is taken closed on the right).
"""
from __future__ import annotations

import numpy as np


def n_basis(knots, p: int) -> int:
    return len(knots) - p - 1


def breakpoints(knots) -> np.ndarray:
    """Distinct knot values t_0 < t_1 < ... < t_{n_el}."""
    return np.unique(np.asarray(knots, dtype=np.float64))


def _degree_tables(knots, p: int, x):
    """All degree-k tables N_{i,k}(x), k = 0..p, as a list of [len(x), nk-1-k] arrays."""
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nk = len(t)
    N0 = np.zeros((len(x), nk - 1))
    for i in range(nk - 1):
        N0[:, i] = (t[i] <= x) & (x < t[i + 1])
    # R4: x equal to the last knot belongs to the last non-empty span
    last = max(i for i in range(nk - 1) if t[i] < t[i + 1])
    at_end = x == t[-1]
    N0[at_end, :] = 0.0
    N0[at_end, last] = 1.0
    tables = [N0]
    for k in range(1, p + 1):
        prev = tables[-1]
        cur = np.zeros((len(x), nk - 1 - k))
        for i in range(nk - 1 - k):
            d1 = t[i + k] - t[i]
            d2 = t[i + k + 1] - t[i + 1]
            if d1 > 0:
                cur[:, i] += (x - t[i]) / d1 * prev[:, i]
            if d2 > 0:
                cur[:, i] += (t[i + k + 1] - x) / d2 * prev[:, i + 1]
        tables.append(cur)
    return tables


def basis_matrix(knots, p: int, x, deriv: int = 0) -> np.ndarray:
    """[len(x), m] matrix of b_j(x) (deriv=0) or b_j'(x) (deriv=1), all j = 0..m-1."""
    t = np.asarray(knots, dtype=np.float64)
    m = n_basis(t, p)
    tables = _degree_tables(t, p, x)
    if deriv == 0:
        return tables[p][:, :m].copy()
    if deriv != 1:
        raise ValueError("only first derivatives are needed by the method")
    lower = tables[p - 1]
    out = np.zeros((lower.shape[0], m))
    for i in range(m):
        d1 = t[i + p] - t[i]
        d2 = t[i + p + 1] - t[i + 1]
        if d1 > 0:
            out[:, i] += p / d1 * lower[:, i]
        if d2 > 0:
            out[:, i] -= p / d2 * lower[:, i + 1]
    return out


def support(knots, p: int, j: int):
    """Closed support [xi_j, xi_{j+p+1}] of b_j."""
    t = np.asarray(knots, dtype=np.float64)
    return t[j], t[j + p + 1]


def gauss_points(knots, nper: int):
    """Gauss-Legendre points and weights, ``nper`` per non-empty knot span."""
    g, gw = np.polynomial.legendre.leggauss(nper)
    br = breakpoints(knots)
    xs, ws = [], []
    for a, b in zip(br[:-1], br[1:]):
        xs.append(0.5 * (b - a) * g + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * gw)
    return np.concatenate(xs), np.concatenate(ws)


def galerkin_1d(knots, p: int, a: int, b: int) -> np.ndarray:
    """G^{ab}_{ij} = int_0^1 b_i^{(a)} b_j^{(b)} dxi for all i, j = 0..m-1, by Gauss
    quadrature with p+1 points per span (exact: the integrand has degree <= 2p)."""
    x, w = gauss_points(knots, p + 1)
    Ba = basis_matrix(knots, p, x, a)
    Bb = basis_matrix(knots, p, x, b)
    return Ba.T @ (w[:, None] * Bb)
