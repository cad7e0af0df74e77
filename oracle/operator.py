"""The MF-WQ operator of the model problem -div(K grad u) + alpha u = f
(Sections 2.2-3.2).  CPU oracle, test infrastructure only.

K~ = sum_{alpha,beta=1..3} W^(alpha,beta) D^(alpha,beta) B^(beta)          (Section 3.2)

with, for direction l (x = 1 fastest, Kronecker order of eq. ordering):
    B^(beta)        = B_3^(b3) (x) B_2^(b2) (x) B_1^(b1),   b_l = [l == beta]
    W^(alpha,beta)  = W_3^{a3 b3} (x) W_2^{a2 b2} (x) W_1^{a1 b1},   a_l = [l == alpha]
    D^(alpha,beta)  = diag(C_{alpha beta}(x_q))
where B_l^(0) = B_l, B_l^(1) = B-dot_l and W_l^{ab} are the 1D weights of the
rule for int b_i^{(a)} b_j^{(b)} (eq. exactness_K).

With a reaction coefficient alpha (``set_alpha``) the operator is K~ + M~, where
M~ = W^(00) D B is the weighted-quadrature mass matrix of Section 3.1 (eq. WDB):
B = B_3 (x) B_2 (x) B_1, W^(00) = W_3^{00} (x) W_2^{00} (x) W_1^{00} and
D = diag(alpha(x_q) det J(x_q)) (the mass integrand pulled back to the
parametric domain).

With ``rule="gauss"`` the same factorisation holds for standard Gauss
quadrature (p + 1 points per element, test factors w_q b_i^{(a)}(x_q); the
remark after rem:memory, eq. WDBgaussian): the Gauss-quadrature Galerkin matrix.

``assemble`` builds the operator explicitly as a scipy.sparse matrix (small sizes only);
``apply`` / ``apply_T`` evaluate K~ v and K~^T v with one 1D product per mode
(eq. sum-factorization) and no fusion.  ``rhs`` is the load vector of reading
R6: b_i = sum_q W^(00)_{iq} det J(x_q) f(F(x_q)) (weighted-quadrature mass rule,
Section 3.1, eq. main).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import SYM_PAIRS, coefficient_planes, coefficient_tensor, map_and_jacobian
from .wq import Space1D

_PLANE = {}
for _c, (_a, _b) in enumerate(SYM_PAIRS):
    _PLANE[(_a, _b)] = _c
    _PLANE[(_b, _a)] = _c


def ab_indices(alpha: int, beta: int):
    """Per-direction (a_l, b_l) for the pair (alpha, beta), 0-based directions."""
    return [(int(l == alpha), int(l == beta)) for l in range(3)]


def mode(A, X, axis):
    """Apply the matrix A along ``axis`` of the 3D array X (axis 2 = x, 0 = z)."""
    return np.moveaxis(np.tensordot(A, X, axes=(1, axis)), 0, axis)


class Problem:
    """Spaces, geometry and coefficient planes of one single-patch problem."""

    def __init__(self, knots3, p, ctrl, K_fn=None, rule="wq", weights=None):
        self.p = p
        self.spaces = [Space1D(k, p, rule) for k in knots3]
        S1, S2, S3 = self.spaces
        self.n = (S1.n, S2.n, S3.n)
        self.nq = (S1.nq, S2.nq, S3.nq)
        self.N = S1.n * S2.n * S3.n
        self.Nq = S1.nq * S2.nq * S3.nq
        self.F, self.J = map_and_jacobian(self.spaces, ctrl, weights)
        self.Cm = None                          # reaction diagonal alpha det J (None: alpha = 0)
        self.set_K(K_fn(self.F) if K_fn is not None else None)

    def set_K(self, K):
        self.K = K
        C, self.detJ = coefficient_tensor(self.J, K)
        self.C = coefficient_planes(C)          # (6, nq3, nq2, nq1)

    def set_alpha(self, alpha_q):
        """Reaction coefficient alpha of the model problem at the quadrature
        points ([nq3, nq2, nq1] or flat), or None for alpha = 0.  The diagonal of
        Algorithm 1 is c_q = alpha(x_q) det J(x_q): the mass integrand
        alpha b_i b_j over the physical domain, pulled back by F."""
        if alpha_q is None:
            self.Cm = None
        else:
            self.Cm = np.asarray(alpha_q, dtype=np.float64).reshape(self.detJ.shape) * self.detJ

    # -- factors -----------------------------------------------------------
    def Wk(self, alpha, beta):
        ab = ab_indices(alpha, beta)
        S = self.spaces
        return [S[l].W[ab[l]] for l in range(3)]

    def Bk(self, beta):
        S = self.spaces
        return [S[l].B[int(l == beta)] for l in range(3)]

    def plane(self, alpha, beta):
        return self.C[_PLANE[(alpha, beta)]]

    # -- explicit assembly (small sizes) -----------------------------------
    def assemble(self, C=None):
        C = self.C if C is None else C
        K = None
        for al in range(3):
            for be in range(3):
                W1, W2, W3 = self.Wk(al, be)
                B1, B2, B3 = self.Bk(be)
                Wk = sp.kron(sp.csr_matrix(W3), sp.kron(sp.csr_matrix(W2), sp.csr_matrix(W1)))
                Bk = sp.kron(sp.csr_matrix(B3), sp.kron(sp.csr_matrix(B2), sp.csr_matrix(B1)))
                D = sp.diags(C[_PLANE[(al, be)]].ravel())
                term = (Wk @ D @ Bk).tocsr()
                K = term if K is None else K + term
        if self.Cm is not None:
            K = K + self.assemble_mass()
        return K.tocsr()

    def assemble_mass(self):
        """M~ = W^(00) D B (eq. WDB) as a sparse matrix."""
        S = self.spaces
        Wk = sp.kron(sp.csr_matrix(S[2].W[(0, 0)]),
                     sp.kron(sp.csr_matrix(S[1].W[(0, 0)]), sp.csr_matrix(S[0].W[(0, 0)])))
        Bk = sp.kron(sp.csr_matrix(S[2].B[0]), sp.kron(sp.csr_matrix(S[1].B[0]), sp.csr_matrix(S[0].B[0])))
        return (Wk @ sp.diags(self.Cm.ravel()) @ Bk).tocsr()

    # -- matrix-free products ---------------------------------------------
    def _shape(self, v, q=False, dtype=np.float64):
        n = self.nq if q else self.n
        return np.asarray(v, dtype=dtype).reshape(n[2], n[1], n[0])

    def grad_at_quad(self, v, dtype=np.float64):
        """v~^(beta) = B^(beta) v for beta = 1..3 (Algorithm 2, first step)."""
        V = self._shape(v, dtype=dtype)
        out = []
        for be in range(3):
            B1, B2, B3 = self.Bk(be)
            out.append(mode(B3, mode(B2, mode(B1, V, 2), 1), 0))
        return out

    def test_contract(self, alpha, beta, Q):
        W1, W2, W3 = self.Wk(alpha, beta)
        return mode(W3, mode(W2, mode(W1, Q, 2), 1), 0)

    def test_contract_T(self, alpha, beta, Y):
        W1, W2, W3 = self.Wk(alpha, beta)
        return mode(W3.T, mode(W2.T, mode(W1.T, Y, 2), 1), 0)

    def apply(self, v, dtype=np.float64):
        """w = K~ v following Algorithm 2 step by step (plus M~ v when alpha is set).
        dtype=np.longdouble evaluates the same steps in extended precision (the
        FP64 factors converted exactly), for residuals of reference solves."""
        g = self.grad_at_quad(v, dtype)
        w = np.zeros((self.n[2], self.n[1], self.n[0]), dtype=dtype)
        for be in range(3):
            for al in range(3):
                w += self.test_contract(al, be, self.plane(al, be) * g[be])
        if self.Cm is not None:
            w += self.mass_apply(v, dtype).reshape(w.shape)
        return w.ravel()

    def values_at_quad(self, v, dtype=np.float64):
        """v~ = (B_3 (x) B_2 (x) B_1) v, the values of v_h at the points (Algorithm 1, first step)."""
        S = self.spaces
        return mode(S[2].B[0], mode(S[1].B[0], mode(S[0].B[0], self._shape(v, dtype=dtype), 2), 1), 0)

    def mass_apply(self, v, dtype=np.float64):
        """w = M~ v by the three steps of Algorithm 1: values at the points, the
        diagonal D = diag(alpha det J), the W^(00) rules."""
        vt = self.values_at_quad(v, dtype)
        vtt = self.Cm * vt
        return self.W00(vtt).ravel()

    def mass_apply_T(self, v, dtype=np.float64):
        """w = M~^T v = B^T D W^(00)^T v."""
        S = self.spaces
        Y = self.Cm * self.W00_T(self._shape(v, dtype=dtype))
        return mode(S[2].B[0].T, mode(S[1].B[0].T, mode(S[0].B[0].T, Y, 2), 1), 0).ravel()

    def apply_T(self, v, dtype=np.float64):
        """w = K~^T v = sum_{alpha,beta} B^(beta)^T D^(alpha,beta) W^(alpha,beta)^T v
        (dtype as in ``apply``)."""
        Y = self._shape(v, dtype=dtype)
        w = np.zeros((self.n[2], self.n[1], self.n[0]), dtype=dtype)
        for be in range(3):
            acc = np.zeros((self.nq[2], self.nq[1], self.nq[0]), dtype=dtype)
            for al in range(3):
                acc += self.plane(al, be) * self.test_contract_T(al, be, Y)
            B1, B2, B3 = self.Bk(be)
            w += mode(B3.T, mode(B2.T, mode(B1.T, acc, 2), 1), 0)
        if self.Cm is not None:
            w += self.mass_apply_T(v, dtype).reshape(w.shape)
        return w.ravel()

    # -- rounding-error scales (reading R11) ---------------------------------
    def apply_abs(self, v):
        """Entry-wise rounding-error scale of ``apply``: the same chain on the
        absolute values of every factor and of v, sum_ab |W^(ab)| |D^(ab)| |B^(b)| |v|
        (plus |W^(00)| |D_alpha| |B| |v| with a reaction term).  Any evaluation order
        of K~ v in floating point differs from the exact product by at most a small
        multiple of the unit roundoff times this, entry by entry."""
        V = np.abs(self._shape(v))
        w = np.zeros((self.n[2], self.n[1], self.n[0]))
        for be in range(3):
            B1, B2, B3 = (np.abs(B) for B in self.Bk(be))
            g = mode(B3, mode(B2, mode(B1, V, 2), 1), 0)
            for al in range(3):
                W1, W2, W3 = (np.abs(W) for W in self.Wk(al, be))
                w += mode(W3, mode(W2, mode(W1, np.abs(self.plane(al, be)) * g, 2), 1), 0)
        if self.Cm is not None:
            S = self.spaces
            g = mode(np.abs(S[2].B[0]), mode(np.abs(S[1].B[0]), mode(np.abs(S[0].B[0]), V, 2), 1), 0)
            w += self._W00_abs(np.abs(self.Cm) * g)
        return w.ravel()

    def apply_T_abs(self, v):
        """Entry-wise rounding-error scale of ``apply_T``: sum_ab |B^(b)|^T |D^(ab)| |W^(ab)|^T |v|."""
        Y = np.abs(self._shape(v))
        w = np.zeros((self.n[2], self.n[1], self.n[0]))
        for be in range(3):
            acc = np.zeros((self.nq[2], self.nq[1], self.nq[0]))
            for al in range(3):
                W1, W2, W3 = (np.abs(W) for W in self.Wk(al, be))
                acc += np.abs(self.plane(al, be)) * mode(W3.T, mode(W2.T, mode(W1.T, Y, 2), 1), 0)
            B1, B2, B3 = (np.abs(B) for B in self.Bk(be))
            w += mode(B3.T, mode(B2.T, mode(B1.T, acc, 2), 1), 0)
        if self.Cm is not None:
            S = self.spaces
            Q = np.abs(self.Cm) * mode(np.abs(S[2].W[(0, 0)]).T, mode(np.abs(S[1].W[(0, 0)]).T,
                                                                         mode(np.abs(S[0].W[(0, 0)]).T, Y, 2), 1), 0)
            w += mode(np.abs(S[2].B[0]).T, mode(np.abs(S[1].B[0]).T, mode(np.abs(S[0].B[0]).T, Q, 2), 1), 0)
        return w.ravel()

    def rhs_abs(self, f_q):
        """Entry-wise rounding-error scale of ``rhs``: |W^(00)| |det J f|."""
        return self._W00_abs(np.abs(self.detJ * np.asarray(f_q).reshape(self.detJ.shape))).ravel()

    def _W00_abs(self, Q):
        S = self.spaces
        return mode(np.abs(S[2].W[(0, 0)]), mode(np.abs(S[1].W[(0, 0)]), mode(np.abs(S[0].W[(0, 0)]), Q, 2), 1), 0)

    def explicit_row(self, i):
        """Row i of K~ from the definition eq. Kwq, without forming the matrix:
        K~_ij = sum_{ab} sum_q w^(ab)_{iq} C_ab(x_q) d_b b_j(x_q)."""
        n1, n2, n3 = self.n
        i1, i2, i3 = i % n1, (i // n1) % n2, i // (n1 * n2)
        row = np.zeros(self.N)
        for al in range(3):
            for be in range(3):
                W1, W2, W3 = self.Wk(al, be)
                Q = np.einsum("c,b,a->cba", W3[i3], W2[i2], W1[i1]) * self.plane(al, be)
                B1, B2, B3 = self.Bk(be)
                row += np.einsum("cba,ck,bj,ai->kji", Q, B3, B2, B1, optimize=True).ravel()
        if self.Cm is not None:            # M~_ij = sum_q w^(00)_{iq} c_q b_j(x_q) (eq. Mwq)
            S = self.spaces
            Q = np.einsum("c,b,a->cba", S[2].W[(0, 0)][i3], S[1].W[(0, 0)][i2], S[0].W[(0, 0)][i1]) * self.Cm
            row += np.einsum("cba,ck,bj,ai->kji", Q, S[2].B[0], S[1].B[0], S[0].B[0], optimize=True).ravel()
        return row

    # -- load vector and mass-type pieces ----------------------------------
    def W00(self, Q):
        S = self.spaces
        return mode(S[2].W[(0, 0)], mode(S[1].W[(0, 0)], mode(S[0].W[(0, 0)], Q, 2), 1), 0)

    def W00_T(self, Y):
        S = self.spaces
        return mode(S[2].W[(0, 0)].T, mode(S[1].W[(0, 0)].T, mode(S[0].W[(0, 0)].T, Y, 2), 1), 0)

    def rhs(self, f_q):
        """Reading R6: b = W^(00) (det J f) with f sampled at the quadrature points."""
        return self.W00(self.detJ * np.asarray(f_q).reshape(self.detJ.shape)).ravel()

    def rhs_from(self, f_fn):
        return self.rhs(f_fn(self.F))
