"""Fast Diagonalization (FD) preconditioner.  CPU oracle, test infrastructure only.

The paper uses "the simplest version" of the FD preconditioner of its reference
[Sangalli2016] (Section 4) and defines it only by citation.  Reading R7: the
preconditioner is the parametric-domain Laplacian with exact 1D Galerkin
matrices of the interior B-splines, in the Kronecker order of eq. ordering,

    P = K_3 (x) M_2 (x) M_1 + M_3 (x) K_2 (x) M_1 + M_3 (x) M_2 (x) K_1,

inverted by fast diagonalization (Lynch, Rice and Thomas 1964): with the
generalized eigenpairs K_l U_l = M_l U_l Lambda_l, U_l^T M_l U_l = I,

    P^{-1} = (U_3 (x) U_2 (x) U_1) diag(1 / (lam1_i + lam2_j + lam3_k)) (U_3 (x) U_2 (x) U_1)^T.

For the model problem with a reaction term alpha u, a constant shift sigma (a
representative value of alpha det J) adds sigma M_3 (x) M_2 (x) M_1 to P; in
the same eigenbasis that term is sigma I, so the diagonal becomes
lam1_i + lam2_j + lam3_k + sigma.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .operator import mode


class FD:
    def __init__(self, spaces, shift: float = 0.0):
        self.shift = float(shift)
        self.M = [s.M for s in spaces]
        self.K = [s.K for s in spaces]
        self.n = tuple(s.n for s in spaces)
        self.lam, self.U = [], []
        for K, M in zip(self.K, self.M):
            lam, U = sla.eigh(K, M)
            self.lam.append(lam)
            self.U.append(U)
        l1, l2, l3 = self.lam
        self.D = l3[:, None, None] + l2[None, :, None] + l1[None, None, :] + self.shift

    def apply(self, r):
        """z = P^{-1} r by the six mode products and the diagonal scaling."""
        U1, U2, U3 = self.U
        R = np.asarray(r, dtype=np.float64).reshape(self.n[2], self.n[1], self.n[0])
        Rh = mode(U3.T, mode(U2.T, mode(U1.T, R, 2), 1), 0)
        Rh = Rh / self.D
        return mode(U3, mode(U2, mode(U1, Rh, 2), 1), 0).ravel()

    def apply_abs(self, r):
        """Entry-wise rounding-error scale of ``apply``: the same six mode
        products on |U_l|, |U_l^T|, |r| and the scaling by 1 / |diagonal|."""
        A1, A2, A3 = (np.abs(U) for U in self.U)
        R = np.abs(np.asarray(r, dtype=np.float64)).reshape(self.n[2], self.n[1], self.n[0])
        Rh = mode(A3.T, mode(A2.T, mode(A1.T, R, 2), 1), 0) / np.abs(self.D)
        return mode(A3, mode(A2, mode(A1, Rh, 2), 1), 0).ravel()

    def P_apply(self, v):
        """P v from the Kronecker form (no eigen-decomposition)."""
        M1, M2, M3 = self.M
        K1, K2, K3 = self.K
        V = np.asarray(v, dtype=np.float64).reshape(self.n[2], self.n[1], self.n[0])
        out = mode(K3, mode(M2, mode(M1, V, 2), 1), 0)
        out += mode(M3, mode(K2, mode(M1, V, 2), 1), 0)
        out += mode(M3, mode(M2, mode(K1, V, 2), 1), 0)
        if self.shift:
            out += self.shift * mode(M3, mode(M2, mode(M1, V, 2), 1), 0)
        return out.ravel()

    def P_matrix(self):
        M1, M2, M3 = (sp.csr_matrix(m) for m in self.M)
        K1, K2, K3 = (sp.csr_matrix(k) for k in self.K)
        P = (sp.kron(K3, sp.kron(M2, M1)) + sp.kron(M3, sp.kron(K2, M1))
             + sp.kron(M3, sp.kron(M2, K1)))
        if self.shift:
            P = P + self.shift * sp.kron(M3, sp.kron(M2, M1))
        return P.tocsr()
