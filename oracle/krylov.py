"""Right-preconditioned BiCGStab (van der Vorst 1992), the Krylov method the
paper uses for the non-symmetric WQ systems (Section 4).  CPU oracle, test
infrastructure only.

Reading R8: x0 = 0 unless given, shadow residual r^ = r0, stop when the
recurrence residual satisfies |r|_2 / |b|_2 <= tol (then confirmed with the true
residual b - A x; the iteration continues if the confirmation fails).
"""
from __future__ import annotations

import numpy as np


def bicgstab(A, b, M=None, tol=1e-10, maxit=1000, x0=None):
    """Solve A x = b with right preconditioner M (x = M y).  ``A`` and ``M`` are
    callables.  Returns (x, iterations, relres, history)."""
    M = M or (lambda r: r)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x) if x0 is not None else b.copy()
    if nb == 0:
        return x, 0, 0.0, []
    rh = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    hist = []
    for it in range(1, maxit + 1):
        rho = rh @ r
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = M(p)
        v = A(ph)
        alpha = rho / (rh @ v)
        s = r - alpha * v
        if np.linalg.norm(s) / nb <= tol:
            # half step: x + alpha ph is returned only if its true residual
            # confirms; otherwise x is left as it was and the full step below
            # adds alpha ph (once) together with omega sh.
            x_half = x + alpha * ph
            rel = np.linalg.norm(b - A(x_half)) / nb
            if rel <= tol:
                hist.append(rel)
                return x_half, it, rel, hist
        sh = M(s)
        t = A(sh)
        omega = (t @ s) / (t @ t)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho_old = rho
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol:
            true = np.linalg.norm(b - A(x)) / nb
            if true <= tol:
                return x, it, true, hist
            r = b - A(x)
    return x, maxit, np.linalg.norm(b - A(x)) / nb, hist


def refined_solve(apply_ext, solve, b, steps=4):
    """Reference solution of A x = b to (nearly) full FP64 accuracy by iterative
    refinement (Wilkinson 1963; Moler 1967): x_0 = solve(b), then
    x_{k+1} = x_k + solve(r_k) with the residual r_k = b - A x_k formed in
    extended precision (``apply_ext`` returns A x as numpy longdouble, 64-bit
    significand) and rounded to FP64 once.  Each correction is as accurate as
    ``solve`` (an FP64 solve to relative residual t gives about cond(A) t
    relative accuracy), so the error contracts by that factor per step until
    the extended-precision residual, about cond(A) 2^-64 relative, limits it:
    below FP64 rounding up to cond(A) ~ 1e7, where an FP64 residual alone
    stalls near cond(A) 1e-16.  Returns (x, relative extended residual of x,
    relative size of the last correction); the residual cannot fall below that
    of x* rounded to FP64 (about 1e-16 |A| |x| / |b|), the last correction is
    the convergence certificate."""
    b = np.asarray(b, dtype=np.float64)
    bl = b.astype(np.longdouble)
    x = solve(b)
    step = np.inf
    for _ in range(steps):
        r = bl - apply_ext(x)
        d = solve(np.asarray(r, dtype=np.float64))
        x = x + d
        step = float(np.linalg.norm(d) / np.linalg.norm(x))
    r = bl - apply_ext(x)
    return x, float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(bl * bl))), step
