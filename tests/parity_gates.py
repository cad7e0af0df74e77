"""Element-wise parity measures shared by the GPU tests (test helpers only).

max_rel:   max_i |got_i - ref_i| / max_i |ref_i|   (every entry against the
           largest reference entry: a single wrong entry anywhere, e.g. at a
           tile seam, shows at its own size instead of being averaged away as
           in a 2-norm ratio)
per_entry: max_i |got_i - ref_i| / scale_i         (every entry against its own
           rounding-error scale, e.g. the oracle's chain on absolute values)
norm_rel:  |got - ref|_2 / |ref|_2                 (solutions and stated
           low-precision errors)
"""
import numpy as np


def _a(x):
    return np.asarray(x, dtype=np.float64).ravel()


def max_rel(got, ref) -> float:
    g, r = _a(got), _a(ref)
    assert g.shape == r.shape, (g.shape, r.shape)
    assert np.isfinite(g).all(), "non-finite entries"
    return float(np.abs(g - r).max() / np.abs(r).max())


def per_entry(got, ref, scale) -> float:
    g, r, s = _a(got), _a(ref), _a(scale)
    assert g.shape == r.shape == s.shape
    assert np.isfinite(g).all(), "non-finite entries"
    assert (s > 0).all(), "rounding scale must be positive"
    return float((np.abs(g - r) / s).max())


def norm_rel(got, ref) -> float:
    g, r = _a(got), _a(ref)
    return float(np.linalg.norm(g - r) / np.linalg.norm(r))


def reference_solve(pr, b, transpose=False, shift=0.0):
    """The oracle's reference solution of K~ x = b (or K~^T x = b) for an
    oracle Problem ``pr`` (reaction term included when set): FP64 BiCGStab with
    the FD preconditioner (shifted by ``shift``), refined with residuals of the
    matrix-free operator in extended precision (reading R10)."""
    from oracle.fd import FD
    from oracle.krylov import bicgstab, refined_solve
    fd = FD(pr.spaces, shift=shift)
    A = pr.apply_T if transpose else pr.apply
    Ae = (lambda x: pr.apply_T(x, np.longdouble)) if transpose else (lambda x: pr.apply(x, np.longdouble))
    x, r, step = refined_solve(Ae, lambda rr: bicgstab(A, rr, fd.apply, tol=1e-14, maxit=500)[0], b, steps=6)
    # converged: the last correction is at the level the extended residual allows
    # (about cond(K~) 2^-64 |K~| |x| / |b|, up to 1e-13 at cond ~ 1e7), a hundred
    # times below the 1e-10 gate; the residual of an FP64 vector cannot fall below
    # ~1e-16 |K~| |x| / |b|
    assert step <= 1e-12 and r <= 1e-12, (step, r)
    return x


def oracle_fp64_solve_error(pr, b, xref, transpose=False, shift=0.0, tol=1e-14):
    """Relative error of the oracle's own FP64 BiCGStab (to relative residual
    ``tol``) against the refined reference: the floor FP64 arithmetic leaves on
    this system.  A GPU solve at the same tolerance is held to 1e-10, or to
    three times this floor, or to the normwise bound kappa_2 times its own
    oracle residual (forward_error_bound), whichever is largest."""
    from oracle.fd import FD
    from oracle.krylov import bicgstab
    fd = FD(pr.spaces, shift=shift)
    A = pr.apply_T if transpose else pr.apply
    x = bicgstab(A, b, fd.apply, tol=tol, maxit=500)[0]
    return norm_rel(x, xref)


def forward_error_bound(pr, rel_residual, max_n=4000) -> float:
    """kappa_2(K~) times a relative residual: the normwise bound on the relative
    error of any solution with that residual (K~ assembled by the oracle, dense
    condition number; 0 when N > max_n, where it is not computed).  An FP64
    solve of a system with kappa ~ 1e7 fixes the solution only to about this
    level, whatever its arithmetic order (reading R10)."""
    if pr.N > max_n:
        return 0.0
    return float(np.linalg.cond(pr.assemble().toarray())) * rel_residual
