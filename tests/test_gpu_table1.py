"""Table 1 of the paper (tab:k_refinement, Section 4) at its coarse levels, on
the GPU: the thick quarter ring with the oscillating solution of
eq. (exact-solution), K = I, solved by the library's FD-preconditioned BiCGStab
with the paper's error-matched stopping rule (eq. stopping_criterion):
|r_k|_2 / |b|_2 <= eta |u - u_h|_H1 / |u|_H1, eta = 0.1, where u_h is the
Galerkin solution (here: the library's solve to relative residual 1e-12) and its
relative H1 error is integrated by the oracle (p + 3 Gauss points per element,
exact gradient).  The paper's printed errors (tests/golden/table1_h1_errors.txt)
are those of the solution stopped by that rule; the ring here is the spline
interpolant of the ring map (order p + 1), not the paper's NURBS ring, so they
are matched within 25% (as the oracle's own pin does).  The stopped solution's
error stays within 5% of the Galerkin error, in fewer iterations."""
import os

import numpy as np
import pytest

import synth
from oracle.errors import errors

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = [(16, p) for p in range(2, 8)] + [(32, p) for p in (2, 3, 4)]
ETA = 0.1


def paper_value(ne, p):
    rows = np.loadtxt(os.path.join(HERE, "golden", "table1_h1_errors.txt"))
    return {int(r[0]): r[1:] for r in rows}[p][{16: 0, 32: 1, 64: 2, 128: 3, 256: 4}[ne]]


@pytest.mark.parametrize("ne,p", CASES)
def test_table1_with_the_error_matched_stopping_rule(ne, p):
    from paper_1712_08565_amd import problem, wqfd
    wl = synth.Workload(f"ring{ne}_p{p}", ne, p, "ring_interp", 0.0, "identity", "paper")
    print(f"[table1] h = 1/{ne}, p = {p}", flush=True)
    dp = problem.build(wl, wqfd.WQ_F64, wqfd.WQ_F64)
    kn, ctrl = wl.knots(), wl.ctrl()
    xg, it_g, res_g = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-12, maxit=3000)
    e_g = errors(kn, p, ctrl, xg.cpu().numpy(), synth.u_paper, synth.grad_u_paper)[1]
    tol = ETA * e_g
    x, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=tol, maxit=3000)
    e = errors(kn, p, ctrl, x.cpu().numpy(), synth.u_paper, synth.grad_u_paper)[1]
    ref = paper_value(ne, p)
    print(f"[table1] h = 1/{ne}, p = {p}: Galerkin error {e_g:.3e} ({it_g} it); stopping rule tol {tol:.2e}: "
          f"{it} it, error {e:.3e}; paper {ref:.1e} (ratio {e / ref:.2f})", flush=True)
    assert res <= tol and it <= it_g, (res, tol, it, it_g)
    assert abs(e / e_g - 1) < 0.05, (e, e_g)
    assert abs(e / ref - 1) < 0.25, (e, ref)
