"""Partial reproduction of the k-refinement study (Table 1 of the paper): the
Dirichlet problem on the thick quarter ring with the oscillating manufactured
solution of eq. (exact-solution), K = I, alpha = 0, solved by the library on the
GPU (FP64 BiCGStab + FD to relative residual 1e-12, i.e. the Galerkin solution),
and its relative H1 error integrated by the oracle (p + 3 Gauss points per
element in physical coordinates).  Prints one row per (h, p) beside the paper's
value.  Test infrastructure (not collected by pytest):

    python tests/table1_study.py --cases 16:2,16:3,32:2,32:3          # GPU solves + errors
    python tests/table1_study.py --cases 16:2 --solutions DIR         # errors of saved solutions only

--geometry ring_interp (default) interpolates the ring map at the Greville
abscissae (order p + 1 in h); --geometry ring places the control points at the
images of the Greville abscissae (order 2), which limits the error from p = 6 at
32^3 elements.  The paper uses an exact NURBS ring.
--eta 0.1 also solves with the paper's error-matched stopping rule
(eq. stopping_criterion: relative residual <= eta times the Galerkin solution's
relative H1 error) and reports that solution's error and iteration count.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.errors import errors  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def paper_table():
    """{p: [H1 error at h = 2^-4 .. 2^-8]} from tests/golden/table1_h1_errors.txt."""
    rows = np.loadtxt(os.path.join(HERE, "golden", "table1_h1_errors.txt"))
    return {int(r[0]): list(r[1:]) for r in rows}


def solve_on_gpu(ne, p, geometry, rtol=1e-12, dp=None):
    import torch
    from paper_1712_08565_amd import problem, wqfd
    if dp is None:
        wl = synth.Workload(f"ring{ne}_p{p}", ne, p, geometry, 0.0, "identity", "paper")
        dp = problem.build(wl, wqfd.WQ_F64, wqfd.WQ_F64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=rtol, maxit=3000, raise_on_noconv=False)
    torch.cuda.synchronize()
    return x.cpu().numpy(), it, res, time.perf_counter() - t0, dp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="16:2,16:3,16:4,32:2,32:3,32:4", help="n_el:p pairs")
    ap.add_argument("--solutions", default="", help="directory of saved x_ne{n_el}_p{p}.npy (skip the GPU)")
    ap.add_argument("--geometry", default="ring_interp", choices=("ring_interp", "ring"))
    ap.add_argument("--eta", type=float, default=0.0, help="also solve with the error-matched stopping rule")
    args = ap.parse_args()
    paper = paper_table()
    print(f"{'h':>6} {'p':>2} {'rel H1 error':>12} {'paper':>8}  solve")
    for ne, p in ((int(a), int(b)) for a, b in (c.split(":") for c in args.cases.split(","))):
        if args.solutions:
            x, info = np.load(os.path.join(args.solutions, f"x_ne{ne}_p{p}.npy")), "saved"
        else:
            x, it, res, t, dp = solve_on_gpu(ne, p, args.geometry)
            info = f"{it} it, relres {res:.1e}, {1e3 * t:.1f} ms"
        k = synth.uniform_knots(ne, p)
        kn = (k, k, k)
        ctrl = synth.control_net(args.geometry, kn, p, 0.0, 0)
        h1 = errors(kn, p, ctrl, x, synth.u_paper, synth.grad_u_paper)[1]
        if args.eta > 0 and not args.solutions:
            xe, ite, rese, te, _ = solve_on_gpu(ne, p, args.geometry, rtol=args.eta * h1, dp=dp)
            he = errors(kn, p, ctrl, xe, synth.u_paper, synth.grad_u_paper)[1]
            info += f"; stopping rule (eta {args.eta}): {ite} it, {1e3 * te:.1f} ms, error {he:.2e}"
        col = {16: 0, 32: 1, 64: 2, 128: 3, 256: 4}.get(ne)
        ref = paper[p][col] if (p in paper and col is not None) else float("nan")
        print(f"2^-{int(np.log2(ne)):d} {p:2d} {h1:12.2e} {ref:8.1e}  {info}", flush=True)


if __name__ == "__main__":
    main()
