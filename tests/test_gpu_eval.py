"""GPU parity of the Gauss-point evaluator (wq_eval_setup / wq_eval_slab, the
error measure of Section 4, Table 1) against the oracle's point values
(oracle.errors.gauss_point_values) on the same seeded coefficients, element by
element: mapped points to 1e-14, w |det J|, u_h and the physical gradient to
1e-12 of their maximum, on the rational (NURBS) ring, a polynomial ring with
non-uniform knots, the twisted cube and p = 8; whole range and a sub-slab.
The relative H1 and L2 errors of a Galerkin solution integrated from the GPU's
point values equal the oracle's error integral to 1e-10."""
import numpy as np
import pytest

import synth
from oracle.errors import errors, gauss_point_values

pytestmark = pytest.mark.gpu

CASES = ["nurbs8_p3", "ring8nu_p5", "twist5_p4", "ring6_p8", "nurbs6nu_p4"]


def host(t):
    return t.detach().double().cpu().numpy()


def rel_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(b).max())


@pytest.mark.parametrize("name", CASES)
def test_eval_points_match_oracle(name):
    import torch
    from paper_1712_08565_amd import wqfd
    wl = synth.workload(name)
    kn, ctrl, w = wl.knots(), wl.ctrl(), wl.weights()
    ng = wl.p + 3
    print(f"[eval] {name}: p = {wl.p}, ng = {ng}", flush=True)
    E = wqfd.wq_eval_setup(wl.p, kn, ctrl, ng, weights=w)
    n = [e + wl.p - 2 for e in E.ne]
    u = synth.random_vector(int(np.prod(n)), 51)
    F, wq, uh, gx = gauss_point_values(kn, wl.p, ctrl, u, ng, w)
    ud = torch.as_tensor(u, device="cuda")
    for e0, e1 in ((0, E.ne[2]), (1, min(3, E.ne[2]))):
        X, wdet, uhd, grad = wqfd.wq_eval_slab(E, ud, e0, e1)
        sl = slice(e0 * ng, e1 * ng)
        eX = float(np.abs(host(X).T - F[sl].reshape(-1, 3)).max())
        ew = rel_max(host(wdet), wq[sl].ravel())
        eu = rel_max(host(uhd), uh[sl].ravel())
        eg = rel_max(host(grad).T, gx[sl].reshape(-1, 3))
        print(f"[eval] {name} elements [{e0}, {e1}): X {eX:.1e}, w|det J| {ew:.1e}, u_h {eu:.1e}, grad {eg:.1e}",
              flush=True)
        assert eX <= 1e-14 and ew <= 1e-12 and eu <= 1e-12 and eg <= 1e-12, (eX, ew, eu, eg)


@pytest.mark.parametrize("name", ["nurbs8_p3", "ring8_p4"])
def test_h1_error_from_gpu_points_equals_oracle(name):
    """The error of a Galerkin solution (the paper's problem, GPU solve to
    1e-13), integrated over slabs from the GPU's point values with torch,
    against the oracle's integral of the same coefficients."""
    import torch
    from paper_1712_08565_amd import problem, wqfd
    wl = synth.workload(name)
    kn, ctrl, w = wl.knots(), wl.ctrl(), wl.weights()
    dp = problem.build(wl, wqfd.WQ_F64, wqfd.WQ_F64)
    x, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-13)
    E = wqfd.wq_eval_setup(wl.p, kn, ctrl, wl.p + 3, weights=w)
    s = torch.zeros(4, dtype=torch.float64, device="cuda")
    for e0 in range(0, E.ne[2], 3):
        X, wdet, uh, grad = wqfd.wq_eval_slab(E, x, e0, min(E.ne[2], e0 + 3))
        P = X.t()
        ue, ge = synth.u_paper(P), synth.grad_u_paper(P)
        s += torch.stack([torch.sum(wdet * (uh - ue) ** 2), torch.sum(wdet * ue ** 2),
                          torch.sum(wdet * torch.sum((grad.t() - ge) ** 2, 1)), torch.sum(wdet * torch.sum(ge ** 2, 1))])
    l2, h1 = float(torch.sqrt(s[0] / s[1])), float(torch.sqrt(s[2] / s[3]))
    l2o, h1o = errors(kn, wl.p, ctrl, host(x), synth.u_paper, synth.grad_u_paper, weights=w)
    print(f"[eval] {name}: H1 {h1:.6e} (oracle {h1o:.6e}), L2 {l2:.6e} (oracle {l2o:.6e})", flush=True)
    assert abs(h1 / h1o - 1) <= 1e-10 and abs(l2 / l2o - 1) <= 1e-10, (h1, h1o, l2, l2o)
