"""Full-size parity on the benchmark workload (thick quarter ring, 64^3 elements,
p = 3 and 6), through the same entry points and launch configuration the
benchmark times.  The oracle cannot assemble K~ at this size, so:
  * apply: sampled rows of K~ from the oracle's definition (eq. Kwq) at corner,
    edge, tile-seam and random DOFs, each compared with the GPU result on the
    rounding scale sum_j |K_ij v_j| (<= 1e-12);
  * transposed apply: <K~ v, u> = <v, K~^T u> (<= 1e-13 relative);
  * FD and load vector: the oracle's full vectors (<= 1e-12 relative);
  * FP64 solve: the oracle's matrix-free residual of the GPU solution <= 1e-10;
  * reaction term (p = 3, the bench's alpha): sampled rows of K~ + M~ the same
    way, and the transpose identity.
"""
import numpy as np
import pytest

import synth
from oracle.fd import FD
from oracle.operator import Problem

pytestmark = pytest.mark.gpu

_cache = {}


def setup(name):
    if name in _cache:
        return _cache[name]
    import torch
    from paper_1712_08565_amd import problem
    from paper_1712_08565_amd.wqfd import WQ_F64
    wl = synth.workload(name)
    print(f"[fullsize] setup {name}", flush=True)
    dp = problem.build(wl, WQ_F64, WQ_F64)
    pr = Problem(wl.knots(), wl.p, wl.ctrl(), wl.K_field())
    torch.cuda.synchronize()
    _cache[name] = (wl, dp, pr)
    return _cache[name]


def sample_rows(n, p, count=24, seed=7):
    """DOF indices at the corners, on the edges, next to 16-point tile seams
    (quadrature tiles of 16 points cover about 8 elements) and at random."""
    n1, n2, n3 = n
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (n1 - 1, n2 - 1, n3 - 1), (0, n2 - 1, n3 // 2), (n1 - 1, 0, 0), (n1 // 2, n2 // 2, n3 - 1)]
    for t in (7, 8, 15, 16):
        pts.append((min(t, n1 - 1), min(t + p, n2 - 1), min(2 * t, n3 - 1)))
    while len(pts) < count:
        pts.append(tuple(int(rng.integers(0, m)) for m in (n1, n2, n3)))
    return [i1 + n1 * (i2 + n2 * i3) for i1, i2, i3 in pts]


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda", dtype=torch.float64)


@pytest.mark.parametrize("name", ["ring64_p3", "ring64_p6"])
def test_fullsize_apply_sampled_rows(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    v = synth.random_vector(pr.N, 42)
    w = wqfd.wq_apply(dp.A, dev(v)).cpu().numpy()
    worst = 0.0
    for i in sample_rows(pr.n, wl.p):
        row = pr.explicit_row(i)
        ref = float(row @ v)
        scale = float(np.abs(row) @ np.abs(v))
        worst = max(worst, abs(w[i] - ref) / scale)
    print(f"[fullsize] {name}: worst sampled-row error / rounding scale {worst:.2e}", flush=True)
    assert worst <= 1e-12, f"{worst:.3e}"


@pytest.mark.parametrize("name", ["ring64_p3", "ring64_p6"])
def test_fullsize_transpose_identity(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    v = synth.random_vector(pr.N, 43)
    u = synth.random_vector(pr.N, 44)
    Kv = wqfd.wq_apply(dp.A, dev(v)).cpu().numpy()
    KTu = wqfd.wq_apply_T(dp.A, dev(u)).cpu().numpy()
    d = abs(Kv @ u - v @ KTu) / (np.linalg.norm(Kv) * np.linalg.norm(u))
    assert d <= 1e-13, f"{d:.3e}"


@pytest.mark.parametrize("name", ["ring64_p3", "ring64_p6"])
def test_fullsize_fd_and_rhs(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    r = synth.random_vector(pr.N, 45)
    z = wqfd.fd_apply(dp.P, dev(r)).cpu().numpy()
    zr = FD(pr.spaces).apply(r)
    e_fd = float(np.linalg.norm(z - zr) / np.linalg.norm(zr))
    b_ref = pr.rhs_from(wl.f())
    e_b = float(np.linalg.norm(dp.b.cpu().numpy() - b_ref) / np.linalg.norm(b_ref))
    assert e_fd <= 1e-12 and e_b <= 1e-12, (f"{e_fd:.3e}", f"{e_b:.3e}")


@pytest.mark.parametrize("name", ["ring64_p3", "ring64_p6"])
def test_fullsize_solve_residual(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    x, it, rel = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-10)
    xh = x.cpu().numpy()
    b = pr.rhs_from(wl.f())
    res = float(np.linalg.norm(b - pr.apply(xh)) / np.linalg.norm(b))
    print(f"[fullsize] {name}: {it} iterations, reported {rel:.2e}, oracle residual {res:.2e}", flush=True)
    assert res <= 1e-10, f"{res:.3e}"


def test_fullsize_reaction_sampled_rows():
    import torch
    from paper_1712_08565_amd import problem, wqfd
    from paper_1712_08565_amd.wqfd import WQ_F64
    wl, _, pr = setup("ring64_p3")
    alpha_fn = synth.alpha_field(10.0 * wl.n_el ** 2)
    dp = problem.build(wl, WQ_F64, WQ_F64)
    problem.set_reaction(dp, alpha_fn)
    pr.set_alpha(alpha_fn(pr.F))
    try:
        v = synth.random_vector(pr.N, 42)
        u = synth.random_vector(pr.N, 44)
        w = wqfd.wq_apply(dp.A, dev(v)).cpu().numpy()
        KTu = wqfd.wq_apply_T(dp.A, dev(u)).cpu().numpy()
        worst = 0.0
        for i in sample_rows(pr.n, wl.p):
            row = pr.explicit_row(i)
            worst = max(worst, abs(w[i] - float(row @ v)) / float(np.abs(row) @ np.abs(v)))
        d = abs(w @ u - v @ KTu) / (np.linalg.norm(w) * np.linalg.norm(u))
        print(f"[fullsize] ring64_p3 + alpha: worst sampled row / rounding scale {worst:.2e}, "
              f"transpose identity {d:.2e}", flush=True)
        assert worst <= 1e-12 and d <= 1e-13, (worst, d)
    finally:
        pr.set_alpha(None)
        del dp
        torch.cuda.empty_cache()
