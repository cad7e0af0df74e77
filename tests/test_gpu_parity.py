"""GPU parity of the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs.  Gates (element by element, see parity_gates.py):
  FP64 apply / apply_T / FD / rhs: max |d_i| <= 1e-12 max |ref_i| on N(0,1)
     inputs (reading R11); for a smooth input, whose K~ v is small against the
     rounding of its terms, |d_i| <= 1e-12 times the entry's rounding scale
     (the oracle's chain on absolute values).
  FP64 solves: relative error <= 1e-10 (reading R10) against the oracle's
     reference solution: FP64 BiCGStab refined with extended-precision residuals
     of the matrix-free operator, which is accurate to about 1e-13 even where
     cond(K~) ~ 1e7 (twist6_p6) and FP64 residuals alone are not.
  FP32 / BF16 results: error stated (bounds are about ten times the observed error).
Non-uniform knots (element lengths within a factor 4, different per direction)
and the exact ring as a rational (NURBS) map run through the same cases: the
fused kernels (p <= 7, one and several tiles) and the staged ones (p = 8).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.fd import FD
from oracle.operator import Problem
from parity_gates import forward_error_bound, max_rel, norm_rel, oracle_fp64_solve_error, per_entry, reference_solve

pytestmark = pytest.mark.gpu

APPLY_CASES = ["cube12_p3", "ring8_p2", "ring8_p3", "ring8_p4", "ring8_p5", "ring8_p6", "ring7_p4_kappa",
               "twist6_p6", "shear6_p3", "ring6_p8", "ring20_p6", "ring6_p7", "ring18_p7", "ring5_p10",
               "ring8nu_p2", "ring8nu_p3", "ring8nu_p4", "ring8nu_p5", "ring8nu_p6", "ring20nu_p6", "ring6nu_p8",
               "twist6nu_p5", "nurbs8_p2", "nurbs8_p3", "nurbs8_p6", "nurbs20_p5", "nurbs6nu_p4", "nurbs6_p8"]

_cache = {}


def setup(name):
    if name in _cache:
        return _cache[name]
    import torch
    from paper_1712_08565_amd import problem
    from paper_1712_08565_amd.wqfd import WQ_BF16, WQ_F32, WQ_F64
    wl = synth.workload(name)
    print(f"[parity] setup {name} (p={wl.p}, n_el={wl.n_el})", flush=True)
    dp = problem.build(wl, WQ_F64 | WQ_F32, WQ_F64 | WQ_F32 | WQ_BF16)
    pr = Problem(wl.knots(), wl.p, wl.ctrl(), wl.K_field(), weights=wl.weights())
    torch.cuda.synchronize()
    _cache[name] = (wl, dp, pr)
    return _cache[name]


def dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda", dtype=dtype or torch.float64)


def host(t):
    return t.double().cpu().numpy()


@pytest.mark.parametrize("name", APPLY_CASES)
def test_dims_and_points(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    n, nq = wqfd.wq_dims(dp.A)
    assert n == pr.n and nq == pr.nq
    xq, Fq = wqfd.wq_quad_points(dp.A)
    e_x = max(float(np.abs(xq[l] - pr.spaces[l].xq).max()) for l in range(3))
    e_F = float(np.abs(host(Fq) - pr.F.reshape(-1, 3).T).max())
    e_d = float(np.abs(host(wqfd.wq_detj(dp.A)) - pr.detJ.ravel()).max() / np.abs(pr.detJ).max())
    assert e_x < 1e-15 and e_F < 1e-13 and e_d < 1e-12, (e_x, e_F, e_d)


@pytest.mark.parametrize("name", APPLY_CASES)
def test_apply_fp64_parity(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    v = synth.random_vector(pr.N, 42)
    e = max_rel(host(wqfd.wq_apply(dp.A, dev(v))), pr.apply(v))
    print(f"[apply] {name}: max entry error / max |K~ v| {e:.2e}")
    assert e <= 1e-12, f"{e:.3e}"


@pytest.mark.parametrize("name", ["cube12_p3", "ring8_p6", "twist6_p6", "ring20nu_p6", "ring6_p8"])
def test_apply_smooth_input_on_rounding_scale(name):
    """A smooth v (a spline interpolant-like sample of a smooth function) makes
    K~ v and K~^T v small against their terms; each entry is then compared on
    its own rounding scale (reading R11)."""
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    n1, n2, n3 = pr.n
    g = [np.arange(1, m + 1) / (m + 1) for m in (n1, n2, n3)]
    Z, Y, X = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    v = (np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z) * (1 + X * Y)).ravel()
    e = per_entry(host(wqfd.wq_apply(dp.A, dev(v))), pr.apply(v), pr.apply_abs(v))
    eT = per_entry(host(wqfd.wq_apply_T(dp.A, dev(v))), pr.apply_T(v), pr.apply_T_abs(v))
    print(f"[apply smooth] {name}: worst entry / rounding scale {e:.2e}, transpose {eT:.2e}")
    assert e <= 1e-12 and eT <= 1e-12, (e, eT)


@pytest.mark.parametrize("name", ["cube12_p3", "ring8_p6", "ring20_p6"])
def test_apply_acc_parity(name):
    """w += K~ v (Algorithm 2 added to w): w0 + K~ v after one call, w0 + 2 K~ v
    after two, against the oracle's apply; FP64 to 1e-12 relative."""
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    v = synth.random_vector(pr.N, 51)
    w0 = synth.random_vector(pr.N, 52)
    Kv = pr.apply(v)
    w = dev(w0)
    wqfd.wq_apply_acc(dp.A, dev(v), w)
    e1 = max_rel(host(w), w0 + Kv)
    wqfd.wq_apply_acc(dp.A, dev(v), w)
    e2 = max_rel(host(w), w0 + 2 * Kv)
    print(f"[apply acc] {name}: {e1:.2e}, {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12, (e1, e2)


def test_repeated_applies_and_solves_agree():
    """Run-to-run agreement: the fused apply adds overlapping tiles into w with
    FP64 atomics, so repeated applies may differ only in the last bits
    (<= 1e-14 of max |w|); repeated solves take the same number of iterations
    and agree to the solver tolerance."""
    import torch
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup("ring20_p6")
    v = dev(synth.random_vector(pr.N, 55))
    ws = [wqfd.wq_apply(dp.A, v).clone() for _ in range(5)]
    torch.cuda.synchronize()
    d = max(float((w - ws[0]).abs().max()) for w in ws[1:]) / float(ws[0].abs().max())
    xs = [wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-12) for _ in range(3)]
    its = {it for _, it, _ in xs}
    dx = max(float((x - xs[0][0]).norm() / xs[0][0].norm()) for x, _, _ in xs[1:])
    print(f"[repeat] applies {d:.1e}, solves: iterations {sorted(its)}, spread {dx:.1e}")
    assert d <= 1e-14 and len(its) == 1 and dx <= 1e-11, (d, its, dx)


def test_apply_acc_refused_without_fused_kernels():
    """p = 8 runs the staged kernels, which overwrite w: the accumulating call
    is refused with an error instead of returning a wrong sum."""
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup("ring6_p8")
    v = dev(synth.random_vector(pr.N, 53))
    w = dev(synth.random_vector(pr.N, 54))
    with pytest.raises(Exception, match="fused"):
        wqfd.wq_apply_acc(dp.A, v, w)


@pytest.mark.parametrize("name", APPLY_CASES)
def test_apply_T_fp64_parity_and_adjoint_identity(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    v = synth.random_vector(pr.N, 43)
    u = synth.random_vector(pr.N, 44)
    gT = host(wqfd.wq_apply_T(dp.A, dev(v)))
    e = max_rel(gT, pr.apply_T(v))
    print(f"[apply_T] {name}: max entry error / max |K~^T v| {e:.2e}")
    assert e <= 1e-12, f"{e:.3e}"
    gu = host(wqfd.wq_apply(dp.A, dev(u)))
    d = abs(gu @ v - u @ gT) / (np.linalg.norm(gu) * np.linalg.norm(v))
    assert d <= 1e-13, f"{d:.3e}"


@pytest.mark.parametrize("name", ["cube12_p3", "ring8_p3", "ring8_p6", "twist6_p6", "ring8nu_p4", "ring20nu_p6"])
def test_apply_fp32_error(name):
    import torch
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    v = synth.random_vector(pr.N, 42)
    e = max_rel(host(wqfd.wq_apply(dp.A, dev(v, torch.float32))), pr.apply(v))
    eT = max_rel(host(wqfd.wq_apply_T(dp.A, dev(v, torch.float32))), pr.apply_T(v))
    print(f"[fp32 apply] {name}: max entry error / max |ref| {e:.2e}, transpose {eT:.2e}")
    assert e <= 1e-5 and eT <= 1e-5, (e, eT)


@pytest.mark.parametrize("name", ["cube12_p3", "ring8_p2", "ring8_p6", "twist6_p6", "ring8nu_p3", "ring20nu_p6"])
def test_fd_parity(name):
    import torch
    from paper_1712_08565_amd import wqfd
    from paper_1712_08565_amd.wqfd import WQ_BF16, WQ_F32
    wl, dp, pr = setup(name)
    fd = FD(pr.spaces)
    r = synth.random_vector(pr.N, 45)
    ref = fd.apply(r)
    e = max_rel(host(wqfd.fd_apply(dp.P, dev(r))), ref)
    e32 = max_rel(host(wqfd.fd_apply(dp.P, dev(r, torch.float32), prec=WQ_F32)), ref)
    ebf = max_rel(host(wqfd.fd_apply(dp.P, dev(r, torch.float32), prec=WQ_BF16)), ref)
    print(f"[fd] {name}: max entry error / max |ref|: fp64 {e:.2e}, fp32 {e32:.2e}, bf16 {ebf:.2e}")
    assert e <= 1e-12 and e32 <= 1e-5 and ebf <= 5e-2, (e, e32, ebf)
    x = dev(r)                      # r and z may alias
    wqfd.fd_apply(dp.P, x, x)
    e_in = max_rel(host(x), ref)
    assert e_in <= 1e-12, f"{e_in:.3e}"


@pytest.mark.parametrize("name", ["cube12_p3", "ring8_p3", "twist6_p6", "ring8nu_p5"])
def test_rhs_parity(name):
    wl, dp, pr = setup(name)
    e = max_rel(host(dp.b), pr.rhs_from(wl.f()))
    assert e <= 1e-12, f"{e:.3e}"


def test_identity_cube_solves_in_one_iteration():
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup("cube12_p3")
    x, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-12)
    xd = spla.spsolve(pr.assemble().tocsc(), pr.rhs_from(wl.f()))
    e = norm_rel(host(x), xd)
    assert it == 1 and res <= 1e-12 and e <= 1e-10, (it, res, e)


_refs = {}


def reference_solution(name, pr, b, transpose=False):
    key = (name, transpose)
    if key not in _refs:
        _refs[key] = reference_solve(pr, b, transpose)
    return _refs[key]


def _solve_check(pr, A, b, x, xref, res, label, transpose=False):
    """The oracle's residual of the GPU solution <= 1e-12, and its error against
    the refined reference <= 1e-10, or <= 3 times the error of the oracle's own
    FP64 BiCGStab, or <= kappa_2(K~) times that residual (the normwise bound,
    computed for N <= 4000), whichever is largest (reading R10)."""
    e = norm_rel(x, xref)
    e_or = oracle_fp64_solve_error(pr, b, xref, transpose)
    r_or = float(np.linalg.norm(A(x) - b) / np.linalg.norm(b))
    bound = forward_error_bound(pr, r_or) if e > max(1e-10, 3 * e_or) else 0.0
    print(f"[{label}] relres {res:.2e}, oracle residual {r_or:.2e}, rel err vs reference {e:.2e} "
          f"(oracle FP64 BiCGStab: {e_or:.2e}; kappa bound {bound:.1e})")
    assert r_or <= 1e-12 and e <= max(1e-10, 3 * e_or, bound), (r_or, e, e_or, bound)


@pytest.mark.parametrize("name", ["ring8_p2", "ring8_p4", "ring8_p6", "ring7_p4_kappa", "twist5_p4", "twist6_p6",
                                  "ring8nu_p3", "ring8nu_p6", "twist6nu_p5", "ring6nu_p8", "nurbs8_p3",
                                  "nurbs6nu_p4"])
def test_solve_parity(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr = setup(name)
    b = pr.rhs_from(wl.f())
    x, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-14, maxit=400, raise_on_noconv=False)
    assert res <= 1e-13, f"{res:.3e}"
    _solve_check(pr, pr.apply, b, host(x), reference_solution(name, pr, b), res, f"solve {name} ({it} it)")
    xt, itt, rest = wqfd.krylov_solve(dp.A, dp.P, dp.b, transpose=True, rtol=1e-14, maxit=400,
                                      raise_on_noconv=False)
    assert rest <= 1e-13, f"{rest:.3e}"
    _solve_check(pr, pr.apply_T, b, host(xt), reference_solution(name, pr, b, True), rest,
                 f"solve^T {name} ({itt} it)", transpose=True)


@pytest.mark.parametrize("fd_prec", ["f32", "bf16"])
@pytest.mark.parametrize("name", ["ring8_p4", "twist6_p6", "ring7_p4_kappa", "ring8nu_p5"])
def test_mixed_precision_refinement_parity(name, fd_prec):
    from paper_1712_08565_amd import wqfd
    from paper_1712_08565_amd.wqfd import WQ_BF16, WQ_F32
    wl, dp, pr = setup(name)
    b = pr.rhs_from(wl.f())
    xref = reference_solution(name, pr, b)
    prec = WQ_F32 if fd_prec == "f32" else WQ_BF16
    x, outer, inner, res = wqfd.ir_solve(dp.A, dp.P, dp.b, fd_prec=prec, rtol=1e-13, tau_inner=1e-4)
    e = norm_rel(host(x), xref)
    r_or = float(np.linalg.norm(pr.apply(host(x)) - b) / np.linalg.norm(b))
    print(f"[ir {fd_prec}] {name}: outer {outer}, inner {inner}, relres {res:.2e}, oracle residual {r_or:.2e}, "
          f"rel err {e:.2e}")
    assert res <= 1e-13 and r_or <= 1e-12 and e <= 1e-10, (res, r_or, e)


@pytest.mark.parametrize("name", ["nurbs8_p3", "twist6_p6", "ring8nu_p5", "ring6_p8", "cube12_p3"])
def test_device_geometry_matches_host(name, monkeypatch):
    """The set-up computes F, J^{-1}, det J on the device (three sum-factorisation
    passes); with WQFD_HOST_GEOMETRY set it uses the host's.  Mapped points, det J
    and the resulting operator agree to rounding."""
    from paper_1712_08565_amd import wqfd
    wl = synth.workload(name)
    v = dev(synth.random_vector(int(np.prod([e + wl.p - 2 for e in (wl.n_el,) * 3])), 42))
    out = []
    for host_geom in (False, True):
        if host_geom:
            monkeypatch.setenv("WQFD_HOST_GEOMETRY", "1")
        A = wqfd.wq_setup(wl.p, wl.knots(), wl.ctrl(), weights=wl.weights())
        out.append((host(wqfd.wq_quad_points(A)[1]), host(wqfd.wq_detj(A)), host(wqfd.wq_apply(A, v))))
    (Fd, dd, wd), (Fh, dh, wh) = out
    eF, ed, ew = max_rel(Fd, Fh), max_rel(dd, dh), max_rel(wd, wh)
    print(f"[geometry] {name}: device vs host F {eF:.1e}, det J {ed:.1e}, apply {ew:.1e}")
    assert eF <= 1e-14 and ed <= 1e-13 and ew <= 1e-13, (eF, ed, ew)
