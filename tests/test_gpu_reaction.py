"""GPU parity of the reaction term alpha u of the model problem
-div(K grad u) + alpha u = f (the mass apply of Algorithm 1 inside the fused
kernels, staged passes for p = 8, the shifted FD, dJ/dalpha), through the C ABI,
against the CPU FP64 oracle on the same seeded inputs.  Gates as for the
stiffness, element by element: FP64 results max |d_i| <= 1e-12 max |ref_i|
(the reaction part alone, as the difference of two applies, <= 1e-11); FP32
apply <= 1e-5; solves: error <= 1e-10 against the oracle's reference solution
(BiCGStab refined with extended-precision residuals) at residual 1e-14.  alpha is scaled with n_el^2
so that M~ and K~ have the same size and a mistake in either shows.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import adjoint
from oracle.fd import FD
from oracle.operator import Problem
from parity_gates import forward_error_bound, max_rel, norm_rel, oracle_fp64_solve_error, reference_solve

pytestmark = pytest.mark.gpu

CASES = ["cube12_p3", "ring8_p2", "ring8_p6", "twist6_p6", "ring6_p8", "ring20_p6", "ring18_p7", "ring8nu_p4",
         "ring6nu_p8"]
_cache = {}


def setup(name):
    if name in _cache:
        return _cache[name]
    import torch
    from paper_1712_08565_amd import problem
    from paper_1712_08565_amd.wqfd import WQ_BF16, WQ_F32, WQ_F64
    wl = synth.workload(name)
    print(f"[reaction] setup {name} (p={wl.p}, n_el={wl.n_el})", flush=True)
    dp = problem.build(wl, WQ_F64 | WQ_F32, WQ_F64 | WQ_F32 | WQ_BF16)
    alpha_fn = synth.alpha_field(10.0 * wl.n_el ** 2)
    alpha_q, sigma = problem.set_reaction(dp, alpha_fn)
    pr = Problem(wl.knots(), wl.p, wl.ctrl(), wl.K_field())
    pr.set_alpha(alpha_fn(pr.F))
    torch.cuda.synchronize()
    _cache[name] = (wl, dp, pr, sigma)
    return _cache[name]


rel = max_rel


def dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda", dtype=dtype or torch.float64)


def host(t):
    return t.double().cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_reaction_apply_parity(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr, _ = setup(name)
    v = synth.random_vector(pr.N, 61)
    u = synth.random_vector(pr.N, 62)
    w = host(wqfd.wq_apply(dp.A, dev(v)))
    wT = host(wqfd.wq_apply_T(dp.A, dev(v)))
    e, eT = rel(w, pr.apply(v)), rel(wT, pr.apply_T(v))
    # the reaction part alone: the standalone mass apply, and the fused difference
    Mv = pr.mass_apply(v)
    e_m = rel(host(wqfd.wq_apply_mass(dp.A, dev(v))), Mv)
    wqfd.wq_set_alpha(dp.A, None)
    w0 = host(wqfd.wq_apply(dp.A, dev(v)))
    w0T = host(wqfd.wq_apply_T(dp.A, dev(v)))
    wqfd.wq_set_alpha(dp.A, synth.alpha_field(10.0 * wl.n_el ** 2)(dp.Fq.t()).contiguous())
    e_d, e_dT = rel(w - w0, Mv), rel(wT - w0T, pr.mass_apply_T(v))
    gu = host(wqfd.wq_apply(dp.A, dev(u)))
    d = abs(gu @ v - u @ wT) / (np.linalg.norm(gu) * np.linalg.norm(v))
    print(f"[reaction] {name}: apply {e:.2e}, apply_T {eT:.2e}, mass {e_m:.2e}, "
          f"fused mass part {e_d:.2e} / {e_dT:.2e}, adjoint identity {d:.2e}")
    assert e <= 1e-12 and eT <= 1e-12 and e_m <= 1e-12, (e, eT, e_m)
    assert e_d <= 1e-11 and e_dT <= 1e-11 and d <= 1e-13, (e_d, e_dT, d)


@pytest.mark.parametrize("name", ["cube12_p3", "ring8_p6", "twist6_p6", "ring6_p8"])
def test_reaction_apply_fp32_error(name):
    import torch
    from paper_1712_08565_amd import wqfd
    wl, dp, pr, _ = setup(name)
    v = synth.random_vector(pr.N, 63)
    e = rel(host(wqfd.wq_apply(dp.A, dev(v, torch.float32))), pr.apply(v))
    eT = rel(host(wqfd.wq_apply_T(dp.A, dev(v, torch.float32))), pr.apply_T(v))
    em = rel(host(wqfd.wq_apply_mass(dp.A, dev(v, torch.float32))), pr.mass_apply(v))
    print(f"[reaction fp32] {name}: apply {e:.2e}, transpose {eT:.2e}, mass {em:.2e}")
    assert e <= 1e-5 and eT <= 1e-5 and em <= 1e-5, (e, eT, em)


def test_reaction_accumulating_apply():
    from paper_1712_08565_amd import wqfd
    wl, dp, pr, _ = setup("ring20_p6")
    v = synth.random_vector(pr.N, 64)
    w0 = synth.random_vector(pr.N, 65)
    w = dev(w0)
    wqfd.wq_apply_acc(dp.A, dev(v), w)
    e = rel(host(w), w0 + pr.apply(v))
    assert e <= 1e-12, f"{e:.3e}"


def test_reaction_removed_restores_stiffness():
    """alpha = NULL: the operator is K~ again.  The fused kernels add
    overlapping tiles into w with atomics, so two applies agree to rounding
    (not bit for bit): <= 1e-14 relative."""
    import torch
    from paper_1712_08565_amd import problem, wqfd
    from paper_1712_08565_amd.wqfd import WQ_F64
    wl = synth.workload("ring8_p3")
    dp = problem.build(wl, WQ_F64, WQ_F64)
    v = dev(synth.random_vector(int(np.prod(wqfd.wq_dims(dp.A)[0])), 66))
    ref = wqfd.wq_apply(dp.A, v)
    problem.set_reaction(dp, synth.alpha_field(100.0))
    with_alpha = wqfd.wq_apply(dp.A, v)
    problem.set_reaction(dp, None)
    again = wqfd.wq_apply(dp.A, v)
    torch.cuda.synchronize()
    d_alpha = float((with_alpha - ref).norm() / ref.norm())
    d_again = float((again - ref).norm() / ref.norm())
    assert d_alpha > 1e-3 and d_again <= 1e-14, (d_alpha, d_again)
    with pytest.raises(Exception, match="reaction"):
        wqfd.wq_apply_mass(dp.A, v)


@pytest.mark.parametrize("name", ["cube12_p3", "twist6_p6", "ring8nu_p4"])
def test_fd_shift_is_the_library_mean_of_alpha_det_J(name):
    """The FD shift sigma (reading R15) is the mean of c_q = alpha det J over the
    quadrature points, computed by the library (wq_alpha_mean): against the
    oracle's diagonal, 1e-14 relative; refused without a reaction term."""
    from paper_1712_08565_amd import wqfd
    wl, dp, pr, sigma = setup(name)
    ref = float(pr.Cm.mean())
    print(f"[alpha mean] {name}: library {sigma:.15e}, oracle {ref:.15e}")
    assert abs(sigma - ref) <= 1e-14 * abs(ref), (sigma, ref)
    assert abs(wqfd.wq_alpha_mean(dp.A) - sigma) == 0.0


def test_alpha_mean_refused_without_reaction_term():
    from paper_1712_08565_amd import problem, wqfd
    from paper_1712_08565_amd.wqfd import WQ_F64
    dp = problem.build(synth.workload("cube5_p2"), WQ_F64, WQ_F64)
    with pytest.raises(Exception, match="reaction"):
        wqfd.wq_alpha_mean(dp.A)


@pytest.mark.parametrize("name", ["cube12_p3", "ring8_p6", "twist6_p6"])
def test_shifted_fd_parity(name):
    import torch
    from paper_1712_08565_amd import wqfd
    from paper_1712_08565_amd.wqfd import WQ_BF16, WQ_F32
    wl, dp, pr, sigma = setup(name)
    fd = FD(pr.spaces, shift=sigma)
    r = synth.random_vector(pr.N, 67)
    ref = fd.apply(r)
    e = rel(host(wqfd.fd_apply(dp.P, dev(r))), ref)
    e32 = rel(host(wqfd.fd_apply(dp.P, dev(r, torch.float32), prec=WQ_F32)), ref)
    ebf = rel(host(wqfd.fd_apply(dp.P, dev(r, torch.float32), prec=WQ_BF16)), ref)
    print(f"[shifted fd] {name} (sigma {sigma:.3e}): fp64 {e:.2e}, fp32 {e32:.2e}, bf16 {ebf:.2e}")
    assert e <= 1e-12 and e32 <= 1e-5 and ebf <= 5e-2, (e, e32, ebf)


def test_fd_shift_rejects_bad_values():
    from paper_1712_08565_amd import wqfd
    wl, dp, pr, sigma = setup("cube12_p3")
    for bad in (float("nan"), float("inf"), -1e30):
        with pytest.raises(Exception, match="shift"):
            wqfd.fd_set_shift(dp.P, bad)
    # the rejected calls left the shift in place
    r = synth.random_vector(pr.N, 68)
    e = rel(host(wqfd.fd_apply(dp.P, dev(r))), FD(pr.spaces, shift=sigma).apply(r))
    assert e <= 1e-12, f"{e:.3e}"


def test_reaction_identity_cube_one_iteration():
    """Identity cube, K = I, constant alpha: K~ + M~ is the shifted FD operator
    exactly, so one preconditioned iteration solves it."""
    import torch
    from paper_1712_08565_amd import problem, wqfd
    from paper_1712_08565_amd.wqfd import WQ_F64
    wl = synth.workload("cube12_p3")
    dp = problem.build(wl, WQ_F64, WQ_F64)
    alpha_q, sigma = problem.set_reaction(dp, lambda X: 0 * X[..., 0] + 300.0)
    assert abs(sigma - 300.0) < 1e-9
    x, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-12)
    pr = Problem(wl.knots(), wl.p, wl.ctrl())
    pr.set_alpha(np.full(pr.Nq, 300.0))
    xd = spla.spsolve(pr.assemble().tocsc(), pr.rhs_from(wl.f()))
    e = norm_rel(host(x), xd)
    assert it == 1 and res <= 1e-12 and e <= 1e-10, (it, res, e)


def _solve_check(pr, b, x, xref, label, transpose=False, shift=0.0):
    """The oracle's residual of the GPU solution <= 1e-12, and its error against
    the oracle's reference solution <= 1e-10, or <= 3 times the error of the
    oracle's own FP64 BiCGStab, or <= kappa_2(K~ + M~) times that residual (the
    normwise bound, computed for N <= 4000), whichever is largest (reading R10)."""
    e = norm_rel(x, xref)
    e_or = oracle_fp64_solve_error(pr, b, xref, transpose, shift)
    A = pr.apply_T if transpose else pr.apply
    r_or = float(np.linalg.norm(A(x) - b) / np.linalg.norm(b))
    bound = forward_error_bound(pr, r_or) if e > max(1e-10, 3 * e_or) else 0.0
    print(f"[{label}] oracle residual {r_or:.2e}, rel err vs reference {e:.2e} (oracle FP64 BiCGStab: {e_or:.2e}; "
          f"kappa bound {bound:.1e})")
    assert r_or <= 1e-12 and e <= max(1e-10, 3 * e_or, bound), (r_or, e, e_or, bound)


@pytest.mark.parametrize("name", ["ring8_p2", "ring8_p4", "twist5_p4", "twist6_p6"])
def test_reaction_solve_parity(name):
    from paper_1712_08565_amd import wqfd
    wl, dp, pr, sigma = setup(name)
    b = pr.rhs_from(wl.f())
    x, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-14, maxit=400, raise_on_noconv=False)
    xt, itt, rest = wqfd.krylov_solve(dp.A, dp.P, dp.b, transpose=True, rtol=1e-14, maxit=400,
                                      raise_on_noconv=False)
    assert res <= 1e-13 and rest <= 1e-13, (res, rest)
    _solve_check(pr, b, host(x), reference_solve(pr, b, False, sigma), f"reaction solve {name} ({it} it)",
                 shift=sigma)
    _solve_check(pr, b, host(xt), reference_solve(pr, b, True, sigma), f"reaction solve^T {name} ({itt} it)",
                 transpose=True, shift=sigma)


@pytest.mark.parametrize("fd_prec", ["f32", "bf16"])
def test_reaction_mixed_precision_refinement(fd_prec):
    from paper_1712_08565_amd import wqfd
    from paper_1712_08565_amd.wqfd import WQ_BF16, WQ_F32
    wl, dp, pr, sigma = setup("ring8_p4")
    prec = WQ_F32 if fd_prec == "f32" else WQ_BF16
    x, outer, inner, res = wqfd.ir_solve(dp.A, dp.P, dp.b, fd_prec=prec, rtol=1e-13, tau_inner=1e-4)
    print(f"[reaction ir {fd_prec}] outer {outer}, inner {inner}, relres {res:.2e}")
    assert res <= 1e-13, f"{res:.3e}"
    b = pr.rhs_from(wl.f())
    _solve_check(pr, b, host(x), reference_solve(pr, b, False, sigma), f"reaction ir {fd_prec}", shift=sigma)


@pytest.mark.parametrize("name", ["ring8_p3", "twist6_p6", "ring6_p8"])
def test_grad_alpha_parity(name):
    """dJ/dalpha = -det J (W^(00)T lam) (B u) is a pointwise product, so each
    entry is gated on its own rounding scale det J (|W^(00)|T |lam|)(|B| |u|)
    (the weights grow with p and mix signs): <= 1e-12, the level to which the
    two sides' independently computed det J agree on curved maps.  At p = 8 the
    two sides' minimum-norm weights W^(00) themselves agree only to about 1e-11
    of max |W| (ill-conditioned local systems, reading R2; pinned on the CPU),
    a difference the exactness conditions leave free and that a product with
    a random lam sees in full: <= 1e-10 there."""
    from paper_1712_08565_amd import wqfd
    from oracle.operator import mode
    wl, dp, pr, _ = setup(name)
    lam = synth.random_vector(pr.N, 69)
    u = synth.random_vector(pr.N, 70)
    g = host(wqfd.wq_grad_alpha(dp.A, dev(lam), dev(u)))
    ref = adjoint.grad_alpha(pr, lam, u).ravel()
    S = pr.spaces
    aW = mode(np.abs(S[2].W[(0, 0)]).T, mode(np.abs(S[1].W[(0, 0)]).T,
                                             mode(np.abs(S[0].W[(0, 0)]).T, np.abs(pr._shape(lam)), 2), 1), 0)
    aB = mode(np.abs(S[2].B[0]), mode(np.abs(S[1].B[0]), mode(np.abs(S[0].B[0]), np.abs(pr._shape(u)), 2), 1), 0)
    scale = (np.abs(pr.detJ) * aW * aB).ravel()
    nz = scale > 0                      # B u vanishes on the boundary points: both sides exactly 0 there
    e_pt = float(np.max(np.abs(g[nz] - ref[nz]) / scale[nz]))
    print(f"[grad alpha] {name}: max-relative {rel(g, ref):.2e}, worst entry / rounding scale {e_pt:.2e}")
    tol = 1e-12 if wl.p <= 7 else 1e-10
    assert e_pt <= tol and np.all(g[~nz] == 0), f"{e_pt:.3e}"
