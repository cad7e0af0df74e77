"""Pins of the oracle's adjoint gradients (dJ/dK_q, dJ/df_q for
J = 1/2 |u - u_obs|^2 with K~(K) u = b(f)) against facts that do not re-type
their formulas:

* central finite differences of J through an independent direct solve
  (scipy spsolve on the explicitly assembled K~), along seeded random
  directions and at single quadrature points;
* Euler homogeneity: K~ is linear in K, so u(cK) = u(K) / c and
  sum_q K_q dJ/dK_q = -<u - u_obs, u>; b is linear in f, so
  sum_q f_q dJ/df_q = <u - u_obs, u>;
* u_obs = u gives a zero gradient;
* a plausible mistake (the chain rule through eq. C taken with J^{-1} and
  J^{-T} swapped) fails the finite-difference pin on a twisted geometry;
* dJ/dalpha_q of the reaction term against central differences, and the same
  gradient with det J dropped (a planted mistake) failing them.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import adjoint
from oracle.geometry import SYM_PAIRS
from oracle.operator import Problem


def make(wl):
    pr = Problem(wl.knots(), wl.p, wl.ctrl(), None)
    if wl.k_kind == "scalar":
        K = synth.kappa_field(seed=1, sigma=0.5, ell=0.1, M=512)(pr.F)
        K_obs = synth.kappa_field(seed=2, sigma=0.5, ell=0.1, M=512)(pr.F)
    else:
        K = synth.sym6_field()(pr.F)
        K_obs = synth.sym6_field(seeds=(8, 9, 10))(pr.F)
    f_q = wl.f()(pr.F)
    return pr, np.asarray(K, dtype=np.float64), np.asarray(K_obs, dtype=np.float64), np.asarray(f_q)


def solve(pr, K, f_q):
    pr.set_K(K)
    A = pr.assemble().tocsc()
    return A, spla.spsolve(A, pr.rhs(f_q))


def J_of(pr, K, f_q, u_obs):
    _, u = solve(pr, K, f_q)
    return 0.5 * float(np.sum((u - u_obs) ** 2))


def gradients(pr, K, f_q, u_obs, kind):
    A, u = solve(pr, K, f_q)
    lam = spla.spsolve(A.T.tocsc(), u - u_obs)
    gK = adjoint.grad_kappa(pr, lam, u) if kind == "scalar" else adjoint.grad_sym6(pr, lam, u)
    gf = adjoint.grad_f(pr, lam)
    return u, gK, gf


CASES = [synth.Workload("ring4_p3_kappa", 4, 3, "ring", 0.02, "scalar", "paper"),
         synth.Workload("twist4_p3_sym6", 4, 3, "twist", 0.0, "sym6", "smooth")]


@pytest.fixture(scope="module", params=CASES, ids=lambda w: w.name)
def case(request):
    wl = request.param
    pr, K, K_obs, f_q = make(wl)
    _, u_obs = solve(pr, K_obs, f_q)
    u, gK, gf = gradients(pr, K, f_q, u_obs, wl.k_kind)
    return dict(wl=wl, pr=pr, K=K, f_q=f_q, u_obs=u_obs, u=u, gK=gK, gf=gf)


def _dir_K(K, kind, seed=3):
    rng = np.random.default_rng(seed)
    if kind == "scalar":
        return rng.uniform(-1, 1, K.shape)
    d = rng.uniform(-1, 1, K.shape)
    return d


def _gK_dot(gK, d, kind):
    # gK: scalar (nq3, nq2, nq1) or (6, nq3, nq2, nq1); d in the layout of K
    if kind == "scalar":
        return float(np.sum(gK * d))
    return float(sum(np.sum(gK[c] * d[..., c]) for c in range(6)))


def test_gradient_K_matches_central_differences(case):
    pr, K, f_q, u_obs, kind = case["pr"], case["K"], case["f_q"], case["u_obs"], case["wl"].k_kind
    d = _dir_K(K, kind)
    eps = 1e-6 * np.abs(K).max()
    fd = (J_of(pr, K + eps * d, f_q, u_obs) - J_of(pr, K - eps * d, f_q, u_obs)) / (2 * eps)
    an = _gK_dot(case["gK"], d, kind)
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_gradient_f_matches_central_differences(case):
    pr, K, f_q, u_obs = case["pr"], case["K"], case["f_q"], case["u_obs"]
    d = np.random.default_rng(3).uniform(-1, 1, f_q.shape)
    eps = 1e-6 * np.abs(f_q).max()
    fd = (J_of(pr, K, f_q + eps * d, u_obs) - J_of(pr, K, f_q - eps * d, u_obs)) / (2 * eps)
    an = float(np.sum(case["gf"] * d))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_gradient_single_point(case):
    """Perturb K (and f) at the quadrature point of largest sensitivity only."""
    pr, K, f_q, u_obs, kind = case["pr"], case["K"], case["f_q"], case["u_obs"], case["wl"].k_kind
    gK = case["gK"] if kind == "scalar" else case["gK"][0]
    q = np.unravel_index(np.argmax(np.abs(gK)), gK.shape)
    d = np.zeros(K.shape)
    if kind == "scalar":
        d[q] = 1.0
    else:
        d[q + (0,)] = 1.0
    eps = 1e-6 * abs(K[q] if kind == "scalar" else K[q + (0,)])
    fd = (J_of(pr, K + eps * d, f_q, u_obs) - J_of(pr, K - eps * d, f_q, u_obs)) / (2 * eps)
    assert abs(fd - gK[q]) <= 1e-6 * abs(gK[q]), (fd, gK[q])
    qf = np.unravel_index(np.argmax(np.abs(case["gf"])), f_q.shape)
    df = np.zeros(f_q.shape)
    df[qf] = 1.0
    e2 = 1e-6 * np.abs(f_q).max()
    fd = (J_of(pr, K, f_q + e2 * df, u_obs) - J_of(pr, K, f_q - e2 * df, u_obs)) / (2 * e2)
    assert abs(fd - case["gf"][qf]) <= 1e-6 * abs(case["gf"][qf])


def test_euler_homogeneity(case):
    u, u_obs, K, f_q, kind = case["u"], case["u_obs"], case["K"], case["f_q"], case["wl"].k_kind
    r = float(np.dot(u - u_obs, u))
    sK = _gK_dot(case["gK"], K, kind)
    sf = float(np.sum(case["gf"] * f_q))
    assert abs(sK + r) <= 1e-10 * abs(r), (sK, r)
    assert abs(sf - r) <= 1e-10 * abs(r), (sf, r)


def test_zero_gradient_at_observation(case):
    pr, K, f_q, kind = case["pr"], case["K"], case["f_q"], case["wl"].k_kind
    _, gK, gf = gradients(pr, K, f_q, case["u"], kind)
    assert np.abs(gK).max() <= 1e-12 * np.abs(case["gK"]).max()
    assert np.abs(gf).max() <= 1e-12 * np.abs(case["gf"]).max()


def test_swapped_chain_rule_fails_finite_differences():
    """The planted mistake H = det J J^{-1} g J^{-T} (instead of J^{-T} g J^{-1})
    must be caught by the directional finite-difference pin on the twisted cube."""
    wl = CASES[1]
    pr, K, K_obs, f_q = make(wl)
    _, u_obs = solve(pr, K_obs, f_q)
    A, u = solve(pr, K, f_q)
    lam = spla.spsolve(A.T.tocsc(), u - u_obs)
    g = adjoint.grad_C_full(pr, lam, u)
    gm = np.moveaxis(np.moveaxis(g, 0, -1), 0, -1)
    Ji = np.linalg.inv(pr.J)
    H = pr.detJ[..., None, None] * (Ji @ gm @ np.swapaxes(Ji, -1, -2))       # the mistake
    wrong = np.empty((6,) + pr.detJ.shape)
    for c, (a, b) in enumerate(SYM_PAIRS):
        wrong[c] = H[..., a, b] if a == b else H[..., a, b] + H[..., b, a]
    d = _dir_K(K, "sym6")
    eps = 1e-6 * np.abs(K).max()
    fd = (J_of(pr, K + eps * d, f_q, u_obs) - J_of(pr, K - eps * d, f_q, u_obs)) / (2 * eps)
    right = _gK_dot(adjoint.grad_sym6(pr, lam, u), d, "sym6")
    bad = _gK_dot(wrong, d, "sym6")
    assert abs(fd - right) <= 1e-6 * abs(right)
    assert abs(fd - bad) > 1e-3 * abs(fd)


def test_gradient_alpha_matches_central_differences():
    wl = synth.Workload("ring4_p3", 4, 3, "ring", 0.02, "identity", "paper")
    pr = Problem(wl.knots(), wl.p, wl.ctrl(), None)
    f_q = np.asarray(wl.f()(pr.F))
    alpha = np.asarray(synth.alpha_field(30.0)(pr.F))
    pr.set_alpha(np.asarray(synth.alpha_field(60.0)(pr.F)))
    _, u_obs = solve(pr, None, f_q)

    def J_alpha(a):
        pr.set_alpha(a)
        _, u = solve(pr, None, f_q)
        return 0.5 * float(np.sum((u - u_obs) ** 2))
    pr.set_alpha(alpha)
    A, u = solve(pr, None, f_q)
    lam = spla.spsolve(A.T.tocsc(), u - u_obs)
    g = adjoint.grad_alpha(pr, lam, u)
    d = np.random.default_rng(4).uniform(-1, 1, alpha.shape)
    eps = 1e-4 * np.abs(alpha).max()        # J ~ 1e3 |dJ|: a smaller step loses digits to cancellation
    fd = (J_alpha(alpha + eps * d) - J_alpha(alpha - eps * d)) / (2 * eps)
    an = float(np.sum(g * d))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    # single quadrature point
    q = (pr.nq[2] // 2, pr.nq[1] // 3, pr.nq[0] // 2)
    e = np.zeros_like(alpha)
    e[q] = 1.0
    eps1 = 1e-2 * alpha[q]
    fd1 = (J_alpha(alpha + eps1 * e) - J_alpha(alpha - eps1 * e)) / (2 * eps1)
    assert abs(fd1 - g[q]) <= 1e-4 * abs(g[q]), (fd1, g[q])
    # planted mistake: the gradient without det J
    wrong = float(np.sum(g / pr.detJ * d))
    assert abs(fd - wrong) > 1e-2 * abs(fd)
