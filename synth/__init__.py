"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *defines* inputs: knot vectors, control nets, coefficient
fields, source terms and random vectors.  It contains none of the method's
arithmetic (no B-spline evaluation, no quadrature, no operator), so both the
CPU oracle and the GPU path can draw from it without sharing any code of the
method itself.

Workloads stand in for the paper's experiments (Section 4): the thick quarter
ring ``1 <= x1^2 + x2^2 <= 4, x1, x2 >= 0, 0 <= x3 <= 1`` and the oscillating
manufactured solution of eq. (exact-solution).  The paper represents the ring
with NURBS; here every geometry is a *polynomial* spline whose control points
sit at the images of the Greville abscissae (an O(h^2) spline approximation of
the target map that reproduces affine maps exactly), optionally perturbed by a
smooth seeded field that vanishes on the boundary.

Field functions accept either numpy arrays or torch tensors (of shape
``(..., 3)``) and return the same kind, so large coefficient fields can be
evaluated on the device.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, Optional, Tuple

import numpy as np

__all__ = [
    "uniform_knots", "nonuniform_knots", "greville", "control_net", "Workload", "WORKLOADS",
    "workload", "random_vector", "kappa_field", "sym6_field", "alpha_field",
    "u_sine", "grad_u_sine", "f_sine", "u_paper", "grad_u_paper", "f_paper", "f_smooth",
]


# ----------------------------------------------------------------------------
# array-namespace helpers (numpy or torch)
# ----------------------------------------------------------------------------
def _ns(x):
    if isinstance(x, np.ndarray):
        return np
    import torch  # noqa: WPS433  (only when a tensor is passed)
    return torch


def _stack(xp, parts, axis=-1):
    return xp.stack(parts, axis) if xp is np else xp.stack(parts, dim=axis)


# ----------------------------------------------------------------------------
# knots and control nets
# ----------------------------------------------------------------------------
def uniform_knots(n_el: int, p: int) -> np.ndarray:
    """Open knot vector on [0, 1] with ``n_el`` equal elements and simple interior
    knots (maximum regularity C^{p-1}, Section 2.1).  Length ``n_el + 2p + 1``."""
    inner = np.arange(1, n_el) / n_el
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def nonuniform_knots(n_el: int, p: int, seed: int, ratio: float = 4.0) -> np.ndarray:
    """Open knot vector with ``n_el`` elements of seeded random lengths (log-uniform
    within a factor ``ratio`` of each other) and simple interior knots: the
    non-uniform meshes the paper's algorithms are written for (Section 4)."""
    rng = np.random.default_rng(seed)
    h = np.exp(rng.uniform(-0.5, 0.5, n_el) * math.log(ratio))
    br = np.cumsum(h / h.sum())[:-1]
    return np.concatenate([np.zeros(p + 1), br, np.ones(p + 1)])


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae: the average of the p knots following knot k."""
    knots = np.asarray(knots, dtype=np.float64)
    m = len(knots) - p - 1
    return np.array([knots[k + 1:k + p + 1].mean() for k in range(m)])


def _map_identity(g1, g2, g3):
    return g1, g2, g3


def _map_ring(g1, g2, g3):
    r = 1.0 + g1
    t = 0.5 * math.pi * g2
    return r * np.cos(t), r * np.sin(t), g3


def _shear_matrix():
    # non-symmetric, det > 0 (affine sheared cube used for the C-convention pin)
    return np.array([[1.0, 0.3, 0.1], [0.2, 1.2, -0.15], [0.05, 0.25, 0.9]])


def _ring_homogeneous(g1, g2, g3):
    """Homogeneous coordinates (w x, w y, w z, w) of the exact thick quarter ring
    (1 <= r <= 2, 0 <= theta <= pi/2, 0 <= z <= 1) as a rational map: r = 1 + xi1,
    z = xi3, and in xi2 the quarter circle as the rational quadratic Bezier curve
    with control points (1, 0), (1, 1), (0, 1) and weights 1, 1/sqrt(2), 1.  Every
    component is a polynomial of degree <= 2 in xi2 and <= 1 in xi1 and xi3."""
    c = math.sqrt(0.5)
    b0, b1, b2 = (1.0 - g2) ** 2, 2.0 * g2 * (1.0 - g2), g2 ** 2
    w = b0 + c * b1 + b2
    r = 1.0 + g1
    return r * (b0 + c * b1), r * (c * b1 + b2), g3 * w, w


def nurbs_net(kind: str, knots3, p: int):
    """(P [k3, k2, k1, 3], w [k3, k2, k1]) of a rational map of degree p on the
    given knots: 'ring_nurbs' is the exact thick quarter ring.  Each homogeneous
    component is a product of polynomials of degree <= 2 <= p in one variable
    each, so it is the tensor product of the 1D interpolants at the Greville
    abscissae, which reproduce those polynomials exactly in the spline space."""
    if kind != "ring_nurbs":
        raise ValueError(f"unknown rational geometry {kind!r}")
    from scipy.interpolate import make_interp_spline

    def interp(l, f):
        g = greville(knots3[l], p)
        return make_interp_spline(g, f(g), k=p, t=np.asarray(knots3[l], dtype=np.float64)).c

    one = lambda g: np.ones_like(g)                                      # noqa: E731
    c = math.sqrt(0.5)
    b0 = lambda g: (1.0 - g) ** 2                                        # noqa: E731
    b1 = lambda g: 2.0 * g * (1.0 - g)                                   # noqa: E731
    b2 = lambda g: g ** 2                                                # noqa: E731
    r1, o1 = interp(0, lambda g: 1.0 + g), interp(0, one)
    X2 = interp(1, lambda g: b0(g) + c * b1(g))
    Y2 = interp(1, lambda g: c * b1(g) + b2(g))
    W2 = interp(1, lambda g: b0(g) + c * b1(g) + b2(g))
    z3, o3 = interp(2, lambda g: g), interp(2, one)
    outer = lambda a3, a2, a1: np.einsum("k,j,i->kji", a3, a2, a1)       # noqa: E731
    w = outer(o3, W2, o1)
    P = np.stack([outer(o3, X2, r1), outer(o3, Y2, r1), outer(z3, W2, o1)], -1) / w[..., None]
    return np.ascontiguousarray(P), np.ascontiguousarray(w)


def _map_shear(g1, g2, g3):
    A = _shear_matrix()
    X = np.stack([g1, g2, g3], -1) @ A.T
    return X[..., 0], X[..., 1], X[..., 2]


def _twist_angle(g3, c):
    return (math.pi / 6.0) * (g3 + (c / (2.0 * math.pi)) * np.sin(2.0 * math.pi * g3))


def _map_twist(c):
    def f(g1, g2, g3):
        th = _twist_angle(g3, c)
        a, b = g1 - 0.5, g2 - 0.5
        return 0.5 + a * np.cos(th) - b * np.sin(th), 0.5 + a * np.sin(th) + b * np.cos(th), g3
    return f


def control_net(kind: str, knots3, p: int, noise: float = 0.0, seed: int = 0,
                twist_seed: int = 4) -> np.ndarray:
    """Control points ``P[k3, k2, k1, :]`` (x index fastest) of a degree-p
    polynomial spline map of [0,1]^3 onto the named domain.

    kind: 'identity' (unit cube), 'ring' (thick quarter ring extruded in z),
    'shear' (affine, non-symmetric Jacobian), 'twist' (cube twisted about the
    vertical axis, up to 30 degrees at the top); these place the control points
    at the images of the Greville abscissae (second order in h).  'ring_interp'
    is the ring map interpolated at the Greville abscissae by the spline of the
    same knots (scipy.interpolate.make_interp_spline along each axis), accurate
    to order p + 1 in h.  'ring_nurbs' gives the Euclidean control points of the
    exact ring as a rational map (its weights from ``nurbs_net``).
    ``noise`` adds 0.02-style smooth perturbations that vanish on the boundary:
    eta_c(g) = sum_{a,b,c in {1,2}} r sin(a pi g1) sin(b pi g2) sin(c pi g3) / 8,
    r ~ U(-1, 1) from ``seed``.
    """
    g = [greville(k, p) for k in knots3]
    G3, G2, G1 = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    if kind == "identity":
        X = _map_identity(G1, G2, G3)
    elif kind == "ring":
        X = _map_ring(G1, G2, G3)
    elif kind == "ring_interp":
        from scipy.interpolate import make_interp_spline
        V = np.stack(_map_ring(G1, G2, G3), -1)           # values at the Greville grid [k3, k2, k1, 3]
        for axis, (k, gl) in zip((2, 1, 0), zip(knots3, g)):
            c = make_interp_spline(gl, V, k=p, t=np.asarray(k, dtype=np.float64), axis=axis).c
            V = np.moveaxis(c, 0, axis)                    # (the coefficients come with that axis first)
        X = (V[..., 0], V[..., 1], V[..., 2])
    elif kind == "ring_nurbs":
        X = tuple(np.moveaxis(nurbs_net(kind, knots3, p)[0], -1, 0))
    elif kind == "shear":
        X = _map_shear(G1, G2, G3)
    elif kind == "twist":
        c = np.random.default_rng(twist_seed).uniform(-0.5, 0.5)
        X = _map_twist(c)(G1, G2, G3)
    else:
        raise ValueError(f"unknown geometry kind {kind!r}")
    P = np.stack(X, -1).astype(np.float64)
    if noise:
        rng = np.random.default_rng(seed)
        r = rng.uniform(-1.0, 1.0, size=(3, 2, 2, 2))
        eta = np.zeros_like(P)
        for a in (1, 2):
            for b in (1, 2):
                for c in (1, 2):
                    s = np.sin(a * math.pi * G1) * np.sin(b * math.pi * G2) * np.sin(c * math.pi * G3)
                    for comp in range(3):
                        eta[..., comp] += r[comp, a - 1, b - 1, c - 1] * s / 8.0
        P = P + noise * eta
    return np.ascontiguousarray(P)


# ----------------------------------------------------------------------------
# coefficient fields K(x) (random Fourier features of a squared-exponential
# Gaussian field) and source terms f(x)
# ----------------------------------------------------------------------------
class _RFF:
    """g(x) = sqrt(2/M) sum_m cos(w_m . x + phi_m), w ~ N(0, ell^-2 I), phi ~ U[0, 2pi):
    a unit-variance Gaussian field with squared-exponential covariance of length ell."""

    def __init__(self, seed: int, ell: float, M: int):
        rng = np.random.default_rng(seed)
        self.w = rng.normal(0.0, 1.0 / ell, size=(M, 3))
        self.phi = rng.uniform(0.0, 2.0 * math.pi, size=M)
        self.M = M

    def __call__(self, x, chunk: int = 1 << 16):
        xp = _ns(x)
        shape = x.shape[:-1]
        flat = x.reshape(-1, 3)
        if xp is np:
            w, phi = self.w, self.phi
            out = np.empty(flat.shape[0])
            for s in range(0, flat.shape[0], chunk):
                out[s:s + chunk] = np.cos(flat[s:s + chunk] @ w.T + phi).sum(1)
        else:
            w = xp.as_tensor(self.w, dtype=flat.dtype, device=flat.device)
            phi = xp.as_tensor(self.phi, dtype=flat.dtype, device=flat.device)
            out = xp.empty(flat.shape[0], dtype=flat.dtype, device=flat.device)
            for s in range(0, flat.shape[0], chunk * 16):
                out[s:s + chunk * 16] = xp.cos(flat[s:s + chunk * 16] @ w.T + phi).sum(1)
        return (out * math.sqrt(2.0 / self.M)).reshape(shape)


def kappa_field(seed: int = 1, sigma: float = 0.5, ell: float = 0.1, M: int = 512) -> Callable:
    """Log-normal isotropic conductivity kappa(x) = exp(sigma g(x)); K = kappa I."""
    g = _RFF(seed, ell, M)

    def kappa(x):
        xp = _ns(x)
        return xp.exp(sigma * g(x))
    return kappa


def sym6_field(seeds=(5, 6, 7), ell: float = 0.25, M: int = 64,
               evals=(1.0, 0.5, 0.25)) -> Callable:
    """Full anisotropic SPD K(x) = Q diag(evals) Q^T with Q a z-y-x Euler rotation
    whose angles are (pi/4) tanh(g_i(x)).  Returns the six stored components in
    the order (K11, K22, K33, K12, K13, K23), stacked on the last axis."""
    gs = [_RFF(s, ell, M) for s in seeds]

    def K6(x):
        xp = _ns(x)
        a, b, c = [(math.pi / 4.0) * xp.tanh(g(x)) for g in gs]
        ca, sa, cb, sb, cc, sc = xp.cos(a), xp.sin(a), xp.cos(b), xp.sin(b), xp.cos(c), xp.sin(c)
        # Q = Rz(a) Ry(b) Rx(c)
        Q = [[ca * cb, ca * sb * sc - sa * cc, ca * sb * cc + sa * sc],
             [sa * cb, sa * sb * sc + ca * cc, sa * sb * cc - ca * sc],
             [-sb, cb * sc, cb * cc]]
        d = evals

        def k(i, j):
            return sum(Q[i][r] * d[r] * Q[j][r] for r in range(3))
        return _stack(xp, [k(0, 0), k(1, 1), k(2, 2), k(0, 1), k(0, 2), k(1, 2)])
    return K6


def alpha_field(scale: float = 1.0) -> Callable:
    """Smooth positive reaction coefficient of the model problem
    -div(K grad u) + alpha u = f:
    alpha(x) = scale (1 + 0.5 sin(pi x1) cos(pi x2) + 0.25 x3^2) >= scale / 2."""
    def alpha(x):
        xp = _ns(x)
        return scale * (1.0 + 0.5 * xp.sin(math.pi * x[..., 0]) * xp.cos(math.pi * x[..., 1])
                        + 0.25 * x[..., 2] * x[..., 2])
    return alpha


def u_sine(x):
    """u = sin(pi x1) sin(pi x2) sin(pi x3), zero on the unit cube's boundary."""
    xp = _ns(x)
    return xp.sin(math.pi * x[..., 0]) * xp.sin(math.pi * x[..., 1]) * xp.sin(math.pi * x[..., 2])


def f_sine(x):
    """-Laplace(u_sine) = 3 pi^2 u_sine."""
    return 3.0 * math.pi ** 2 * u_sine(x)


def u_paper(x):
    """The oscillating manufactured solution of eq. (exact-solution)."""
    xp = _ns(x)
    x1, x2, x3 = x[..., 0], x[..., 1], x[..., 2]
    rho = x1 * x1 + x2 * x2
    k = 5.0 * math.pi
    return xp.sin(k * x1) * xp.sin(k * x2) * xp.sin(k * x3) * (rho - 1.0) * (rho - 4.0)


def grad_u_paper(x):
    """Gradient of u_paper in closed form, shape (..., 3).  With s_l = sin(k x_l),
    c_l = cos(k x_l), g(rho) = (rho - 1)(rho - 4), g'(rho) = 2 rho - 5:
    du/dx1 = k c1 s2 s3 g + s1 s2 s3 g' 2 x1, du/dx2 likewise, du/dx3 = k s1 s2 c3 g."""
    xp = _ns(x)
    x1, x2, x3 = x[..., 0], x[..., 1], x[..., 2]
    k = 5.0 * math.pi
    s1, s2, s3 = xp.sin(k * x1), xp.sin(k * x2), xp.sin(k * x3)
    c1, c2, c3 = xp.cos(k * x1), xp.cos(k * x2), xp.cos(k * x3)
    rho = x1 * x1 + x2 * x2
    g = (rho - 1.0) * (rho - 4.0)
    gp = 2.0 * rho - 5.0
    s = s1 * s2 * s3
    return _stack(xp, [k * c1 * s2 * s3 * g + s * gp * 2.0 * x1,
                       k * s1 * c2 * s3 * g + s * gp * 2.0 * x2,
                       k * s1 * s2 * c3 * g])


def grad_u_sine(x):
    """Gradient of u_sine, shape (..., 3)."""
    xp = _ns(x)
    a, b, c = (math.pi * x[..., l] for l in range(3))
    return _stack(xp, [math.pi * xp.cos(a) * xp.sin(b) * xp.sin(c),
                       math.pi * xp.sin(a) * xp.cos(b) * xp.sin(c),
                       math.pi * xp.sin(a) * xp.sin(b) * xp.cos(c)])


def f_paper(x):
    """-Laplace(u_paper) in closed form.  With s = sin(k x1) sin(k x2) sin(k x3),
    g(rho) = (rho - 1)(rho - 4), rho = x1^2 + x2^2:
    Lap u = g Lap s + 2 grad s . grad g + s Lap g,
    Lap s = -3 k^2 s, grad g = g'(rho) (2 x1, 2 x2, 0), Lap g = 16 rho - 20."""
    xp = _ns(x)
    x1, x2, x3 = x[..., 0], x[..., 1], x[..., 2]
    k = 5.0 * math.pi
    s1, s2, s3 = xp.sin(k * x1), xp.sin(k * x2), xp.sin(k * x3)
    c1, c2 = xp.cos(k * x1), xp.cos(k * x2)
    s = s1 * s2 * s3
    rho = x1 * x1 + x2 * x2
    g = (rho - 1.0) * (rho - 4.0)
    gp = 2.0 * rho - 5.0
    grad_dot = gp * (2.0 * x1 * k * c1 * s2 * s3 + 2.0 * x2 * k * s1 * c2 * s3)
    lap = -3.0 * k * k * s * g + 2.0 * grad_dot + s * (16.0 * rho - 20.0)
    return -lap


def f_smooth(x):
    """A smooth, non-vanishing source: 1 + sin(pi x1) cos(pi x2) exp(x3)."""
    xp = _ns(x)
    return 1.0 + xp.sin(math.pi * x[..., 0]) * xp.cos(math.pi * x[..., 1]) * xp.exp(x[..., 2])


def random_vector(n: int, seed: int = 42) -> np.ndarray:
    """Seeded N(0,1) FP64 vector (apply benchmarks and parity tests)."""
    return np.random.default_rng(seed).standard_normal(n)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_el: int
    p: int
    geometry: str               # identity | ring | ring_interp | ring_nurbs | shear | twist
    noise: float = 0.0          # control-net perturbation amplitude
    k_kind: str = "identity"    # identity | scalar | sym6
    source: str = "sine"        # sine | paper | smooth
    geom_seed: int = 0
    knot_seed: Optional[int] = None   # None: uniform knots; else non-uniform, seeds knot_seed + l per direction

    def knots(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        if self.knot_seed is not None:
            return tuple(nonuniform_knots(self.n_el, self.p, self.knot_seed + l) for l in range(3))
        k = uniform_knots(self.n_el, self.p)
        return (k, k.copy(), k.copy())

    def ctrl(self) -> np.ndarray:
        return control_net(self.geometry, self.knots(), self.p, self.noise, self.geom_seed)

    def weights(self) -> Optional[np.ndarray]:
        """Control weights of a rational map, None for a polynomial one."""
        if self.geometry == "ring_nurbs":
            return nurbs_net(self.geometry, self.knots(), self.p)[1]
        return None

    def K_field(self) -> Optional[Callable]:
        if self.k_kind == "identity":
            return None
        if self.k_kind == "scalar":
            return kappa_field(seed=1, sigma=0.5, ell=0.1, M=512 if self.n_el <= 64 else 128)
        if self.k_kind == "sym6":
            return sym6_field()
        raise ValueError(self.k_kind)

    def f(self) -> Callable:
        return {"sine": f_sine, "paper": f_paper, "smooth": f_smooth}[self.source]

    @property
    def n(self) -> int:
        return self.n_el + self.p - 2


def _mk() -> Dict[str, Workload]:
    w = {}
    # unit cube, identity geometry, K = I, u = sin sin sin
    w["cube12_p3"] = Workload("cube12_p3", 12, 3, "identity")
    # thick quarter ring + 0.02 smooth noise, K = I, oscillating source of eq. (exact-solution)
    for p in (2, 3, 4, 5, 6):
        w[f"ring64_p{p}"] = Workload(f"ring64_p{p}", 64, p, "ring", 0.02, "identity", "paper")
    w["ring96_p5"] = Workload("ring96_p5", 96, 5, "ring", 0.02, "identity", "paper")
    # heterogeneous log-normal kappa (sigma 0.5, correlation length 0.1)
    w["ring48_p4_kappa"] = Workload("ring48_p4_kappa", 48, 4, "ring", 0.02, "scalar", "paper")
    # twisted cube, full anisotropic K per quadrature point
    w["twist128_p6"] = Workload("twist128_p6", 128, 6, "twist", 0.0, "sym6", "smooth")
    # structure-matched miniatures (explicit assembly is affordable)
    for p in (2, 3, 4, 5, 6):
        w[f"ring8_p{p}"] = Workload(f"ring8_p{p}", 8, p, "ring", 0.02, "identity", "paper")
    w["ring7_p4_kappa"] = Workload("ring7_p4_kappa", 7, 4, "ring", 0.02, "scalar", "paper")
    w["twist6_p6"] = Workload("twist6_p6", 6, 6, "twist", 0.0, "sym6", "smooth")
    w["twist5_p4"] = Workload("twist5_p4", 5, 4, "twist", 0.0, "sym6", "smooth")
    w["ring6_p8"] = Workload("ring6_p8", 6, 8, "ring", 0.02, "identity", "paper")
    # the highest degree of the paper's study (staged kernels)
    w["ring5_p10"] = Workload("ring5_p10", 5, 10, "ring", 0.02, "identity", "paper")
    # highest degree of the fused kernels: one tile, and several tiles with a ragged last one (n_q = 51)
    w["ring6_p7"] = Workload("ring6_p7", 6, 7, "ring", 0.02, "identity", "paper")
    w["ring18_p7"] = Workload("ring18_p7", 18, 7, "ring", 0.02, "identity", "paper")
    # several 16-point tiles per direction and a ragged last tile (n_q = 53)
    w["ring20_p6"] = Workload("ring20_p6", 20, 6, "ring", 0.02, "identity", "paper")
    w["shear6_p3"] = Workload("shear6_p3", 6, 3, "shear", 0.0, "identity", "sine")
    # non-uniform knots (element lengths within a factor 4, different per direction)
    for p in (2, 3, 4, 5, 6):
        w[f"ring8nu_p{p}"] = Workload(f"ring8nu_p{p}", 8, p, "ring", 0.02, "identity", "paper", knot_seed=200 + 10 * p)
    w["ring20nu_p6"] = Workload("ring20nu_p6", 20, 6, "ring", 0.02, "identity", "paper", knot_seed=300)
    w["ring6nu_p8"] = Workload("ring6nu_p8", 6, 8, "ring", 0.02, "identity", "paper", knot_seed=310)
    w["twist6nu_p5"] = Workload("twist6nu_p5", 6, 5, "twist", 0.0, "sym6", "smooth", knot_seed=320)
    w["ring64nu_p4"] = Workload("ring64nu_p4", 64, 4, "ring", 0.02, "identity", "paper", knot_seed=330)
    w["cube5_p2"] = Workload("cube5_p2", 5, 2, "identity")
    # the exact ring as a rational (NURBS) map, the paper's source; several tiles with a ragged tail at p = 5
    for p in (2, 3, 6):
        w[f"nurbs8_p{p}"] = Workload(f"nurbs8_p{p}", 8, p, "ring_nurbs", 0.0, "identity", "paper")
    w["nurbs20_p5"] = Workload("nurbs20_p5", 20, 5, "ring_nurbs", 0.0, "identity", "paper")
    w["nurbs6nu_p4"] = Workload("nurbs6nu_p4", 6, 4, "ring_nurbs", 0.0, "scalar", "paper", knot_seed=340)
    w["nurbs6_p8"] = Workload("nurbs6_p8", 6, 8, "ring_nurbs", 0.0, "identity", "paper")
    return w


WORKLOADS: Dict[str, Workload] = _mk()


def workload(name: str) -> Workload:
    return WORKLOADS[name]
