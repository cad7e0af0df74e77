// Host setup of the MF-WQ operator and the FD preconditioner (FP64, CPU).
//
//  * B-splines: de Boor's triangular recurrence over the non-zero span
//    functions, derivatives from the degree p-1 values (Section 2.1).
//  * Quadrature points: all breakpoints, midpoints of the interior elements,
//    and p+1 equispaced interior points in the first and last element
//    (n_q = 2 n_el + 2p + 1; the paper only says "a few more" points are
//    needed there, Section 2.2).
//  * Weights: for every interior test function i and derivative pair (a, b),
//    the minimum-2-norm solution of the exactness conditions
//        sum_{q in supp b_i} w_q b_j^{(b)}(x_q) = int b_i^{(a)} b_j^{(b)},  |j - i| <= p,
//    for all m trial B-splines (eqs. exactness1d, weights-support, exactness_K),
//    computed with a one-sided (Hestenes) Jacobi SVD after scaling each
//    equation to unit norm, relative rank cut-off 1e-12.
//  * Right-hand sides: Gauss-Legendre with p+1 points per element (exact).
//  * Geometry: F and J = dF/dxi at the quadrature points by sum factorisation
//    over the non-zero B-splines of each direction (Section 2.1).
//  * FD: Cholesky of M_l and cyclic Jacobi on L^{-1} K_l L^{-T} (Golub & Van Loan).
#include "host_setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <thread>

#include "../../include/wqfd.h"

namespace wqfd {

namespace {

constexpr double kPi = 3.14159265358979323846;

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute the derivative at the converged node
        double p0 = 1.0, p1 = 0.0;
        for (int j = 1; j <= n; ++j) {
            double p2 = p1;
            p1 = p0;
            p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

int find_span(const std::vector<double>& U, int p, int m, double x) {
    if (x >= U[m]) return m - 1;
    if (x <= U[p]) return p;
    int lo = p, hi = m;  // U[lo] <= x < U[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x < U[mid]) hi = mid; else lo = mid;
    }
    return lo;
}

// r - sum_s a[s] x[s] with every product split exactly by an FMA and the sum
// accumulated as a double-double (error-free TwoSum), rounded once at the end:
// accurate as if computed in twice the working precision.
double dot_residual(double r, const double* a, size_t stride, const double* x, int n) {
#pragma clang fp contract(off)
    // (no contraction: the error-free transformations need each product and
    // sum rounded on its own)
    double hi = r, lo = 0.0;
    for (int s = 0; s < n; ++s) {
        const double pr = a[(size_t)s * stride] * x[s];
        const double pe = std::fma(a[(size_t)s * stride], x[s], -pr);   // exact: a x = pr + pe
        const double t = hi - pr;                                         // TwoSum(hi, -pr)
        const double bb = t - hi;
        lo += (hi - (t - bb)) + (-pr - bb) - pe;
        hi = t;
    }
    return hi + lo;
}

// Minimum-norm solution of A w = r, A is nt x ns (row-major), via one-sided
// Jacobi on the columns of A^T, then one refinement step of the two
// conditions that define the minimum-norm solution, w = A^T z and A w = r:
// with f = A^T z - w and g = r - A w (both exactly rounded), the correction
// w += f + pinv(A) (g - A f).  On graded knots and at high degree the local
// systems reach condition numbers of 1e7 and more; without the step the
// solution leaks into the null space of A.  Returns the numerical rank.
int min_norm_solve(int nt, int ns, const std::vector<double>& A, const std::vector<double>& r,
                   std::vector<double>& w) {
    // M = A^T  (ns x nt), column k = equation k
    std::vector<double> M(ns * nt), V(nt * nt, 0.0);
    for (int t = 0; t < nt; ++t)
        for (int s = 0; s < ns; ++s) M[s * nt + t] = A[t * ns + s];
    for (int k = 0; k < nt; ++k) V[k * nt + k] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int c1 = 0; c1 < nt - 1; ++c1) {
            for (int c2 = c1 + 1; c2 < nt; ++c2) {
                double al = 0, be = 0, ga = 0;
                for (int s = 0; s < ns; ++s) {
                    double x = M[s * nt + c1], y = M[s * nt + c2];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                if (ga == 0.0) continue;
                double rel = std::fabs(ga) / std::sqrt(al * be);
                off = std::max(off, rel);
                if (rel < 1e-17) continue;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                for (int s = 0; s < ns; ++s) {
                    double x = M[s * nt + c1], y = M[s * nt + c2];
                    M[s * nt + c1] = c * x - sn * y;
                    M[s * nt + c2] = sn * x + c * y;
                }
                for (int k = 0; k < nt; ++k) {
                    double x = V[k * nt + c1], y = V[k * nt + c2];
                    V[k * nt + c1] = c * x - sn * y;
                    V[k * nt + c2] = sn * x + c * y;
                }
            }
        }
        if (off < 1e-15) break;
    }
    // A^T V = M with V orthogonal and the columns m_k of M orthogonal, so
    // A = V M^T and pinv(A) y = sum_k m_k (v_k . y) / |m_k|^2 over the kept k
    std::vector<double> sig2(nt);
    double smax = 0.0;
    for (int k = 0; k < nt; ++k) {
        double s2 = 0;
        for (int s = 0; s < ns; ++s) s2 += M[s * nt + k] * M[s * nt + k];
        sig2[k] = s2;
        smax = std::max(smax, std::sqrt(s2));
    }
    std::vector<char> keep(nt);
    int rank = 0;
    for (int k = 0; k < nt; ++k) {
        keep[k] = std::sqrt(sig2[k]) > 1e-12 * smax;
        rank += keep[k];
    }
    auto pinv = [&](const std::vector<double>& y, std::vector<double>& out) {   // out = pinv(A) y (ns)
        out.assign(ns, 0.0);
        for (int k = 0; k < nt; ++k) {
            if (!keep[k]) continue;
            double vy = 0;
            for (int t = 0; t < nt; ++t) vy += V[t * nt + k] * y[t];
            const double f = vy / sig2[k];
            for (int s = 0; s < ns; ++s) out[s] += f * M[s * nt + k];
        }
    };
    auto pinvT = [&](const std::vector<double>& x, std::vector<double>& out) {  // out = pinv(A^T) x (nt)
        out.assign(nt, 0.0);
        for (int k = 0; k < nt; ++k) {
            if (!keep[k]) continue;
            double mx = 0;
            for (int s = 0; s < ns; ++s) mx += M[s * nt + k] * x[s];
            const double f = mx / sig2[k];
            for (int t = 0; t < nt; ++t) out[t] += f * V[t * nt + k];
        }
    };
    pinv(r, w);
    std::vector<double> z, f(ns), g(nt), h(nt), dv;
    {
        pinvT(w, z);
        for (int s = 0; s < ns; ++s) f[s] = -dot_residual(w[s], &A[s], ns, z.data(), nt);    // A^T z - w
        for (int t = 0; t < nt; ++t) g[t] = dot_residual(r[t], &A[(size_t)t * ns], 1, w.data(), ns);  // r - A w
        for (int t = 0; t < nt; ++t) {
            double af = 0;
            for (int s = 0; s < ns; ++s) af += A[(size_t)t * ns + s] * f[s];
            h[t] = g[t] - af;
        }
        pinv(h, dv);
        for (int s = 0; s < ns; ++s) w[s] += f[s] + dv[s];
    }
    return rank;
}

}  // namespace

int eval_nonzero(const std::vector<double>& U, int p, int m, double x, double* N, double* dN) {
    const int mu = find_span(U, p, m, x);
    double left[kMaxDegree + 2], right[kMaxDegree + 2], Nm[kMaxDegree + 2];
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        if (j == p)
            for (int r = 0; r < p; ++r) Nm[r] = N[r];  // degree p-1: functions mu-p+1..mu
        left[j] = x - U[mu + 1 - j];
        right[j] = U[mu + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
    for (int r = 0; r <= p; ++r) {
        const int i = mu - p + r;
        double d = 0.0;
        if (r >= 1) d += Nm[r - 1] / (U[i + p] - U[i]);
        if (r <= p - 1) d -= Nm[r] / (U[i + p + 1] - U[i + 1]);
        dN[r] = p * d;
    }
    return mu;
}

int build_space(int p, int nknots, const double* knots, bool with_weights, Space1D& S,
                std::string& err, int rule) {
    char buf[256];
    if (p < 2 || p > kMaxDegree) {
        snprintf(buf, sizeof buf, "degree p = %d outside [2, %d]", p, kMaxDegree);
        err = buf;
        return WQ_EINVAL;
    }
    if (!knots || nknots < 2 * p + 4) {
        err = "knot vector too short (need at least 3 elements)";
        return WQ_EINVAL;
    }
    S = Space1D();
    S.p = p;
    S.knots.assign(knots, knots + nknots);
    S.m = nknots - p - 1;
    S.n = S.m - 2;
    const auto& U = S.knots;
    for (int i = 0; i <= p; ++i) {
        if (U[i] != 0.0 || U[nknots - 1 - i] != 1.0) {
            err = "knot vector is not open on [0, 1] (p+1 end knots equal to 0 and 1)";
            return WQ_EINVAL;
        }
    }
    for (int i = p + 1; i < nknots - p - 1; ++i) {
        if (!(U[i] > U[i - 1]) || !(U[i] < 1.0)) {
            err = "interior knots must be strictly increasing and simple (maximum regularity)";
            return WQ_EINVAL;
        }
    }
    S.breaks.push_back(0.0);
    for (int i = p + 1; i < nknots - p - 1; ++i) S.breaks.push_back(U[i]);
    S.breaks.push_back(1.0);
    S.n_el = (int)S.breaks.size() - 1;
    if (S.n_el < 3) {
        err = "need at least 3 elements per direction";
        return WQ_EINVAL;
    }
    // quadrature points
    const auto& br = S.breaks;
    std::vector<double> gx, gw;                   // Gauss-Legendre rule on [-1, 1], p + 1 points
    gauss_legendre(p + 1, gx, gw);
    std::vector<double> xq, wq;                   // wq: Gauss weights of the points (Gauss rule)
    if (rule == kRuleGauss) {
        std::vector<int> ord(p + 1);                  // nodes in ascending order
        for (int g = 0; g <= p; ++g) ord[g] = g;
        std::sort(ord.begin(), ord.end(), [&](int u, int v) { return gx[u] < gx[v]; });
        for (int e = 0; e < S.n_el; ++e) {
            const double lo = br[e], h = br[e + 1] - br[e];
            for (int g : ord) {
                xq.push_back(lo + 0.5 * h * (gx[g] + 1.0));
                wq.push_back(0.5 * h * gw[g]);
            }
        }
    } else {
        xq.assign(br.begin(), br.end());
        for (int e = 1; e < S.n_el - 1; ++e) xq.push_back(0.5 * (br[e] + br[e + 1]));
        for (int e : {0, S.n_el - 1}) {
            const double h = br[e + 1] - br[e];
            for (int k = 1; k <= p + 1; ++k) xq.push_back(br[e] + k * h / (p + 2));
        }
        std::sort(xq.begin(), xq.end());
    }
    S.xq = xq;
    S.nq = (int)xq.size();
    const int m = S.m, n = S.n, nq = S.nq;
    // basis matrices
    double Nv[kMaxDegree + 2], dNv[kMaxDegree + 2];
    for (int d = 0; d < 2; ++d) {
        S.Bfull[d].assign((size_t)nq * m, 0.0);
        S.B[d].assign((size_t)nq * n, 0.0);
    }
    for (int q = 0; q < nq; ++q) {
        const int mu = eval_nonzero(U, p, m, xq[q], Nv, dNv);
        for (int r = 0; r <= p; ++r) {
            const int j = mu - p + r;
            S.Bfull[0][(size_t)q * m + j] = Nv[r];
            S.Bfull[1][(size_t)q * m + j] = dNv[r];
            if (j >= 1 && j <= m - 2) {
                S.B[0][(size_t)q * n + j - 1] = Nv[r];
                S.B[1][(size_t)q * n + j - 1] = dNv[r];
            }
        }
    }
    // 1D Galerkin integrals G^{ab} (m x m) with p+1 Gauss points per element
    std::vector<double> G[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) G[a][b].assign((size_t)m * m, 0.0);
    for (int e = 0; e < S.n_el; ++e) {
        const double lo = br[e], hi = br[e + 1], h = hi - lo;
        for (int g = 0; g <= p; ++g) {
            const double x = lo + 0.5 * h * (gx[g] + 1.0), wt = 0.5 * h * gw[g];
            const int mu = eval_nonzero(U, p, m, x, Nv, dNv);
            const double* F[2] = {Nv, dNv};
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int r = 0; r <= p; ++r)
                        for (int c = 0; c <= p; ++c)
                            G[a][b][(size_t)(mu - p + r) * m + (mu - p + c)] += wt * F[a][r] * F[b][c];
        }
    }
    S.Mi.assign((size_t)n * n, 0.0);
    S.Ki.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            S.Mi[(size_t)i * n + j] = G[0][0][(size_t)(i + 1) * m + j + 1];
            S.Ki[(size_t)i * n + j] = G[1][1][(size_t)(i + 1) * m + j + 1];
        }
    if (!with_weights) return WQ_OK;
    if (rule == kRuleGauss) {                     // W^{ab}_iq = w_q b_i^{(a)}(x_q), any b
        for (int a = 0; a < 2; ++a) {
            S.W[a][0].assign((size_t)n * nq, 0.0);
            for (int i = 0; i < n; ++i)
                for (int q = 0; q < nq; ++q) S.W[a][0][(size_t)i * nq + q] = wq[q] * S.B[a][(size_t)q * n + i];
            S.W[a][1] = S.W[a][0];
        }
        return WQ_OK;
    }
    // weights
    double worst = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            auto& W = S.W[a][b];
            W.assign((size_t)n * nq, 0.0);
            for (int i = 1; i <= m - 2; ++i) {
                const double lo = U[i], hi = U[i + p + 1];
                std::vector<int> Sq, Tj;
                for (int q = 0; q < nq; ++q)
                    if (xq[q] >= lo && xq[q] <= hi) Sq.push_back(q);
                for (int j = std::max(0, i - p); j <= std::min(m - 1, i + p); ++j) Tj.push_back(j);
                const int ns = (int)Sq.size(), nt = (int)Tj.size();
                std::vector<double> A((size_t)nt * ns), r(nt), As((size_t)nt * ns), rs(nt), w;
                for (int t = 0; t < nt; ++t) {
                    double nrm = 0;
                    for (int s = 0; s < ns; ++s) {
                        A[t * ns + s] = S.Bfull[b][(size_t)Sq[s] * m + Tj[t]];
                        nrm += A[t * ns + s] * A[t * ns + s];
                    }
                    r[t] = G[a][b][(size_t)i * m + Tj[t]];
                    const double sc = nrm > 0 ? 1.0 / std::sqrt(nrm) : 0.0;
                    for (int s = 0; s < ns; ++s) As[t * ns + s] = A[t * ns + s] * sc;
                    rs[t] = r[t] * sc;
                }
                min_norm_solve(nt, ns, As, rs, w);
                double rmax = 0, res = 0;
                for (int t = 0; t < nt; ++t) {
                    double acc = -r[t];
                    for (int s = 0; s < ns; ++s) acc += A[t * ns + s] * w[s];
                    res = std::max(res, std::fabs(acc));
                    rmax = std::max(rmax, std::fabs(r[t]));
                }
                const double rel = res / std::max(rmax, 1e-300);
                worst = std::max(worst, rel);
                if (rel > 1e-9) {
                    snprintf(buf, sizeof buf,
                             "weighted-quadrature exactness system (a=%d, b=%d, i=%d) not solvable: "
                             "relative residual %.3e",
                             a, b, i, rel);
                    err = buf;
                    return WQ_ESINGULAR;
                }
                for (int s = 0; s < ns; ++s) W[(size_t)(i - 1) * nq + Sq[s]] = w[s];
            }
        }
    S.max_exactness_residual = worst;
    return WQ_OK;
}

int gauss_space(int p, int nknots, const double* knots, int ng, GaussSpace1D& G, std::string& err) {
    if (ng < 1 || ng > 32) {
        err = "Gauss points per element must be in 1..32";
        return WQ_EINVAL;
    }
    Space1D S;
    int rc = build_space(p, nknots, knots, false, S, err);
    if (rc) return rc;
    std::vector<double> gx, gw;
    gauss_legendre(ng, gx, gw);
    G.p = p;
    G.m = S.m;
    G.n_el = S.n_el;
    G.ng = ng;
    G.nq = S.n_el * ng;
    G.first.resize(G.nq);
    G.B.resize((size_t)G.nq * (p + 1));
    G.D.resize((size_t)G.nq * (p + 1));
    G.w.resize(G.nq);
    for (int e = 0; e < S.n_el; ++e) {
        const double a = S.breaks[e], b = S.breaks[e + 1];
        for (int g = 0; g < ng; ++g) {
            // ascending points inside the element (the rule's nodes run from +1 down)
            const double t = gx[ng - 1 - g];
            const int q = e * ng + g;
            const double x = 0.5 * (a + b) + 0.5 * (b - a) * t;
            const int mu = eval_nonzero(S.knots, p, S.m, x, &G.B[(size_t)q * (p + 1)], &G.D[(size_t)q * (p + 1)]);
            G.first[q] = mu - p;
            G.w[q] = 0.5 * (b - a) * gw[ng - 1 - g];
        }
    }
    return WQ_OK;
}

namespace {

// Sum factorization of a control net with NC components per point (x, y, z, and
// for a rational map the weight last, the first three multiplied by it): value
// and parametric gradient of every component at the quadrature points of plane
// k3 range [k_begin, k_end) with stride, handed to `at(q, value[NC], grad[NC][3])`.
template <int NC, typename At>
void sum_factorize(const Space1D* sp, const double* ctrl, int tid, int nthreads, At&& at) {
    const Space1D &S1 = sp[0], &S2 = sp[1], &S3 = sp[2];
    const int p = S1.p;
    const int m1 = S1.m, m2 = S2.m;
    const int nq1 = S1.nq, nq2 = S2.nq, nq3 = S3.nq;
    struct Nz {
        std::vector<int> first;
        std::vector<double> v, d;
    } nz[3];
    for (int l = 0; l < 3; ++l) {
        const Space1D& S = sp[l];
        nz[l].first.resize(S.nq);
        nz[l].v.resize((size_t)S.nq * (p + 1));
        nz[l].d.resize((size_t)S.nq * (p + 1));
        for (int q = 0; q < S.nq; ++q) {
            int mu = eval_nonzero(S.knots, p, S.m, S.xq[q], &nz[l].v[(size_t)q * (p + 1)],
                                  &nz[l].d[(size_t)q * (p + 1)]);
            nz[l].first[q] = mu - p;
        }
    }
    // per quad plane: z contraction, then y, then x
    std::vector<double> Pz0((size_t)m2 * m1 * NC), Pz1((size_t)m2 * m1 * NC);
    std::vector<double> Y00((size_t)m1 * NC), Y01((size_t)m1 * NC), Y10((size_t)m1 * NC);
    for (int k = tid; k < nq3; k += nthreads) {
        std::fill(Pz0.begin(), Pz0.end(), 0.0);
        std::fill(Pz1.begin(), Pz1.end(), 0.0);
        const int f3 = nz[2].first[k];
        for (int r = 0; r <= p; ++r) {
            const double bv = nz[2].v[(size_t)k * (p + 1) + r], bd = nz[2].d[(size_t)k * (p + 1) + r];
            const double* P = ctrl + (size_t)(f3 + r) * m2 * m1 * NC;
            for (size_t t = 0; t < (size_t)m2 * m1 * NC; ++t) {
                Pz0[t] += bv * P[t];
                Pz1[t] += bd * P[t];
            }
        }
        for (int q2 = 0; q2 < nq2; ++q2) {
            std::fill(Y00.begin(), Y00.end(), 0.0);
            std::fill(Y01.begin(), Y01.end(), 0.0);
            std::fill(Y10.begin(), Y10.end(), 0.0);
            const int f2 = nz[1].first[q2];
            for (int r = 0; r <= p; ++r) {
                const double bv = nz[1].v[(size_t)q2 * (p + 1) + r], bd = nz[1].d[(size_t)q2 * (p + 1) + r];
                const double* A0 = &Pz0[(size_t)(f2 + r) * m1 * NC];
                const double* A1 = &Pz1[(size_t)(f2 + r) * m1 * NC];
                for (int t = 0; t < m1 * NC; ++t) {
                    Y00[t] += bv * A0[t];
                    Y01[t] += bd * A0[t];
                    Y10[t] += bv * A1[t];
                }
            }
            for (int q1 = 0; q1 < nq1; ++q1) {
                const int f1 = nz[0].first[q1];
                double Fv[NC], G[NC][3];
                for (int a = 0; a < NC; ++a) Fv[a] = G[a][0] = G[a][1] = G[a][2] = 0.0;
                for (int r = 0; r <= p; ++r) {
                    const double bv = nz[0].v[(size_t)q1 * (p + 1) + r], bd = nz[0].d[(size_t)q1 * (p + 1) + r];
                    const int j = f1 + r;
                    for (int a = 0; a < NC; ++a) {
                        Fv[a] += bv * Y00[j * NC + a];
                        G[a][0] += bd * Y00[j * NC + a];
                        G[a][1] += bv * Y01[j * NC + a];
                        G[a][2] += bv * Y10[j * NC + a];
                    }
                }
                at(((size_t)k * nq2 + q2) * nq1 + q1, Fv, G);
            }
        }
    }
}

// det J, J^{-1} (plane 3 r + c) and F of one point; false if det J <= 0
inline bool store_point(size_t q, size_t Nq, const double (&Fv)[3], const double (&J)[3][3], double* detJ,
                        double* Jinv, double* F) {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    double Ji[3][3];
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    detJ[q] = det;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Jinv[(size_t)(3 * r + c) * Nq + q] = Ji[r][c];
    for (int a = 0; a < 3; ++a) F[(size_t)a * Nq + q] = Fv[a];
    return det > 0.0;
}

}  // namespace

int geometry_at_quad(const Space1D* sp, const double* ctrl, const double* weights, double* detJ, double* Jinv,
                     double* F, std::string& err, int nthreads) {
    const size_t Nq = (size_t)sp[0].nq * sp[1].nq * sp[2].nq;
    const size_t M = (size_t)sp[0].m * sp[1].m * sp[2].m;
    std::vector<int> bad(nthreads, 0);
    std::vector<double> hom;
    if (weights) {
        // homogeneous control net (w P, w): the rational map is the quotient of
        // two polynomial splines, F = (sum w_k P_k b_k) / (sum w_k b_k)
        for (size_t k = 0; k < M; ++k)
            if (!(weights[k] > 0.0)) {
                err = "rational map: every control weight must be positive";
                return WQ_EINVAL;
            }
        hom.resize(M * 4);
        for (size_t k = 0; k < M; ++k) {
            for (int a = 0; a < 3; ++a) hom[4 * k + a] = weights[k] * ctrl[3 * k + a];
            hom[4 * k + 3] = weights[k];
        }
    }
    auto work = [&](int tid) {
        if (!weights) {
            sum_factorize<3>(sp, ctrl, tid, nthreads, [&](size_t q, const double (&Fv)[3], const double (&J)[3][3]) {
                if (!store_point(q, Nq, Fv, J, detJ, Jinv, F)) bad[tid] = 1;
            });
            return;
        }
        // quotient rule: dF_a/dxi_b = (dP_a/dxi_b - F_a dW/dxi_b) / W
        sum_factorize<4>(sp, hom.data(), tid, nthreads,
                         [&](size_t q, const double (&Pv)[4], const double (&G)[4][3]) {
                             const double iw = 1.0 / Pv[3];
                             double Fv[3], J[3][3];
                             for (int a = 0; a < 3; ++a) Fv[a] = Pv[a] * iw;
                             for (int a = 0; a < 3; ++a)
                                 for (int b = 0; b < 3; ++b) J[a][b] = (G[a][b] - Fv[a] * G[3][b]) * iw;
                             if (!store_point(q, Nq, Fv, J, detJ, Jinv, F)) bad[tid] = 1;
                         });
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nthreads; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& t : th) t.join();
    for (int b : bad)
        if (b) {
            err = "geometry map is not orientation preserving: det J <= 0 at a quadrature point";
            return WQ_EGEOM;
        }
    return WQ_OK;
}

int gen_eig(int n, const std::vector<double>& K, const std::vector<double>& M, std::vector<double>& lam,
            std::vector<double>& U, std::string& err) {
    // Cholesky M = L L^T (lower, row-major)
    std::vector<double> L((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = M[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) {
            err = "FD: 1D mass matrix is not positive definite";
            return WQ_ESINGULAR;
        }
        const double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = M[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = s / ljj;
        }
    }
    // X = L^{-1} K (forward substitution per column)
    std::vector<double> X((size_t)n * n), A((size_t)n * n);
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            double s = K[(size_t)i * n + c];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * X[(size_t)k * n + c];
            X[(size_t)i * n + c] = s / L[(size_t)i * n + i];
        }
    // A = X L^{-T} = (L^{-1} X^T)^T
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            double s = X[(size_t)c * n + i];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * A[(size_t)c * n + k];
            A[(size_t)c * n + i] = s / L[(size_t)i * n + i];
        }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
            A[(size_t)i * n + j] = A[(size_t)j * n + i] = s;
        }
    // cyclic Jacobi: A = Q diag Q^T
    std::vector<double> Q((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
            for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        }
        if (off <= 1e-32 * diag) break;
        for (int pp = 0; pp < n - 1; ++pp)
            for (int qq = pp + 1; qq < n; ++qq) {
                const double apq = A[(size_t)pp * n + qq];
                if (apq == 0.0) continue;
                const double app = A[(size_t)pp * n + pp], aqq = A[(size_t)qq * n + qq];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(1.0 + theta * theta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = A[(size_t)k * n + pp], akq = A[(size_t)k * n + qq];
                    A[(size_t)k * n + pp] = c * akp - s * akq;
                    A[(size_t)k * n + qq] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = A[(size_t)pp * n + k], aqk = A[(size_t)qq * n + k];
                    A[(size_t)pp * n + k] = c * apk - s * aqk;
                    A[(size_t)qq * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q[(size_t)k * n + pp], qkq = Q[(size_t)k * n + qq];
                    Q[(size_t)k * n + pp] = c * qkp - s * qkq;
                    Q[(size_t)k * n + qq] = s * qkp + c * qkq;
                }
            }
    }
    // sort ascending
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
    lam.resize(n);
    std::vector<double> Qs((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        lam[k] = A[(size_t)order[k] * n + order[k]];
        for (int i = 0; i < n; ++i) Qs[(size_t)i * n + k] = Q[(size_t)i * n + order[k]];
    }
    // U = L^{-T} Q (back substitution per column)
    U.assign((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            double s = Qs[(size_t)i * n + c];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * U[(size_t)k * n + c];
            U[(size_t)i * n + c] = s / L[(size_t)i * n + i];
        }
    return WQ_OK;
}

}  // namespace wqfd
