// Host-side (FP64, CPU) setup of the MF-WQ operator and the FD preconditioner:
// spline spaces, quadrature points, weighted-quadrature weights, geometry at the
// quadrature points and the 1D generalized eigenproblems.  Nothing here touches
// the GPU; the C-ABI layer uploads the results.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace wqfd {

constexpr int kMaxDegree = 10;

// Quadrature rule of the operator: weighted quadrature (Section 2.2), or the
// standard Gauss rule with p + 1 points per element, whose test factor is
// W_iq = w_q b_i^{(a)}(x_q) for every trial derivative order (the remark after
// rem:memory, eq. WDBgaussian).
enum Rule { kRuleWQ = 0, kRuleGauss = 1 };

// One direction of the tensor-product space (Section 2.1): open knot vector
// with simple interior knots, m B-splines of degree p, n = m - 2 interior ones,
// nq quadrature points (Section 2.2).
struct Space1D {
    int p = 0, m = 0, n = 0, nq = 0, n_el = 0;
    std::vector<double> knots;    // m + p + 1
    std::vector<double> breaks;   // n_el + 1 distinct knot values
    std::vector<double> xq;       // nq quadrature points, ascending
    // dense matrices, row-major
    std::vector<double> Bfull[2]; // [nq][m]   b_j^{(d)}(x_q), all j
    std::vector<double> B[2];     // [nq][n]   interior columns j = 1..m-2
    std::vector<double> W[2][2];  // [n][nq]   W^{ab}: a = test, b = trial derivative
    std::vector<double> Mi, Ki;   // [n][n]    interior 1D Galerkin mass / stiffness
    double max_exactness_residual = 0.0;
};

// Validates the knot vector and builds everything above for the given rule.
// Returns 0 or a negative wqfd error code with a message in `err`.
int build_space(int p, int nknots, const double* knots, bool with_weights, Space1D& out,
                std::string& err, int rule = kRuleWQ);

// Tensor Gauss rule of ng points per element and direction, for evaluating a
// discrete solution (the error measure of Section 4): per point the first of
// the p+1 B-splines that are non-zero there, their values and derivatives, and
// the Gauss weight scaled to the element.  Points ascend.
struct GaussSpace1D {
    int p = 0, m = 0, n_el = 0, ng = 0, nq = 0;   // nq = n_el ng
    std::vector<int> first;                      // [nq]
    std::vector<double> B, D;                    // [nq][p+1]
    std::vector<double> w;                       // [nq]
};
int gauss_space(int p, int nknots, const double* knots, int ng, GaussSpace1D& out, std::string& err);

// Values and first derivatives of the p+1 B-splines that are non-zero on the
// knot span containing x (span index returned; x == 1 uses the last span).
int eval_nonzero(const std::vector<double>& knots, int p, int m, double x, double* N, double* dN);

// Geometry at the quadrature points: detJ [Nq] and J^{-1} [9][Nq] (row-major
// 3x3 per point, entry (r, c) in plane 3 r + c) and F [3][Nq], from control
// points ctrl[m3][m2][m1][3] and, for a rational (NURBS) map, positive weights
// [m3][m2][m1] (null: polynomial map).  Returns 0, WQ_EINVAL for a weight
// <= 0, or WQ_EGEOM if det J <= 0 somewhere.
int geometry_at_quad(const Space1D* sp, const double* ctrl, const double* weights, double* detJ,
                     double* Jinv, double* F, std::string& err, int nthreads);

// Generalized symmetric eigenproblem K U = M U diag(lam), U^T M U = I by
// Cholesky of M and cyclic Jacobi on L^{-1} K L^{-T}.  U row-major [n][n]
// with eigenvector k in column k.  Returns 0 or WQ_ESINGULAR.
int gen_eig(int n, const std::vector<double>& K, const std::vector<double>& M,
            std::vector<double>& lam, std::vector<double>& U, std::string& err);

}  // namespace wqfd
