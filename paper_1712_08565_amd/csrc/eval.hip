// Evaluation of a discrete solution and of the geometry map at tensor Gauss
// points, one slab of elements along z at a time: the error measure of the
// k-refinement study (Section 4, Table 1) needs the solution's gradient and the
// weights w |det J| at (p + 3)^3 points per element, more points than the
// operator's own quadrature and, at 256^3 elements, more than is worth holding
// at once.
//
// One thread per point evaluates, from the homogeneous control net (w P, w) of
// the map (polynomial maps carry w = 1) and the coefficient vector u of the
// interior B-splines (the homogeneous Dirichlet space of Section 2.1), the
// values and parametric gradients of the map's numerator and denominator and of
// u_h = sum_j u_j b_j, each as a sum over the (p + 1)^3 B-splines that are
// non-zero at the point (x innermost, with the y and z factors applied per
// row).  Then F = P / W, J = (dP - F dW^T) / W (the quotient rule of a rational
// map), grad_x u_h = J^{-T} grad_xi u_h.
#include <hip/hip_runtime.h>

#include "device.h"

namespace wqfd {

namespace {

struct EvalArgs {
    EvalOp E;
    const double* u = nullptr;
    int q3_begin = 0;               // first quadrature plane of the slab
    size_t npts = 0;                // points of the slab: nq1 nq2 (planes)
    double* X = nullptr;            // [3][npts]
    double* wdet = nullptr;         // [npts]
    double* uh = nullptr;           // [npts]
    double* grad = nullptr;         // [3][npts]
};

template <int P>
__global__ __launch_bounds__(256) void eval_kernel(EvalArgs a) {
    const EvalOp& E = a.E;
    const int nq1 = E.nq[0], nq2 = E.nq[1];
    const int m1 = E.m[0], m2 = E.m[1], m3 = E.m[2];
    const int n1 = E.n[0], n2 = E.n[1];
    const size_t npl = (size_t)nq1 * nq2;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.npts;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int q1 = (int)(idx % nq1);
        const int q2 = (int)((idx / nq1) % nq2);
        const int q3 = a.q3_begin + (int)(idx / npl);
        const int f1 = E.first[0][q1], f2 = E.first[1][q2], f3 = E.first[2][q3];
        const double* bx = E.B[0] + (size_t)q1 * (P + 1);
        const double* dx = E.D[0] + (size_t)q1 * (P + 1);
        const double* by = E.B[1] + (size_t)q2 * (P + 1);
        const double* dy = E.D[1] + (size_t)q2 * (P + 1);
        const double* bz = E.B[2] + (size_t)q3 * (P + 1);
        const double* dz = E.D[2] + (size_t)q3 * (P + 1);
        double G[4][4], U[4];           // [component][value, d/dxi1, d/dxi2, d/dxi3]
        for (int c = 0; c < 4; ++c) G[c][0] = G[c][1] = G[c][2] = G[c][3] = U[c] = 0.0;
        for (int c = 0; c <= P; ++c) {
            const int k3 = f3 + c;
            const bool in3 = k3 >= 1 && k3 <= m3 - 2;
            for (int b = 0; b <= P; ++b) {
                const int k2 = f2 + b;
                const bool in23 = in3 && k2 >= 1 && k2 <= m2 - 2;
                const double* row = E.ctrl + (((size_t)k3 * m2 + k2) * m1 + f1) * 4;
                const long long ub = ((long long)(k3 - 1) * n2 + (k2 - 1)) * n1 + (f1 - 1);   // u index of (f1, k2, k3)
                double S[4] = {0, 0, 0, 0}, Sd[4] = {0, 0, 0, 0}, Su = 0.0, Sud = 0.0;
#pragma unroll
                for (int i = 0; i <= P; ++i) {
                    const double vb = bx[i], vd = dx[i];
#pragma unroll
                    for (int comp = 0; comp < 4; ++comp) {
                        const double pc = row[4 * i + comp];
                        S[comp] += vb * pc;
                        Sd[comp] += vd * pc;
                    }
                    const int k1 = f1 + i;
                    if (in23 && k1 >= 1 && k1 <= m1 - 2) {
                        const double uv = a.u[ub + i];
                        Su += vb * uv;
                        Sud += vd * uv;
                    }
                }
                const double yz = by[b] * bz[c], dyz = dy[b] * bz[c], ydz = by[b] * dz[c];
                for (int comp = 0; comp < 4; ++comp) {
                    G[comp][0] += yz * S[comp];
                    G[comp][1] += yz * Sd[comp];
                    G[comp][2] += dyz * S[comp];
                    G[comp][3] += ydz * S[comp];
                }
                U[0] += yz * Su;
                U[1] += yz * Sud;
                U[2] += dyz * Su;
                U[3] += ydz * Su;
            }
        }
        const double iw = 1.0 / G[3][0];
        double F[3], J[3][3];
        for (int r = 0; r < 3; ++r) F[r] = G[r][0] * iw;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) J[r][c] = (G[r][c + 1] - F[r] * G[3][c + 1]) * iw;
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double id = 1.0 / det;
        // J^{-1} by cofactors; grad_x u_h = J^{-T} grad_xi u_h
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
        const size_t n = a.npts;
        for (int r = 0; r < 3; ++r) {
            a.X[r * n + idx] = F[r];
            a.grad[r * n + idx] = Ji[0][r] * U[1] + Ji[1][r] * U[2] + Ji[2][r] * U[3];
        }
        a.uh[idx] = U[0];
        a.wdet[idx] = E.w[0][q1] * E.w[1][q2] * E.w[2][q3] * fabs(det);
    }
}

}  // namespace

hipError_t launch_eval_slab(const EvalOp& E, const double* u, int e3_begin, int e3_end, double* X, double* wdet,
                            double* uh, double* grad, hipStream_t s) {
    EvalArgs a;
    a.E = E;
    a.u = u;
    a.q3_begin = e3_begin * E.ng;
    a.npts = (size_t)E.nq[0] * E.nq[1] * (size_t)(e3_end - e3_begin) * E.ng;
    a.X = X;
    a.wdet = wdet;
    a.uh = uh;
    a.grad = grad;
    if (a.npts == 0) return hipSuccess;
    size_t blocks = (a.npts + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    const dim3 grid((unsigned)blocks), block(256);
    switch (E.p) {
        case 2: hipLaunchKernelGGL(eval_kernel<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(eval_kernel<3>, grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL(eval_kernel<4>, grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL(eval_kernel<5>, grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL(eval_kernel<6>, grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL(eval_kernel<7>, grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL(eval_kernel<8>, grid, block, 0, s, a); break;
        case 9: hipLaunchKernelGGL(eval_kernel<9>, grid, block, 0, s, a); break;
        case 10: hipLaunchKernelGGL(eval_kernel<10>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wqfd
