// Geometry at the quadrature points on the device (Section 2.1; the set-up step
// that the paper calls the main cost of its set-up): F, J^{-1} and det J at every
// quadrature point from the homogeneous control net (w P, w) of a polynomial
// (w = 1) or rational map, by sum factorisation in three passes:
//   z: Z[q3][k2][k1] = (sum_r B3 P, sum_r B-dot3 P)            8 values (4 components)
//   y: Y[q3][q2][k1] = (sum_b B2 Z0, sum_b B-dot2 Z0, sum_b B2 Z1)  12 values
//   x: at (q1, q2, q3): value and the three parametric derivatives of each
//      component (16 values), then the quotient rule F = P / W,
//      J = (dP - F dW^T) / W, det J and J^{-1} by cofactors.
// Each pass is one thread per output row entry, reading the p + 1 non-zero
// B-splines of its point from per-direction tables (first index, values,
// derivatives).  The same computation, inside the apply, is what computing the
// coefficients on the fly (the memory remark of Section 3.2) would cost.
#include <hip/hip_runtime.h>

#include "device.h"

namespace wqfd {

namespace {

constexpr int kGT = 256;

inline unsigned grid_of(size_t n) {
    size_t g = (n + kGT - 1) / kGT;
    return (unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

template <int P>
__global__ __launch_bounds__(kGT) void geom_z(GeomArgs a) {
    const int m1 = a.m[0], m2 = a.m[1], nq3 = a.nq[2];
    const size_t total = (size_t)nq3 * m2 * m1;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t col = idx % ((size_t)m2 * m1);
        const int q3 = (int)(idx / ((size_t)m2 * m1));
        const int f3 = a.first[2][q3];
        const double* b = a.B[2] + (size_t)q3 * (P + 1);
        const double* d = a.D[2] + (size_t)q3 * (P + 1);
        double z0[4] = {0, 0, 0, 0}, z1[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            const double* c = a.ctrl + ((size_t)(f3 + r) * m2 * m1 + col) * 4;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                z0[k] += b[r] * c[k];
                z1[k] += d[r] * c[k];
            }
        }
        double* o = a.Z + idx * 8;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[k] = z0[k];
            o[4 + k] = z1[k];
        }
    }
}

template <int P>
__global__ __launch_bounds__(kGT) void geom_y(GeomArgs a) {
    const int m1 = a.m[0], m2 = a.m[1], nq2 = a.nq[1], nq3 = a.nq[2];
    const size_t total = (size_t)nq3 * nq2 * m1;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int k1 = (int)(idx % m1);
        const size_t t = idx / m1;
        const int q2 = (int)(t % nq2);
        const int q3 = (int)(t / nq2);
        const int f2 = a.first[1][q2];
        const double* b = a.B[1] + (size_t)q2 * (P + 1);
        const double* d = a.D[1] + (size_t)q2 * (P + 1);
        double y00[4] = {0, 0, 0, 0}, y01[4] = {0, 0, 0, 0}, y10[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            const double* z = a.Z + (((size_t)q3 * m2 + (f2 + r)) * m1 + k1) * 8;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                y00[k] += b[r] * z[k];
                y01[k] += d[r] * z[k];
                y10[k] += b[r] * z[4 + k];
            }
        }
        double* o = a.Y + idx * 12;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[k] = y00[k];
            o[4 + k] = y01[k];
            o[8 + k] = y10[k];
        }
    }
}

template <int P>
__global__ __launch_bounds__(kGT) void geom_x(GeomArgs a) {
    const int m1 = a.m[0], nq1 = a.nq[0], nq2 = a.nq[1];
    const size_t Nq = a.Nq;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < Nq; q += (size_t)gridDim.x * blockDim.x) {
        const int q1 = (int)(q % nq1);
        const size_t row = q / nq1;                 // q3 nq2 + q2
        const int f1 = a.first[0][q1];
        const double* b = a.B[0] + (size_t)q1 * (P + 1);
        const double* d = a.D[0] + (size_t)q1 * (P + 1);
        double G[4][4];                             // [component][value, d/dxi1, d/dxi2, d/dxi3]
#pragma unroll
        for (int k = 0; k < 4; ++k) G[k][0] = G[k][1] = G[k][2] = G[k][3] = 0.0;
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            const double* y = a.Y + (row * m1 + (f1 + r)) * 12;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                G[k][0] += b[r] * y[k];
                G[k][1] += d[r] * y[k];
                G[k][2] += b[r] * y[4 + k];
                G[k][3] += b[r] * y[8 + k];
            }
        }
        const double iw = 1.0 / G[3][0];
        double F[3], J[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r) F[r] = G[r][0] * iw;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) J[r][c] = (G[r][c + 1] - F[r] * G[3][c + 1]) * iw;
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
        a.detJ[q] = det;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) a.Jinv[(size_t)(3 * r + c) * Nq + q] = Ji[r][c];
#pragma unroll
        for (int r = 0; r < 3; ++r) a.F[(size_t)r * Nq + q] = F[r];
        if (!(det > 0.0)) atomicOr(a.bad, 1);
        (void)nq2;
    }
}

template <int P>
hipError_t run(const GeomArgs& a, hipStream_t s) {
    const size_t nz = (size_t)a.nq[2] * a.m[1] * a.m[0], ny = (size_t)a.nq[2] * a.nq[1] * a.m[0];
    hipLaunchKernelGGL(geom_z<P>, dim3(grid_of(nz)), dim3(kGT), 0, s, a);
    hipLaunchKernelGGL(geom_y<P>, dim3(grid_of(ny)), dim3(kGT), 0, s, a);
    hipLaunchKernelGGL(geom_x<P>, dim3(grid_of(a.Nq)), dim3(kGT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

size_t geometry_scratch_bytes(const int m[3], const int nq[3]) {
    const size_t z = (size_t)nq[2] * m[1] * m[0] * 8, y = (size_t)nq[2] * nq[1] * m[0] * 12;
    return (z + y) * sizeof(double);
}

hipError_t launch_geometry(const GeomArgs& a, hipStream_t s) {
    switch (a.p) {
        case 2: return run<2>(a, s);
        case 3: return run<3>(a, s);
        case 4: return run<4>(a, s);
        case 5: return run<5>(a, s);
        case 6: return run<6>(a, s);
        case 7: return run<7>(a, s);
        case 8: return run<8>(a, s);
        case 9: return run<9>(a, s);
        case 10: return run<10>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace wqfd
