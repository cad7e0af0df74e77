// MF-WQ stiffness operator on gfx950: Algorithm 2 of Section 3.2,
//     K~ v = sum_{a,b} W^(a,b) D^(a,b) B^(b) v,
// evaluated by sum factorisation (eq. sum-factorization): banded 1D
// contractions along z, y and x with the basis matrices B_l / B-dot_l, a
// pointwise product with the coefficient planes C_ab(x_q), then banded
// contractions with the weight matrices W_l^{ab}.  Also the transpose, the
// coefficient set-up C = det J J^{-1} K J^{-T} (eq. C), the load vector and the
// adjoint gradients with respect to K and f.  With a reaction coefficient
// alpha the operator also carries the mass term of Algorithm 1 (Section 3.1),
// M~ v = W^(00) diag(alpha det J) B v (eq. WDB), plus dJ/dalpha.
//
// This file holds the staged form: one launch per 1D contraction, with
// intermediates in device memory.  Each launch streams its input once with
// coalesced accesses along x.
#include <hip/hip_runtime.h>

#include "buffer_store.h"
#include "device.h"

namespace wqfd {

namespace {

constexpr int kThreads = 256;

// ab index pairs: direction l gets a_l = [l == alpha], b_l = [l == beta];
// weight variant v = 2 a + b; coefficient plane of the symmetric pair.
__host__ __device__ inline int plane_of(int a, int b) {
    if (a == b) return a;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

enum { kPlain = 0, kMulIn = 1, kMulOut = 2 };

// out[...] (+)= sum_s coef[r][s] * in[... start[r] + s ...] along AXIS
// (0 = x, 1 = y, 2 = z); input dims (d0, d1, d2) with x fastest; output has R
// entries along AXIS.  kMulIn multiplies each input by mul (same layout as in),
// kMulOut multiplies the sum by mul (same layout as out).
template <typename T, int AXIS, int MODE>
__global__ __launch_bounds__(kThreads) void band_axis_kernel(
    const T* __restrict__ in, const T* __restrict__ mul, T* __restrict__ out, int d0, int d1, int d2,
    int R, const int* __restrict__ start, const T* __restrict__ coef, int L, int accumulate) {
    const int o0 = AXIS == 0 ? R : d0;
    const int o1 = AXIS == 1 ? R : d1;
    const int o2 = AXIS == 2 ? R : d2;
    const size_t total = (size_t)o0 * o1 * o2;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(idx % o0);
        const size_t t = idx / o0;
        const int y = (int)(t % o1);
        const int z = (int)(t / o1);
        const int r = AXIS == 0 ? x : (AXIS == 1 ? y : z);
        const int st = start[r];
        const T* cf = coef + (size_t)r * L;
        size_t base, stride;
        if (AXIS == 0) {
            base = ((size_t)z * d1 + y) * d0 + st;
            stride = 1;
        } else if (AXIS == 1) {
            base = ((size_t)z * d1 + st) * d0 + x;
            stride = (size_t)d0;
        } else {
            base = ((size_t)st * d1 + y) * d0 + x;
            stride = (size_t)d0 * d1;
        }
        T sum = 0;
        for (int s = 0; s < L; ++s) {
            T val = in[base + s * stride];
            if (MODE == kMulIn) val *= mul[base + s * stride];
            sum += cf[s] * val;
        }
        if (MODE == kMulOut) sum *= mul[idx];
        out[idx] = accumulate ? out[idx] + sum : sum;
    }
}

inline int grid_for(size_t total) {
    size_t g = (total + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

template <typename T, int MODE = kPlain>
hipError_t band(int axis, const Band<T>& b, const T* in, const T* mul, T* out, int d0, int d1, int d2,
                bool acc, hipStream_t s) {
    const int dims[3] = {d0, d1, d2};
    size_t total = (size_t)b.rows;
    for (int a = 0; a < 3; ++a)
        if (a != axis) total *= dims[a];
    const int g = grid_for(total);
    switch (axis) {
        case 0:
            hipLaunchKernelGGL((band_axis_kernel<T, 0, MODE>), dim3(g), dim3(kThreads), 0, s, in, mul, out, d0, d1,
                               d2, b.rows, b.start, b.c, b.L, (int)acc);
            break;
        case 1:
            hipLaunchKernelGGL((band_axis_kernel<T, 1, MODE>), dim3(g), dim3(kThreads), 0, s, in, mul, out, d0, d1,
                               d2, b.rows, b.start, b.c, b.L, (int)acc);
            break;
        default:
            hipLaunchKernelGGL((band_axis_kernel<T, 2, MODE>), dim3(g), dim3(kThreads), 0, s, in, mul, out, d0, d1,
                               d2, b.rows, b.start, b.c, b.L, (int)acc);
            break;
    }
    return hipGetLastError();
}

#define WQ_TRY(...)                            \
    do {                                       \
        hipError_t e_ = (__VA_ARGS__);         \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

// Scratch layout shared by the staged forward and transposed applies.
template <typename T>
struct Staged {
    T *g[3], *A, *Bq, *Z[4], *X;
    Staged(const WqOp& op, void* base) {
        const size_t n1 = op.n[0], n2 = op.n[1], nq1 = op.nq[0], nq2 = op.nq[1], nq3 = op.nq[2];
        T* p = reinterpret_cast<T*>(base);
        for (int k = 0; k < 3; ++k) {
            g[k] = p;
            p += op.Nq;
        }
        A = p;                    // nq3 nq2 n1
        p += nq3 * nq2 * n1;
        Bq = p;                   // nq3 nq2 n1
        p += nq3 * nq2 * n1;
        X = p;                    // nq3 nq2 nq1
        p += nq3 * nq2 * nq1;
        for (int k = 0; k < 4; ++k) {
            Z[k] = p;             // nq3 n2 n1 (z-quadrature, xy-DOF)
            p += nq3 * n2 * n1;
        }
    }
    static size_t elems(const WqOp& op) {
        const size_t n1 = op.n[0], n2 = op.n[1], nq1 = op.nq[0], nq2 = op.nq[1], nq3 = op.nq[2];
        return 3 * op.Nq + 2 * nq3 * nq2 * n1 + nq3 * nq2 * nq1 + 4 * nq3 * n2 * n1;
    }
};

// v~^(beta) = B^(beta) v for beta = x, y, z (first step of Algorithm 2).
template <typename T>
hipError_t trial_gradient(const WqOp& op, const OpTables<T>& tb, const T* v, Staged<T>& st, hipStream_t s) {
    const int n1 = op.n[0], n2 = op.n[1], n3 = op.n[2];
    const int nq2 = op.nq[1], nq3 = op.nq[2];
    const Dir1D<T>&dx = tb.dir[0], &dy = tb.dir[1], &dz = tb.dir[2];
    T* Tz0 = st.Z[0];   // [nq3][n2][n1]  B3 v
    T* Tz1 = st.Z[1];   // [nq3][n2][n1]  B-dot3 v
    WQ_TRY(band<T>(2, dz.B[0], v, nullptr, Tz0, n1, n2, n3, false, s));
    WQ_TRY(band<T>(2, dz.B[1], v, nullptr, Tz1, n1, n2, n3, false, s));
    // beta = x: B3 B2 Bdot1
    WQ_TRY(band<T>(1, dy.B[0], Tz0, nullptr, st.A, n1, n2, nq3, false, s));
    WQ_TRY(band<T>(0, dx.B[1], st.A, nullptr, st.g[0], n1, nq2, nq3, false, s));
    // beta = y: B3 Bdot2 B1
    WQ_TRY(band<T>(1, dy.B[1], Tz0, nullptr, st.Bq, n1, n2, nq3, false, s));
    WQ_TRY(band<T>(0, dx.B[0], st.Bq, nullptr, st.g[1], n1, nq2, nq3, false, s));
    // beta = z: Bdot3 B2 B1
    WQ_TRY(band<T>(1, dy.B[0], Tz1, nullptr, st.A, n1, n2, nq3, false, s));
    WQ_TRY(band<T>(0, dx.B[0], st.A, nullptr, st.g[2], n1, nq2, nq3, false, s));
    return hipSuccess;
}

template <typename T>
hipError_t apply_staged(const WqOp& op, const OpTables<T>& tb, const T* C, const T* Cm, const T* v, T* w,
                        hipStream_t s) {
    Staged<T> st(op, op.scratch);
    const int n1 = op.n[0], n2 = op.n[1];
    const int nq1 = op.nq[0], nq2 = op.nq[1], nq3 = op.nq[2];
    WQ_TRY(trial_gradient(op, tb, v, st, s));
    // reaction term: values at the points, X = B3 B2 B1 v, from B3 v (in Z[0])
    // before the test passes reuse Z[0]
    if (Cm) {
        WQ_TRY(band<T>(1, tb.dir[1].B[0], st.Z[0], nullptr, st.A, n1, op.n[1], nq3, false, s));
        WQ_TRY(band<T>(0, tb.dir[0].B[0], st.A, nullptr, st.X, n1, nq2, nq3, false, s));
    }
    bool zset[4] = {false, false, false, false};
    for (int be = 0; be < 3; ++be)
        for (int al = 0; al < 3; ++al) {
            int var[3];
            for (int l = 0; l < 3; ++l) var[l] = 2 * (l == al) + (l == be);
            const T* Cp = C + (size_t)plane_of(al, be) * op.Nq;
            // x: W1 (C .* v~)  -> [nq3][nq2][n1]
            WQ_TRY(band<T, kMulIn>(0, tb.dir[0].W[var[0]], st.g[be], Cp, st.A, nq1, nq2, nq3, false, s));
            // y: W2           -> [nq3][n2][n1], grouped by the z weight variant
            const int grp = var[2];
            WQ_TRY(band<T>(1, tb.dir[1].W[var[1]], st.A, nullptr, st.Z[grp], n1, nq2, nq3, zset[grp], s));
            zset[grp] = true;
        }
    if (Cm) {   // W1^{00} (c .* X), then W2^{00} into the W3^{00} group
        WQ_TRY(band<T, kMulIn>(0, tb.dir[0].W[0], st.X, Cm, st.A, nq1, nq2, nq3, false, s));
        WQ_TRY(band<T>(1, tb.dir[1].W[0], st.A, nullptr, st.Z[0], n1, nq2, nq3, zset[0], s));
    }
    for (int grp = 0; grp < 4; ++grp)
        WQ_TRY(band<T>(2, tb.dir[2].W[grp], st.Z[grp], nullptr, w, n1, n2, nq3, grp > 0, s));
    return hipSuccess;
}

template <typename T>
hipError_t apply_T_staged(const WqOp& op, const OpTables<T>& tb, const T* C, const T* Cm, const T* v, T* w,
                          hipStream_t s) {
    Staged<T> st(op, op.scratch);
    const int n1 = op.n[0], n2 = op.n[1], n3 = op.n[2];
    const int nq1 = op.nq[0], nq2 = op.nq[1], nq3 = op.nq[2];
    const Dir1D<T>&dx = tb.dir[0], &dy = tb.dir[1], &dz = tb.dir[2];
    // z: W3^T v for the four variants -> [nq3][n2][n1]
    for (int grp = 0; grp < 4; ++grp) WQ_TRY(band<T>(2, dz.WT[grp], v, nullptr, st.Z[grp], n1, n2, n3, false, s));
    // reaction term first: w = B^T (c .* W^(00)T v)
    if (Cm) {
        WQ_TRY(band<T>(1, dy.WT[0], st.Z[0], nullptr, st.A, n1, n2, nq3, false, s));
        WQ_TRY(band<T, kMulOut>(0, dx.WT[0], st.A, Cm, st.X, n1, nq2, nq3, false, s));
        WQ_TRY(band<T>(0, dx.BT[0], st.X, nullptr, st.A, nq1, nq2, nq3, false, s));
        WQ_TRY(band<T>(1, dy.BT[0], st.A, nullptr, st.Bq, n1, nq2, nq3, false, s));
        WQ_TRY(band<T>(2, dz.BT[0], st.Bq, nullptr, w, n1, n2, nq3, false, s));
    }
    // psi_beta = sum_alpha C_ab (W^(ab)^T v)
    for (int be = 0; be < 3; ++be)
        for (int al = 0; al < 3; ++al) {
            int var[3];
            for (int l = 0; l < 3; ++l) var[l] = 2 * (l == al) + (l == be);
            const T* Cp = C + (size_t)plane_of(al, be) * op.Nq;
            WQ_TRY(band<T>(1, dy.WT[var[1]], st.Z[var[2]], nullptr, st.A, n1, n2, nq3, false, s));
            WQ_TRY(band<T, kMulOut>(0, dx.WT[var[0]], st.A, Cp, st.g[be], n1, nq2, nq3, al > 0, s));
        }
    // w = sum_beta B^(beta)^T psi_beta
    for (int be = 0; be < 3; ++be) {
        const int d1 = be == 0, d2 = be == 1, d3 = be == 2;
        WQ_TRY(band<T>(0, dx.BT[d1], st.g[be], nullptr, st.A, nq1, nq2, nq3, false, s));     // [nq3][nq2][n1]
        WQ_TRY(band<T>(1, dy.BT[d2], st.A, nullptr, st.X, n1, nq2, nq3, false, s));          // [nq3][n2][n1]
        WQ_TRY(band<T>(2, dz.BT[d3], st.X, nullptr, w, n1, n2, nq3, be > 0 || Cm, s));        // [n3][n2][n1]
    }
    return hipSuccess;
}

// C = det J J^{-1} K J^{-T} per quadrature point (eq. C); writes FP64 planes
// and, when c32 != nullptr, an FP32 copy.
__global__ __launch_bounds__(kThreads) void set_coef_kernel(const double* __restrict__ detJ,
                                                            const double* __restrict__ Jinv, int k_kind,
                                                            const double* __restrict__ Kq,
                                                            double* __restrict__ c64, float* __restrict__ c32,
                                                            size_t Nq) {
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < Nq; q += (size_t)gridDim.x * blockDim.x) {
        double Ji[3][3], K[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Ji[r][c] = Jinv[(size_t)(3 * r + c) * Nq + q];
        if (k_kind == 0) {
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) K[r][c] = r == c ? 1.0 : 0.0;
        } else if (k_kind == 1) {
            const double k = Kq[q];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) K[r][c] = r == c ? k : 0.0;
        } else {
            K[0][0] = Kq[q];
            K[1][1] = Kq[Nq + q];
            K[2][2] = Kq[2 * Nq + q];
            K[0][1] = K[1][0] = Kq[3 * Nq + q];
            K[0][2] = K[2][0] = Kq[4 * Nq + q];
            K[1][2] = K[2][1] = Kq[5 * Nq + q];
        }
        // M = Ji K ; C = det M Ji^T
        double M[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[r][c] = Ji[r][0] * K[0][c] + Ji[r][1] * K[1][c] + Ji[r][2] * K[2][c];
        const double d = detJ[q];
        const int pr[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
        for (int k = 0; k < 6; ++k) {
            const int a = pr[k][0], b = pr[k][1];
            const double v = d * (M[a][0] * Ji[b][0] + M[a][1] * Ji[b][1] + M[a][2] * Ji[b][2]);
            c64[(size_t)k * Nq + q] = v;
            if (c32) c32[(size_t)k * Nq + q] = (float)v;
        }
    }
}

// Gradient of J with respect to C_ab at each point, chained to K:
//   gC_ab = -(W^(ab)^T lam)_q (B^(b) u)_q ;  scalar: sum_ab gC_ab G_ab, G = det Ji Ji^T;
//   sym6: H = det Ji^T gC Ji, diagonal H_aa, off-diagonal H_ab + H_ba;
//   identity kind: the six stored C planes (g_ab + g_ba off the diagonal).
// dJ/dC (the 3 x 3 g at point q) chained through eq. C to the layout of K_q.
__device__ inline void grad_chain(const double (&g)[3][3], const double* __restrict__ detJ,
                                  const double* __restrict__ Jinv, int k_kind, double* __restrict__ out, size_t Nq,
                                  size_t q) {
    if (k_kind == 0) {
        out[q] = g[0][0];
        out[Nq + q] = g[1][1];
        out[2 * Nq + q] = g[2][2];
        out[3 * Nq + q] = g[0][1] + g[1][0];
        out[4 * Nq + q] = g[0][2] + g[2][0];
        out[5 * Nq + q] = g[1][2] + g[2][1];
        return;
    }
    double Ji[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Ji[r][c] = Jinv[(size_t)(3 * r + c) * Nq + q];
    const double d = detJ[q];
    if (k_kind == 1) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double G = Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2];
                acc += g[a][b] * G;
            }
        out[q] = d * acc;
    } else {
        double T[3][3], H[3][3];   // T = g Ji ; H = Ji^T T
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) T[a][c] = g[a][0] * Ji[0][c] + g[a][1] * Ji[1][c] + g[a][2] * Ji[2][c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) H[r][c] = d * (Ji[0][r] * T[0][c] + Ji[1][r] * T[1][c] + Ji[2][r] * T[2][c]);
        out[q] = H[0][0];
        out[Nq + q] = H[1][1];
        out[2 * Nq + q] = H[2][2];
        out[3 * Nq + q] = H[0][1] + H[1][0];
        out[4 * Nq + q] = H[0][2] + H[2][0];
        out[5 * Nq + q] = H[1][2] + H[2][1];
    }
}

__global__ __launch_bounds__(kThreads) void grad_K_kernel(const double* __restrict__ wtl,  // [9][Nq] (al*3+be)
                                                          const double* __restrict__ gu,   // [3][Nq]
                                                          const double* __restrict__ detJ,
                                                          const double* __restrict__ Jinv, int k_kind,
                                                          double* __restrict__ out, size_t Nq) {
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < Nq; q += (size_t)gridDim.x * blockDim.x) {
        double g[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) g[a][b] = -wtl[(size_t)(3 * a + b) * Nq + q] * gu[(size_t)b * Nq + q];
        grad_chain(g, detJ, Jinv, k_kind, out, Nq, q);
    }
}

// Fused gradient expansion (p <= 7, operators with the fused tables).  One
// workgroup per 16 x 16 tile of quadrature columns and a range of quadrature
// planes; each of its four waves takes whole planes on its own (no barrier after
// the factor blocks are in LDS).  Per plane a wave
//   * contracts z in registers: the rows of the tile's test window of
//     W3^(v)T lam (v = 0..3, from the p + 2 planes of lam the plane's weights
//     touch) and of the trial window of B3 u and B-dot3 u;
//   * forms, as products of 16 x 16 blocks on the matrix cores, the y products
//     transposed (C'[i1][q2]) and then the x products (out[q2][q1]): the y
//     result, as it sits in the accumulator registers, is exactly the A operand
//     of the x product, so nothing goes through LDS;
//   * takes the nine values (W^(ab)T lam)_q, the three (B^(b) u)_q and, when
//     dJ/df is wanted, (W^(00)T lam)_q at the lane's four points and writes
//     g_ab = -(W^(ab)T lam)_q (B^(b) u)_q, summed over symmetric pairs and
//     chained to the layout of K_q, and det J (W^(00)T lam)_q.
// No N_q-sized or z-contracted intermediate is written.
typedef double gd4 __attribute__((ext_vector_type(4)));

struct GradFusedArgs {
    const double* tilesX = nullptr;
    const double* tilesY = nullptr;
    const int* JX = nullptr;
    const int* IX = nullptr;
    const int* JY = nullptr;
    const int* IY = nullptr;
    const int* bs3 = nullptr;
    const int* wts3 = nullptr;
    const double* cz = nullptr;     // [nq3][2(p+1) + 4(p+2)]: B3, B-dot3 rows, W3^(v) columns
    const double* lam = nullptr;
    const double* u = nullptr;
    const double* detJ = nullptr;
    const double* Jinv = nullptr;
    double* gK = nullptr;           // dJ/dK (nullptr: not wanted)
    double* gf = nullptr;           // dJ/df (nullptr: not wanted)
    int k_kind = 0;
    int n1 = 0, n2 = 0, n3 = 0, nq1 = 0, nq2 = 0, nq3 = 0, ntx = 0, nty = 0, zchunk = 0;
    size_t Nq = 0;
};

// 16 x 16 x 16 product on the matrix cores: A per lane as a[s] = A[cl][4s + kb]
// (FP64 operand layout: lane l holds row l % 16 of k-block l / 16), B from LDS
// stored [k][n] (lane reads T[4s + kb][cl]); result c[v] = C[kb + 4v][cl].
__device__ inline gd4 mm16(const double (&a)[4], const double* __restrict__ T, int cl, int kb) {
    gd4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], T[(4 * s + kb) * 16 + cl], c, 0, 0, 0);
    return c;
}

// y then x product of one field: D given as the lane's A operand of the y
// product (D[i2 = 4s + kb][i1 = cl]); Ty [i2][q2] and Tx [i1][q1] in LDS.
__device__ inline gd4 yx16(const double (&d)[4], const double* Ty, const double* Tx, int cl, int kb) {
    // one scheduling region per product: measured faster than letting the
    // compiler interleave products (102 vs 122 us on ring 64^3, p = 3)
    asm volatile("" ::: "memory");
    const gd4 y = mm16(d, Ty, cl, kb);                 // y[v] = C'[i1 = kb + 4v][q2 = cl]
    const double ya[4] = {y[0], y[1], y[2], y[3]};     // = A[q2 = cl][i1 = 4s + kb] of the x product
    return mm16(ya, Tx, cl, kb);                       // out[q2 = kb + 4v][q1 = cl]
}

// KK: coefficient kind of the output (0: the six C planes, else chained through
// eq. C).  Memory goes through raw buffer accesses (buffer.h): array bases and
// plane offsets in scalar registers, the lane's 32-bit byte offset in a vector
// register (the launcher checks that N and N_q stay below 2^32 bytes per plane
// set).
template <int P, int KK>
__global__ __launch_bounds__(256) void grad_fused_kernel(GradFusedArgs a) {
    constexpr int RT = P + 1, RO = P + 2, CZ = 2 * RT + 4 * RO;
    // factor blocks as [k][n]: 0-3 W2^(v) [i2][q2]; 4, 5 B2_d [j2][q2]; 6-9 W1^(v) [i1][q1];
    // 10, 11 B1_d [j1][q1] (v = 2 [test derivative] + [trial derivative], d = trial derivative)
    __shared__ double sT[12][256];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cl = lane & 15, kb = lane >> 4;
    const int lin = blockIdx.x;
    const int t1 = lin % a.ntx, t2 = (lin / a.ntx) % a.nty, zc = lin / (a.ntx * a.nty);
    const int k0 = zc * a.zchunk, k1 = min(a.nq3, k0 + a.zchunk);
    if (k0 >= k1) return;                              // uniform over the workgroup
    for (int e = tid; e < 12 * 256; e += 256) {
        const int b = e >> 8, r = (e >> 4) & 15, c = e & 15;
        double val;
        if (b < 4)
            val = a.tilesY[((size_t)t2 * 6 + 2 + b) * 256 + r * 16 + c];           // W_v[i = r][q = c]
        else if (b < 6)
            val = a.tilesY[((size_t)t2 * 6 + (b - 4)) * 256 + c * 16 + r];         // B_d[q = c][j = r]
        else if (b < 10)
            val = a.tilesX[((size_t)t1 * 6 + 2 + (b - 6)) * 256 + r * 16 + c];
        else
            val = a.tilesX[((size_t)t1 * 6 + (b - 10)) * 256 + c * 16 + r];
        sT[b][r * 16 + c] = val;
    }
    __syncthreads();
    // the lane's rows 4s + kb and column cl of the test (I) and trial (J) DOF
    // windows (byte offsets in a plane), clamped into the arrays: the factor
    // blocks are zero beyond n
    const int I1 = a.IX[t1], J1 = a.JX[t1], I2 = a.IY[t2], J2 = a.JY[t2];
    const int i1 = min(I1 + cl, a.n1 - 1), j1 = min(J1 + cl, a.n1 - 1);
    unsigned offL[4], offU[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        offL[s] = 8u * (unsigned)(min(I2 + 4 * s + kb, a.n2 - 1) * a.n1 + i1);
        offU[s] = 8u * (unsigned)(min(J2 + 4 * s + kb, a.n2 - 1) * a.n1 + j1);
    }
    const unsigned plb = 8u * (unsigned)(a.n2 * a.n1);                 // bytes of a DOF plane
    const unsigned pqb = 8u * (unsigned)(a.nq2 * a.nq1);               // bytes of a quadrature plane
    const __amdgpu_buffer_rsrc_t rl = buf_rsrc(a.lam), ru = buf_rsrc(a.u), rd = buf_rsrc(a.detJ);
    const int q1 = 16 * t1 + cl;
    const bool wantK = a.gK != nullptr, wantF = a.gf != nullptr;
    for (int k = k0 + wave; k < k1; k += 4) {
        // keeps the factor operands in LDS (read per product) instead of 96
        // registers held across the loop
        asm volatile("" ::: "memory");
        const double* __restrict__ c = a.cz + (size_t)k * CZ;
        const unsigned kq = (unsigned)k * pqb;
        // the test window's values of lam are loaded first, so that their latency
        // overlaps the trial side's loads and products
        double xl[RO][4];
        const int wb = a.wts3[k];
#pragma unroll
        for (int r = 0; r < RO; ++r) {
            const unsigned so = (unsigned)min(wb + r, a.n3 - 1) * plb;
#pragma unroll
            for (int s = 0; s < 4; ++s) xl[r][s] = buf_load<double>(rl, offL[s], so);
        }
        // trial side: B3 u, B-dot3 u in z, then (B^(b) u) at the lane's points
        gd4 Bu[3];
        if (wantK) {
            double Du[2][4];
#pragma unroll
            for (int s = 0; s < 4; ++s) Du[0][s] = Du[1][s] = 0.0;
            const int bb = a.bs3[k];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const unsigned so = (unsigned)min(bb + r, a.n3 - 1) * plb;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double x = buf_load<double>(ru, offU[s], so);
                    Du[0][s] += c[r] * x;
                    Du[1][s] += c[RT + r] * x;
                }
            }
#pragma unroll
            for (int be = 0; be < 3; ++be) Bu[be] = yx16(Du[be == 2], sT[4 + (be == 1)], sT[10 + (be == 0)], cl, kb);
        }
        // test side: W3^(v)T lam in z (out-of-range planes have zero coefficients, clamped loads)
        double Dl[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) Dl[0][s] = Dl[1][s] = Dl[2][s] = Dl[3][s] = 0.0;
#pragma unroll
        for (int r = 0; r < RO; ++r) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double x = xl[r][s];
                if (wantK) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) Dl[v][s] += c[2 * RT + v * RO + r] * x;
                } else {
                    Dl[0][s] += c[2 * RT + r] * x;
                }
            }
        }
        if (wantF) {
            const gd4 f = yx16(Dl[0], sT[0], sT[6], cl, kb);
            const __amdgpu_buffer_rsrc_t rf = buf_rsrc(a.gf);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q2 = 16 * t2 + kb + 4 * v;
                if (q1 < a.nq1 && q2 < a.nq2) {
                    const unsigned o = 8u * (unsigned)(q2 * a.nq1 + q1);
                    buf_store<double>(buf_load<double>(rd, o, kq) * f[v], rf, o, kq);
                }
            }
        }
        if (!wantK) continue;
        // symmetric accumulation acc[c][v], c in (11, 22, 33, 12, 13, 23): g_ab + g_ba off the diagonal
        double acc[6][4];
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
            for (int be = 0; be < 3; ++be) {
                const int v1 = 2 * (al == 0) + (be == 0), v2 = 2 * (al == 1) + (be == 1),
                          v3 = 2 * (al == 2) + (be == 2);
                const int pc = plane_of(al, be);
                const bool first = al <= be;
                const gd4 w = yx16(Dl[v3], sT[v2], sT[6 + v1], cl, kb);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double g = -w[v] * Bu[be][v];
                    acc[pc][v] = first ? g : acc[pc][v] + g;
                }
            }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int q2 = 16 * t2 + kb + 4 * v;
            if (!(q1 < a.nq1 && q2 < a.nq2)) continue;
            const unsigned o = 8u * (unsigned)(q2 * a.nq1 + q1);
            if (KK == 0) {
#pragma unroll
                for (int pc = 0; pc < 6; ++pc) buf_store<double>(acc[pc][v], buf_rsrc(a.gK + pc * a.Nq), o, kq);
                continue;
            }
            // chain: only the symmetric part M of g reaches dJ/dK (K and J^{-1} J^{-T} are symmetric)
            const double M[3][3] = {{acc[0][v], 0.5 * acc[3][v], 0.5 * acc[4][v]},
                                    {0.5 * acc[3][v], acc[1][v], 0.5 * acc[5][v]},
                                    {0.5 * acc[4][v], 0.5 * acc[5][v], acc[2][v]}};
            double Ji[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) Ji[r][cc] = buf_load<double>(buf_rsrc(a.Jinv + (3 * r + cc) * a.Nq), o, kq);
            const double d = buf_load<double>(rd, o, kq);
            if (KK == 1) {
                double sum = 0.0;
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = 0; be < 3; ++be)
                        sum += M[al][be] * (Ji[al][0] * Ji[be][0] + Ji[al][1] * Ji[be][1] + Ji[al][2] * Ji[be][2]);
                buf_store<double>(d * sum, buf_rsrc(a.gK), o, kq);
            } else {
                double T[3][3];   // T = M J^{-1}; H = det J J^{-T} T, H_rr and 2 H_rc stored
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        T[al][cc] = M[al][0] * Ji[0][cc] + M[al][1] * Ji[1][cc] + M[al][2] * Ji[2][cc];
                constexpr int R[6] = {0, 1, 2, 0, 0, 1}, Cc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
                for (int pc = 0; pc < 6; ++pc) {
                    const int r = R[pc], cc = Cc[pc];
                    const double h = d * (Ji[0][r] * T[0][cc] + Ji[1][r] * T[1][cc] + Ji[2][r] * T[2][cc]);
                    buf_store<double>(pc < 3 ? h : 2.0 * h, buf_rsrc(a.gK + pc * a.Nq), o, kq);
                }
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void mul_kernel(const double* __restrict__ a, double* __restrict__ b,
                                                       size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] *= a[i];
}

// Reaction plane c_q = alpha_q det J_q (FP64, and an FP32 copy when prepared).
__global__ __launch_bounds__(kThreads) void set_alpha_kernel(const double* __restrict__ alpha,
                                                             const double* __restrict__ detJ,
                                                             double* __restrict__ c64, float* __restrict__ c32,
                                                             size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double c = alpha[i] * detJ[i];
        c64[i] = c;
        if (c32) c32[i] = (float)c;
    }
}

// g = -g .* b
__global__ __launch_bounds__(kThreads) void neg_mul_kernel(const double* __restrict__ b, double* __restrict__ g,
                                                           size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        g[i] = -(g[i] * b[i]);
}

// w = M~ v = W^(00) (c .* B v), Algorithm 1: values at the points by z, y, x
// passes, the diagonal folded into the first test pass, then the W^(00) rules.
template <typename T>
hipError_t apply_mass_staged(const WqOp& op, const OpTables<T>& tb, const T* Cm, const T* v, T* w, hipStream_t s) {
    Staged<T> st(op, op.scratch);
    const int n1 = op.n[0], n2 = op.n[1], n3 = op.n[2];
    const int nq1 = op.nq[0], nq2 = op.nq[1], nq3 = op.nq[2];
    const Dir1D<T>&dx = tb.dir[0], &dy = tb.dir[1], &dz = tb.dir[2];
    WQ_TRY(band<T>(2, dz.B[0], v, nullptr, st.Z[0], n1, n2, n3, false, s));
    WQ_TRY(band<T>(1, dy.B[0], st.Z[0], nullptr, st.A, n1, n2, nq3, false, s));
    WQ_TRY(band<T>(0, dx.B[0], st.A, nullptr, st.X, n1, nq2, nq3, false, s));
    WQ_TRY(band<T, kMulIn>(0, dx.W[0], st.X, Cm, st.A, nq1, nq2, nq3, false, s));
    WQ_TRY(band<T>(1, dy.W[0], st.A, nullptr, st.Z[0], n1, nq2, nq3, false, s));
    WQ_TRY(band<T>(2, dz.W[0], st.Z[0], nullptr, w, n1, n2, nq3, false, s));
    return hipSuccess;
}

}  // namespace

size_t wq_scratch_bytes(const WqOp& op, int prec_mask) {
    // staged apply in the widest precision; the staged gradient (operators
    // without the fused tables) also needs its fields (12 N_q FP64), the fused
    // gradient (below 2^32 bytes per plane set) no scratch at all
    size_t e = Staged<double>::elems(op);
    size_t grad = 12 * op.Nq + 2 * (size_t)op.nq[2] * op.nq[1] * op.n[0] + 4 * (size_t)op.nq[2] * op.n[1] * op.n[0];
    const bool fused_grad = op.fused && op.N * 8 <= 0xffffffffull && op.Nq * 8 <= 0xffffffffull;
    if (!fused_grad && grad > e) e = grad;
    (void)prec_mask;
    return e * sizeof(double);
}

hipError_t launch_set_coef(const WqOp& op, int k_kind, const double* K_q, hipStream_t s) {
    hipLaunchKernelGGL(set_coef_kernel, dim3(grid_for(op.Nq)), dim3(kThreads), 0, s, op.detJ, op.Jinv, k_kind, K_q,
                       op.C64, (op.prec_mask & 2) ? op.C32 : nullptr, op.Nq);
    return hipGetLastError();
}

hipError_t launch_apply(const WqOp& op, int prec, const void* v, void* w, bool transpose, hipStream_t s,
                        bool w_zeroed) {
    if (op.fused) {
        if (prec == 1) {
            FusedArgs<double> a = op.fz64;
            a.v = static_cast<const double*>(v);
            a.w = static_cast<double*>(w);
            a.Cm = op.mass ? op.Cm64 : nullptr;
            a.w_zeroed = w_zeroed;
            return transpose ? launch_fused_apply_T<double>(a, op.p, s) : launch_fused_apply<double>(a, op.p, s);
        }
        FusedArgs<float> a = op.fz32;
        a.v = static_cast<const float*>(v);
        a.w = static_cast<float*>(w);
        a.Cm = op.mass ? op.Cm32 : nullptr;
        a.w_zeroed = w_zeroed;
        return transpose ? launch_fused_apply_T<float>(a, op.p, s) : launch_fused_apply<float>(a, op.p, s);
    }
    if (prec == 1) {
        const double* vv = static_cast<const double*>(v);
        double* ww = static_cast<double*>(w);
        const double* cm = op.mass ? op.Cm64 : nullptr;
        return transpose ? apply_T_staged<double>(op, op.t64, op.C64, cm, vv, ww, s)
                         : apply_staged<double>(op, op.t64, op.C64, cm, vv, ww, s);
    }
    const float* vv = static_cast<const float*>(v);
    float* ww = static_cast<float*>(w);
    const float* cm = op.mass ? op.Cm32 : nullptr;
    return transpose ? apply_T_staged<float>(op, op.t32, op.C32, cm, vv, ww, s)
                     : apply_staged<float>(op, op.t32, op.C32, cm, vv, ww, s);
}

hipError_t launch_set_alpha(const WqOp& op, const double* alpha_q, hipStream_t s) {
    hipLaunchKernelGGL(set_alpha_kernel, dim3(grid_for(op.Nq)), dim3(kThreads), 0, s, alpha_q, op.detJ, op.Cm64,
                       (op.prec_mask & 2) ? op.Cm32 : nullptr, op.Nq);
    return hipGetLastError();
}

hipError_t launch_apply_mass(const WqOp& op, int prec, const void* v, void* w, hipStream_t s) {
    if (prec == 1)
        return apply_mass_staged<double>(op, op.t64, op.Cm64, static_cast<const double*>(v), static_cast<double*>(w),
                                         s);
    return apply_mass_staged<float>(op, op.t32, op.Cm32, static_cast<const float*>(v), static_cast<float*>(w), s);
}

// the fused gradient addresses a DOF vector and every quadrature plane set with
// 32-bit byte offsets
static bool grad_fused_ok(const WqOp& op) {
    return op.fused && op.N * 8 <= 0xffffffffull && op.Nq * 8 <= 0xffffffffull;
}

static hipError_t launch_grad_fused(const WqOp& op, const double* lam, const double* u, double* gK, double* gf,
                                    hipStream_t s) {
    if (!grad_fused_ok(op)) return hipErrorInvalidValue;
    const FusedArgs<double>& f = op.fz64;
    GradFusedArgs g;
    g.tilesX = f.tilesX;
    g.tilesY = f.tilesY;
    g.JX = f.JX;
    g.IX = f.IX;
    g.JY = f.JY;
    g.IY = f.IY;
    g.bs3 = f.bs3;
    g.wts3 = f.wts3;
    g.cz = f.cz;
    g.lam = lam;
    g.u = u;
    g.detJ = op.detJ;
    g.Jinv = op.Jinv;
    g.gK = gK;
    g.gf = gf;
    g.k_kind = op.k_kind;
    g.n1 = op.n[0];
    g.n2 = op.n[1];
    g.n3 = op.n[2];
    g.nq1 = op.nq[0];
    g.nq2 = op.nq[1];
    g.nq3 = op.nq[2];
    g.ntx = f.ntx;
    g.nty = f.nty;
    g.Nq = op.Nq;
    // eight planes per workgroup (two per wave); 4, 12 and 16 measured no faster
    g.zchunk = 8;
    const int nz = (g.nq3 + g.zchunk - 1) / g.zchunk;
    const dim3 grid(g.ntx * g.nty * nz), block(256);
#define WQ_GRAD_LAUNCH(P)                                                                      \
    do {                                                                                       \
        if (g.k_kind == 0 || !gK)                                                              \
            hipLaunchKernelGGL((grad_fused_kernel<P, 0>), grid, block, 0, s, g);               \
        else if (g.k_kind == 1)                                                                \
            hipLaunchKernelGGL((grad_fused_kernel<P, 1>), grid, block, 0, s, g);               \
        else                                                                                   \
            hipLaunchKernelGGL((grad_fused_kernel<P, 6>), grid, block, 0, s, g);               \
    } while (0)
    switch (op.p) {
        case 2: WQ_GRAD_LAUNCH(2); break;
        case 3: WQ_GRAD_LAUNCH(3); break;
        case 4: WQ_GRAD_LAUNCH(4); break;
        case 5: WQ_GRAD_LAUNCH(5); break;
        case 6: WQ_GRAD_LAUNCH(6); break;
        case 7: WQ_GRAD_LAUNCH(7); break;
        default: return hipErrorInvalidValue;
    }
#undef WQ_GRAD_LAUNCH
    return hipGetLastError();
}

hipError_t launch_grad_Kf(const WqOp& op, const double* lam, const double* u, double* gK, double* gf,
                          hipStream_t s) {
    if (grad_fused_ok(op)) return launch_grad_fused(op, lam, u, gK, gf, s);
    WQ_TRY(launch_grad_K(op, lam, u, gK, s));
    return launch_grad_f(op, lam, gf, s);
}

hipError_t launch_grad_alpha(const WqOp& op, const double* lam, const double* u, double* g, hipStream_t s) {
    // g = det J W^(00)T lam (the chain of dJ/df), then g = -g .* (B u)
    WQ_TRY(launch_grad_f(op, lam, g, s));
    Staged<double> st(op, op.scratch);
    const int n1 = op.n[0], n2 = op.n[1], n3 = op.n[2];
    const int nq2 = op.nq[1], nq3 = op.nq[2];
    const OpTables<double>& tb = op.t64;
    WQ_TRY(band<double>(2, tb.dir[2].B[0], u, nullptr, st.Z[0], n1, n2, n3, false, s));
    WQ_TRY(band<double>(1, tb.dir[1].B[0], st.Z[0], nullptr, st.A, n1, n2, nq3, false, s));
    WQ_TRY(band<double>(0, tb.dir[0].B[0], st.A, nullptr, st.X, n1, nq2, nq3, false, s));
    hipLaunchKernelGGL(neg_mul_kernel, dim3(grid_for(op.Nq)), dim3(kThreads), 0, s, st.X, g, op.Nq);
    return hipGetLastError();
}

hipError_t launch_rhs(const WqOp& op, const double* f_q, double* b, hipStream_t s) {
    Staged<double> st(op, op.scratch);
    const int n1 = op.n[0], n2 = op.n[1];
    const int nq1 = op.nq[0], nq2 = op.nq[1], nq3 = op.nq[2];
    const OpTables<double>& tb = op.t64;
    WQ_TRY(band<double, kMulIn>(0, tb.dir[0].W[0], f_q, op.detJ, st.A, nq1, nq2, nq3, false, s));
    WQ_TRY(band<double>(1, tb.dir[1].W[0], st.A, nullptr, st.Z[0], n1, nq2, nq3, false, s));
    WQ_TRY(band<double>(2, tb.dir[2].W[0], st.Z[0], nullptr, b, n1, n2, nq3, false, s));
    return hipSuccess;
}

hipError_t launch_grad_f(const WqOp& op, const double* lam, double* gf, hipStream_t s) {
    if (grad_fused_ok(op)) return launch_grad_fused(op, lam, nullptr, nullptr, gf, s);
    Staged<double> st(op, op.scratch);
    const int n1 = op.n[0], n2 = op.n[1], n3 = op.n[2];
    const int nq1 = op.nq[0], nq2 = op.nq[1], nq3 = op.nq[2];
    const OpTables<double>& tb = op.t64;
    WQ_TRY(band<double>(2, tb.dir[2].WT[0], lam, nullptr, st.Z[0], n1, n2, n3, false, s));
    WQ_TRY(band<double>(1, tb.dir[1].WT[0], st.Z[0], nullptr, st.A, n1, n2, nq3, false, s));
    WQ_TRY(band<double, kMulOut>(0, tb.dir[0].WT[0], st.A, op.detJ, gf, n1, nq2, nq3, false, s));
    (void)nq1;
    return hipSuccess;
}

hipError_t launch_grad_K(const WqOp& op, const double* lam, const double* u, double* gK, hipStream_t s) {
    if (grad_fused_ok(op)) return launch_grad_fused(op, lam, u, gK, nullptr, s);
    // fields: wtl [9][Nq] = W^(ab)^T lam, gu [3][Nq] = B^(b) u
    double* base = reinterpret_cast<double*>(op.scratch);
    double* wtl = base;
    double* gu = base + 9 * op.Nq;
    double* tmpA = base + 12 * op.Nq;                                        // nq3 nq2 n1
    double* tmpZ = tmpA + 2 * (size_t)op.nq[2] * op.nq[1] * op.n[0];         // 4 x nq3 n2 n1
    const int n1 = op.n[0], n2 = op.n[1], n3 = op.n[2];
    const int nq2 = op.nq[1], nq3 = op.nq[2];
    const size_t zsz = (size_t)op.nq[2] * op.n[1] * op.n[0];
    const OpTables<double>& tb = op.t64;
    const Dir1D<double>&dx = tb.dir[0], &dy = tb.dir[1], &dz = tb.dir[2];
    // B^(b) u  (same chain as the trial step of the apply)
    double* Tz0 = tmpZ;
    double* Tz1 = tmpZ + zsz;
    WQ_TRY(band<double>(2, dz.B[0], u, nullptr, Tz0, n1, n2, n3, false, s));
    WQ_TRY(band<double>(2, dz.B[1], u, nullptr, Tz1, n1, n2, n3, false, s));
    WQ_TRY(band<double>(1, dy.B[0], Tz0, nullptr, tmpA, n1, n2, nq3, false, s));
    WQ_TRY(band<double>(0, dx.B[1], tmpA, nullptr, gu, n1, nq2, nq3, false, s));
    WQ_TRY(band<double>(1, dy.B[1], Tz0, nullptr, tmpA, n1, n2, nq3, false, s));
    WQ_TRY(band<double>(0, dx.B[0], tmpA, nullptr, gu + op.Nq, n1, nq2, nq3, false, s));
    WQ_TRY(band<double>(1, dy.B[0], Tz1, nullptr, tmpA, n1, n2, nq3, false, s));
    WQ_TRY(band<double>(0, dx.B[0], tmpA, nullptr, gu + 2 * op.Nq, n1, nq2, nq3, false, s));
    // W^(ab)^T lam for the nine pairs
    for (int grp = 0; grp < 4; ++grp)
        WQ_TRY(band<double>(2, dz.WT[grp], lam, nullptr, tmpZ + grp * zsz, n1, n2, n3, false, s));
    for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) {
            int var[3];
            for (int l = 0; l < 3; ++l) var[l] = 2 * (l == al) + (l == be);
            WQ_TRY(band<double>(1, dy.WT[var[1]], tmpZ + var[2] * zsz, nullptr, tmpA, n1, n2, nq3, false, s));
            WQ_TRY(band<double>(0, dx.WT[var[0]], tmpA, nullptr, wtl + (size_t)(3 * al + be) * op.Nq, n1, nq2, nq3,
                                false, s));
        }
    hipLaunchKernelGGL(grad_K_kernel, dim3(grid_for(op.Nq)), dim3(kThreads), 0, s, wtl, gu, op.detJ, op.Jinv,
                       op.k_kind, gK, op.Nq);
    return hipGetLastError();
}

}  // namespace wqfd
