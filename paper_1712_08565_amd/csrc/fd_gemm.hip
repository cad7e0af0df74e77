// Mode products of the Fast Diagonalization preconditioner on the matrix cores
// (gfx950).  One launch applies a small n x n matrix T along one axis of the
// [n3][n2][n1] array:
//     out[i][g] = sum_j T[i][j] in[j][g]
// over all "columns" g (the index pairs of the two other axes): column g sits
// at (g / cdiv) * sa + (g % cdiv) * sc and its element j at + j * sj.
//
// One wave computes a 16 x 16 output block (16 rows i, 16 columns g) over the
// whole contraction length; the workgroup holds the ceil(n / 16) waves of one
// column block, so the input slab is fetched from memory once and the other
// waves read it from the L1 cache.  Every operand of the block is loaded up
// front (no LDS, no barrier): at these sizes (n <= 144, a few MB per pass) the
// pass is bound by memory latency, and a grid of one small workgroup per 16
// columns keeps every CU busy.
//   FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32,
//   BF16: v_mfma_f32_16x16x32_bf16 (FP32 data rounded to bf16 as it is
//         loaded, T pre-converted and zero padded), FP32 accumulation.
// The eigenvalue scaling 1/(l1 + l2 + l3) of the preconditioner is an optional
// epilogue.
#include <hip/hip_runtime.h>

#include "device.h"
#include "fd_gemm.h"

namespace wqfd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int PREC>
struct G;
template <>
struct G<1> {                    // FP64
    using T = double;            // data
    using S = double;            // matrix operand
    using Acc = d4;
    __device__ static int drow(int kb, int v) { return kb + 4 * v; }
};
template <>
struct G<2> {                    // FP32
    using T = float;
    using S = float;
    using Acc = f4;
    __device__ static int drow(int kb, int v) { return 4 * kb + v; }
};
template <>
struct G<4> {                    // BF16 operands, FP32 data
    using T = float;
    using S = __bf16;
    using Acc = f4;
    __device__ static int drow(int kb, int v) { return 4 * kb + v; }
};

// KB = ceil(n / 16): row blocks per column block (= waves per workgroup) and
// 16-wide contraction chunks.
template <int PREC, int KB>
__global__ __launch_bounds__(64 * KB) void fd_mode_mfma(FdModeArgs<typename G<PREC>::T, typename G<PREC>::S> p) {
    using T = typename G<PREC>::T;
    using S = typename G<PREC>::S;
    using Acc = typename G<PREC>::Acc;
    const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
    const int cl = lane & 15, kb = lane >> 4;
    const int n = p.n;
    const int g = blockIdx.x * 16 + cl;                  // this lane's column
    const bool gin = g < p.C;
    const size_t base = gin ? (size_t)(g / p.cdiv) * p.sa + (size_t)(g % p.cdiv) * p.sc : 0;
    const int row = t * 16 + cl;                         // this lane's row of T (A operand)
    Acc acc = Acc{0, 0, 0, 0};
    if constexpr (PREC == 4) {
        // k-step s covers k = 32 s + 8 kb + e, e = 0..7; T is zero padded to a
        // multiple of 64 in both dimensions, so its loads need no guard
        constexpr int NKS = (KB + 1) / 2;
        bf8 a[NKS], b[NKS];
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int k0 = 32 * s + 8 * kb;
            a[s] = *reinterpret_cast<const bf8*>(p.mat + (size_t)row * p.ldT + k0);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + e;
                const float x = (gin && k < n) ? p.in[base + (size_t)k * p.sj] : 0.0f;
                b[s][e] = (__bf16)x;
            }
        }
#pragma unroll
        for (int s = 0; s < NKS; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], b[s], acc, 0, 0, 0);
    } else {
        constexpr int NKS = 4 * KB;                      // k-step s covers k = 4 s + kb
        S a[NKS];
        T b[NKS];
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int k = 4 * s + kb;
            a[s] = (row < n && k < n) ? p.mat[(size_t)row * p.ldT + k] : S(0);
            b[s] = (gin && k < n) ? p.in[base + (size_t)k * p.sj] : T(0);
        }
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            if constexpr (PREC == 1)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
            else
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
        }
    }
    if (!gin) return;
    double l12 = 0.0;
    if (p.l1) {                                          // single-batch pass: g = i2 * n1 + i1
        const int i2 = g / p.n1, i1 = g - i2 * p.n1;
        l12 = p.l1[i1] + p.l2[i2];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = t * 16 + G<PREC>::drow(kb, v);
        if (i < n) {
            T val = acc[v];
            if (p.l1) val = (T)((double)val / (l12 + p.l3[i]));
            p.out[base + (size_t)i * p.sj] = val;
        }
    }
}

template <int PREC, int KB>
hipError_t launch_kb(const FdModeArgs<typename G<PREC>::T, typename G<PREC>::S>& p, hipStream_t s) {
    const int blocks = (p.C + 15) / 16;
    hipLaunchKernelGGL((fd_mode_mfma<PREC, KB>), dim3(blocks), dim3(64 * KB), 0, s, p);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_any(const FdModeArgs<typename G<PREC>::T, typename G<PREC>::S>& p, hipStream_t s) {
    if (p.C <= 0 || p.n <= 0 || p.cdiv <= 0) return hipErrorInvalidValue;
    if (p.l1 && p.cdiv != p.C) return hipErrorInvalidValue;
    switch ((p.n + 15) / 16) {
        case 1: return launch_kb<PREC, 1>(p, s);
        case 2: return launch_kb<PREC, 2>(p, s);
        case 3: return launch_kb<PREC, 3>(p, s);
        case 4: return launch_kb<PREC, 4>(p, s);
        case 5: return launch_kb<PREC, 5>(p, s);
        case 6: return launch_kb<PREC, 6>(p, s);
        case 7: return launch_kb<PREC, 7>(p, s);
        case 8: return launch_kb<PREC, 8>(p, s);
        case 9: return launch_kb<PREC, 9>(p, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Fused passes of the whole preconditioner (FP64 and FP32, n <= 144), three
// launches per application instead of six:
//   xy pass, per z-plane i3 and 16-row block of i2 (the y product first, so the
//   data is read and written along contiguous x rows):
//     Q[i2][j1] = sum_j2 T2[i2][j2] in[i3][j2][j1]    (wave t: columns j1 of block t)
//     out[i3][i2][i1] = sum_j1 Q[i2][j1] T1[i1][j1]   (Q through LDS; wave t: i1 of block t)
//   z pass, per 16-column block of g = (i2, i1):
//     Y[i3][g] = sum_j3 T3f[i3][j3] in[j3][g] / (l1[i1] + l2[i2] + l3[i3])
//     out[i3][g] = sum_j3 T3b[i3][j3] Y[j3][g]       (Y through LDS; in may be out)
// The small matrices are passed transposed (Tt[j][i] = T[i][j]), so that the 16
// lanes of an operand column read 16 consecutive entries.
// One wave per 16-wide block (KB = ceil(n / 16) waves).  Every operand that
// does not depend on the first product, the second product's matrix included,
// is loaded before the first product (for KB <= PRELOAD_KB; larger blocks load
// the second matrix after it, to bound registers), and contraction steps past
// the true length are skipped.
constexpr int FLD = 17;                                  // padded row of 16-column LDS blocks
constexpr int PRELOAD_KB = 6;

template <int PREC>
__device__ inline typename G<PREC>::Acc mma_step(typename G<PREC>::T a, typename G<PREC>::T b,
                                                 typename G<PREC>::Acc c) {
    if constexpr (PREC == 1)
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int PREC, int KB>
__global__ __launch_bounds__(64 * KB) void fd_xy_pass(const typename G<PREC>::T* __restrict__ in,
                                                      typename G<PREC>::T* __restrict__ out,
                                                      const typename G<PREC>::T* __restrict__ T1t,
                                                      const typename G<PREC>::T* __restrict__ T2t, int n1, int n2) {
    using T = typename G<PREC>::T;
    using Acc = typename G<PREC>::Acc;
    constexpr int NKS = 4 * KB;
    constexpr int LDQ = 16 * KB + 1;                     // odd row length of the Q block
    constexpr bool PRE = KB <= PRELOAD_KB;
    __shared__ T sQ[16 * LDQ];
    const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
    const int cl = lane & 15, kb = lane >> 4;
    const int r0 = blockIdx.x * 16;                      // first i2 of this block
    const size_t pl = (size_t)blockIdx.y * n1 * n2;       // z-plane offset
    const int ks2 = (n2 + 3) >> 2, ks1 = (n1 + 3) >> 2;  // contraction steps of the two products
    const int i2a = r0 + cl, jc = 16 * t + cl;           // A row (i2) and B column (j1, then i1)
    T a[NKS], b[NKS], c[PRE ? NKS : 1];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int k = 4 * s + kb;
        a[s] = (i2a < n2 && k < n2) ? T2t[(size_t)k * n2 + i2a] : T(0);
        b[s] = (jc < n1 && k < n2) ? in[pl + (size_t)k * n1 + jc] : T(0);
        if constexpr (PRE) c[s] = (jc < n1 && k < n1) ? T1t[(size_t)k * n1 + jc] : T(0);
    }
    Acc q = Acc{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NKS; ++s)
        if (s < ks2) q = mma_step<PREC>(a[s], b[s], q);
#pragma unroll
    for (int v = 0; v < 4; ++v) sQ[G<PREC>::drow(kb, v) * LDQ + jc] = q[v];   // columns >= n1 hold zeros
    __syncthreads();
    Acc r = Acc{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int k = 4 * s + kb;
        a[s] = sQ[cl * LDQ + k];
        if constexpr (!PRE) b[s] = (jc < n1 && k < n1) ? T1t[(size_t)k * n1 + jc] : T(0);
    }
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        if constexpr (PRE) {
            if (s < ks1) r = mma_step<PREC>(a[s], c[s], r);
        } else {
            if (s < ks1) r = mma_step<PREC>(a[s], b[s], r);
        }
    }
    if (jc >= n1) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i2 = r0 + G<PREC>::drow(kb, v);
        if (i2 < n2) out[pl + (size_t)i2 * n1 + jc] = r[v];
    }
}

template <int PREC, int KB>
__global__ __launch_bounds__(64 * KB) void fd_z_pass(const typename G<PREC>::T* in, typename G<PREC>::T* out,
                                                     const typename G<PREC>::T* __restrict__ T3ft,
                                                     const typename G<PREC>::T* __restrict__ T3bt,
                                                     const double* __restrict__ l1, const double* __restrict__ l2,
                                                     const double* __restrict__ l3, int n1, int n2, int n3) {
    using T = typename G<PREC>::T;
    using Acc = typename G<PREC>::Acc;
    constexpr int NKS = 4 * KB;
    constexpr bool PRE = KB <= PRELOAD_KB;
    __shared__ T sY[16 * KB * FLD];
    const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
    const int cl = lane & 15, kb = lane >> 4;
    const int C = n1 * n2;
    const int g = blockIdx.x * 16 + cl;
    const bool gin = g < C;
    const int i3r = 16 * t + cl;                         // row of T3 (A operand)
    const int ks3 = (n3 + 3) >> 2;
    T a[NKS], b[NKS], c[PRE ? NKS : 1];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int k = 4 * s + kb;                        // j3
        a[s] = (i3r < n3 && k < n3) ? T3ft[(size_t)k * n3 + i3r] : T(0);
        b[s] = (gin && k < n3) ? in[(size_t)k * C + g] : T(0);
        if constexpr (PRE) c[s] = (i3r < n3 && k < n3) ? T3bt[(size_t)k * n3 + i3r] : T(0);
    }
    Acc y = Acc{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NKS; ++s)
        if (s < ks3) y = mma_step<PREC>(a[s], b[s], y);
    double l12 = 0.0;
    if (gin) {
        const int i2 = g / n1, i1 = g - i2 * n1;
        l12 = l1[i1] + l2[i2];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i3 = 16 * t + G<PREC>::drow(kb, v);
        sY[(16 * t + G<PREC>::drow(kb, v)) * FLD + cl] =
            (gin && i3 < n3) ? (T)((double)y[v] / (l12 + l3[i3])) : T(0);
    }
    __syncthreads();                                     // every read of `in` by this block is done
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int k = 4 * s + kb;
        if constexpr (!PRE) a[s] = (i3r < n3 && k < n3) ? T3bt[(size_t)k * n3 + i3r] : T(0);
        b[s] = sY[k * FLD + cl];
    }
    Acc z = Acc{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        if constexpr (PRE) {
            if (s < ks3) z = mma_step<PREC>(c[s], b[s], z);
        } else {
            if (s < ks3) z = mma_step<PREC>(a[s], b[s], z);
        }
    }
    if (!gin) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i3 = 16 * t + G<PREC>::drow(kb, v);
        if (i3 < n3) out[(size_t)i3 * C + g] = z[v];
    }
}

template <int PREC, int KB>
hipError_t fused_kb(const FdFusedArgs<typename G<PREC>::T>& f, hipStream_t s) {
    using T = typename G<PREC>::T;
    hipError_t e;
    // forward x and y
    dim3 gxy((f.n2 + 15) / 16, f.n3);
    // (T = U^T forward, U backward; each passed transposed)
    hipLaunchKernelGGL((fd_xy_pass<PREC, KB>), gxy, dim3(64 * KB), 0, s, f.r, f.tmp, f.U[0], f.U[1], f.n1, f.n2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // forward z, scaling, backward z (in place on tmp)
    dim3 gz((f.n1 * f.n2 + 15) / 16);
    hipLaunchKernelGGL((fd_z_pass<PREC, KB>), gz, dim3(64 * KB), 0, s, (const T*)f.tmp, f.tmp, f.U[2], f.UT[2],
                       f.l1, f.l2, f.l3, f.n1, f.n2, f.n3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // backward x and y
    hipLaunchKernelGGL((fd_xy_pass<PREC, KB>), gxy, dim3(64 * KB), 0, s, (const T*)f.tmp, f.z, f.UT[0], f.UT[1], f.n1,
                       f.n2);
    return hipGetLastError();
}

template <int PREC>
hipError_t fused_any(const FdFusedArgs<typename G<PREC>::T>& f, hipStream_t s) {
    const int nmax = f.n1 > f.n2 ? (f.n1 > f.n3 ? f.n1 : f.n3) : (f.n2 > f.n3 ? f.n2 : f.n3);
    switch ((nmax + 15) / 16) {
        case 1: return fused_kb<PREC, 1>(f, s);
        case 2: return fused_kb<PREC, 2>(f, s);
        case 3: return fused_kb<PREC, 3>(f, s);
        case 4: return fused_kb<PREC, 4>(f, s);
        case 5: return fused_kb<PREC, 5>(f, s);
        case 6: return fused_kb<PREC, 6>(f, s);
        case 7: return fused_kb<PREC, 7>(f, s);
        case 8: return fused_kb<PREC, 8>(f, s);
        case 9: return fused_kb<PREC, 9>(f, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fd_mode(const FdModeArgs<double, double>& p, hipStream_t s) { return launch_any<1>(p, s); }
hipError_t launch_fd_mode(const FdModeArgs<float, float>& p, hipStream_t s) { return launch_any<2>(p, s); }
hipError_t launch_fd_mode(const FdModeArgs<float, __bf16>& p, hipStream_t s) { return launch_any<4>(p, s); }
hipError_t launch_fd_fused(const FdFusedArgs<double>& f, hipStream_t s) { return fused_any<1>(f, s); }
hipError_t launch_fd_fused(const FdFusedArgs<float>& f, hipStream_t s) { return fused_any<2>(f, s); }

}  // namespace wqfd
