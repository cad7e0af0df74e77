// Fast Diagonalization preconditioner apply on gfx950 (Section 4, by citation
// of Lynch, Rice and Thomas):
//     z = (U3 x U2 x U1) diag(1 / (l1_i + l2_j + l3_k)) (U3 x U2 x U1)^T r,
// as six dense mode products with the n x n eigenvector matrices, run on the
// matrix cores:
//   FP64: v_mfma_f64_16x16x4f64   (double in/out, FP64 accumulate)
//   FP32: v_mfma_f32_16x16x4f32   (float in/out, FP32 accumulate)
//   BF16: v_mfma_f32_16x16x32_bf16 (float in/out, bf16 operands, FP32 accumulate)
// The diagonal scaling is fused into the epilogue of the third forward product.
//
// Mode products:
//   x (contiguous axis):   out[r][i]    = sum_j T[i][j] in[r][j],     r over n2 n3 rows
//   y, z (strided axis):   out[a][i][c] = sum_j T[i][j] in[a][j][c],  c contiguous
// with T = U^T (forward) or T = U (backward); U row-major, eigenvector k in column k.
//
// MFMA register layouts (16x16 output tile, 64 lanes, lane l):
//   A operand (16 x K):  row l % 16, k block l / 16
//   B operand (K x 16):  k block l / 16, column l % 16
//   D (16 x 16, 4 values v per lane), column l % 16 and row
//       FP32 / BF16:  4 (l / 16) + v
//       FP64:         (l / 16) + 4 v
//   (checked on gfx950 with known integer inputs).
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "device.h"
#include "fd_gemm.h"

namespace wqfd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;       // waves per workgroup
constexpr int kTilesI = 4;      // 16-row tiles of the output index i per wave

// ---------------------------------------------------------------- element traits
template <int PREC>
struct Tr;
template <>
struct Tr<1> {   // FP64
    using T = double;
    using Acc = d4;
    __device__ static Acc mfma(T a, T b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int drow(int kb, int v) { return kb + 4 * v; }
};
template <>
struct Tr<2> {   // FP32
    using T = float;
    using Acc = f4;
    __device__ static Acc mfma(T a, T b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int kb, int v) { return 4 * kb + v; }
};

__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }

// eigenvalue scaling 1 / (l1[i1] + l2[i2] + l3[i3]) for the third forward product
struct Scale {
    const double* l1 = nullptr;
    const double* l2 = nullptr;
    const double* l3 = nullptr;
    int n1 = 0, n2 = 0;
};

__device__ inline double scale_at(const Scale& sc, int i3, int c) {
    const int i2 = c / sc.n1, i1 = c - i2 * sc.n1;
    return 1.0 / (sc.l1[i1] + sc.l2[i2] + sc.l3[i3]);
}

// T[i][j] = trans ? U[j][i] : U[i][j]
template <typename T>
__device__ inline T tmat(const T* __restrict__ U, int n, int i, int j, int trans) {
    if (i >= n || j >= n) return T(0);
    return trans ? U[(size_t)j * n + i] : U[(size_t)i * n + j];
}

// ---------------------------------------------------------------- strided axis, FP64 / FP32
template <int PREC>
__global__ __launch_bounds__(64 * kWaves) void mode_strided_kernel(const typename Tr<PREC>::T* __restrict__ in,
                                                                   typename Tr<PREC>::T* __restrict__ out,
                                                                   const typename Tr<PREC>::T* __restrict__ U,
                                                                   int n, int C, int trans, Scale sc) {
    using T = typename Tr<PREC>::T;
    using Acc = typename Tr<PREC>::Acc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = (blockIdx.x * kWaves + wave) * 16;
    if (c0 >= C) return;
    const int ibase = blockIdx.y * (16 * kTilesI);
    const size_t a = blockIdx.z;
    const T* src = in + a * (size_t)n * C;
    T* dst = out + a * (size_t)n * C;
    const int col = c0 + (lane & 15);
    const int kb = lane >> 4;
    Acc acc[kTilesI];
    for (int t = 0; t < kTilesI; ++t) acc[t] = Acc{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 4) {
        const int j = k0 + kb;
        const T b = (j < n && col < C) ? src[(size_t)j * C + col] : T(0);
#pragma unroll
        for (int t = 0; t < kTilesI; ++t) {
            const T av = tmat<T>(U, n, ibase + t * 16 + (lane & 15), j, trans);
            acc[t] = Tr<PREC>::mfma(av, b, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < kTilesI; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ibase + t * 16 + Tr<PREC>::drow(kb, v);
            if (i < n && col < C) {
                T val = acc[t][v];
                if (sc.l1) val = (T)((double)val * scale_at(sc, i, col));
                dst[(size_t)i * C + col] = val;
            }
        }
}

// ---------------------------------------------------------------- contiguous axis (x), FP64 / FP32
template <int PREC>
__global__ __launch_bounds__(64 * kWaves) void mode_x_kernel(const typename Tr<PREC>::T* __restrict__ in,
                                                             typename Tr<PREC>::T* __restrict__ out,
                                                             const typename Tr<PREC>::T* __restrict__ U, int n,
                                                             int rows, int trans) {
    using T = typename Tr<PREC>::T;
    using Acc = typename Tr<PREC>::Acc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * kWaves + wave) * 16;
    if (r0 >= rows) return;
    const int ibase = blockIdx.y * (16 * kTilesI);
    const int kb = lane >> 4;
    const int row = r0 + (lane & 15);
    Acc acc[kTilesI];
    for (int t = 0; t < kTilesI; ++t) acc[t] = Acc{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 4) {
        const int j = k0 + kb;
        const T av = (j < n && row < rows) ? in[(size_t)row * n + j] : T(0);
#pragma unroll
        for (int t = 0; t < kTilesI; ++t) {
            const T bv = tmat<T>(U, n, ibase + t * 16 + (lane & 15), j, trans);
            acc[t] = Tr<PREC>::mfma(av, bv, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < kTilesI; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + Tr<PREC>::drow(kb, v);
            const int i = ibase + t * 16 + (lane & 15);
            if (r < rows && i < n) out[(size_t)r * n + i] = acc[t][v];
        }
}

// ---------------------------------------------------------------- BF16 operands, FP32 data
// Tb: bf16 copy of T (already transposed as needed), padded to npad x npad with zeros.
__global__ __launch_bounds__(64 * kWaves) void mode_strided_bf16_kernel(const float* __restrict__ in,
                                                                        float* __restrict__ out,
                                                                        const __bf16* __restrict__ Tb, int n,
                                                                        int npad, int C, Scale sc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = (blockIdx.x * kWaves + wave) * 16;
    if (c0 >= C) return;
    const int ibase = blockIdx.y * (16 * kTilesI);
    const size_t a = blockIdx.z;
    const float* src = in + a * (size_t)n * C;
    float* dst = out + a * (size_t)n * C;
    const int col = c0 + (lane & 15);
    const int kb = lane >> 4;
    f4 acc[kTilesI];
    for (int t = 0; t < kTilesI; ++t) acc[t] = f4{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 32) {
        bf8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = k0 + 8 * kb + e;
            b[e] = to_bf16((j < n && col < C) ? src[(size_t)j * C + col] : 0.0f);
        }
#pragma unroll
        for (int t = 0; t < kTilesI; ++t) {
            const int i = ibase + t * 16 + (lane & 15);
            bf8 av = *reinterpret_cast<const bf8*>(Tb + (size_t)i * npad + k0 + 8 * kb);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < kTilesI; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ibase + t * 16 + 4 * kb + v;
            if (i < n && col < C) {
                float val = acc[t][v];
                if (sc.l1) val = (float)((double)val * scale_at(sc, i, col));
                dst[(size_t)i * C + col] = val;
            }
        }
}

__global__ __launch_bounds__(64 * kWaves) void mode_x_bf16_kernel(const float* __restrict__ in,
                                                                  float* __restrict__ out,
                                                                  const __bf16* __restrict__ Tb, int n, int npad,
                                                                  int rows) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * kWaves + wave) * 16;
    if (r0 >= rows) return;
    const int ibase = blockIdx.y * (16 * kTilesI);
    const int kb = lane >> 4;
    const int row = r0 + (lane & 15);
    f4 acc[kTilesI];
    for (int t = 0; t < kTilesI; ++t) acc[t] = f4{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 32) {
        bf8 av;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = k0 + 8 * kb + e;
            av[e] = to_bf16((j < n && row < rows) ? in[(size_t)row * n + j] : 0.0f);
        }
#pragma unroll
        for (int t = 0; t < kTilesI; ++t) {
            const int i = ibase + t * 16 + (lane & 15);
            bf8 bv = *reinterpret_cast<const bf8*>(Tb + (size_t)i * npad + k0 + 8 * kb);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < kTilesI; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 4 * kb + v;
            const int i = ibase + t * 16 + (lane & 15);
            if (r < rows && i < n) out[(size_t)r * n + i] = acc[t][v];
        }
}

inline dim3 grid_cols(int C, int n, int A) {
    const int per = 16 * kWaves;
    return dim3((C + per - 1) / per, (n + 16 * kTilesI - 1) / (16 * kTilesI), A);
}

template <int PREC>
hipError_t fd_apply_t(const FdPc& P, const typename Tr<PREC>::T* r, typename Tr<PREC>::T* z, void* scratch,
                      hipStream_t s) {
    using T = typename Tr<PREC>::T;
    const int n1 = P.n[0], n2 = P.n[1], n3 = P.n[2];
    T* tmp = reinterpret_cast<T*>(scratch);
    const T* U[3];
    for (int l = 0; l < 3; ++l) U[l] = PREC == 1 ? (const T*)P.U64[l] : (const T*)P.U32[l];
    const dim3 blk(64 * kWaves);
    Scale none;
    Scale sc;
    sc.l1 = P.lam[0];
    sc.l2 = P.lam[1];
    sc.l3 = P.lam[2];
    sc.n1 = n1;
    sc.n2 = n2;
    const int rows_x = n2 * n3;
    const dim3 gx((rows_x + 16 * kWaves - 1) / (16 * kWaves), (n1 + 16 * kTilesI - 1) / (16 * kTilesI));
    // forward: T = U^T
    hipLaunchKernelGGL(mode_x_kernel<PREC>, gx, blk, 0, s, r, tmp, U[0], n1, rows_x, 1);
    hipLaunchKernelGGL(mode_strided_kernel<PREC>, grid_cols(n1, n2, n3), blk, 0, s, tmp, z, U[1], n2, n1, 1, none);
    hipLaunchKernelGGL(mode_strided_kernel<PREC>, grid_cols(n1 * n2, n3, 1), blk, 0, s, z, tmp, U[2], n3, n1 * n2,
                       1, sc);
    // backward: T = U
    hipLaunchKernelGGL(mode_x_kernel<PREC>, gx, blk, 0, s, tmp, z, U[0], n1, rows_x, 0);
    hipLaunchKernelGGL(mode_strided_kernel<PREC>, grid_cols(n1, n2, n3), blk, 0, s, z, tmp, U[1], n2, n1, 0, none);
    hipLaunchKernelGGL(mode_strided_kernel<PREC>, grid_cols(n1 * n2, n3, 1), blk, 0, s, tmp, z, U[2], n3, n1 * n2,
                       0, none);
    return hipGetLastError();
}

hipError_t fd_apply_bf16(const FdPc& P, const float* r, float* z, void* scratch, hipStream_t s) {
    const int n1 = P.n[0], n2 = P.n[1], n3 = P.n[2];
    float* tmp = reinterpret_cast<float*>(scratch);
    const dim3 blk(64 * kWaves);
    Scale none;
    Scale sc;
    sc.l1 = P.lam[0];
    sc.l2 = P.lam[1];
    sc.l3 = P.lam[2];
    sc.n1 = n1;
    sc.n2 = n2;
    // Ubf[l] holds two padded npad x npad bf16 matrices: T = U^T then T = U
    int npad[3];
    const __bf16 *Tf[3], *Tb[3];
    for (int l = 0; l < 3; ++l) {
        npad[l] = (P.n[l] + 63) / 64 * 64;   // rows and columns padded as stored by fd_setup
        Tf[l] = reinterpret_cast<const __bf16*>(P.Ubf[l]);
        Tb[l] = Tf[l] + (size_t)npad[l] * npad[l];
    }
    const int rows_x = n2 * n3;
    const dim3 gx((rows_x + 16 * kWaves - 1) / (16 * kWaves), (n1 + 16 * kTilesI - 1) / (16 * kTilesI));
    hipLaunchKernelGGL(mode_x_bf16_kernel, gx, blk, 0, s, r, tmp, Tf[0], n1, npad[0], rows_x);
    hipLaunchKernelGGL(mode_strided_bf16_kernel, grid_cols(n1, n2, n3), blk, 0, s, tmp, z, Tf[1], n2, npad[1], n1,
                       none);
    hipLaunchKernelGGL(mode_strided_bf16_kernel, grid_cols(n1 * n2, n3, 1), blk, 0, s, z, tmp, Tf[2], n3, npad[2],
                       n1 * n2, sc);
    hipLaunchKernelGGL(mode_x_bf16_kernel, gx, blk, 0, s, tmp, z, Tb[0], n1, npad[0], rows_x);
    hipLaunchKernelGGL(mode_strided_bf16_kernel, grid_cols(n1, n2, n3), blk, 0, s, z, tmp, Tb[1], n2, npad[1], n1,
                       none);
    hipLaunchKernelGGL(mode_strided_bf16_kernel, grid_cols(n1 * n2, n3, 1), blk, 0, s, tmp, z, Tb[2], n3, npad[2],
                       n1 * n2, none);
    return hipGetLastError();
}

// Six LDS-tiled mode products (fd_gemm.hip): x, y, z forward with U^T (scaling
// fused into z), then x, y, z backward with U.  Ping-pongs between z and the
// scratch buffer (N values), so r and z may alias.
template <typename T, typename S>
hipError_t fd_apply_gemm(const FdPc& P, const T* r, T* z, void* scratch, const S* const Tf[3], const S* const Tb[3],
                         const int ld[3], hipStream_t s) {
    const int n1 = P.n[0], n2 = P.n[1], n3 = P.n[2];
    T* tmp = reinterpret_cast<T*>(scratch);
    auto mode = [&](int axis, const T* in, T* out, const S* mat, bool scale) {
        FdModeArgs<T, S> a;
        a.in = in;
        a.out = out;
        a.mat = mat;
        a.ldT = ld[axis];
        if (axis == 0) {                    // columns (i3, i2): contiguous rows of length n1
            a.n = n1;
            a.C = n2 * n3;
            a.cdiv = a.C;
            a.sj = 1;
            a.sc = (size_t)n1;
        } else if (axis == 1) {             // columns (i3, i1)
            a.n = n2;
            a.C = n1 * n3;
            a.cdiv = n1;
            a.sj = (size_t)n1;
            a.sc = 1;
            a.sa = (size_t)n1 * n2;
        } else {                            // columns (i2, i1)
            a.n = n3;
            a.C = n1 * n2;
            a.cdiv = a.C;
            a.sj = (size_t)n1 * n2;
            a.sc = 1;
        }
        if (scale) {
            a.l1 = P.lam[0];
            a.l2 = P.lam[1];
            a.l3 = P.lam[2];
            a.n1 = n1;
        }
        return launch_fd_mode(a, s);
    };
    hipError_t e;
    if ((e = mode(0, r, tmp, Tf[0], false)) != hipSuccess) return e;
    if ((e = mode(1, tmp, z, Tf[1], false)) != hipSuccess) return e;
    if ((e = mode(2, z, tmp, Tf[2], true)) != hipSuccess) return e;
    if ((e = mode(0, tmp, z, Tb[0], false)) != hipSuccess) return e;
    if ((e = mode(1, z, tmp, Tb[1], false)) != hipSuccess) return e;
    return mode(2, tmp, z, Tb[2], false);
}

}  // namespace

hipError_t launch_fd_apply(const FdPc& P, int prec, const void* r, void* z, void* scratch, hipStream_t s) {
    const bool small = P.n[0] <= 144 && P.n[1] <= 144 && P.n[2] <= 144;
    if (small && P.ldp && (prec == 1 || prec == 2) && !std::getenv("WQFD_FD_MODES")) {
        if (prec == 1) {
            FdFusedArgs<double> f;
            f.r = static_cast<const double*>(r);
            f.z = static_cast<double*>(z);
            f.tmp = reinterpret_cast<double*>(scratch);
            for (int l = 0; l < 3; ++l) {
                f.U[l] = P.Up64[l];
                f.UT[l] = P.UTp64[l];
            }
            f.l1 = P.lam[0];
            f.l2 = P.lam[1];
            f.l3 = P.lam[2];
            f.n1 = P.n[0];
            f.n2 = P.n[1];
            f.n3 = P.n[2];
            f.ldp = P.ldp;
            return launch_fd_fused(f, s);
        }
        FdFusedArgs<float> f;
        f.r = static_cast<const float*>(r);
        f.z = static_cast<float*>(z);
        f.tmp = reinterpret_cast<float*>(scratch);
        for (int l = 0; l < 3; ++l) {
            f.U[l] = P.Up32[l];
            f.UT[l] = P.UTp32[l];
        }
        f.l1 = P.lam[0];
        f.l2 = P.lam[1];
        f.l3 = P.lam[2];
        f.n1 = P.n[0];
        f.n2 = P.n[1];
        f.n3 = P.n[2];
        f.ldp = P.ldp;
        return launch_fd_fused(f, s);
    }
    if (small && prec == 4 && !std::getenv("WQFD_FD_MODES")) {
        FdFusedBf16Args f;
        f.r = static_cast<const float*>(r);
        f.z = static_cast<float*>(z);
        f.tmp = reinterpret_cast<float*>(scratch);
        for (int l = 0; l < 3; ++l) {
            f.ld[l] = (P.n[l] + 63) / 64 * 64;              // as stored by fd_setup
            f.n[l] = P.n[l];
            f.Tf[l] = reinterpret_cast<const __bf16*>(P.Ubf[l]);
            f.Tb[l] = f.Tf[l] + (size_t)f.ld[l] * f.ld[l];
        }
        f.l1 = P.lam[0];
        f.l2 = P.lam[1];
        f.l3 = P.lam[2];
        f.n1 = P.n[0];
        f.n2 = P.n[1];
        f.n3 = P.n[2];
        return launch_fd_fused_bf16(f, s);
    }
    if (small) {
        if (prec == 1) {
            const double* Tf[3] = {P.UT64[0], P.UT64[1], P.UT64[2]};
            const double* Tb[3] = {P.U64[0], P.U64[1], P.U64[2]};
            const int ld[3] = {P.n[0], P.n[1], P.n[2]};
            return fd_apply_gemm<double, double>(P, static_cast<const double*>(r), static_cast<double*>(z), scratch, Tf, Tb,
                                                 ld, s);
        }
        if (prec == 2) {
            const float* Tf[3] = {P.UT32[0], P.UT32[1], P.UT32[2]};
            const float* Tb[3] = {P.U32[0], P.U32[1], P.U32[2]};
            const int ld[3] = {P.n[0], P.n[1], P.n[2]};
            return fd_apply_gemm<float, float>(P, static_cast<const float*>(r), static_cast<float*>(z), scratch, Tf, Tb, ld,
                                               s);
        }
        const __bf16 *Tf[3], *Tb[3];
        int ld[3];
        for (int l = 0; l < 3; ++l) {
            ld[l] = (P.n[l] + 63) / 64 * 64;
            Tf[l] = reinterpret_cast<const __bf16*>(P.Ubf[l]);
            Tb[l] = Tf[l] + (size_t)ld[l] * ld[l];
        }
        return fd_apply_gemm<float, __bf16>(P, static_cast<const float*>(r), static_cast<float*>(z), scratch, Tf, Tb, ld,
                                            s);
    }
    if (prec == 1) return fd_apply_t<1>(P, static_cast<const double*>(r), static_cast<double*>(z), scratch, s);
    if (prec == 2) return fd_apply_t<2>(P, static_cast<const float*>(r), static_cast<float*>(z), scratch, s);
    return fd_apply_bf16(P, static_cast<const float*>(r), static_cast<float*>(z), scratch, s);
}

}  // namespace wqfd
