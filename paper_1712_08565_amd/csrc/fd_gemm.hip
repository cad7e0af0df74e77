// LDS-tiled mode products of the Fast Diagonalization preconditioner on the
// matrix cores (gfx950).  One launch applies a small n x n matrix T along one
// axis of the [n3][n2][n1] array:
//     out[a][i][c] = sum_j T[i][j] in[a][j][c]
// where element (j, c) of batch a sits at a * sa + j * sj + c * sc (y and z
// modes: sj = row length, sc = 1; x mode: sj = 1, sc = n).  A workgroup owns
// all n output rows (MT 16-row tiles) and 64 columns c; T and the input are
// staged through LDS in K chunks, double buffered, with both operands stored
// k-contiguous so every MFMA fragment is one LDS read per lane.
//   FP64: v_mfma_f64_16x16x4f64, 4 k-steps per 16-wide chunk
//   FP32: v_mfma_f32_16x16x4f32
//   BF16: v_mfma_f32_16x16x32_bf16 (FP32 data converted to bf16 at staging,
//         T pre-converted), one k-step per 32-wide chunk, FP32 accumulation.
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
    using S = double;            // staged operand
    using Acc = d4;
    static constexpr int BK = 16;
    __device__ static int drow(int kb, int v) { return kb + 4 * v; }
};
template <>
struct G<2> {                    // FP32
    using T = float;
    using S = float;
    using Acc = f4;
    static constexpr int BK = 16;
    __device__ static int drow(int kb, int v) { return 4 * kb + v; }
};
template <>
struct G<4> {                    // BF16 operands, FP32 data
    using T = float;
    using S = __bf16;
    using Acc = f4;
    static constexpr int BK = 32;
    __device__ static int drow(int kb, int v) { return 4 * kb + v; }
};

constexpr int BN = 64;

template <int PREC, int MT>
__global__ __launch_bounds__(256) void fd_mode_gemm(FdModeArgs<typename G<PREC>::T, typename G<PREC>::S> p) {
    using T = typename G<PREC>::T;
    using S = typename G<PREC>::S;
    using Acc = typename G<PREC>::Acc;
    constexpr int BK = G<PREC>::BK;
    constexpr int LDK = BK + (sizeof(S) == 8 ? 1 : (sizeof(S) == 4 ? 1 : 8));   // padded k length
    constexpr int BM = 16 * MT;
    __shared__ __attribute__((aligned(16))) S sA[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) S sB[2][BN * LDK];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cl = lane & 15, kb = lane >> 4;
    const int c0 = blockIdx.x * BN;
    const size_t abase = (size_t)blockIdx.y * p.sa;
    const T* __restrict__ in = p.in + abase;
    T* __restrict__ out = p.out + abase;
    const int n = p.n, C = p.C;
    const int nchunk = (n + BK - 1) / BK;

    // staging registers for the next chunk
    constexpr int AE = (BM * BK + 255) / 256;      // A elements per thread
    constexpr int BE = (BN * BK) / 256;            // B elements per thread
    S ra[AE], rb[BE];

    auto load_chunk = [&](int ch) {
        const int k0 = ch * BK;
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid + e * 256;
            const int i = idx / BK, k = idx % BK;
            S v = S(0);
            if (idx < BM * BK && i < n && k0 + k < n) v = p.mat[(size_t)i * p.ldT + k0 + k];
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = tid + e * 256;
            int c, k;
            if (p.sc == 1) {            // contiguous along c
                k = idx / BN;
                c = idx % BN;
            } else {                    // contiguous along k
                c = idx / BK;
                k = idx % BK;
            }
            T v = T(0);
            if (c0 + c < C && k0 + k < n) v = in[(size_t)(k0 + k) * p.sj + (size_t)(c0 + c) * p.sc];
            rb[e] = (S)v;
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid + e * 256;
            if (idx < BM * BK) sA[buf][(idx / BK) * LDK + idx % BK] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = tid + e * 256;
            int c, k;
            if (p.sc == 1) {
                k = idx / BN;
                c = idx % BN;
            } else {
                c = idx / BK;
                k = idx % BK;
            }
            sB[buf][c * LDK + k] = rb[e];
        }
    };

    Acc acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = Acc{0, 0, 0, 0};

    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunk) load_chunk(ch + 1);
        const S* A = sA[buf];
        const S* B = sB[buf] + (wave * 16 + cl) * LDK;
        if constexpr (PREC == 4) {
            const bf8 b = *reinterpret_cast<const bf8*>(B + 8 * kb);
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const bf8 a = *reinterpret_cast<const bf8*>(A + (t * 16 + cl) * LDK + 8 * kb);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < BK / 4; ++s) {
                const S b = B[4 * s + kb];
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    const S a = A[(t * 16 + cl) * LDK + 4 * s + kb];
                    if constexpr (PREC == 1)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
                    else
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        if (ch + 1 < nchunk) {
            // buf ^ 1 was last read in the previous chunk, before the barrier below
            store_chunk(buf ^ 1);
            __syncthreads();
        }
    }
    // epilogue: optional eigenvalue scaling, bounds-checked store
    const int c = c0 + wave * 16 + cl;
    if (c >= C) return;
    double l12 = 0.0;
    if (p.l1) {
        const int i2 = c / p.n1, i1 = c - i2 * p.n1;
        l12 = p.l1[i1] + p.l2[i2];
    }
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = t * 16 + G<PREC>::drow(kb, v);
            if (i < n) {
                T val = acc[t][v];
                if (p.l1) val = (T)((double)val / (l12 + p.l3[i]));
                out[(size_t)i * p.sj + (size_t)c * p.sc] = val;
            }
        }
}

template <int PREC, int MT>
hipError_t launch_mt(const FdModeArgs<typename G<PREC>::T, typename G<PREC>::S>& p, int batches, hipStream_t s) {
    dim3 grid((p.C + BN - 1) / BN, batches);
    hipLaunchKernelGGL((fd_mode_gemm<PREC, MT>), grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_any(const FdModeArgs<typename G<PREC>::T, typename G<PREC>::S>& p, int batches, hipStream_t s) {
    switch ((p.n + 15) / 16) {
        case 1: return launch_mt<PREC, 1>(p, batches, s);
        case 2: return launch_mt<PREC, 2>(p, batches, s);
        case 3: return launch_mt<PREC, 3>(p, batches, s);
        case 4: return launch_mt<PREC, 4>(p, batches, s);
        case 5: return launch_mt<PREC, 5>(p, batches, s);
        case 6: return launch_mt<PREC, 6>(p, batches, s);
        case 7: return launch_mt<PREC, 7>(p, batches, s);
        case 8: return launch_mt<PREC, 8>(p, batches, s);
        case 9: return launch_mt<PREC, 9>(p, batches, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fd_mode(const FdModeArgs<double, double>& p, int batches, hipStream_t s) {
    return launch_any<1>(p, batches, s);
}
hipError_t launch_fd_mode(const FdModeArgs<float, float>& p, int batches, hipStream_t s) {
    return launch_any<2>(p, batches, s);
}
hipError_t launch_fd_mode(const FdModeArgs<float, __bf16>& p, int batches, hipStream_t s) {
    return launch_any<4>(p, batches, s);
}

}  // namespace wqfd
