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

#include <type_traits>

#include "buffer.h"
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
// The small matrices are passed transposed (Tt[j][i] = T[i][j]) and zero-padded
// to ldp x ldp, ldp = 16 KB: an operand column is 16 consecutive entries and no
// load needs a bounds check.  Data loads are unconditional too: rows and columns
// past the extents are clamped to the last one (finite values that meet the
// zero padding of the matrix, or land in outputs that are not stored).  All
// loads are raw buffer loads with the step offset in a scalar register, issued
// a fixed number of steps ahead of their product (software pipelined).
// One wave per 16-wide block (KB = ceil(n / 16) waves), one plane (xy) or
// column block (z) per workgroup, one barrier per workgroup.  Contraction
// steps past the true length are skipped.
constexpr int FLD = 17;                                  // padded row of 16-column LDS blocks

// Workgroup barrier that waits only for this wave's LDS operations: global loads
// in flight (the pipelined operands) stay in flight across it, where the release
// fence of __syncthreads() would drain them.
__device__ inline void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int PREC>
__device__ inline typename G<PREC>::Acc mma_step(typename G<PREC>::T a, typename G<PREC>::T b,
                                                 typename G<PREC>::Acc c) {
    if constexpr (PREC == 1)
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Accumulator and product of one wave: a 16 x 16 block (v_mfma_f64_16x16x4f64 or
// v_mfma_f32_16x16x4f32), or, SMALL (FP64 only), four 4 x 4 blocks
// (v_mfma_f64_4x4x4f64, a quarter of the matrix-core time) for a block of the
// output with at most 4 rows or columns inside the array.  Lane layout of the
// four-block product, lane = 16 kb + cl: A_b[i][k] at i = cl & 3, b = cl >> 2,
// k = kb; B_b[k][j] at j = cl & 3, b = cl >> 2, k = kb; D_b[i][j] at lane
// 16 i + 4 b + j.  With the A operand the same in all four blocks (rows i of
// a 4-row block) the lane holds D row kb, column cl; with B the same in all four
// (columns j of a 4-column block) it holds row 4 (cl >> 2) + kb, column cl & 3.
template <int PREC, bool SMALL>
struct WaveMM {
    using T = typename G<PREC>::T;
    using Acc = typename G<PREC>::Acc;
    __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
    __device__ static Acc mma(T a, T b, Acc c) { return mma_step<PREC>(a, b, c); }
};
template <>
struct WaveMM<1, true> {
    using Acc = double;
    __device__ static Acc zero() { return 0.0; }
    __device__ static Acc mma(double a, double b, double c) { return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0); }
};

// The operands of a contraction step live in rings of R = DL + 1 registers, not
// in arrays over the whole contraction, so a wave holds few registers (FP64:
// 47-52 in the xy pass, 60-66 in the z pass) and several workgroups share a CU,
// one's load latency, barrier and stores overlapping another's products.  Step
// s of the first matrix and of the data go to slot s % R, DL steps ahead of
// their product; once the first matrix's last step is issued, the second
// matrix's steps follow in the same ring (step j in slot (NKS + j) % R), so its
// first DL steps are in flight across the barrier.  The intermediate (Q or Y) is
// read from LDS LA steps ahead of its product.  (Measured against arrays over
// the whole contraction with one or two planes per workgroup: FP64 n = 65 26.1
// -> 24.6 us per application, n = 99 63 -> 58, n = 132 171 -> 136.)
template <int PREC, int KB>
__global__ __launch_bounds__(64 * KB) void fd_xy_pass(const typename G<PREC>::T* __restrict__ in,
                                                      typename G<PREC>::T* __restrict__ out,
                                                      const typename G<PREC>::T* __restrict__ T1t,
                                                      const typename G<PREC>::T* __restrict__ T2t, int n1, int n2,
                                                      int n3) {
    using T = typename G<PREC>::T;
    constexpr int NKS = 4 * KB;
    constexpr int LDP = 16 * KB;
    constexpr int LDQ = 16 * KB + 1;
    constexpr int DL = 6, R = DL + 1, LA = 4;        // load lead, LDS lead (measured: 6 and 4 best)
    __shared__ T sQ[16 * LDQ];
    const int lane = threadIdx.x & 63, t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cl = lane & 15, kb = lane >> 4;
    // workgroup -> (row block, plane): consecutive workgroups are dealt
    // round-robin to the eight XCDs, so hand each XCD a contiguous run of
    // (row block, plane) items: the row blocks of a plane, which all read the
    // whole plane, then mostly share one XCD's L2
    int r0, z;
    {
        const int nrb = gridDim.x, nblk = gridDim.x * gridDim.y, b = blockIdx.x + blockIdx.y * gridDim.x;
        const int base = nblk / 8, rem = nblk % 8, xcd = b % 8, slot = b / 8;
        const int lin = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + slot;
        r0 = (lin % nrb) * 16;
        z = lin / nrb;
    }
    const int tl = (n1 - 1) >> 4;
    if (t > tl) {
        lds_sync();
        return;
    }
    const bool rr = PREC == 1 && n2 - r0 <= 4, rc = PREC == 1 && t == tl && n1 - 16 * tl <= 4;
    auto body = [&](auto small_tag) {
        constexpr bool SMALL = decltype(small_tag)::value;
        using MM = WaveMM<PREC, SMALL>;
        using Acc = typename MM::Acc;
        const unsigned psz = (unsigned)(n1 * n2);
        const int ks2 = (n2 + 3) >> 2, ks1 = (n1 + 3) >> 2;
        const int arow = rr ? (cl & 3) : cl;
        const int jc = 16 * t + (rc ? (cl & 3) : cl);
        const __amdgpu_buffer_rsrc_t rin = buf_rsrc(in), r1 = buf_rsrc(T1t), r2 = buf_rsrc(T2t);
        const int jcc = min(jc, n1 - 1);
        const unsigned vo = (unsigned)((kb * n1 + jcc) * sizeof(T));
        const unsigned va = (unsigned)((kb * LDP + r0 + arow) * sizeof(T)), vc = (unsigned)((kb * LDP + jc) * sizeof(T));
        constexpr unsigned kstep = 4 * LDP * sizeof(T);
        const unsigned zo = (unsigned)(z * psz * sizeof(T));
        T a[R], b[R], aq[LA + 1];
        Acc q = MM::zero();
        auto load_step = [&](int s) {                    // T2 and data of step s, or T1 step s - NKS
            if (s < NKS) {
                a[s % R] = buf_load<T>(r2, va, s * kstep);
                if (4 * s + 3 < n2)
                    b[s % R] = buf_load<T>(rin, vo, zo + (unsigned)(4 * s * n1 * sizeof(T)));
                else if (s < ks2)
                    b[s % R] = buf_load<T>(rin, (unsigned)((min(4 * s + kb, n2 - 1) * n1 + jcc) * sizeof(T)), zo);
                else
                    b[s % R] = T(0);
            } else if (s - NKS < NKS) {
                a[s % R] = buf_load<T>(r1, vc, (s - NKS) * kstep);
            }
        };
#pragma unroll
        for (int s = 0; s < DL; ++s) load_step(s);
#pragma unroll
        for (int m = 0; m < NKS; ++m) {
            __builtin_amdgcn_sched_barrier(0);
            load_step(m + DL);
            __builtin_amdgcn_sched_barrier(0);
            if (m < ks2) q = MM::mma(a[m % R], b[m % R], q);
        }
        const int qrow = rr ? kb : 4 * (cl >> 2) + kb;
        if constexpr (SMALL) {
            sQ[qrow * LDQ + jc] = q;
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) sQ[G<PREC>::drow(kb, v) * LDQ + jc] = q[v];
        }
        lds_sync();
        if (z >= n3) return;
#pragma unroll
        for (int j = 0; j < LA; ++j) aq[j] = sQ[arow * LDQ + 4 * j + kb];
        Acc r = MM::zero();
#pragma unroll
        for (int j = 0; j < NKS; ++j) {
            __builtin_amdgcn_sched_barrier(0);
            load_step(NKS + j + DL);
            if (j + LA < NKS) aq[(j + LA) % (LA + 1)] = sQ[arow * LDQ + 4 * (j + LA) + kb];
            __builtin_amdgcn_sched_barrier(0);
            if (j < ks1) r = MM::mma(aq[j % (LA + 1)], a[(NKS + j) % R], r);
        }
        if (jc < n1) {
            T* op = out + (size_t)z * psz + jc;
            if constexpr (SMALL) {
                if (r0 + qrow < n2) op[(size_t)(r0 + qrow) * n1] = r;
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i2 = r0 + G<PREC>::drow(kb, v);
                    if (i2 < n2) op[(size_t)i2 * n1] = r[v];
                }
            }
        }
    };
    if constexpr (PREC == 1) {
        if (rr || rc)
            body(std::true_type{});
        else
            body(std::false_type{});
    } else {
        body(std::false_type{});
    }
}

template <int PREC, int KB>
__global__ __launch_bounds__(64 * KB) void fd_z_pass(const typename G<PREC>::T* in, typename G<PREC>::T* out,
                                                     const typename G<PREC>::T* __restrict__ T3ft,
                                                     const typename G<PREC>::T* __restrict__ T3bt,
                                                     const double* __restrict__ l1, const double* __restrict__ l2,
                                                     const double* __restrict__ l3, int n1, int n2, int n3) {
    using T = typename G<PREC>::T;
    constexpr int NKS = 4 * KB;
    constexpr int LDP = 16 * KB;
    constexpr int DL = 6, R = DL + 1, LA = 4;        // load lead, LDS lead (measured: 6 and 4 best)
    __shared__ T sY[16 * KB * FLD];
    const int lane = threadIdx.x & 63, t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cl = lane & 15, kb = lane >> 4;
    const int tl = (n3 - 1) >> 4;
    if (t > tl) {
        lds_sync();
        return;
    }
    const bool rs = PREC == 1 && t == tl && n3 - 16 * tl <= 4;
    auto body = [&](auto small_tag) {
        constexpr bool SMALL = decltype(small_tag)::value;
        using MM = WaveMM<PREC, SMALL>;
        using Acc = typename MM::Acc;
        constexpr int NV = SMALL ? 1 : 4;
        const int C = n1 * n2;
        const int i3r = 16 * t + (SMALL ? (cl & 3) : cl);
        const int ks3 = (n3 + 3) >> 2;
        const __amdgpu_buffer_rsrc_t rin = buf_rsrc(in), rf = buf_rsrc(T3ft), rb = buf_rsrc(T3bt);
        const unsigned va = (unsigned)((kb * LDP + i3r) * sizeof(T));
        constexpr unsigned kstep = 4 * LDP * sizeof(T);
        auto row_of = [&](int v) { return 16 * t + (SMALL ? kb : G<PREC>::drow(kb, v)); };
        auto get = [](const Acc& c, int v) -> T {
            if constexpr (SMALL) return c; else return c[v];
        };
        const int g = blockIdx.x * 16 + cl;
        const bool gin = g < C;
        const int gc = min(g, C - 1);
        const unsigned vo = (unsigned)((kb * C + gc) * sizeof(T));
        double l12 = 0.0, l3v[NV];
        if (gin) {
            const int i2 = g / n1, i1 = g - i2 * n1;
            l12 = l1[i1] + l2[i2];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) l3v[v] = row_of(v) < n3 ? l3[row_of(v)] : 1.0;
        T a[R], b[R], by[LA + 1];
        Acc y = MM::zero();
        auto load_step = [&](int s) {                    // T3f and data of step s, or T3b step s - NKS
            if (s < NKS) {
                a[s % R] = buf_load<T>(rf, va, s * kstep);
                if (4 * s + 3 < n3)
                    b[s % R] = buf_load<T>(rin, vo, (unsigned)(4 * s * C * sizeof(T)));
                else if (s < ks3)
                    b[s % R] = buf_load<T>(rin, (unsigned)((min(4 * s + kb, n3 - 1) * C + gc) * sizeof(T)), 0u);
                else
                    b[s % R] = T(0);
            } else if (s - NKS < NKS) {
                a[s % R] = buf_load<T>(rb, va, (s - NKS) * kstep);
            }
        };
#pragma unroll
        for (int s = 0; s < DL; ++s) load_step(s);
#pragma unroll
        for (int m = 0; m < NKS; ++m) {
            __builtin_amdgcn_sched_barrier(0);
            load_step(m + DL);
            __builtin_amdgcn_sched_barrier(0);
            if (m < ks3) y = MM::mma(a[m % R], b[m % R], y);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int i3 = row_of(v);
            sY[i3 * FLD + cl] = (gin && i3 < n3) ? (T)((double)get(y, v) / (l12 + l3v[v])) : T(0);
        }
        lds_sync();                                      // every read of `in` by this block is done: in may be out
#pragma unroll
        for (int j = 0; j < LA; ++j) by[j] = sY[(4 * j + kb) * FLD + cl];
        Acc zz = MM::zero();
#pragma unroll
        for (int j = 0; j < NKS; ++j) {
            __builtin_amdgcn_sched_barrier(0);
            load_step(NKS + j + DL);
            if (j + LA < NKS) by[(j + LA) % (LA + 1)] = sY[(4 * (j + LA) + kb) * FLD + cl];
            __builtin_amdgcn_sched_barrier(0);
            if (j < ks3) zz = MM::mma(a[(NKS + j) % R], by[j % (LA + 1)], zz);
        }
        if (gin) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int i3 = row_of(v);
                if (i3 < n3) out[(size_t)i3 * C + g] = get(zz, v);
            }
        }
    };
    if constexpr (PREC == 1) {
        if (rs)
            body(std::true_type{});
        else
            body(std::false_type{});
    } else {
        body(std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// BF16 variant of the fused passes: FP32 data, bf16 operands rounded as they are
// loaded, FP32 accumulation, v_mfma_f32_16x16x32_bf16 (k-step s covers
// k = 32 s + 8 kb + e, e = 0..7, so an operand is eight consecutive values of a
// row).  The matrices are the bf16 copies of fd_setup: T = U^T and T = U,
// row-major and zero padded to ld = 64 ceil(n / 64) in both dimensions (rows
// and columns past n are zero, so clamped data rows and columns contribute
// nothing).  Intermediates go through LDS in FP32, stored so that every MFMA
// operand is one 16-byte read.  NS = ceil(n / 32) steps (at most NSM); the
// workgroup has 2 NSM waves, waves past ceil(n / 16) only join the barrier.
__device__ inline bf8 to_bf8(const float (&x)[8]) {
    bf8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (__bf16)x[e];
    return r;
}

__device__ inline bf8 lds_bf8(const float* p) {             // 8 consecutive FP32 values, 16-byte aligned
    const float4 lo = *reinterpret_cast<const float4*>(p), hi = *reinterpret_cast<const float4*>(p + 4);
    const float x[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    return to_bf8(x);
}

__device__ inline bf8 mat_bf8(const __bf16* T, int ld, int row, int k0) {
    return *reinterpret_cast<const bf8*>(T + (size_t)row * ld + k0);
}

// xy pass: per z-plane and 16-row block of i2,
//   Q[i2][j1] = sum_j2 T2[i2][j2] in[z][j2][j1],   out[z][i2][i1] = sum_j1 Q[i2][j1] T1[i1][j1]
template <int NSM>
__global__ __launch_bounds__(128 * NSM) void fd_xy_pass_bf16(const float* __restrict__ in, float* __restrict__ out,
                                                            const __bf16* __restrict__ T1, const __bf16* __restrict__ T2,
                                                            int ld1, int ld2, int n1, int n2) {
    constexpr int LDQ = 32 * NSM + 4;                    // row of Q in LDS (16-byte aligned rows)
    __shared__ __align__(16) float sQ[16 * LDQ];
    const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
    const int cl = lane & 15, kb = lane >> 4;
    // workgroup -> (row block, plane): consecutive workgroups are dealt
    // round-robin to the eight XCDs, so hand each XCD a contiguous run of
    // (row block, plane) items: the row blocks of a plane, which all read the
    // whole plane, then mostly share one XCD's L2
    int r0, z;
    {
        const int nrb = gridDim.x, nblk = gridDim.x * gridDim.y, b = blockIdx.x + blockIdx.y * gridDim.x;
        const int base = nblk / 8, rem = nblk % 8, xcd = b % 8, slot = b / 8;
        const int lin = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + slot;
        r0 = (lin % nrb) * 16;
        z = lin / nrb;
    }
    const size_t pbase = (size_t)z * n1 * n2;
    const int kb1 = (n1 + 15) >> 4;                      // waves with columns j1 / i1
    const int ns1 = (n1 + 31) >> 5, ns2 = (n2 + 31) >> 5;
    const bool active = t < kb1;                         // wave-uniform
    const int jc = 16 * t + cl, jcc = min(jc, n1 - 1);
    // columns of Q past the last wave's block are read by the second product
    // (multiplied by zero padding of T1): clear them
    for (int idx = threadIdx.x; idx < 16 * (32 * ns1 - 16 * kb1); idx += blockDim.x) {
        const int w = 32 * ns1 - 16 * kb1;
        sQ[(idx / w) * LDQ + 16 * kb1 + idx % w] = 0.0f;
    }
    if (active) {
        f4 q = f4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NSM; ++s) {
            if (s < ns2) {
                const bf8 a = mat_bf8(T2, ld2, r0 + cl, 32 * s + 8 * kb);
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = in[pbase + (size_t)min(32 * s + 8 * kb + e, n2 - 1) * n1 + jcc];
                q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, to_bf8(x), q, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) sQ[(4 * kb + v) * LDQ + jc] = q[v];
    }
    __syncthreads();
    if (!active) return;
    f4 r = f4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
        if (s < ns1) {
            const bf8 a = lds_bf8(sQ + cl * LDQ + 32 * s + 8 * kb);
            const bf8 b = mat_bf8(T1, ld1, jc, 32 * s + 8 * kb);
            r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, r, 0, 0, 0);
        }
    }
    if (jc < n1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i2 = r0 + 4 * kb + v;
            if (i2 < n2) out[pbase + (size_t)i2 * n1 + jc] = r[v];
        }
    }
}

// z pass: per 16-column block of g = (i2, i1),
//   Y[i3][g] = sum_j3 T3f[i3][j3] in[j3][g] / (l1[i1] + l2[i2] + l3[i3]),   out[i3][g] = sum_j3 T3b[i3][j3] Y[j3][g]
// (Y kept transposed in LDS; every read of `in` precedes the block's writes, so in may be out)
template <int NSM>
__global__ __launch_bounds__(128 * NSM) void fd_z_pass_bf16(const float* in, float* out, const __bf16* __restrict__ Tf,
                                                           const __bf16* __restrict__ Tb, int ld3,
                                                           const double* __restrict__ l1, const double* __restrict__ l2,
                                                           const double* __restrict__ l3, int n1, int n2, int n3) {
    constexpr int LDY = 32 * NSM + 4;
    __shared__ __align__(16) float sY[16 * LDY];         // Y^T: [column g][i3]
    const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
    const int cl = lane & 15, kb = lane >> 4;
    const int C = n1 * n2;
    const int g = blockIdx.x * 16 + cl;
    const bool gin = g < C;
    const int gc = min(g, C - 1);
    const int kb3 = (n3 + 15) >> 4, ns3 = (n3 + 31) >> 5;
    const bool active = t < kb3;
    const int i3r = 16 * t + cl;
    for (int idx = threadIdx.x; idx < 16 * (32 * ns3 - 16 * kb3); idx += blockDim.x) {
        const int w = 32 * ns3 - 16 * kb3;
        sY[(idx / w) * LDY + 16 * kb3 + idx % w] = 0.0f;
    }
    if (active) {
        f4 y = f4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NSM; ++s) {
            if (s < ns3) {
                const bf8 a = mat_bf8(Tf, ld3, i3r, 32 * s + 8 * kb);
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = in[(size_t)min(32 * s + 8 * kb + e, n3 - 1) * C + gc];
                y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, to_bf8(x), y, 0, 0, 0);
            }
        }
        double l12 = 0.0;
        if (gin) {
            const int i2 = g / n1, i1 = g - i2 * n1;
            l12 = l1[i1] + l2[i2];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i3 = 16 * t + 4 * kb + v;
            sY[cl * LDY + i3] = (gin && i3 < n3) ? (float)((double)y[v] / (l12 + l3[i3])) : 0.0f;
        }
    }
    __syncthreads();
    if (!active) return;
    f4 o = f4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NSM; ++s) {
        if (s < ns3) {
            const bf8 a = mat_bf8(Tb, ld3, i3r, 32 * s + 8 * kb);
            const bf8 b = lds_bf8(sY + cl * LDY + 32 * s + 8 * kb);
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, o, 0, 0, 0);
        }
    }
    if (gin) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i3 = 16 * t + 4 * kb + v;
            if (i3 < n3) out[(size_t)i3 * C + g] = o[v];
        }
    }
}

template <int NSM>
hipError_t fused_bf16_ns(const FdFusedBf16Args& f, hipStream_t s) {
    hipError_t e;
    const dim3 blk(128 * NSM);
    const dim3 gxy((f.n2 + 15) / 16, f.n3);
    const dim3 gz((f.n1 * f.n2 + 15) / 16);
    hipLaunchKernelGGL(fd_xy_pass_bf16<NSM>, gxy, blk, 0, s, f.r, f.tmp, f.Tf[0], f.Tf[1], f.ld[0], f.ld[1], f.n1,
                       f.n2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(fd_z_pass_bf16<NSM>, gz, blk, 0, s, (const float*)f.tmp, f.tmp, f.Tf[2], f.Tb[2], f.ld[2],
                       f.l1, f.l2, f.l3, f.n1, f.n2, f.n3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(fd_xy_pass_bf16<NSM>, gxy, blk, 0, s, (const float*)f.tmp, f.z, f.Tb[0], f.Tb[1], f.ld[0],
                       f.ld[1], f.n1, f.n2);
    return hipGetLastError();
}

template <int PREC, int KB>
hipError_t fused_kb(const FdFusedArgs<typename G<PREC>::T>& f, hipStream_t s) {
    using T = typename G<PREC>::T;
    if (f.ldp != 16 * KB) return hipErrorInvalidValue;   // matrices padded for this block count
    hipError_t e;
    const dim3 gxy((f.n2 + 15) / 16, f.n3), gz((f.n1 * f.n2 + 15) / 16), blk(64 * KB);
    // forward y and x (T = U^T forward, U backward; each passed transposed)
    hipLaunchKernelGGL((fd_xy_pass<PREC, KB>), gxy, blk, 0, s, f.r, f.tmp, f.U[0], f.U[1], f.n1, f.n2, f.n3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // forward z, scaling, backward z (in place on tmp)
    hipLaunchKernelGGL((fd_z_pass<PREC, KB>), gz, blk, 0, s, (const T*)f.tmp, f.tmp, f.U[2], f.UT[2], f.l1, f.l2,
                       f.l3, f.n1, f.n2, f.n3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // backward y and x
    hipLaunchKernelGGL((fd_xy_pass<PREC, KB>), gxy, blk, 0, s, (const T*)f.tmp, f.z, f.UT[0], f.UT[1], f.n1, f.n2,
                       f.n3);
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
hipError_t launch_fd_fused_bf16(const FdFusedBf16Args& f, hipStream_t s) {
    const int nmax = f.n1 > f.n2 ? (f.n1 > f.n3 ? f.n1 : f.n3) : (f.n2 > f.n3 ? f.n2 : f.n3);
    for (int l = 0; l < 3; ++l)
        if (f.ld[l] % 64 || f.ld[l] < 32 * ((f.n[l] + 31) / 32)) return hipErrorInvalidValue;
    switch ((nmax + 31) / 32) {
        case 1: return fused_bf16_ns<1>(f, s);
        case 2: return fused_bf16_ns<2>(f, s);
        case 3: return fused_bf16_ns<3>(f, s);
        case 4: return fused_bf16_ns<4>(f, s);
        case 5: return fused_bf16_ns<5>(f, s);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_fd_fused(const FdFusedArgs<float>& f, hipStream_t s) { return fused_any<2>(f, s); }

}  // namespace wqfd
