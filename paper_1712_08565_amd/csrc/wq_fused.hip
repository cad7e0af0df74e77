// Fused MF-WQ stiffness apply (Algorithm 2, Section 3.2) for gfx950.
//
// One workgroup owns a 16 x 16 tile of quadrature columns (q1, q2) and a
// contiguous range of quadrature planes k, and streams through k:
//
//   trial (v~^b = B^(b) v):  each DOF plane j3 entering the z window is
//       contracted in x and y on the matrix cores (two 16x16x16 products for
//       x, three for y), giving U_x = (B2 x B-dot1) v, U_y = (B-dot2 x B1) v,
//       U_0 = (B2 x B1) v at the tile's columns; every thread keeps the last
//       p+1 planes of its column in registers and forms
//         v~^x = sum_j3 B3 U_x,  v~^y = sum_j3 B3 U_y,  v~^z = sum_j3 B-dot3 U_0.
//   pointwise: psi_ab = C_ab(x_q) v~^b, the six coefficient planes streamed
//       from HBM once, coalesced along x.
//   test, z first: every thread accumulates W3^{a3 b3}[i3][k] psi_ab into a
//       register window of the p+2 output planes i3 that plane k touches.
//   test, x and y: when plane i3 leaves the window, the nine fields of the
//       tile are contracted with W2^{a2 b2} (y) and W1^{a1 b1} (x) on the matrix
//       cores and the 16 x 16 DOF block is added to w with atomics (tiles and
//       z ranges overlap in the DOFs they touch).
//
// The banded 1D factors restricted to a tile are stored as dense 16 x 16
// blocks (DOF footprints of 16 quadrature points fit in 16 for p <= 7), held in
// LDS for the whole kernel.  FP64 uses v_mfma_f64_16x16x4f64, FP32
// v_mfma_f32_16x16x4f32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "device.h"
#include "fused.h"

namespace wqfd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int LD = 17;            // padded row length of 16 x 16 LDS blocks
constexpr int BLK = 16 * LD;
constexpr int kMaxZ = 64;         // longest z range of one workgroup (the launcher caps zchunk)

template <typename T>
struct MF;
template <>
struct MF<double> {
    using acc = d4;
    __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int drow(int kb, int v) { return kb + 4 * v; }
};
template <>
struct MF<float> {
    using acc = f4;
    __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int kb, int v) { return 4 * kb + v; }
};

// 16x16x16 product accumulated into c.  A[m][k] = At[m][k]; B[k][n] = Bt[k][n]
// (BT = false) or Bt[n][k] (BT = true).
template <typename T, bool BT>
__device__ inline typename MF<T>::acc gemm16(const T* At, const T* Bt, typename MF<T>::acc c, int cl, int kb) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const T a = At[cl * LD + 4 * s + kb];
        const T b = BT ? Bt[cl * LD + 4 * s + kb] : Bt[(4 * s + kb) * LD + cl];
        c = MF<T>::mma(a, b, c);
    }
    return c;
}

// Workgroup barrier that waits only for this wave's LDS operations: global loads
// already in flight (coefficient planes, the next DOF plane) stay in flight
// across it, unlike __syncthreads(), whose release fence drains them.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <typename T>
__device__ inline void store16(T* tile, const typename MF<T>::acc& c, int cl, int kb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) tile[MF<T>::drow(kb, v) * LD + cl] = c[v];
}

// 512 threads: two per quadrature column.  Threads 0..255 (waves 0-3) carry
// the test fields f = 3 alpha + beta = 0..4, threads 256..511 (waves 4-7) the
// fields 5..8, which halves the per-thread register windows; the x/y work of a
// retired output plane is spread over all eight waves.
template <typename T, int P>
__global__ __launch_bounds__(512, 1) void wq_apply_fused_kernel(FusedArgs<T> a) {
    constexpr int RT = P + 1;              // trial window (DOF planes)
    constexpr int RO = P + 2;              // test window (output planes)
    constexpr int CZ = 2 * RT + 4 * RO;    // z coefficients per quadrature plane
    __shared__ T sCoef[12][BLK];           // 0,1 B1t_d  2,3 B2t_d  4..7 W1t_v  8..11 W2t_v
    __shared__ T sT[6][BLK];               // V, A_0, A_1, U_x, U_y, U_0
    __shared__ T sP[9][BLK];               // psi_f of the plane being retired
    __shared__ T sR[8][BLK];               // per-wave partial output blocks
    __shared__ T sZ[kMaxZ * CZ];            // z coefficients of this workgroup's planes
    __shared__ int sB3[kMaxZ], sW3[kMaxZ];  // z window starts of these planes

    using acc_t = typename MF<T>::acc;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = tid >> 8, ct = tid & 255;
    const int cl = lane & 15, kb = lane >> 4;
    const int q1l = ct & 15, q2l = ct >> 4;

    // workgroup -> (t1, t2, zc); consecutive blocks are dealt round-robin to the
    // eight XCDs, so hand each XCD a contiguous run of neighbouring tiles
    const int nblk = gridDim.x, b = blockIdx.x;
    const int base = nblk / 8, rem = nblk % 8, xcd = b % 8, slot = b / 8;
    const int lin = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + slot;
    const int t1 = lin % a.ntx;
    const int t2 = (lin / a.ntx) % a.nty;
    const int zc = lin / (a.ntx * a.nty);
    const int k0 = zc * a.zchunk;
    const int k1 = min(a.nq3, k0 + a.zchunk);
    if (k0 >= k1) return;

    const int Q1 = t1 * 16, Q2 = t2 * 16;
    const int q1 = Q1 + q1l, q2 = Q2 + q2l;
    const bool active = q1 < a.nq1 && q2 < a.nq2;
    const int J1 = a.JX[t1], I1 = a.IX[t1], J2 = a.JY[t2], I2 = a.IY[t2];

    // coefficient blocks of this tile
    for (int idx = tid; idx < 12 * 256; idx += 512) {
        const int tl = idx >> 8, e = idx & 255;
        const T* src;
        if (tl < 2) src = a.tilesX + ((size_t)t1 * 6 + tl) * 256;
        else if (tl < 4) src = a.tilesY + ((size_t)t2 * 6 + (tl - 2)) * 256;
        else if (tl < 8) src = a.tilesX + ((size_t)t1 * 6 + 2 + (tl - 4)) * 256;
        else src = a.tilesY + ((size_t)t2 * 6 + 2 + (tl - 8)) * 256;
        sCoef[tl][(e >> 4) * LD + (e & 15)] = src[e];
    }

    // z coefficients and window starts of planes k0..k1-1, staged once: per-plane
    // scalar loads would miss the scalar cache and stall every LDS wait
    for (int idx = tid; idx < (k1 - k0) * CZ; idx += 512) sZ[idx] = a.cz[(size_t)k0 * CZ + idx];
    for (int idx = tid; idx < k1 - k0; idx += 512) {
        sB3[idx] = a.bs3[k0 + idx];
        sW3[idx] = a.wts3[k0 + idx];
    }

    // this thread's entry V[j2][j1] of DOF plane j3 (zero outside the mesh;
    // only the first half of the workgroup stages V)
    const int vj1 = J1 + q1l, vj2 = J2 + q2l;
    const bool vin = half == 0 && vj1 < a.n1 && vj2 < a.n2;
    auto load_v = [&](int j3) -> T {
        return (vin && j3 < a.n3) ? a.v[((size_t)j3 * a.n2 + vj2) * a.n1 + vj1] : T(0);
    };
    // trial contraction of a DOF plane onto the tile's columns
    auto trial_plane = [&](T val, T& ux, T& uy, T& u0) {
        if (half == 0) sT[0][q2l * LD + q1l] = val;           // V[j2][j1]
        lds_barrier();
        if (wave < 2) {                                        // A_d[j2][q1] = sum_j1 V[j2][j1] B1_d[q1][j1]
            acc_t c = {0, 0, 0, 0};
            c = gemm16<T, true>(sT[0], sCoef[wave], c, cl, kb);
            store16<T>(sT[1 + wave], c, cl, kb);
        }
        lds_barrier();
        if (wave >= 2 && wave < 5) {                           // U[q2][q1] = sum_j2 B2_d[q2][j2] A[j2][q1]
            const int u = wave - 2;                            // 0: U_x, 1: U_y, 2: U_0
            const T* At = sCoef[2 + (u == 1 ? 1 : 0)];         // U_y uses B-dot2
            const T* Bt = sT[u == 0 ? 2 : 1];                  // U_x uses A_1 (B-dot1)
            acc_t c = {0, 0, 0, 0};
            c = gemm16<T, false>(At, Bt, c, cl, kb);
            store16<T>(sT[3 + u], c, cl, kb);
        }
        lds_barrier();
        ux = sT[3][q2l * LD + q1l];
        uy = sT[4][q2l * LD + q1l];
        u0 = sT[5][q2l * LD + q1l];
    };

    // x/y test contraction of output plane i3 and atomic update of w.  A field
    // is contracted in x first (X = psi_f W1^T) and the y product takes X
    // straight from the accumulator registers as its B operand (the K index of
    // step s held by lane group kb is the accumulator row drow(kb, s), so W2 is
    // read with the same row mapping).  Waves 0-5 take one field each
    // (xx, xz, zx, zz, xy, zy), wave 6 the pair {yx, yz} sharing W2^2, wave 7 yy.
    auto xpart = [&](acc_t& X, int f) {
        const int al = f / 3, be = f % 3;
        const int v1 = 2 * (al == 0) + (be == 0);
        X = gemm16<T, true>(sP[f], sCoef[4 + v1], X, cl, kb);
    };
    auto ypart = [&](acc_t& Z, const acc_t& X, int v2) {
        const T* A = sCoef[8 + v2];
#pragma unroll
        for (int s = 0; s < 4; ++s) Z = MF<T>::mma(A[cl * LD + MF<T>::drow(kb, s)], X[s], Z);
    };
    auto flush = [&](int i3, const T* vals) {
        if (i3 < 0 || i3 >= a.n3) return;                      // uniform across the workgroup
        if (half == 0) {
#pragma unroll
            for (int f = 0; f < 5; ++f) sP[f][q2l * LD + q1l] = vals[f];
        } else {
#pragma unroll
            for (int f = 0; f < 4; ++f) sP[5 + f][q2l * LD + q1l] = vals[f];
        }
        lds_barrier();
        {
            // (field, y variant) per wave; wave 6 adds a second field
            constexpr int fw[8] = {0, 2, 6, 8, 1, 7, 3, 4};
            constexpr int vw[8] = {0, 0, 0, 0, 1, 1, 2, 3};
            acc_t X = {0, 0, 0, 0}, Z = {0, 0, 0, 0};
            xpart(X, fw[wave]);
            if (wave == 6) xpart(X, 5);
            ypart(Z, X, vw[wave]);
            store16<T>(sR[wave], Z, cl, kb);
        }
        lds_barrier();
        if (half == 0) {
            T s = T(0);
#pragma unroll
            for (int w = 0; w < 8; ++w) s += sR[w][q2l * LD + q1l];
            const int i1 = I1 + q1l, i2 = I2 + q2l;
            if (i1 < a.n1 && i2 < a.n2 && s != T(0)) atomicAdd(&a.w[((size_t)i3 * a.n2 + i2) * a.n1 + i1], s);
        }
        lds_barrier();
    };

    T Ux[RT], Uy[RT], U0[RT];
    T acc[5][RO];                                              // half 0: fields 0..4, half 1: 5..8
#pragma unroll
    for (int f = 0; f < 5; ++f)
#pragma unroll
        for (int s = 0; s < RO; ++s) acc[f][s] = T(0);

    lds_barrier();
    int tbase = sB3[0];
    int obase = sW3[0];
#pragma unroll
    for (int s = 0; s < RT; ++s) trial_plane(load_v(tbase + s), Ux[s], Uy[s], U0[s]);
    T vnext = load_v(tbase + RT);                              // next plane to enter the window

    // coefficient planes this half needs: half 0 (C11, C22, C12, C13), half 1 (C33, C13, C23)
    const size_t Nq = a.Nq;
    const size_t col = (size_t)q2 * a.nq1 + q1;
    const size_t plane = (size_t)a.nq1 * a.nq2;
    const int cpl[4] = {half == 0 ? 0 : 2, half == 0 ? 1 : 4, half == 0 ? 3 : 5, 4};
    const int ncp = half == 0 ? 4 : 3;
    T Cn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        Cn[c] = (active && c < ncp) ? a.C[cpl[c] * Nq + (size_t)k0 * plane + col] : T(0);
    for (int k = k0; k < k1; ++k) {
        // plane k's coefficients were loaded one plane ahead; issue plane k+1's now
        T C[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) C[c] = Cn[c];
        if (k + 1 < k1) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                Cn[c] = (active && c < ncp) ? a.C[cpl[c] * Nq + (size_t)(k + 1) * plane + col] : T(0);
        }
        const int bk = sB3[k - k0], wk = sW3[k - k0];
        while (tbase < bk) {                                   // slide the trial window
#pragma unroll
            for (int s = 0; s < RT - 1; ++s) {
                Ux[s] = Ux[s + 1];
                Uy[s] = Uy[s + 1];
                U0[s] = U0[s + 1];
            }
            const T vcur = vnext;
            vnext = load_v(tbase + RT + 1);                    // issue the following load early
            trial_plane(vcur, Ux[RT - 1], Uy[RT - 1], U0[RT - 1]);
            ++tbase;
        }
        while (obase < wk) {                                   // retire the oldest output plane
            T vals[5];
#pragma unroll
            for (int f = 0; f < 5; ++f) vals[f] = acc[f][0];
            flush(obase, vals);
#pragma unroll
            for (int f = 0; f < 5; ++f) {
#pragma unroll
                for (int s = 0; s < RO - 1; ++s) acc[f][s] = acc[f][s + 1];
                acc[f][RO - 1] = T(0);
            }
            ++obase;
        }
        const T* cz = sZ + (size_t)(k - k0) * CZ;
        T g[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int s = 0; s < RT; ++s) {
            g[0] += cz[s] * Ux[s];
            g[1] += cz[s] * Uy[s];
            g[2] += cz[RT + s] * U0[s];
        }
        // psi_ab = C_ab g_b; the z weight variant of field (alpha, beta) is
        // 2 [alpha = z] + [beta = z]
        T psi[5];
        int v3[5];
        if (half == 0) {        // xx, xy, xz, yx, yy with C = (C11, C22, C12, C13)
            psi[0] = C[0] * g[0]; v3[0] = 0;
            psi[1] = C[2] * g[1]; v3[1] = 0;
            psi[2] = C[3] * g[2]; v3[2] = 1;
            psi[3] = C[2] * g[0]; v3[3] = 0;
            psi[4] = C[1] * g[1]; v3[4] = 0;
        } else {                // yz, zx, zy, zz with C = (C33, C13, C23)
            psi[0] = C[2] * g[2]; v3[0] = 1;
            psi[1] = C[1] * g[0]; v3[1] = 2;
            psi[2] = C[2] * g[1]; v3[2] = 2;
            psi[3] = C[0] * g[2]; v3[3] = 3;
            psi[4] = T(0);        v3[4] = 0;
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const T* cw = cz + 2 * RT + v3[f] * RO;
#pragma unroll
            for (int s = 0; s < RO; ++s) acc[f][s] += cw[s] * psi[f];
        }
    }
#pragma unroll
    for (int s = 0; s < RO; ++s) {
        T vals[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) vals[f] = acc[f][s];
        flush(obase + s, vals);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void zero_kernel(T* __restrict__ w, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) w[i] = T(0);
}

// Length of the z range of one workgroup.  The grid is tiles x ranges
// workgroups; each range also pays for the p + 2 halo planes at its two ends,
// and the launch runs in ceil(workgroups / resident slots) rounds, so the
// estimated time is rounds x (zchunk / 2 + p + 3) DOF-plane steps.  Ranges are
// capped at kMaxZ quadrature planes (the kernel stages their z factors in LDS).
int choose_zchunk(int nq3, int tiles, int slots, int p) {
    int best = kMaxZ, best_cost = -1;
    for (int nzc = (nq3 + kMaxZ - 1) / kMaxZ; nzc <= nq3; ++nzc) {
        const int zc = (nq3 + nzc - 1) / nzc;
        const long rounds = ((long)tiles * nzc + slots - 1) / slots;
        const long cost = rounds * (zc + 2 * (p + 3));          // in half DOF-plane steps
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = zc;
        }
        if (zc <= p + 2) break;
    }
    return best;
}

template <typename T, int P>
hipError_t launch_p(FusedArgs<T> a, hipStream_t s) {
    if (a.zchunk <= 0) {
        static std::atomic<int> occ{0};
        if (occ.load() == 0) {
            int o = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, wq_apply_fused_kernel<T, P>, 512, 0);
            if (e != hipSuccess) return e;
            occ.store(o > 0 ? o : 1);
        }
        int dev = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        a.zchunk = choose_zchunk(a.nq3, a.ntx * a.nty, std::max(1, cus * occ.load()), P);
    }
    if (a.zchunk > kMaxZ) return hipErrorInvalidValue;
    const int nzc = (a.nq3 + a.zchunk - 1) / a.zchunk;
    hipLaunchKernelGGL((wq_apply_fused_kernel<T, P>), dim3(a.ntx * a.nty * nzc), dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_fused_apply(const FusedArgs<T>& a, int p, hipStream_t s) {
    const size_t N = (size_t)a.n1 * a.n2 * a.n3;
    size_t g = (N + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(zero_kernel<T>, dim3((unsigned)g), dim3(256), 0, s, a.w, N);
    switch (p) {
        case 2: return launch_p<T, 2>(a, s);
        case 3: return launch_p<T, 3>(a, s);
        case 4: return launch_p<T, 4>(a, s);
        case 5: return launch_p<T, 5>(a, s);
        case 6: return launch_p<T, 6>(a, s);
        case 7: return launch_p<T, 7>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fused_apply<double>(const FusedArgs<double>&, int, hipStream_t);
template hipError_t launch_fused_apply<float>(const FusedArgs<float>&, int, hipStream_t);

}  // namespace wqfd
