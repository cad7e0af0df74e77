// Fused MF-WQ stiffness apply (Algorithm 2, Section 3.2) for gfx950.
//
// One workgroup owns a 16 x 16 tile of quadrature columns (q1, q2) and a
// contiguous range of quadrature planes k, and streams through k:
//
//   trial (v~^b = B^(b) v):  each DOF plane j3 entering the z window is
//       contracted in x (B1 and B-dot1, by the MFMA waves on the vector units
//       with the exact band of p+1 functions per point) and then in y (by the
//       column waves as the plane enters their window, exact band again),
//       giving U_x = (B2 x B-dot1) v, U_y = (B-dot2 x B1) v, U_0 = (B2 x B1) v
//       at the tile's columns; every thread keeps the last p+1 planes of its
//       column in registers and forms
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
// Reaction term (the mass apply of Algorithm 1, M~ = W^(00) D B): its values
// at the points are B3 applied to U_0, the window the z-derivative waves already
// hold, and its x and y test rules W1^{00}, W2^{00} are those of the field zz.
// So the z-derivative waves add c_q (B3 . window) times the W3^{00} column into
// the zz ring, and nothing else changes; the transposed kernel mirrors this.
//
// The banded 1D factors restricted to a tile are stored as dense 16 x 16
// blocks (DOF footprints of 16 quadrature points fit in 16 for p <= 7), held in
// LDS for the whole kernel.  FP64 uses v_mfma_f64_16x16x4f64, FP32
// v_mfma_f32_16x16x4f32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "buffer.h"
#include "device.h"
#include "fused.h"

namespace wqfd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int LD = 17;            // padded row length of 16 x 16 LDS blocks
constexpr int BLK = 16 * LD;
constexpr int kMaxZ = FUSED_MAX_Z;   // longest z range of one workgroup

// s_waitcnt immediate for gfx9: vmcnt 0, expcnt and lgkmcnt left at their maxima
constexpr int kVmcnt0 = 0x0F70;

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

// Calls f(std::integral_constant<int, i>) for a wave-uniform i in [LO, HI) by a
// binary tree of scalar branches, so that f touches one fixed element of a
// register array.  (A run-time index into such an array makes the compiler
// place it in scratch memory or select over every element; the empty volatile
// asm keeps each leaf a branch target instead of a select.)
template <int LO, int HI, typename F>
__device__ __forceinline__ void slot_dispatch(int i, F&& f) {
    if constexpr (HI - LO == 1) {
        f(std::integral_constant<int, LO>{});
        asm volatile("");
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (i < MID)
            slot_dispatch<LO, MID>(i, f);
        else
            slot_dispatch<MID, HI>(i, f);
    }
}

// 16x16x16 product accumulated into c.  A[m][k] = At[m][k]; B[k][n] = Bt[k][n]
// (BT = false) or Bt[n][k] (BT = true).
template <typename T, bool BT>
__device__ inline typename MF<T>::acc gemm16(const T* At, const T* Bt, typename MF<T>::acc c, int cl, int kb) {
    T a[4], b[4];                        // all operands first: one LDS round trip
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        a[s] = At[cl * LD + 4 * s + kb];
        b[s] = BT ? Bt[cl * LD + 4 * s + kb] : Bt[(4 * s + kb) * LD + cl];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) c = MF<T>::mma(a[s], b[s], c);
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

// Set-up of a workgroup: the tile's twelve factor blocks (three entries per
// thread) and the range's z coefficients.  All loads are issued together and
// written to LDS afterwards, so the set-up costs one memory latency.
template <typename T, int CZ>
struct SetupRegs {
    static constexpr int ZL = (kMaxZ * CZ + 1023) / 1024;
    T cv[3];
    T zv[ZL];
};

template <typename T>
__device__ inline const T* setup_src(const FusedArgs<T>& a, int tl, int t1, int t2) {
    if (tl < 2) return a.tilesX + ((size_t)t1 * 6 + tl) * 256;                 // B1_d
    if (tl < 4) return a.tilesY + ((size_t)t2 * 6 + (tl - 2)) * 256;           // B2_d
    if (tl < 8) return a.tilesX + ((size_t)t1 * 6 + 2 + (tl - 4)) * 256;       // W1_v
    return a.tilesY + ((size_t)t2 * 6 + 2 + (tl - 8)) * 256;                   // W2_v
}

template <typename T, int CZ>
__device__ inline void setup_load(SetupRegs<T, CZ>& su, const FusedArgs<T>& a, int tid, int t1, int t2, int k0,
                                  int k1, const T* cz) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int idx = tid + 1024 * i;
        su.cv[i] = setup_src(a, idx >> 8, t1, t2)[idx & 255];
    }
    const int nz = (k1 - k0) * CZ;
#pragma unroll
    for (int i = 0; i < SetupRegs<T, CZ>::ZL; ++i) {
        const int idx = tid + 1024 * i;
        su.zv[i] = idx < nz ? cz[(size_t)k0 * CZ + idx] : T(0);
    }
}

template <typename T, int CZ>
__device__ inline void setup_store(const SetupRegs<T, CZ>& su, T (*sCoef)[BLK], T* sZ, int tid, int k0, int k1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int idx = tid + 1024 * i, e = idx & 255;
        sCoef[idx >> 8][(e >> 4) * LD + (e & 15)] = su.cv[i];
    }
    const int nz = (k1 - k0) * CZ;
#pragma unroll
    for (int i = 0; i < SetupRegs<T, CZ>::ZL; ++i) {
        const int idx = tid + 1024 * i;
        if (idx < nz) sZ[idx] = su.zv[i];
    }
}

// 1024 threads in two roles, one barrier per interval (one quadrature plane).
//   Column waves 0-11: wave group beta = wave / 4 (trial derivative direction x,
//     y, z) owns the fields f = 3 alpha + beta, alpha = x, y, z, of all 256
//     columns; a thread keeps the window of the p+1 trial planes of U_beta
//     (U_x, U_y or U_0) it needs, the coefficients C_(alpha beta) of the
//     current plane and a register ring of the p+2 output planes per field.
//   MFMA waves 12-15: one interval behind the column waves, they turn staged DOF
//     planes into U planes (a ring of NU planes in LDS), contract retired
//     output planes in x and y, and add the 16 x 16 DOF block to w.
// Every buffer a role writes in an interval is read by the other role only
// after the closing barrier, and is not rewritten before the reader's interval
// has ended; the schedule is computed identically by every wave.
template <typename T, int P, bool MASS>
__global__ __launch_bounds__(1024, 1) void wq_apply_fused_kernel(FusedArgs<T> a) {
    constexpr int RT = P + 1;              // trial window (DOF planes)
    constexpr int RO = P + 2;              // test window (output planes)
    constexpr int CZ = 2 * RT + 4 * RO;    // z coefficients per quadrature plane
    constexpr int NU = 3;                  // U planes in flight
    __shared__ T sCoef[12][BLK];           // 0,1 B1t_d  2,3 B2t_d  4..7 W1t_v  8..11 W2t_v
    __shared__ T sV[2][BLK];               // staged DOF planes
    __shared__ T sA[NU][2][BLK];           // x products A_0, A_1 of produced planes
    __shared__ T sP[2][9][BLK];            // psi_f of retired output planes
    __shared__ T sR[2][5][BLK];            // partial output blocks of the x/y test contraction
    __shared__ T sZ[kMaxZ * CZ];           // z coefficients of this workgroup's planes

    using acc_t = typename MF<T>::acc;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: role branches are scalar
    const bool mrole = wave >= 12;         // MFMA role (wave-uniform)
    const int ct = tid & 255;              // column of a column thread / lane slot of an MFMA thread
    const int cl = lane & 15, kb = lane >> 4;
    const int q1l = ct & 15, q2l = ct >> 4;
    const int beta = wave >> 2;            // column waves: 0, 1, 2
    const int mw = wave - 12;              // MFMA waves: 0..3

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
    const int J1 = __builtin_amdgcn_readfirstlane(a.JX[t1]), I1 = __builtin_amdgcn_readfirstlane(a.IX[t1]);
    const int J2 = __builtin_amdgcn_readfirstlane(a.JY[t2]), I2 = __builtin_amdgcn_readfirstlane(a.IY[t2]);

    // coefficient blocks of this tile and z coefficients: loads issued here, LDS
    // written just before the first barrier
    SetupRegs<T, CZ> su;
    setup_load(su, a, tid, t1, t2, k0, k1, a.cz);
    const int r0 = a.sched_off[zc], nrec = a.sched_off[zc + 1] - r0;
    // the range's interval records, one per lane (at most 64, checked on the
    // host); interval r's fields are read with readlane into scalar registers
    const int* lrec = a.sched + FUSED_REC * (size_t)(r0 + (lane < nrec ? lane : 0));
    const int Rf = lrec[0], Rred = lrec[2], Rts = lrec[3], Rev = lrec[4], Rczo = lrec[5], Rc0 = lrec[6],
              Rc1 = lrec[7];

    // ---- MFMA-role helpers ------------------------------------------------
    // A operand for a product whose B operand is an accumulator: the K index of
    // step s held by lane group kb is the accumulator row drow(kb, s)
    auto ld_accA = [&](T (&av)[4], const T* A) {
#pragma unroll
        for (int s = 0; s < 4; ++s) av[s] = A[cl * LD + MF<T>::drow(kb, s)];
    };
    auto mm_acc = [&](acc_t& Z, const T (&av)[4], const acc_t& X) {
#pragma unroll
        for (int s = 0; s < 4; ++s) Z = MF<T>::mma(av[s], X[s], Z);
    };
    auto v1_of = [](int f) { return 2 * (f / 3 == 0) + (f % 3 == 0); };   // 2[alpha = x] + [beta = x]

    // ---- column-role state ------------------------------------------------
    T Uw[RT];                               // trial window of U_beta
    T acc[3][RO];                           // output ring of fields 3 alpha + beta
#pragma unroll
    for (int s = 0; s < RT; ++s) Uw[s] = T(0);
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int s = 0; s < RO; ++s) acc[al][s] = T(0);
    // coefficient planes C_(alpha beta) of this thread's three fields
    // (stored planes C11, C22, C33, C12, C13, C23 = 0..5; the offsets are wave-uniform)
    const int pidx = __builtin_amdgcn_readfirstlane(beta == 0 ? 0x430 : beta == 1 ? 0x513 : 0x254);
    const size_t Nq = a.Nq;
    const size_t plane = (size_t)a.nq1 * a.nq2;
    const size_t poff[3] = {((pidx >> 0) & 15) * Nq, ((pidx >> 4) & 15) * Nq, ((pidx >> 8) & 15) * Nq};
    // Coefficients are loaded one interval ahead (an interval covers at most two
    // quadrature planes) into two register slots, each reloaded right after its
    // use at a fixed point of the interval.  The loads are unconditional (columns
    // outside the grid read a clamped address; their trial values are exactly 0),
    // so every interval issues the same loads in the same order and a use waits
    // only for its own slot, not for the loads issued after it.
    const unsigned cbyte = (unsigned)(min(q2, a.nq2 - 1) * a.nq1 + min(q1, a.nq1 - 1)) * (unsigned)sizeof(T);
    const unsigned pbytes = (unsigned)(plane * sizeof(T));
    // With the reaction term a fourth slot holds c_q = alpha det J for the z group;
    // the x and y groups load their third plane into it again (a cache hit, value
    // unused), so every column wave keeps the same load sequence.
    constexpr int NC = MASS ? 4 : 3;
    __amdgpu_buffer_rsrc_t rC[NC];
    rC[0] = buf_rsrc(a.C + poff[0]);
    rC[1] = buf_rsrc(a.C + poff[1]);
    rC[2] = buf_rsrc(a.C + poff[2]);
    if constexpr (MASS) rC[3] = buf_rsrc(beta == 2 ? a.Cm : a.C + poff[2]);
    auto cload3 = [&](T (&dst)[NC], int kq) {             // kq: a plane of this range
#pragma unroll
        for (int al = 0; al < NC; ++al) dst[al] = buf_load<T>(rC[al], cbyte, (unsigned)kq * pbytes);
    };

    // one quadrature plane of column work: g = (z trial row) . window,
    // psi_alpha = C_(alpha beta) g, ring += (z test rows) psi; czo = offset of
    // the plane's z coefficients
    auto valu_plane = [&](int czo, const T (&C)[NC]) {
        const T* cz = sZ + czo;
        const T* ct3 = cz + (beta == 2 ? RT : 0);               // B3 row, or B-dot3 for beta = z
        T g = T(0);
#pragma unroll
        for (int s = 0; s < RT; ++s) g += ct3[s] * Uw[s];
        // z weight variant of field (alpha, beta): 2 [alpha = z] + [beta = z]
        const T* w01 = cz + 2 * RT + (beta == 2 ? 1 : 0) * RO;
        const T* w2 = cz + 2 * RT + (beta == 2 ? 3 : 2) * RO;
        const T p0 = C[0] * g, p1 = C[1] * g, p2 = C[2] * g;
#pragma unroll
        for (int s = 0; s < RO; ++s) {
            acc[0][s] += w01[s] * p0;
            acc[1][s] += w01[s] * p1;
            acc[2][s] += w2[s] * p2;
        }
        if constexpr (MASS) {
            if (beta == 2) {                                    // reaction: value (B3 row) x c_q x W3^{00}
                T gm = T(0);
#pragma unroll
                for (int s = 0; s < RT; ++s) gm += cz[s] * Uw[s];
                const T pm = C[3] * gm;
                const T* w00 = cz + 2 * RT;
#pragma unroll
                for (int s = 0; s < RO; ++s) acc[2][s] += w00[s] * pm;
            }
        }
    };

    // band starts (MFMA waves: of point q1 = tid % 16; column waves: of q2) and
    // the column waves' first coefficient slots, loaded with the set-up
    const int bX = a.bandX[t1 * 16 + (tid & 15)], bY = a.bandY[t2 * 16 + q2l];
    T Cs[2][NC];
    if (!mrole) {
        cload3(Cs[0], k0);
        cload3(Cs[1], min(k0 + 1, k1 - 1));
    }
    setup_store(su, sCoef, sZ, tid, k0, k1);
    lds_barrier();

    // ---- the interval loop: every wave walks the same host-computed records ----
    if (mrole) {
        // wave 15 (contraction, reduction and atomics) ends each interval last:
        // it gets the first issue slots of its SIMD
        if (mw == 3) __builtin_amdgcn_s_setprio(2);
        // x/y test contraction of the plane retired in the previous interval.
        // Fields sharing the y weight variant v2 = 2[alpha = y] + [beta = y] are
        // summed after their x products (X = sum_f psi_f W1^(v1_f)T, Z = W2^(v2) X):
        //   wave 12: {xx, xz};  wave 13: {zx, zz} (v2 = 0);  wave 14: {xy, zy} (v2 = 1);
        //   wave 15: {yx, yz} (v2 = 2); {yy} (v2 = 3) runs on column wave 2, whose SIMD
        //   holds the MFMA wave with no staging or reduction duties.
        // The factor operands are the same in every interval and stay in registers.
        // Wave 15 also sums the partial blocks and adds them to w: it issues no
        // loads, so its atomics never delay a wait for loaded data.
        const int fa = mw == 0 ? 0 : mw == 1 ? 6 : mw == 2 ? 1 : 3;
        const int fb = mw == 0 ? 2 : mw == 1 ? 8 : mw == 2 ? 7 : 5;
        const int v2 = mw == 0 ? 0 : mw == 1 ? 0 : mw == 2 ? 1 : 2;
        T ba[4], bb[4], w2a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ba[q] = sCoef[4 + v1_of(fa)][cl * LD + 4 * q + kb];
            bb[q] = sCoef[4 + v1_of(fb)][cl * LD + 4 * q + kb];
        }
        ld_accA(w2a, sCoef[8 + v2]);
        // x products of the staged plane on the vector units, exact band:
        // thread (q1, j2) = (mt & 15, mt >> 4) forms A_d[j2][q1] =
        // sum_s B1_d[q1][js + s] V[j2][js + s] over the p + 1 functions at point q1
        const int mt = tid - 768, xq1 = mt & 15, xj2 = mt >> 4;
        const int jsx = bX;
        T cb0[RT], cb1[RT];
#pragma unroll
        for (int s = 0; s < RT; ++s) {
            cb0[s] = sCoef[0][xq1 * LD + jsx + s];
            cb1[s] = sCoef[1][xq1 * LD + jsx + s];
        }
        // waves 12 and 13 stage the DOF planes (entries lane + 64 (2 mw + q) of the
        // 16 x 16 block); each plane is loaded at the previous staging, at least one
        // interval earlier, from a clamped address, and masked when it is stored
        const bool stager = mw < 2;
        T vq[2];
        unsigned voff[2];
        bool vok[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = lane + 64 * (2 * mw + q);
            const int j1 = J1 + (e & 15), j2 = J2 + (e >> 4);
            vok[q] = j1 < a.n1 && j2 < a.n2;
            voff[q] = (unsigned)(min(j2, a.n2 - 1) * a.n1 + min(j1, a.n1 - 1));
        }
        const unsigned vpbytes = (unsigned)((size_t)a.n1 * a.n2 * sizeof(T));
        const __amdgpu_buffer_rsrc_t rV = buf_rsrc(a.v);
        auto vload = [&](int j3) {
            const unsigned so = (unsigned)min(max(j3, 0), a.n3 - 1) * vpbytes;
#pragma unroll
            for (int q = 0; q < 2; ++q) vq[q] = buf_load<T>(rV, voff[q] * (unsigned)sizeof(T), so);
        };
        if (stager && nrec > 0) vload(__builtin_amdgcn_readlane(Rts, 0));
        for (int r = 0; r < nrec; ++r) {
            const int fl = __builtin_amdgcn_readlane(Rf, r), red_i3 = __builtin_amdgcn_readlane(Rred, r),
                      ts = __builtin_amdgcn_readlane(Rts, r);
            if ((fl >> 7) & 1) {                                 // produce: x products of plane tprod
                const int vs = (fl >> 17) & 1, us = (fl >> 18) & 3;
                T a0 = T(0), a1 = T(0);
#pragma unroll
                for (int s = 0; s < RT; ++s) {
                    const T vv = sV[vs][xj2 * LD + jsx + s];
                    a0 += cb0[s] * vv;
                    a1 += cb1[s] * vv;
                }
                sA[us][0][xj2 * LD + xq1] = a0;
                sA[us][1][xj2 * LD + xq1] = a1;
            }
            if ((fl >> 9) & 1) {
                const int ps = (fl >> 14) & 1, rs = (fl >> 16) & 1;
                T xa[4], xb[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    xa[q] = sP[ps][fa][cl * LD + 4 * q + kb];
                    xb[q] = sP[ps][fb][cl * LD + 4 * q + kb];
                }
                acc_t X = {0, 0, 0, 0}, Z = {0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q) X = MF<T>::mma(xa[q], ba[q], X);
#pragma unroll
                for (int q = 0; q < 4; ++q) X = MF<T>::mma(xb[q], bb[q], X);
                mm_acc(Z, w2a, X);
                store16<T>(sR[rs][mw], Z, cl, kb);
            }
            if (stager && ((fl >> 8) & 1)) {
                const int sl = (fl >> 20) & 1;
                const bool zin = ts >= 0 && ts < a.n3;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int e = lane + 64 * (2 * mw + q);
                    sV[sl][(e >> 4) * LD + (e & 15)] = (vok[q] && zin) ? vq[q] : T(0);
                }
                vload(ts + 1);
            }
            if (mw == 3 && ((fl >> 10) & 1)) {
                const int rs = (fl >> 15) & 1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = lane + 64 * q;
                    const int el = (e >> 4) * LD + (e & 15);
                    const T sum = sR[rs][0][el] + sR[rs][1][el] + sR[rs][2][el] + sR[rs][3][el] + sR[rs][4][el];
                    const int i1 = I1 + (e & 15), i2 = I2 + (e >> 4);
                    if (i1 < a.n1 && i2 < a.n2 && sum != T(0))
                        atomicAdd(&a.w[((size_t)red_i3 * a.n2 + i2) * a.n1 + i1], sum);
                }
            }
            lds_barrier();
        }
    } else {
        // Besides their planes, column waves form the entering U value themselves
        // (y products with the exact band: U_beta[q2][q1] = sum_s B2_e[q2][js + s]
        // A_b[js + s][q1]; beta = x: B2 A_1, y: B-dot2 A_0, z: B2 A_0) and wave 2
        // contracts the {yy} field of the retired plane.
        const int jsy = bY;
        const T* cbY = sCoef[beta == 1 ? 3 : 2] + q2l * LD + jsy;
        const int ab = beta == 0 ? 1 : 0;
        // slot j holds plane kq + j of the interval.  The first interval's slots
        // are waited for before the loop, so the waits inside it are set by the
        // loop's own load order alone (use of a slot: the other slot's three
        // loads may still be in flight).
        __builtin_amdgcn_s_waitcnt(kVmcnt0);
        for (int r = 0; r < nrec; ++r) {
            const int fl = __builtin_amdgcn_readlane(Rf, r), ev = __builtin_amdgcn_readlane(Rev, r);
            const int czo = __builtin_amdgcn_readlane(Rczo, r), cn0 = __builtin_amdgcn_readlane(Rc0, r),
                      cn1 = __builtin_amdgcn_readlane(Rc1, r);
            if (wave == 2 && ((fl >> 9) & 1)) {
                const int ps = (fl >> 14) & 1, rs = (fl >> 16) & 1;
                const T* Bt = sCoef[4 + v1_of(4)];
                acc_t X = {0, 0, 0, 0}, Z = {0, 0, 0, 0};
                {
                    T xv[4], bv[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        xv[q] = sP[ps][4][cl * LD + 4 * q + kb];
                        bv[q] = Bt[cl * LD + 4 * q + kb];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) X = MF<T>::mma(xv[q], bv[q], X);
                }
                T wv[4];
                ld_accA(wv, sCoef[8 + 3]);
                mm_acc(Z, wv, X);
                store16<T>(sR[rs][4], Z, cl, kb);
            }

#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if ((ev >> (3 * j)) & 1) {                       // window entry
#pragma unroll
                    for (int s = 0; s < RT - 1; ++s) Uw[s] = Uw[s + 1];
                    const T* A = sA[(fl >> 11) & 3][ab] + jsy * LD + q1l;
                    T u = T(0);
#pragma unroll
                    for (int s = 0; s < RT; ++s) u += cbY[s] * A[s * LD];
                    Uw[RT - 1] = u;
                }
                if ((ev >> (3 * j + 1)) & 1) {                   // retirement
                    if ((fl >> 6) & 1) {
                        const int ps = (fl >> 13) & 1;
#pragma unroll
                        for (int al = 0; al < 3; ++al) sP[ps][3 * al + beta][q2l * LD + q1l] = acc[al][0];
                    }
#pragma unroll
                    for (int al = 0; al < 3; ++al) {
#pragma unroll
                        for (int s = 0; s < RO - 1; ++s) acc[al][s] = acc[al][s + 1];
                        acc[al][RO - 1] = T(0);
                    }
                }
                if ((ev >> (3 * j + 2)) & 1) valu_plane(czo + j * CZ, Cs[j]);
                cload3(Cs[j], j ? cn1 : cn0);                    // plane j of the next interval
            }
            lds_barrier();
        }
    }
}

// ---------------------------------------------------------------------------
// Fused transposed apply w = K~^T v = sum_ab B^(b)T D^(ab) W^(ab)T v, the same
// pipeline with the roles of the factors exchanged:
//   input side (MFMA waves): each DOF plane i3 of v entering the z window is
//     transformed in x and y with the transposed weights of all nine fields,
//       Y_f[q2][q1] = sum_i2 W2^(v2)[i2][q2] sum_i1 W1^(v1)[i1][q1] V[i2][i1],
//     (one x product per weight variant v1 shared by its fields), into a ring
//     of NU planes of nine blocks in LDS;
//   column waves (group beta): keep the last p+2 planes of Y_(alpha beta),
//     alpha = x, y, z, per column, contract them with W3 (z), form
//     phi_beta = sum_alpha C_(alpha beta) Y_(alpha beta) and accumulate
//     B3^(b3)T phi_beta into a ring of the p+1 output planes it touches;
//   retired output planes (3 fields): x and y products with the transposed B
//     factors (fields x and z share B2 and are summed before it) and atomics.
// From p = FUSED_RING_MIN_P the column waves' windows are fixed register rings
// (an entering plane is written into its slot, a retired slot is emptied in
// place, slots from the interval records and z rows stored in slot order):
// shifting them costs about the same issue time, but spills registers there.
// Operands with transposed LDS reads use the accumulator row mapping as K
// index, as in the forward kernel.
template <typename T, int P, bool MASS>
__global__ __launch_bounds__(1024, 1) void wq_apply_T_fused_kernel(FusedArgs<T> a) {
    constexpr int RT = P + 1;              // output ring (DOF planes, B band)
    constexpr int RO = P + 2;              // input window (DOF planes, W band)
    constexpr int CZ = 2 * RT + 4 * RO;    // z coefficients per quadrature plane
    constexpr int NU = 3;                  // input planes in flight
    constexpr bool RING = P >= FUSED_RING_MIN_P;   // windows as fixed register rings
    __shared__ T sCoef[12][BLK];           // 0,1 B1t_d  2,3 B2t_d  4..7 W1t_v  8..11 W2t_v
    __shared__ T sV[2][BLK];               // staged planes of v (input block IX, IY)
    __shared__ T sU[NU][9][BLK];           // Y_f of produced planes
    __shared__ T sP[2][3][BLK];            // phi_beta of retired output planes
    __shared__ T sR[2][2][BLK];            // partial output blocks
    __shared__ T sZ[kMaxZ * CZ];           // z coefficients of this workgroup's planes

    using acc_t = typename MF<T>::acc;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: role branches are scalar
    const bool mrole = wave >= 12;
    const int ct = tid & 255;
    const int cl = lane & 15, kb = lane >> 4;
    const int q1l = ct & 15, q2l = ct >> 4;
    const int beta = wave >> 2;
    const int mw = wave - 12;

    const int nblk = gridDim.x, b = blockIdx.x;
    const int base = nblk / 8, rem = nblk % 8, xcd = b % 8, slot = b / 8;
    const int lin = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + slot;
    const int t1 = lin % a.ntx;
    const int t2 = (lin / a.ntx) % a.nty;
    const int zc = lin / (a.ntx * a.nty);
    const int k0 = zc * a.zchunk;
    const int k1 = min(a.nq3, k0 + a.zchunk);
    if (k0 >= k1) return;

    const int q1 = t1 * 16 + q1l, q2 = t2 * 16 + q2l;
    const int J1 = __builtin_amdgcn_readfirstlane(a.JX[t1]), I1 = __builtin_amdgcn_readfirstlane(a.IX[t1]);
    const int J2 = __builtin_amdgcn_readfirstlane(a.JY[t2]), I2 = __builtin_amdgcn_readfirstlane(a.IY[t2]);

    SetupRegs<T, CZ> su;
    setup_load(su, a, tid, t1, t2, k0, k1, a.czT);
    const int r0 = a.schedT_off[zc], nrec = a.schedT_off[zc + 1] - r0;
    // the range's interval records, one per lane (at most 64, checked on the
    // host); interval r's fields are read with readlane into scalar registers
    const int* lrec = a.schedT + FUSED_REC * (size_t)(r0 + (lane < nrec ? lane : 0));
    const int Rf = lrec[0], Rred = lrec[2], Rts = lrec[3], Rev = lrec[4], Rczo = lrec[5], Rc0 = lrec[6],
              Rc1 = lrec[7];

    // A operand read transposed from a [k][m] LDS block, K index = accumulator row
    auto ld_accAt = [&](T (&av)[4], const T* A) {
#pragma unroll
        for (int s = 0; s < 4; ++s) av[s] = A[MF<T>::drow(kb, s) * LD + cl];
    };
    auto mm_acc = [&](acc_t& Z, const T (&av)[4], const acc_t& X) {
#pragma unroll
        for (int s = 0; s < 4; ++s) Z = MF<T>::mma(av[s], X[s], Z);
    };
    // x product with the B operand read as [k][n] from LDS: c += A[m][k] B[k][n]
    auto mm_x = [&](acc_t& c, const T* A, const T* B) {
        T av[4], bv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            av[s] = A[cl * LD + 4 * s + kb];
            bv[s] = B[(4 * s + kb) * LD + cl];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) c = MF<T>::mma(av[s], bv[s], c);
    };

    setup_store(su, sCoef, sZ, tid, k0, k1);
    lds_barrier();

    if (mrole) {
        // the MFMA waves' chains are the long ones of an interval (measured: a
        // higher issue priority helps up to p = 5)
        if constexpr (P <= 5) __builtin_amdgcn_s_setprio(1);
        // MFMA waves.  Input planes: the x product with W1^(v1), then the y
        // products of the fields with that v1 (field f = 3 alpha + beta has
        // v1 = 2[alpha = x] + [beta = x], v2 = 2[alpha = y] + [beta = y]):
        //   wave 12: v1 = 0 -> {yy, yz, zy, zz};  wave 13: v1 = 1 -> {yx, zx};
        //   wave 14: v1 = 2 -> {xy, xz} and v1 = 3 -> {xx}.
        // Retired planes: wave 13 field y (B1, then B-dot2), wave 15 fields x and z
        // (X = R_x B-dot1 + R_z B1, then B2), wave 15 also reduces and adds to w.
        // Wave 14 stages the planes of v (each loaded at the previous staging).
        const bool stager = mw == 2;
        T vq[4];
        unsigned voff[4];
        bool vok[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = lane + 64 * q;
            const int i1 = I1 + (e & 15), i2 = I2 + (e >> 4);
            vok[q] = i1 < a.n1 && i2 < a.n2;
            voff[q] = (unsigned)(min(i2, a.n2 - 1) * a.n1 + min(i1, a.n1 - 1));
        }
        const unsigned vpbytes = (unsigned)((size_t)a.n1 * a.n2 * sizeof(T));
        const __amdgpu_buffer_rsrc_t rV = buf_rsrc(a.v);
        auto vload = [&](int i3) {
            const unsigned so = (unsigned)min(max(i3, 0), a.n3 - 1) * vpbytes;
#pragma unroll
            for (int q = 0; q < 4; ++q) vq[q] = buf_load<T>(rV, voff[q] * (unsigned)sizeof(T), so);
        };
        if (stager && nrec > 0) vload(__builtin_amdgcn_readlane(Rts, 0));
        // y products of one x result: fields given as (f, v2) pairs
        auto yprods = [&](const acc_t& A, int us, int f, int v2) {
            T wv[4];
            ld_accAt(wv, sCoef[8 + v2]);
            acc_t Y = {0, 0, 0, 0};
            mm_acc(Y, wv, A);
            store16<T>(sU[us][f], Y, cl, kb);
        };
        for (int r = 0; r < nrec; ++r) {
            const int fl = __builtin_amdgcn_readlane(Rf, r), red_i3 = __builtin_amdgcn_readlane(Rred, r),
                      ts = __builtin_amdgcn_readlane(Rts, r);
            if (((fl >> 7) & 1) && mw < 3) {
                const int vs = (fl >> 17) & 1, us = (fl >> 18) & 3;
                if (mw == 0) {
                    acc_t A = {0, 0, 0, 0};
                    mm_x(A, sV[vs], sCoef[4 + 0]);
                    yprods(A, us, 4, 3);
                    yprods(A, us, 5, 2);
                    yprods(A, us, 7, 1);
                    yprods(A, us, 8, 0);
                } else if (mw == 1) {
                    acc_t A = {0, 0, 0, 0};
                    mm_x(A, sV[vs], sCoef[4 + 1]);
                    yprods(A, us, 3, 2);
                    yprods(A, us, 6, 0);
                } else {
                    acc_t A2 = {0, 0, 0, 0}, A3 = {0, 0, 0, 0};
                    mm_x(A2, sV[vs], sCoef[4 + 2]);
                    mm_x(A3, sV[vs], sCoef[4 + 3]);
                    yprods(A2, us, 1, 1);
                    yprods(A2, us, 2, 0);
                    yprods(A3, us, 0, 0);
                }
            }
            if (((fl >> 9) & 1) && (mw == 1 || mw == 3)) {
                const int ps = (fl >> 14) & 1, rs = (fl >> 16) & 1;
                acc_t X = {0, 0, 0, 0}, Z = {0, 0, 0, 0};
                T wv[4];
                if (mw == 1) {                                   // beta = y: B1, then B-dot2
                    mm_x(X, sP[ps][1], sCoef[0]);
                    ld_accAt(wv, sCoef[3]);
                } else {                                         // beta = x (B-dot1) and z (B1), then B2
                    mm_x(X, sP[ps][0], sCoef[1]);
                    mm_x(X, sP[ps][2], sCoef[0]);
                    ld_accAt(wv, sCoef[2]);
                }
                mm_acc(Z, wv, X);
                store16<T>(sR[rs][mw == 1 ? 0 : 1], Z, cl, kb);
            }
            if (stager && ((fl >> 8) & 1)) {
                const int sl = (fl >> 20) & 1;
                const bool zin = ts >= 0 && ts < a.n3;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = lane + 64 * q;
                    sV[sl][(e >> 4) * LD + (e & 15)] = (vok[q] && zin) ? vq[q] : T(0);
                }
                vload(ts + 1);
            }
            if (mw == 3 && ((fl >> 10) & 1)) {
                const int rs = (fl >> 15) & 1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = lane + 64 * q;
                    const int el = (e >> 4) * LD + (e & 15);
                    const T sum = sR[rs][0][el] + sR[rs][1][el];
                    const int j1 = J1 + (e & 15), j2 = J2 + (e >> 4);
                    if (j1 < a.n1 && j2 < a.n2 && sum != T(0))
                        atomicAdd(&a.w[((size_t)red_i3 * a.n2 + j2) * a.n1 + j1], sum);
                }
            }
            lds_barrier();
        }
    } else {
        // column waves: fields (alpha, beta), alpha = x, y, z
        T Yw[3][RO];                        // input window of Y_(alpha beta)
        T orng[RT];                         // output ring of B3^T phi_beta
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
            for (int s = 0; s < RO; ++s) Yw[al][s] = T(0);
#pragma unroll
        for (int s = 0; s < RT; ++s) orng[s] = T(0);
        const int pidx = __builtin_amdgcn_readfirstlane(beta == 0 ? 0x430 : beta == 1 ? 0x513 : 0x254);
        const size_t Nq = a.Nq;
        const size_t plane = (size_t)a.nq1 * a.nq2;
        const size_t poff[3] = {((pidx >> 0) & 15) * Nq, ((pidx >> 4) & 15) * Nq, ((pidx >> 8) & 15) * Nq};
        // coefficient slots loaded one interval ahead, as in the forward kernel
        const unsigned cbyte = (unsigned)(min(q2, a.nq2 - 1) * a.nq1 + min(q1, a.nq1 - 1)) * (unsigned)sizeof(T);
        const unsigned pbytes = (unsigned)(plane * sizeof(T));
        // reaction plane in a fourth slot, loaded as in the forward kernel
        constexpr int NC = MASS ? 4 : 3;
        __amdgpu_buffer_rsrc_t rC[NC];
        rC[0] = buf_rsrc(a.C + poff[0]);
        rC[1] = buf_rsrc(a.C + poff[1]);
        rC[2] = buf_rsrc(a.C + poff[2]);
        if constexpr (MASS) rC[3] = buf_rsrc(beta == 2 ? a.Cm : a.C + poff[2]);
        auto cload3 = [&](T (&dst)[NC], int kq) {
#pragma unroll
            for (int al = 0; al < NC; ++al) dst[al] = buf_load<T>(rC[al], cbyte, (unsigned)kq * pbytes);
        };
        auto valu_plane = [&](int czo, const T (&C)[NC]) {
            const T* cz = sZ + czo;
            // z weight variant of field (alpha, beta): 2 [alpha = z] + [beta = z]
            const T* w01 = cz + 2 * RT + (beta == 2 ? 1 : 0) * RO;
            const T* w2 = cz + 2 * RT + (beta == 2 ? 3 : 2) * RO;
            T y0 = T(0), y1 = T(0), y2 = T(0);
#pragma unroll
            for (int s = 0; s < RO; ++s) {
                y0 += w01[s] * Yw[0][s];
                y1 += w01[s] * Yw[1][s];
                y2 += w2[s] * Yw[2][s];
            }
            const T phi = C[0] * y0 + C[1] * y1 + C[2] * y2;
            const T* bz = cz + (beta == 2 ? RT : 0);                // B3 row, or B-dot3 for beta = z
#pragma unroll
            for (int s = 0; s < RT; ++s) orng[s] += bz[s] * phi;
            if constexpr (MASS) {
                if (beta == 2) {                                // reaction: W3^{00} x c_q x value (B3 row)
                    const T* w00 = cz + 2 * RT;
                    T ym = T(0);
#pragma unroll
                    for (int s = 0; s < RO; ++s) ym += w00[s] * Yw[2][s];
                    const T pm = C[3] * ym;
#pragma unroll
                    for (int s = 0; s < RT; ++s) orng[s] += cz[s] * pm;
                }
            }
        };
        T Cs[2][NC];
        cload3(Cs[0], k0);
        cload3(Cs[1], min(k0 + 1, k1 - 1));
        __builtin_amdgcn_s_waitcnt(kVmcnt0);
        for (int r = 0; r < nrec; ++r) {
            const int fl = __builtin_amdgcn_readlane(Rf, r), ev = __builtin_amdgcn_readlane(Rev, r);
            const int czo = __builtin_amdgcn_readlane(Rczo, r), cn0 = __builtin_amdgcn_readlane(Rc0, r),
                      cn1 = __builtin_amdgcn_readlane(Rc1, r);
            const int es = (ev >> 8) & 15, rs = (ev >> 12) & 15;    // ring slots of the entry / retirement
            const int el = q2l * LD + q1l;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if ((ev >> (3 * j)) & 1) {                       // window entry
                    const int us = (fl >> 11) & 3;
                    if constexpr (RING) {
                        const T y0 = sU[us][beta][el], y1 = sU[us][3 + beta][el], y2 = sU[us][6 + beta][el];
                        slot_dispatch<0, RO>(es, [&](auto c) {
                            Yw[0][c] = y0;
                            Yw[1][c] = y1;
                            Yw[2][c] = y2;
                        });
                    } else {
#pragma unroll
                        for (int al = 0; al < 3; ++al) {
#pragma unroll
                            for (int s = 0; s < RO - 1; ++s) Yw[al][s] = Yw[al][s + 1];
                            Yw[al][RO - 1] = sU[us][3 * al + beta][el];
                        }
                    }
                }
                if ((ev >> (3 * j + 1)) & 1) {                   // retirement
                    if constexpr (RING) {
                        if ((fl >> 6) & 1) {
                            const int ps = (fl >> 13) & 1;
                            slot_dispatch<0, RT>(rs, [&](auto c) { sP[ps][beta][el] = orng[c]; });
                        }
                        slot_dispatch<0, RT>(rs, [&](auto c) { orng[c] = T(0); });
                    } else {
                        if ((fl >> 6) & 1) sP[(fl >> 13) & 1][beta][el] = orng[0];
#pragma unroll
                        for (int s = 0; s < RT - 1; ++s) orng[s] = orng[s + 1];
                        orng[RT - 1] = T(0);
                    }
                }
                if ((ev >> (3 * j + 2)) & 1) valu_plane(czo + j * CZ, Cs[j]);
                cload3(Cs[j], j ? cn1 : cn0);
            }
            lds_barrier();
        }
    }
}

// Clears w: 16-byte stores when w is 16-byte aligned, element stores otherwise
// and for the tail.
template <typename T>
__global__ __launch_bounds__(256) void zero_kernel(T* __restrict__ w, size_t n) {
    constexpr size_t V = 16 / sizeof(T);
    const size_t nv = (reinterpret_cast<uintptr_t>(w) % 16 == 0) ? n / V : 0;
    const size_t stride = (size_t)gridDim.x * 256, i0 = (size_t)blockIdx.x * 256 + threadIdx.x;
    float4* wv = reinterpret_cast<float4*>(w);
    for (size_t i = i0; i < nv; i += stride) wv[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (size_t i = nv * V + i0; i < n; i += stride) w[i] = T(0);
}

template <typename T>
void launch_zero(T* w, size_t n, hipStream_t s) {
    // about eight 16-byte stores per thread: a clear of a few MB is launch-bound,
    // and fewer workgroups start and retire sooner
    size_t g = (n * sizeof(T) / 16 + 2047) / 2048;
    g = g < 1 ? 1 : g > 1024 ? 1024 : g;
    hipLaunchKernelGGL(zero_kernel<T>, dim3((unsigned)g), dim3(256), 0, s, w, n);
}

template <typename T, int P>
hipError_t launch_p(const FusedArgs<T>& a, hipStream_t s) {
    if (a.zchunk <= 0 || a.zchunk > kMaxZ || !a.sched || !a.sched_off) return hipErrorInvalidValue;
    const int nzc = (a.nq3 + a.zchunk - 1) / a.zchunk;
    if (a.Cm)
        hipLaunchKernelGGL((wq_apply_fused_kernel<T, P, true>), dim3(a.ntx * a.nty * nzc), dim3(1024), 0, s, a);
    else
        hipLaunchKernelGGL((wq_apply_fused_kernel<T, P, false>), dim3(a.ntx * a.nty * nzc), dim3(1024), 0, s, a);
    return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_tp(const FusedArgs<T>& a, hipStream_t s) {
    if (a.zchunk <= 0 || a.zchunk > kMaxZ || !a.schedT || !a.schedT_off || !a.czT) return hipErrorInvalidValue;
    const int nzc = (a.nq3 + a.zchunk - 1) / a.zchunk;
    if (a.Cm)
        hipLaunchKernelGGL((wq_apply_T_fused_kernel<T, P, true>), dim3(a.ntx * a.nty * nzc), dim3(1024), 0, s, a);
    else
        hipLaunchKernelGGL((wq_apply_T_fused_kernel<T, P, false>), dim3(a.ntx * a.nty * nzc), dim3(1024), 0, s, a);
    return hipGetLastError();
}

template <int P>
hipError_t slots_p(int* slots) {
    int occ = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, wq_apply_fused_kernel<double, P, false>, 1024, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *slots = std::max(1, std::max(occ, 1) * cus);
    return hipSuccess;
}

}  // namespace

template <typename T>
hipError_t launch_fused_apply(const FusedArgs<T>& a, int p, hipStream_t s) {
    const size_t N = (size_t)a.n1 * a.n2 * a.n3;
    if (!a.w_zeroed) launch_zero(a.w, N, s);
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

template <typename T>
hipError_t launch_fused_apply_T(const FusedArgs<T>& a, int p, hipStream_t s) {
    const size_t N = (size_t)a.n1 * a.n2 * a.n3;
    if (!a.w_zeroed) launch_zero(a.w, N, s);
    switch (p) {
        case 2: return launch_tp<T, 2>(a, s);
        case 3: return launch_tp<T, 3>(a, s);
        case 4: return launch_tp<T, 4>(a, s);
        case 5: return launch_tp<T, 5>(a, s);
        case 6: return launch_tp<T, 6>(a, s);
        case 7: return launch_tp<T, 7>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fused_apply_T<double>(const FusedArgs<double>&, int, hipStream_t);
template hipError_t launch_fused_apply_T<float>(const FusedArgs<float>&, int, hipStream_t);

hipError_t fused_resident_slots(int p, int* slots) {
    switch (p) {
        case 2: return slots_p<2>(slots);
        case 3: return slots_p<3>(slots);
        case 4: return slots_p<4>(slots);
        case 5: return slots_p<5>(slots);
        case 6: return slots_p<6>(slots);
        case 7: return slots_p<7>(slots);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fused_apply<double>(const FusedArgs<double>&, int, hipStream_t);
template hipError_t launch_fused_apply<float>(const FusedArgs<float>&, int, hipStream_t);

}  // namespace wqfd
