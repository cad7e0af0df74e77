// Tables and launcher of the fused MF-WQ apply kernel (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace wqfd {

constexpr int FUSED_MAX_Z = 64;   // longest z range of one workgroup of the fused apply
// From this degree the transposed kernel keeps its z windows as fixed register
// rings (czT then holds every plane's rows in ring slot order; below it the
// windows shift and czT equals cz).  The shifts cost about as much as the ring
// bookkeeping, but from p = 6 on the shifted form spills registers.
constexpr int FUSED_RING_MIN_P = 6;

// Arguments of the fused apply.  Dense 16 x 16 blocks per 16-point tile:
// tilesX[t][6][16][16] (x direction) and tilesY (y direction), in the order
// B_0[q][j], B_1[q][j] (values / derivatives, q = tile quadrature point,
// j = DOF offset from JX[t]) and W_v[i][q] for v = 0..3 (i = DOF offset from
// IX[t]).  In z the banded factors per quadrature plane k: trial window start
// bs3[k], test window start wts3[k] and cz[k][2(p+1) + 4(p+2)] = B3 row,
// B-dot3 row (p+1 each) and the four W3^v columns (p+2 each); czT the same rows
// for the transposed kernel (in ring slot order from FUSED_RING_MIN_P on).
template <typename T>
struct FusedArgs {
    const T* v = nullptr;
    T* w = nullptr;
    const T* C = nullptr;
    const T* Cm = nullptr;          // reaction plane alpha det J [N_q], or nullptr (no reaction term)
    int n1 = 0, n2 = 0, n3 = 0, nq1 = 0, nq2 = 0, nq3 = 0;
    size_t Nq = 0;
    const T* tilesX = nullptr;
    const T* tilesY = nullptr;
    const int* JX = nullptr;
    const int* IX = nullptr;
    const int* JY = nullptr;
    const int* IY = nullptr;
    const int* bandX = nullptr;     // [tile][16] local start of the p + 1 trial functions at each point
    const int* bandY = nullptr;
    const int* bs3 = nullptr;
    const int* wts3 = nullptr;
    const T* cz = nullptr;
    const T* czT = nullptr;
    int ntx = 0, nty = 0, zchunk = 0;
    // interval schedule: records of FUSED_REC ints per interval (see FusedSched),
    // z range r uses records sched_off[r] .. sched_off[r + 1] - 1
    const int* sched = nullptr;
    const int* sched_off = nullptr;
    // the same for the transposed apply (input window W3, output ring B3)
    const int* schedT = nullptr;
    const int* schedT_off = nullptr;
    bool w_zeroed = false;          // w already cleared by the caller
};

// One interval of the fused apply's pipeline (between two workgroup barriers),
// computed on the host.  f packs: bits 0-1 number of quadrature planes; 2-3
// window entry position + 1; 4-5 retirement position + 1; 6 retired plane is
// written; 7 produce a U plane; 8 stage a DOF plane; 9 contract the retired
// plane written last interval; 10 reduce the partials written last interval;
// 11-12 U slot of the entering plane; 13 psi slot written; 14 psi slot read;
// 15 partial slot reduced; 16 partial slot written; 17 V slot read; 18-19 U
// slot written; 20 V slot written.  The column role reads its events already
// split by step: ev bits 3j, 3j + 1, 3j + 2 = window entry, retirement, plane
// k + j processed, at step j = 0, 1; bits 8-11 and 12-15 = the ring slot the
// interval's entry fills and the slot its retirement empties (entry e fills slot
// e mod IN, retirement r empties slot r mod OUT); czo = (k - k0) CZ, the offset of plane k's
// z coefficients in the range's table; cnext0/1 = the planes (clamped to the
// range) whose coefficients are loaded for the next interval.
struct FusedSched {
    int f, k, red_i3, tstage, ev, czo, cnext0, cnext1;
};
constexpr int FUSED_REC = 8;      // ints per interval record
static_assert(sizeof(FusedSched) == FUSED_REC * sizeof(int), "record layout");

// Resident workgroups of the fused FP64 apply kernel of degree p on the
// current device (compute units x workgroups per unit).
hipError_t fused_resident_slots(int p, int* slots);

template <typename T>
hipError_t launch_fused_apply(const FusedArgs<T>& a, int p, hipStream_t s);
template <typename T>
hipError_t launch_fused_apply_T(const FusedArgs<T>& a, int p, hipStream_t s);

}  // namespace wqfd
