// Tables and launcher of the fused MF-WQ apply kernel (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace wqfd {

// Arguments of the fused apply.  Dense 16 x 16 blocks per 16-point tile:
// tilesX[t][6][16][16] (x direction) and tilesY (y direction), in the order
// B_0[q][j], B_1[q][j] (values / derivatives, q = tile quadrature point,
// j = DOF offset from JX[t]) and W_v[i][q] for v = 0..3 (i = DOF offset from
// IX[t]).  In z the banded factors per quadrature plane k: trial window start
// bs3[k], test window start wts3[k] and cz[k][2(p+1) + 4(p+2)] = B3 row,
// B-dot3 row (p+1 each) and the four W3^v columns (p+2 each).
template <typename T>
struct FusedArgs {
    const T* v = nullptr;
    T* w = nullptr;
    const T* C = nullptr;
    int n1 = 0, n2 = 0, n3 = 0, nq1 = 0, nq2 = 0, nq3 = 0;
    size_t Nq = 0;
    const T* tilesX = nullptr;
    const T* tilesY = nullptr;
    const int* JX = nullptr;
    const int* IX = nullptr;
    const int* JY = nullptr;
    const int* IY = nullptr;
    const int* bs3 = nullptr;
    const int* wts3 = nullptr;
    const T* cz = nullptr;
    int ntx = 0, nty = 0, zchunk = 0;
};

template <typename T>
hipError_t launch_fused_apply(const FusedArgs<T>& a, int p, hipStream_t s);

}  // namespace wqfd
