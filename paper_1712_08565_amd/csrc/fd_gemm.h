// Mode-product launcher of the FD preconditioner (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace wqfd {

// out[i][g] = sum_j mat[i][j] in[j][g] for columns g = 0..C-1: column g starts
// at (g / cdiv) * sa + (g % cdiv) * sc, its element j at + j * sj; mat
// row-major with leading dimension ldT (n <= 144).  l1 != nullptr (passes with
// cdiv = C only): divide row i, column g by l1[g % n1] + l2[g / n1] + l3[i].
template <typename T, typename S>
struct FdModeArgs {
    const T* in = nullptr;
    T* out = nullptr;
    const S* mat = nullptr;
    int n = 0, C = 0, cdiv = 1, ldT = 0;
    size_t sa = 0, sj = 0, sc = 0;
    const double* l1 = nullptr;
    const double* l2 = nullptr;
    const double* l3 = nullptr;
    int n1 = 1;
};

// Whole preconditioner application in three fused passes (n <= 144): forward
// x and y per z-plane, forward z + eigenvalue scaling + backward z per column
// block, backward x and y.  U[l] / UT[l] row-major n_l x n_l; tmp: N scratch
// entries; r and z may alias.
template <typename T>
struct FdFusedArgs {
    const T* r = nullptr;
    T* z = nullptr;
    T* tmp = nullptr;
    const T* U[3] = {nullptr, nullptr, nullptr};
    const T* UT[3] = {nullptr, nullptr, nullptr};
    const double* l1 = nullptr;
    const double* l2 = nullptr;
    const double* l3 = nullptr;
    int n1 = 0, n2 = 0, n3 = 0;
    int ldp = 0;                     // U, UT: zero-padded ldp x ldp, ldp = 16 ceil(max n / 16)
};

// BF16 operands (FP32 data and accumulation), the same three passes; Tf[l] / Tb[l]
// are the bf16 T = U^T / T = U of fd_setup, row-major, zero padded to ld[l]
// (a multiple of 64) in both dimensions; n <= 160.
struct FdFusedBf16Args {
    const float* r = nullptr;
    float* z = nullptr;
    float* tmp = nullptr;
    const __bf16* Tf[3] = {nullptr, nullptr, nullptr};
    const __bf16* Tb[3] = {nullptr, nullptr, nullptr};
    int ld[3] = {0, 0, 0};
    int n[3] = {0, 0, 0};
    const double* l1 = nullptr;
    const double* l2 = nullptr;
    const double* l3 = nullptr;
    int n1 = 0, n2 = 0, n3 = 0;
};

hipError_t launch_fd_fused(const FdFusedArgs<double>& f, hipStream_t s);
hipError_t launch_fd_fused_bf16(const FdFusedBf16Args& f, hipStream_t s);
hipError_t launch_fd_fused(const FdFusedArgs<float>& f, hipStream_t s);

hipError_t launch_fd_mode(const FdModeArgs<double, double>& p, hipStream_t s);
hipError_t launch_fd_mode(const FdModeArgs<float, float>& p, hipStream_t s);
hipError_t launch_fd_mode(const FdModeArgs<float, __bf16>& p, hipStream_t s);

}  // namespace wqfd
