// Mode-product launcher of the FD preconditioner (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace wqfd {

// out[a][i][c] = sum_j mat[i][j] in[a][j][c], element (j, c) of batch a at
// a * sa + j * sj + c * sc; mat row-major with leading dimension ldT (n <= 144).
// l1 != nullptr: divide row i, column c by l1[c % n1] + l2[c / n1] + l3[i].
template <typename T, typename S>
struct FdModeArgs {
    const T* in = nullptr;
    T* out = nullptr;
    const S* mat = nullptr;
    int n = 0, C = 0, ldT = 0;
    size_t sa = 0, sj = 0, sc = 0;
    const double* l1 = nullptr;
    const double* l2 = nullptr;
    const double* l3 = nullptr;
    int n1 = 1;
};

hipError_t launch_fd_mode(const FdModeArgs<double, double>& p, int batches, hipStream_t s);
hipError_t launch_fd_mode(const FdModeArgs<float, float>& p, int batches, hipStream_t s);
hipError_t launch_fd_mode(const FdModeArgs<float, __bf16>& p, int batches, hipStream_t s);

}  // namespace wqfd
