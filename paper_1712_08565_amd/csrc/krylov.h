// BiCGStab driver and mixed-precision helpers (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>

namespace wqfd {

// y = Op(x) enqueued on the stream; element type fixed by the caller.
using LinOp = std::function<hipError_t(const void*, void*, hipStream_t)>;

// Device workspace bytes of one BiCGStab run on N unknowns.
size_t krylov_bytes(size_t N, bool fp32);

// Right-preconditioned BiCGStab: A x = b with x = M y.  Returns 0 or a
// negative wqfd error code (message in err).  Synchronises once per iteration.
// A_acc (optional): the operator adding its product into a zeroed output; the
// iteration then clears the two product outputs inside its vector updates.
// confirm: check a converged recurrence residual against the true residual
// b - A x before returning (the inner solves of iterative refinement skip it:
// the outer loop forms the true residual in FP64 anyway).
template <typename T>
int bicgstab(const LinOp& A, const LinOp& M, size_t N, const T* b, T* x, bool x0_zero, double tol, int maxit,
             void* ws, int* iters, double* relres, std::string& err, hipStream_t s, const LinOp* A_acc = nullptr,
             bool confirm = true);

// failed true-residual confirmations that restarted a recurrence, calling thread
int bicgstab_restart_count();

int norm2(const double* x, size_t N, void* part_ws, double* out, std::string& err, hipStream_t s);
size_t norm2_ws_bytes();
// sum of x[0..N) into *out (host); part_ws: norm2_ws_bytes() of device memory
int sum_all(const double* x, size_t N, void* part_ws, double* out, std::string& err, hipStream_t s);
hipError_t launch_resid(const double* b, double* y, size_t n, hipStream_t s);
hipError_t launch_fill0_f32(float* x, size_t n, hipStream_t s);

}  // namespace wqfd
