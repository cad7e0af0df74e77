// Device-side data of the MF-WQ operator and the FD preconditioner, and the
// launch wrappers of the HIP kernels (gfx950).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "fused.h"

namespace wqfd {

// Banded 1D operator with `rows` rows over `cols` columns.  Row r has its
// non-zeros inside columns [start[r], start[r] + L); start is clamped so the
// window stays inside [0, cols).  Coefficients are stored [rows][L].
template <typename T>
struct Band {
    int rows = 0, cols = 0, L = 0;
    const int* start = nullptr;
    const T* c = nullptr;
};

// All banded 1D factors of one direction, in one precision.
//   B[d]  : n_q x n   values (d = 0) or derivatives (d = 1) of interior B-splines
//   W[v]  : n   x n_q weights, v = 2 a + b (a test, b trial derivative order)
//   BT[d] : n   x n_q transpose of B[d]
//   WT[v] : n_q x n   transpose of W[v]
template <typename T>
struct Dir1D {
    Band<T> B[2], W[4], BT[2], WT[4];
};

template <typename T>
struct OpTables {
    Dir1D<T> dir[3];
};

struct WqOp {
    int p = 0;
    int n[3] = {0, 0, 0}, nq[3] = {0, 0, 0};
    size_t N = 0, Nq = 0;
    int prec_mask = 0;
    int k_kind = 0;
    // device arrays (carved from the caller's workspace)
    double* detJ = nullptr;     // [Nq]
    double* Jinv = nullptr;     // [9][Nq]
    double* F = nullptr;        // [3][Nq]
    double* C64 = nullptr;      // [6][Nq] (C11, C22, C33, C12, C13, C23)
    float* C32 = nullptr;       // [6][Nq]
    double* Cm64 = nullptr;     // [Nq] reaction plane alpha det J (mass term of Algorithm 1)
    float* Cm32 = nullptr;      // [Nq]
    bool mass = false;          // reaction term set (wq_set_alpha)
    void* scratch = nullptr;    // apply intermediates (bytes: scratch_bytes)
    size_t scratch_bytes = 0;
    void* red = nullptr;        // reduction partials (norm2_ws_bytes())
    OpTables<double> t64;
    OpTables<float> t32;
    bool fused = false;         // fused apply available (p <= 7 and tile footprints fit)
    FusedArgs<double> fz64;     // fused-apply tables (v, w filled per call)
    FusedArgs<float> fz32;
    std::vector<double> xq[3];  // host copy of the quadrature points
};

struct FdPc {
    int n[3] = {0, 0, 0};
    size_t N = 0;
    int prec_mask = 0;
    double* U64[3] = {nullptr, nullptr, nullptr};   // row-major n x n (eigenvector k = column k)
    double* UT64[3] = {nullptr, nullptr, nullptr};  // transposes, row-major
    float* U32[3] = {nullptr, nullptr, nullptr};
    float* UT32[3] = {nullptr, nullptr, nullptr};
    uint16_t* Ubf[3] = {nullptr, nullptr, nullptr};  // bf16 copies (raw bits)
    float* Ubf_padded = nullptr;
    // fused passes (every n <= 144): U and U^T zero-padded to ldp = 16 ceil(max n / 16)
    // in both dimensions, so the kernels read them without bounds checks
    int ldp = 0;
    double* Up64[3] = {nullptr, nullptr, nullptr};
    double* UTp64[3] = {nullptr, nullptr, nullptr};
    float* Up32[3] = {nullptr, nullptr, nullptr};
    float* UTp32[3] = {nullptr, nullptr, nullptr};
    double* lam[3] = {nullptr, nullptr, nullptr};    // eigenvalues (device); lam[2] carries the shift
    double shift = 0.0;                              // constant added to the diagonal (reaction term)
    std::vector<double> hlam[3], hU[3];
    void* scratch = nullptr;    // one N-sized buffer of the widest precision
};

// Evaluation tables of a discrete solution at tensor Gauss points (eval.hip):
// per direction the first non-zero B-spline, values and derivatives [nq][p+1]
// and scaled Gauss weights of each point; the homogeneous control net
// [m3][m2][m1][4] = (w P, w) of the geometry map.
struct EvalOp {
    int p = 0, ng = 0;
    int ne[3] = {0, 0, 0}, nq[3] = {0, 0, 0}, m[3] = {0, 0, 0}, n[3] = {0, 0, 0};
    const int* first[3] = {nullptr, nullptr, nullptr};
    const double* B[3] = {nullptr, nullptr, nullptr};
    const double* D[3] = {nullptr, nullptr, nullptr};
    const double* w[3] = {nullptr, nullptr, nullptr};
    const double* ctrl = nullptr;
};

// Geometry at the quadrature points on the device (geom.hip): per direction the
// first non-zero B-spline and the p + 1 values and derivatives at each of the
// nq points, the homogeneous control net [m3][m2][m1][4], intermediates Z
// ([nq3][m2][m1][8]) and Y ([nq3][nq2][m1][12]) in caller memory, outputs det J
// [Nq], J^{-1} [9][Nq], F [3][Nq]; *bad is or-ed with 1 where det J <= 0.
struct GeomArgs {
    int p = 0;
    int m[3] = {0, 0, 0}, nq[3] = {0, 0, 0};
    size_t Nq = 0;
    const int* first[3] = {nullptr, nullptr, nullptr};
    const double* B[3] = {nullptr, nullptr, nullptr};
    const double* D[3] = {nullptr, nullptr, nullptr};
    const double* ctrl = nullptr;
    double* Z = nullptr;
    double* Y = nullptr;
    double* detJ = nullptr;
    double* Jinv = nullptr;
    double* F = nullptr;
    int* bad = nullptr;
};

// ---------------------------------------------------------------- launchers
// MF-WQ operator (wq_kernels.hip)
size_t wq_scratch_bytes(const WqOp& op, int prec_mask);
hipError_t launch_set_coef(const WqOp& op, int k_kind, const double* K_q, hipStream_t s);
// w_zeroed: the caller has cleared w (the fused kernels then skip their own clear)
hipError_t launch_apply(const WqOp& op, int prec, const void* v, void* w, bool transpose, hipStream_t s,
                        bool w_zeroed = false);
hipError_t launch_rhs(const WqOp& op, const double* f_q, double* b, hipStream_t s);
hipError_t launch_grad_K(const WqOp& op, const double* lam, const double* u, double* gK, hipStream_t s);
hipError_t launch_grad_f(const WqOp& op, const double* lam, double* gf, hipStream_t s);
// both in one pass over the quadrature points (fused operators), else one after the other
hipError_t launch_grad_Kf(const WqOp& op, const double* lam, const double* u, double* gK, double* gf,
                          hipStream_t s);
// reaction term: Cm = alpha det J (both prepared precisions), w = M~ v, dJ/dalpha
hipError_t launch_set_alpha(const WqOp& op, const double* alpha_q, hipStream_t s);
hipError_t launch_apply_mass(const WqOp& op, int prec, const void* v, void* w, hipStream_t s);
hipError_t launch_grad_alpha(const WqOp& op, const double* lam, const double* u, double* g, hipStream_t s);

// geometry set-up (geom.hip): bytes of the Z and Y intermediates, and the three passes
size_t geometry_scratch_bytes(const int m[3], const int nq[3]);
hipError_t launch_geometry(const GeomArgs& a, hipStream_t s);

// u_h, grad u_h, F and w |det J| at the Gauss points of elements
// [e3_begin, e3_end) along z (all elements in x and y); outputs [3][n], [n], [n], [3][n]
hipError_t launch_eval_slab(const EvalOp& E, const double* u, int e3_begin, int e3_end, double* X, double* wdet,
                            double* uh, double* grad, hipStream_t s);

// FD preconditioner (fd_kernels.hip).  `scratch` holds the intermediate between
// the passes: N values of the precision's type (at most N * 8 bytes).
hipError_t launch_fd_apply(const FdPc& P, int prec, const void* r, void* z, void* scratch, hipStream_t s);
inline hipError_t launch_fd_apply(const FdPc& P, int prec, const void* r, void* z, hipStream_t s) {
    return launch_fd_apply(P, prec, r, z, P.scratch, s);
}

// BLAS-1 helpers for the Krylov drivers (blas1.hip)
hipError_t launch_cast_f64_to_f32(const double* x, float* y, size_t n, double scale, hipStream_t s);
hipError_t launch_axpy_f32_to_f64(const float* d, double* x, size_t n, double scale, hipStream_t s);
hipError_t launch_axpy_f64(const double* d, double* x, size_t n, double scale, hipStream_t s);

}  // namespace wqfd
