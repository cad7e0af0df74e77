// Right-preconditioned BiCGStab (van der Vorst 1992), the Krylov solver the
// paper uses for the non-symmetric weighted-quadrature systems (Section 4), and
// a mixed-precision iterative-refinement loop around an FP32 inner BiCGStab.
//
// All scalars of the recurrence (rho, alpha, omega, ...) live in device memory
// and are produced by the reduction kernels, so an iteration enqueues its work
// without waiting for the host; the host reads back one small scalar block per
// iteration for the convergence and breakdown tests.  Dot products are
// deterministic two-pass reductions (fixed block partition and order), always
// accumulated in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.h"
#include "krylov.h"

namespace wqfd {

namespace {

constexpr int kT = 256;
constexpr int kU = 4;            // elements of a thread per chunk of kT * kU
constexpr int kMaxBlocks = 1024;

enum Slot {
    S_RHO = 0, S_RHO_OLD, S_ALPHA, S_OMEGA, S_RV, S_TS, S_TT, S_RR, S_BB, S_AUX, S_AUX2, kSlots
};

enum FinalOp { F_STORE = 0, F_ALPHA, F_OMEGA, F_RHO_RR };

inline int nblocks(size_t n) {
    size_t b = (n + (size_t)kT * kU - 1) / ((size_t)kT * kU);
    if (b > kMaxBlocks) b = kMaxBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    __syncthreads();
    return r;
}

// The vector kernels walk the vector in chunks of kT * kU elements, chunks
// assigned to blocks round-robin; a thread's elements of a chunk are kT apart,
// and all their loads are issued before the first use, so a thread waits for
// memory once per chunk instead of once per element.  The kernels are bound by
// that latency, not by bandwidth: a pass over a vector of a few MB at 8 TB/s
// takes well under a microsecond.
template <typename F>
__device__ inline void for_chunks(size_t n, F&& body) {
    for (size_t c = (size_t)blockIdx.x * (kT * kU) + threadIdx.x; c < n; c += (size_t)gridDim.x * (kT * kU))
        body(c);
}

// partial sums of up to three dot products (x_k, y_k)
template <typename T, int K>
__global__ __launch_bounds__(kT) void dot_partial(const T* __restrict__ x0, const T* __restrict__ y0,
                                                  const T* __restrict__ x1, const T* __restrict__ y1,
                                                  const T* __restrict__ x2, const T* __restrict__ y2, size_t n,
                                                  double* __restrict__ part) {
    __shared__ double sh[kT / 64];
    double a0 = 0, a1 = 0, a2 = 0;
    for_chunks(n, [&](size_t c) {
        T u0[kU], v0[kU], u1[kU], v1[kU], u2[kU], v2[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = c + (size_t)u * kT;
            const bool in = i < n;
            u0[u] = in ? x0[i] : T(0);
            v0[u] = in ? y0[i] : T(0);
            if (K > 1) u1[u] = in ? x1[i] : T(0), v1[u] = in ? y1[i] : T(0);
            if (K > 2) u2[u] = in ? x2[i] : T(0), v2[u] = in ? y2[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            a0 += (double)u0[u] * (double)v0[u];
            if (K > 1) a1 += (double)u1[u] * (double)v1[u];
            if (K > 2) a2 += (double)u2[u] * (double)v2[u];
        }
    });
    double r = block_sum(a0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
    if (K > 1) {
        r = block_sum(a1, sh);
        if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = r;
    }
    if (K > 2) {
        r = block_sum(a2, sh);
        if (threadIdx.x == 0) part[2 * gridDim.x + blockIdx.x] = r;
    }
}

// partial sums of x (one per block, fixed partition)
__global__ __launch_bounds__(kT) void sum_partial(const double* __restrict__ x, size_t n, double* __restrict__ part) {
    __shared__ double sh[kT / 64];
    double a = 0;
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) a += x[i];
    const double r = block_sum(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// The scalar block sc is also written to hsc (coherent pinned host memory, its
// device address) and then, once those stores have completed, the marker `mark`
// into hsc[kMark]: the host waits for the marker instead of an event, with no
// copy launch and no end-of-kernel cache write-back for a host wait.
constexpr int kMark = 15;
__device__ inline void to_host(const double* sc, double* hsc, double mark) {
    for (int k = 0; k < kSlots; ++k) hsc[k] = sc[k];
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the scalars' stores have completed
    hsc[kMark] = mark;
}

// single block: sum the partials of K dots and update the scalar block (and,
// with hsc, hand it to the host)
template <int K>
__global__ __launch_bounds__(kT) void dot_final(const double* __restrict__ part, int nb, double* __restrict__ sc,
                                                int slot0, int op, double* __restrict__ hsc, double mark) {
    __shared__ double sh[kT / 64];
    double res[3] = {0, 0, 0};
    for (int k = 0; k < K; ++k) {
        double a = 0;
        for (int i = threadIdx.x; i < nb; i += kT) a += part[k * nb + i];
        res[k] = block_sum(a, sh);
    }
    if (threadIdx.x != 0) return;
    switch (op) {
        case F_STORE:
            for (int k = 0; k < K; ++k) sc[slot0 + k] = res[k];
            break;
        case F_ALPHA:   // res0 = (r^, v)
            sc[S_RV] = res[0];
            sc[S_ALPHA] = sc[S_RHO] / res[0];
            break;
        case F_OMEGA:   // res0 = (t, s), res1 = (t, t)
            sc[S_TS] = res[0];
            sc[S_TT] = res[1];
            sc[S_OMEGA] = res[1] != 0.0 ? res[0] / res[1] : 0.0;
            break;
        case F_RHO_RR:  // res0 = (r^, r), res1 = (r, r)
            sc[S_RHO_OLD] = sc[S_RHO];
            sc[S_RHO] = res[0];
            sc[S_RR] = res[1];
            break;
    }
    if (hsc) to_host(sc, hsc, mark);
}

// Sum of nb partials, identical in every block (same partition and order), so
// a kernel can finish a reduction itself instead of a separate launch.
__device__ inline double sum_partials(const double* __restrict__ part, int nb, double* sh) {
    double a = 0;
    for (int i = threadIdx.x; i < nb; i += kT) a += part[i];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) sh[kT / 64] = a;
    __syncthreads();
    const double r = sh[kT / 64];
    __syncthreads();
    return r;
}

// p = r + beta (p - omega v),  beta = (rho / rho_old) (alpha / omega); v is
// then cleared when the next product accumulates into it
template <typename T>
__global__ __launch_bounds__(kT) void upd_p(T* __restrict__ p, const T* __restrict__ r, T* __restrict__ v,
                                            const double* __restrict__ sc, size_t n, int first, int clear_v) {
    const double beta = first ? 0.0 : (sc[S_RHO] / sc[S_RHO_OLD]) * (sc[S_ALPHA] / sc[S_OMEGA]);
    const double om = sc[S_OMEGA];
    for_chunks(n, [&](size_t c) {
        T rr[kU], pp[kU], vv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = c + (size_t)u * kT;
            const bool in = i < n;
            rr[u] = in ? r[i] : T(0);
            pp[u] = in && !first ? p[i] : T(0);
            vv[u] = in && !first ? v[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = c + (size_t)u * kT;
            if (i < n) {
                p[i] = first ? rr[u] : (T)((double)rr[u] + beta * ((double)pp[u] - om * (double)vv[u]));
                if (clear_v) v[i] = T(0);
            }
        }
    });
}

// alpha = rho / (r^, v) from the partials of (r^, v);  s = r - alpha v;
// t cleared for the next accumulating product
template <typename T>
__global__ __launch_bounds__(kT) void upd_s(T* __restrict__ s, const T* __restrict__ r, const T* __restrict__ v,
                                            T* __restrict__ t, double* __restrict__ sc, const double* __restrict__ part,
                                            int nb, size_t n, int clear_t) {
    __shared__ double sh[kT / 64 + 1];
    const double rv = sum_partials(part, nb, sh);
    const double al = sc[S_RHO] / rv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_RV] = rv;
        sc[S_ALPHA] = al;
    }
    for_chunks(n, [&](size_t c) {
        T rr[kU], vv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = c + (size_t)u * kT;
            rr[u] = i < n ? r[i] : T(0);
            vv[u] = i < n ? v[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = c + (size_t)u * kT;
            if (i < n) {
                s[i] = (T)((double)rr[u] - al * (double)vv[u]);
                if (clear_t) t[i] = T(0);
            }
        }
    });
}

// omega = (t, s) / (t, t) from their partials;  x += alpha p^ + omega s^ ;
// r = s - omega t ; partials of (r^, r) and (r, r) into part_out
template <typename T>
__global__ __launch_bounds__(kT) void upd_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ ph,
                                             const T* __restrict__ sh_, const T* __restrict__ s,
                                             const T* __restrict__ t, const T* __restrict__ rh,
                                             double* __restrict__ sc, const double* __restrict__ part_in, int nb,
                                             size_t n, double* __restrict__ part) {
    __shared__ double sh[kT / 64 + 1];
    const double ts = sum_partials(part_in, nb, sh);
    const double tt = sum_partials(part_in + nb, nb, sh);
    const double om = tt != 0.0 ? ts / tt : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_TS] = ts;
        sc[S_TT] = tt;
        sc[S_OMEGA] = om;
    }
    const double al = sc[S_ALPHA];
    double a0 = 0, a1 = 0;
    for_chunks(n, [&](size_t c) {
        T xx[kU], pp[kU], ss_[kU], ss[kU], tt_[kU], rr[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = c + (size_t)u * kT;
            const bool in = i < n;
            xx[u] = in ? x[i] : T(0);
            pp[u] = in ? ph[i] : T(0);
            ss_[u] = in ? sh_[i] : T(0);
            ss[u] = in ? s[i] : T(0);
            tt_[u] = in ? t[i] : T(0);
            rr[u] = in ? rh[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = c + (size_t)u * kT;
            const T rn = (T)((double)ss[u] - om * (double)tt_[u]);
            if (i < n) {
                x[i] = (T)((double)xx[u] + al * (double)pp[u] + om * (double)ss_[u]);
                r[i] = rn;
            }
            a0 += (double)rr[u] * (double)rn;
            a1 += (double)rn * (double)rn;
        }
    });
    double v = block_sum(a0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
    v = block_sum(a1, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = v;
}

// Initial scalars of the recurrence from the first reduction (rho = (r^, r) in
// S_RHO, (r, r) in S_RHO_OLD, (b, b) in S_ALPHA): rho_old = alpha = omega = 1.
__global__ void init_scalars(double* sc, double* hsc, double mark) {
    const double rr = sc[S_RHO_OLD], bb = sc[S_ALPHA];
    for (int k = 0; k < kSlots; ++k)
        if (k != S_RHO) sc[k] = 0.0;
    sc[S_RHO_OLD] = 1.0;
    sc[S_ALPHA] = 1.0;
    sc[S_OMEGA] = 1.0;
    sc[S_RR] = rr;
    sc[S_BB] = bb;
    to_host(sc, hsc, mark);
}

// y = b - y (true residual) ; copy
template <typename T>
__global__ __launch_bounds__(kT) void resid(const T* __restrict__ b, T* __restrict__ y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) y[i] = b[i] - y[i];
}

template <typename T>
__global__ __launch_bounds__(kT) void copy2(const T* __restrict__ a, T* __restrict__ b, T* __restrict__ c, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) {
        b[i] = a[i];
        if (c) c[i] = a[i];
    }
}

template <typename T>
__global__ __launch_bounds__(kT) void fill0(T* __restrict__ a, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) a[i] = T(0);
}

__global__ __launch_bounds__(kT) void cast_kernel(const double* __restrict__ x, float* __restrict__ y, size_t n,
                                                  double scale) {
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT)
        y[i] = (float)(x[i] * scale);
}

template <typename D>
__global__ __launch_bounds__(kT) void axpy_kernel(const D* __restrict__ d, double* __restrict__ x, size_t n,
                                                  double scale) {
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT)
        x[i] += scale * (double)d[i];
}

thread_local int g_restarts = 0;                 // failed confirmations that restarted (this thread)

// Thread-local pinned host block for the scalar read-back, 16 doubles a slot:
// slots 0 and 1 alternate between iterations (marker: the iteration), slot 2
// the confirmation, slot 3 the restart value, slot 4 the initial scalars,
// slot 5 norms (markers: a per-thread sequence number).  Coherent: the
// reduction kernels' stores to it are not held in the GPU's caches, so they are
// visible to the host once they have completed.  hdev: its device address.
bool host_block(double** h_out, double** hdev_out) {
    static thread_local double* h = nullptr;
    static thread_local double* hdev = nullptr;
    if (!h) {
        double* p = nullptr;
        double* d = nullptr;
        if (hipHostMalloc((void**)&p, 96 * sizeof(double), hipHostMallocCoherent) != hipSuccess) return false;
        if (hipHostGetDevicePointer((void**)&d, p, 0) != hipSuccess || !d) return false;
        for (int i = 0; i < 96; ++i) p[i] = -1.0;
        h = p;
        hdev = d;
    }
    *h_out = h;
    *hdev_out = hdev;
    return true;
}

// marker values of the one-off read-backs (distinct within a thread)
double next_mark() {
    static thread_local double m = 0.0;
    return m += 1.0;
}

// Waits until the reduction kernel has written marker value `want` (the host
// reads coherent pinned memory).  Now and then the stream is queried: an error
// there, or the stream done without the marker, ends the wait with an error.
hipError_t wait_marker(const double* mark, double want, hipStream_t s) {
    const volatile double* m = mark;
    for (unsigned k = 1;; ++k) {
        if (*m == want) return hipSuccess;
        if ((k & 255) == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return q;
            return *m == want ? hipSuccess : hipErrorUnknown;   // (stream done without the marker)
        }
    }
}


#define KR_TRY(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) {                     \
            err = hipGetErrorString(e_);            \
            return WQ_EHIP_CODE;                    \
        }                                           \
    } while (0)

constexpr int WQ_EHIP_CODE = -5;

template <typename T>
struct Vecs {
    T *r, *rh, *p, *v, *s, *t, *ph, *sh;
    double *sc, *part, *part2;
};

template <typename T>
size_t vec_bytes(size_t N) {
    const size_t v = (N * sizeof(T) + 255) / 256 * 256;
    return 8 * v + 256 + (size_t)5 * kMaxBlocks * sizeof(double) + 256;
}

template <typename T>
Vecs<T> carve(void* ws, size_t N) {
    Vecs<T> V;
    char* c = static_cast<char*>(ws);
    const size_t v = (N * sizeof(T) + 255) / 256 * 256;
    T** ptrs[8] = {&V.r, &V.rh, &V.p, &V.v, &V.s, &V.t, &V.ph, &V.sh};
    for (int k = 0; k < 8; ++k) {
        *ptrs[k] = reinterpret_cast<T*>(c);
        c += v;
    }
    V.sc = reinterpret_cast<double*>(c);
    c += 256;
    V.part = reinterpret_cast<double*>(c);
    V.part2 = V.part + 3 * kMaxBlocks;
    return V;
}

}  // namespace

int bicgstab_restart_count() { return g_restarts; }

size_t krylov_bytes(size_t N, bool fp32) { return fp32 ? vec_bytes<float>(N) : vec_bytes<double>(N); }

hipError_t launch_cast_f64_to_f32(const double* x, float* y, size_t n, double scale, hipStream_t s) {
    hipLaunchKernelGGL(cast_kernel, dim3(nblocks(n)), dim3(kT), 0, s, x, y, n, scale);
    return hipGetLastError();
}

hipError_t launch_axpy_f32_to_f64(const float* d, double* x, size_t n, double scale, hipStream_t s) {
    hipLaunchKernelGGL(axpy_kernel<float>, dim3(nblocks(n)), dim3(kT), 0, s, d, x, n, scale);
    return hipGetLastError();
}

hipError_t launch_axpy_f64(const double* d, double* x, size_t n, double scale, hipStream_t s) {
    hipLaunchKernelGGL(axpy_kernel<double>, dim3(nblocks(n)), dim3(kT), 0, s, d, x, n, scale);
    return hipGetLastError();
}

template <typename T>
int bicgstab(const LinOp& A, const LinOp& M, size_t N, const T* b, T* x, bool x0_zero, double tol, int maxit,
             void* ws, int* iters, double* relres, std::string& err, hipStream_t s, const LinOp* A_acc,
             bool confirm) {
    // A_acc: the same operator adding into a cleared output (the update kernels
    // clear v and t just before the products that fill them)
    const LinOp& Aa = A_acc ? *A_acc : A;
    const int clear = A_acc ? 1 : 0;
    Vecs<T> V = carve<T>(ws, N);
    const int nb = nblocks(N);
    const dim3 g(nb), blk(kT);
    double *h = nullptr, *hdev = nullptr;
    if (!host_block(&h, &hdev)) {
        err = "could not allocate pinned host memory";
        return WQ_EHIP_CODE;
    }
    // a failed wait: the stream's error, or the stream done without the marker
    auto wait_fail = [&](hipError_t e) {
        err = e == hipErrorUnknown ? "scalars not received from the device" : hipGetErrorString(e);
        return WQ_EHIP_CODE;
    };
    *iters = 0;
    *relres = 0.0;
    // r = b - A x0 ; r^ = r ; scalars
    if (x0_zero) {
        hipLaunchKernelGGL(fill0<T>, g, blk, 0, s, x, N);
        hipLaunchKernelGGL(copy2<T>, g, blk, 0, s, b, V.r, V.rh, N);
    } else {
        KR_TRY(A(x, V.t, s));
        hipLaunchKernelGGL(copy2<T>, g, blk, 0, s, V.t, V.r, (T*)nullptr, N);
        hipLaunchKernelGGL(resid<T>, g, blk, 0, s, b, V.r, N);
        hipLaunchKernelGGL(copy2<T>, g, blk, 0, s, V.r, V.rh, (T*)nullptr, N);
    }
    hipLaunchKernelGGL((dot_partial<T, 3>), g, blk, 0, s, V.rh, V.r, V.r, V.r, b, b, N, V.part);
    hipLaunchKernelGGL((dot_final<3>), dim3(1), blk, 0, s, V.part, nb, V.sc, (int)S_RHO, (int)F_STORE, nullptr, 0.0);
    // S_RHO = (r^, r), S_RHO_OLD = (r, r), S_ALPHA = (b, b): moved to their slots and the
    // recurrence's initial scalars set on the device, then one read-back
    const double m0 = next_mark();
    hipLaunchKernelGGL(init_scalars, dim3(1), dim3(1), 0, s, V.sc, hdev + 64, m0);
    // Each iteration is enqueued in two halves.  The first (p, p^ = M p, v = A p^,
    // alpha, s, s^ = M s, t = A s^, the partials of omega) touches neither x nor r;
    // the second (omega, x and r, rho) ends with the scalars handed to the host.
    // The next iteration's first half is enqueued before the host waits for the
    // current scalars (when the residual trend predicts that the current one does
    // not converge), so the device keeps working through the read-back.  If
    // the current iteration converged the speculative half is simply not
    // continued (x is the current iterate); if its true residual then fails the
    // confirmation, the recurrence restarts from the true residual (p = r).
    auto first_half = [&](int first) -> hipError_t {
        hipLaunchKernelGGL(upd_p<T>, g, blk, 0, s, V.p, V.r, V.v, V.sc, N, first, clear);
        hipError_t e = M(V.p, V.ph, s);
        if (e == hipSuccess) e = Aa(V.ph, V.v, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((dot_partial<T, 1>), g, blk, 0, s, V.rh, V.v, (const T*)nullptr, (const T*)nullptr,
                           (const T*)nullptr, (const T*)nullptr, N, V.part);
        hipLaunchKernelGGL(upd_s<T>, g, blk, 0, s, V.s, V.r, V.v, V.t, V.sc, V.part, nb, N, clear);
        e = M(V.s, V.sh, s);
        if (e == hipSuccess) e = Aa(V.sh, V.t, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((dot_partial<T, 2>), g, blk, 0, s, V.t, V.s, V.t, V.t, (const T*)nullptr,
                           (const T*)nullptr, N, V.part);
        return hipGetLastError();
    };
    // the first iteration's first half is enqueued before the host waits for the
    // initial scalars (it touches neither x nor r, so an early return leaves them as
    // they are)
    if (maxit >= 1) KR_TRY(first_half(1));
    {
        const hipError_t e = wait_marker(h + 64 + kMark, m0, s);
        if (e != hipSuccess) return wait_fail(e);
    }
    const double bb = h[64 + S_BB], rr0 = h[64 + S_RR];
    if (!std::isfinite(bb) || !std::isfinite(rr0)) {
        err = "non-finite value in the right-hand side or initial residual";
        return -8;
    }
    if (bb == 0.0) {
        hipLaunchKernelGGL(fill0<T>, g, blk, 0, s, x, N);
        return 0;
    }
    const double nbn = std::sqrt(bb);
    if (std::sqrt(rr0) / nbn <= tol) {
        *relres = std::sqrt(rr0) / nbn;
        return 0;
    }
    // residual history for the speculation decision: the next half is enqueued
    // ahead only while this iteration is predicted (geometric trend of the last
    // two residuals, with a factor 4 margin) not to reach the tolerance, so that a
    // solve normally ends without a discarded half
    double rel1 = std::sqrt(rr0) / nbn, rel2 = 0.0;
    // the iterations' scalars arrive in two alternating host slots, each with its
    // iteration number as marker (cleared here: the slots are reused by every solve)
    h[kMark] = h[16 + kMark] = -1.0;
    for (int it = 1; it <= maxit; ++it) {
        double* hb = h + 16 * (it & 1);             // the scalars of this iteration (two host slots)
        hipLaunchKernelGGL(upd_xr<T>, g, blk, 0, s, x, V.r, V.ph, V.sh, V.s, V.t, V.rh, V.sc, V.part, nb, N, V.part2);
        // the reduction kernel writes the scalars to the pinned host block itself
        hipLaunchKernelGGL((dot_final<2>), dim3(1), blk, 0, s, V.part2, nb, V.sc, 0, (int)F_RHO_RR,
                           hdev + 16 * (it & 1), (double)it);
        KR_TRY(hipGetLastError());
        const double q = rel2 > 0.0 ? std::min(1.0, rel1 / rel2) : 1.0;
        const bool spec = it < maxit && rel1 * q > 4.0 * tol;
        if (spec) KR_TRY(first_half(0));            // speculative: the next iteration's first half
        {
            const hipError_t e = wait_marker(hb + kMark, (double)it, s);
            if (e != hipSuccess) return wait_fail(e);
        }
        *iters = it;
        const double rel = std::sqrt(hb[S_RR]) / nbn;
        *relres = rel;
        rel2 = rel1;
        rel1 = rel;
        if (!std::isfinite(rel) || !std::isfinite(hb[S_ALPHA]) || !std::isfinite(hb[S_OMEGA])) {
            KR_TRY(hipStreamSynchronize(s));
            err = "non-finite value in the BiCGStab recurrence";
            return -8;
        }
        if (rel <= tol) {
            if (!confirm) return 0;
            // confirm with the true residual r = b - A x (after the speculative half, in stream order)
            KR_TRY(A(x, V.t, s));
            hipLaunchKernelGGL(resid<T>, g, blk, 0, s, b, V.t, N);
            hipLaunchKernelGGL((dot_partial<T, 2>), g, blk, 0, s, V.t, V.t, V.rh, V.t, (const T*)nullptr,
                               (const T*)nullptr, N, V.part);
            // (the marker comes last in stream order: all queued work, the speculative
            // half included, is done once it is seen)
            const double mc = next_mark();
            hipLaunchKernelGGL((dot_final<2>), dim3(1), blk, 0, s, V.part, nb, V.sc, (int)S_AUX, (int)F_STORE,
                               hdev + 32, mc);
            double* hc = h + 32;
            {
                const hipError_t e = wait_marker(hc + kMark, mc, s);
                if (e != hipSuccess) return wait_fail(e);
            }
            const double tr = std::sqrt(hc[S_AUX]) / nbn;
            *relres = tr;
            if (tr <= tol) return 0;
            if (it == maxit) break;
            // restart from the true residual: r = r_true, rho = (r^, r_true), p = r
            ++g_restarts;
            hipLaunchKernelGGL(copy2<T>, g, blk, 0, s, V.t, V.r, (T*)nullptr, N);
            double* hr = h + 48;                        // (pinned: read by the copy below)
            *hr = hc[S_AUX2];
            KR_TRY(hipMemcpyAsync(V.sc + S_RHO, hr, sizeof(double), hipMemcpyHostToDevice, s));
            KR_TRY(first_half(1));
            rel2 = 0.0;
            continue;
        }
        if (hb[S_RHO] == 0.0 || hb[S_OMEGA] == 0.0 || hb[S_RV] == 0.0) {
            KR_TRY(hipStreamSynchronize(s));
            err = "BiCGStab breakdown (rho, (r^, v) or omega vanished)";
            return -7;
        }
        if (!spec && it < maxit) KR_TRY(first_half(0));
    }
    KR_TRY(hipStreamSynchronize(s));
    err = "BiCGStab reached the iteration limit";
    return -6;
}

template int bicgstab<double>(const LinOp&, const LinOp&, size_t, const double*, double*, bool, double, int,
                              void*, int*, double*, std::string&, hipStream_t, const LinOp*, bool);
template int bicgstab<float>(const LinOp&, const LinOp&, size_t, const float*, float*, bool, double, int, void*,
                             int*, double*, std::string&, hipStream_t, const LinOp*, bool);

// FP64 norm of a vector (two-pass); returns once the stream's work up to it is done.
int norm2(const double* x, size_t N, void* part_ws, double* out, std::string& err, hipStream_t s) {
    double* part = reinterpret_cast<double*>(part_ws);
    double* sc = part + 3 * kMaxBlocks;
    const int nb = nblocks(N);
    hipLaunchKernelGGL((dot_partial<double, 1>), dim3(nb), dim3(kT), 0, s, x, x, (const double*)nullptr,
                       (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, N, part);
    double *h = nullptr, *hdev = nullptr;
    if (!host_block(&h, &hdev)) {
        err = "could not allocate pinned host memory";
        return WQ_EHIP_CODE;
    }
    const double m = next_mark();
    hipLaunchKernelGGL((dot_final<1>), dim3(1), dim3(kT), 0, s, part, nb, sc, 0, (int)F_STORE, hdev + 80, m);
    KR_TRY(hipGetLastError());
    const hipError_t e = wait_marker(h + 80 + kMark, m, s);      // (all queued work is done then)
    if (e != hipSuccess) {
        err = e == hipErrorUnknown ? "norm not received from the device" : hipGetErrorString(e);
        return WQ_EHIP_CODE;
    }
    *out = std::sqrt(h[80]);
    return 0;
}

size_t norm2_ws_bytes() { return (3 * kMaxBlocks + 64) * sizeof(double); }

// FP64 sum of a vector (two-pass, fixed order), synchronising.
int sum_all(const double* x, size_t N, void* part_ws, double* out, std::string& err, hipStream_t s) {
    double* part = reinterpret_cast<double*>(part_ws);
    double* sc = part + 3 * kMaxBlocks;
    const int nb = nblocks(N);
    hipLaunchKernelGGL(sum_partial, dim3(nb), dim3(kT), 0, s, x, N, part);
    hipLaunchKernelGGL((dot_final<1>), dim3(1), dim3(kT), 0, s, part, nb, sc, 0, (int)F_STORE, nullptr, 0.0);
    double h = 0.0;
    KR_TRY(hipMemcpyAsync(&h, sc, sizeof(double), hipMemcpyDeviceToHost, s));
    KR_TRY(hipStreamSynchronize(s));
    *out = h;
    return 0;
}

hipError_t launch_resid(const double* b, double* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(resid<double>, dim3(nblocks(n)), dim3(kT), 0, s, b, y, n);
    return hipGetLastError();
}

hipError_t launch_fill0_f32(float* x, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(fill0<float>, dim3(nblocks(n)), dim3(kT), 0, s, x, n);
    return hipGetLastError();
}

}  // namespace wqfd
