/*
 * wqfd.h -- C ABI of the MI355X (gfx950) matrix-free weighted-quadrature
 * (MF-WQ) isogeometric solver: the WQ stiffness operator of Section 3.2
 * (Algorithm 2), its transpose, the WQ mass operator of the reaction term
 * (Section 3.1, Algorithm 1), the Fast Diagonalization (FD) preconditioner
 * used in Section 4, a right-preconditioned BiCGStab driver (Section 4), mixed-
 * precision refinement, adjoint gradients, and the same operator with standard
 * Gauss quadrature as a baseline (wq_setup_gauss).
 *
 * Model problem (Section 2.1, eq. poisson; alpha = 0 until wq_set_alpha):
 *     -div(K grad u) + alpha u = f on Omega = F([0,1]^3),  u = 0 on the boundary,
 * discretised with degree-p splines of maximum regularity on open knot
 * vectors, homogeneous Dirichlet space of eq. (space): n = m - 2 interior
 * B-splines per direction, N = n1 n2 n3 unknowns, x index fastest (eq. ordering).
 *
 * Conventions shared by every entry point
 *  - Return value: WQ_OK (0) or a negative WQ_E* code; wq_last_error() gives a
 *    thread-local message for the last failure.
 *  - Host pointers are read during the call only (setup copies what it keeps).
 *  - Device pointers (vectors, fields, workspaces) are owned by the caller,
 *    must be 256-byte aligned and must not alias each other unless stated.
 *    A workspace passed to a *_setup call must stay allocated, untouched, until
 *    the handle is destroyed.
 *  - Work is enqueued on the given HIP stream and is asynchronous unless the
 *    function says it synchronises.  Calls that share a handle must not run
 *    concurrently on different streams.
 *  - Layouts: DOF vectors [n3][n2][n1]; quadrature-point fields [nq3][nq2][nq1]
 *    (x fastest), planes of N_q = nq1 nq2 nq3 values, one after another.
 *  - Precision of vector arguments follows the `prec` argument:
 *    WQ_F64 -> double*, WQ_F32 -> float*.
 */
#ifndef WQFD_H
#define WQFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* wq_stream_t;   /* same type as hipStream_t */
typedef struct wq_op_s* wq_op;              /* opaque WQ operator handle */
typedef struct fd_pc_s* fd_pc;              /* opaque FD preconditioner handle */
typedef struct wq_eval_s* wq_eval;          /* opaque Gauss-point evaluator handle */

enum {
    WQ_OK = 0,
    WQ_EINVAL = -1,      /* bad argument: degree, knots, enum, size, null pointer */
    WQ_EGEOM = -2,       /* det J <= 0 at some quadrature point */
    WQ_ESINGULAR = -3,   /* weight system inexact, or FD mass matrix not SPD */
    WQ_ENOMEM = -4,      /* workspace too small */
    WQ_EHIP = -5,        /* HIP runtime error */
    WQ_ENOCONV = -6,     /* iteration limit reached (x holds the last iterate) */
    WQ_EBREAKDOWN = -7,  /* BiCGStab breakdown (rho or omega vanished) */
    WQ_ENONFINITE = -8   /* NaN or Inf met in the iteration */
};

/* precision flags (bit mask at setup, single value per call) */
enum { WQ_F64 = 1, WQ_F32 = 2, WQ_BF16 = 4 };

/* coefficient tensor K at the quadrature points */
enum {
    WQ_K_IDENTITY = 0,   /* K = I; K_q ignored */
    WQ_K_SCALAR = 1,     /* K = kappa I; K_q = kappa, one plane of N_q doubles */
    WQ_K_SYM6 = 6        /* symmetric K; six planes (K11, K22, K33, K12, K13, K23) */
};

/* ------------------------------------------------------------------------ *
 * wq_setup -- build the MF-WQ stiffness operator (Section 3.2, setup of
 * Algorithm 2) from the knot vectors, degree and control points of the
 * geometry map F (Section 2.1).
 *   p            degree, 2 <= p <= 10.
 *   nknots[l]    length of knots[l] (= m_l + p + 1); knots[l] host, open
 *                (p+1 equal end knots, 0 and 1), non-decreasing, interior
 *                knots simple (maximum regularity), at least 3 elements.
 *   ctrl         host [m3][m2][m1][3] FP64 control points (all m_l functions).
 *   k_kind,K_q   coefficient tensor (see WQ_K_*); K_q device FP64 or NULL
 *                for WQ_K_IDENTITY.  May be changed later by wq_set_coef.
 *   prec_mask    which apply precisions to prepare (WQ_F64 | WQ_F32).
 *   ws,ws_bytes  device workspace; ws == NULL makes this a size query that
 *                only writes *ws_needed (all other checks still run).
 * Quadrature points: all breakpoints, interior-element midpoints and p+1
 * equispaced interior points in each end element (n_q = 2 n_el + 2p + 1);
 * weights: minimum-norm solutions of the exactness conditions for all m trial
 * B-splines (eqs. exactness1d, weights-support, exactness_K).
 * C = det(J) J^{-1} K J^{-T} with J = dF/dxi (eq. C).  Synchronises `s`.
 * Deterministic mode: with the environment variable WQFD_STAGED set at set-up
 * the operator uses the staged kernels only (one writer per output, no
 * atomics), so its applies repeat bit for bit; they are slower, and
 * wq_apply_acc is not available.  Otherwise applies for p <= 7 run the fused
 * kernels, whose atomic adds make repeated results differ in the last bits.
 * Errors: WQ_EINVAL, WQ_EGEOM, WQ_ESINGULAR, WQ_ENOMEM, WQ_EHIP.
 * ------------------------------------------------------------------------ */
int wq_setup(int p, const int32_t nknots[3], const double* const knots[3],
             const double* ctrl, int k_kind, const double* K_q, int prec_mask,
             void* ws, size_t ws_bytes, size_t* ws_needed, wq_stream_t s, wq_op* out);

/* The same operator on a rational (NURBS) geometry map, which the paper's
 * experiments use (Section 2.1 notes that the method carries over to NURBS;
 * Section 4 takes the thick quarter ring, which polynomial splines cannot
 * represent exactly): F(xi) = sum_k w_k P_k b_k(xi) / sum_k w_k b_k(xi).
 *   weights      host [m3][m2][m1] FP64 control weights w_k > 0 (WQ_EINVAL
 *                otherwise, or if NULL); ctrl holds the Euclidean points P_k.
 * The discrete space stays the B-spline space of the knot vectors: the map
 * enters only through J, det J and F at the quadrature points (eq. C), so every
 * kernel and every other call works unchanged.  Other arguments and errors as
 * wq_setup. */
int wq_setup_nurbs(int p, const int32_t nknots[3], const double* const knots[3],
                   const double* ctrl, const double* weights, int k_kind, const double* K_q,
                   int prec_mask, void* ws, size_t ws_bytes, size_t* ws_needed, wq_stream_t s,
                   wq_op* out);

/* The same operator with standard Gauss quadrature instead of weighted
 * quadrature (the remark after rem:memory, eq. WDBgaussian): p + 1
 * Gauss-Legendre points per element and direction, test factors
 * W^{ab}_{iq} = w_q b_i^{(a)}(x_q) (independent of the trial order b), so
 * K^GQ = sum_{a,b} W^GQ D B is the Gauss-quadrature Galerkin matrix.  It needs
 * (p+1) n_el points per direction instead of about 2 n_el, hence O(N p^3)
 * coefficient memory and O(N p^4) apply work instead of O(N) and O(N p): a
 * baseline for the weighted-quadrature operator, with the same kernels and
 * every call of this header (apply, transpose, reaction term, solves,
 * gradients; wq_quad_points reports the Gauss points).  Arguments and errors as
 * wq_setup. */
int wq_setup_gauss(int p, const int32_t nknots[3], const double* const knots[3],
                   const double* ctrl, int k_kind, const double* K_q, int prec_mask,
                   void* ws, size_t ws_bytes, size_t* ws_needed, wq_stream_t s, wq_op* out);

/* Sizes: n[l] = m_l - 2 interior B-splines of direction l (the homogeneous
 * Dirichlet space of eq. space, Section 2.1) and nq[l] quadrature points of the
 * weighted-quadrature rule (Section 2.2; n_q = 2 n_el + 2p + 1, or (p+1) n_el
 * for wq_setup_gauss).  N = n[0] n[1] n[2], N_q likewise.  Host outputs. */
int wq_dims(wq_op A, int32_t n[3], int32_t nq[3]);

/* Quadrature points of Section 2.2: xq host [nq1 + nq2 + nq3] parametric
 * coordinates per direction (or NULL); Fq device [3][N_q] their images under the
 * geometry map F of Section 2.1 (or NULL), where a caller evaluates K, alpha
 * and f.  Async on s. */
int wq_quad_points(wq_op A, double* xq, double* Fq, wq_stream_t s);

/* det J(x_q), J = dF/dxi the Jacobian of the geometry map (Section 2.1), at
 * the quadrature points into device [N_q] (FP64): the volume factor of the
 * pulled-back integrands (eq. C; load vector and mass term).  Async on s. */
int wq_detj(wq_op A, double* detj, wq_stream_t s);

/* Recompute the coefficient planes C = det J J^{-1} K J^{-T} from a new K_q
 * (eq. C) without touching the geometry.  Async on s. */
int wq_set_coef(wq_op A, int k_kind, const double* K_q, wq_stream_t s);

/* Reaction coefficient of the model problem -div(K grad u) + alpha u = f
 * (Section 2.1): alpha_q device [N_q] FP64, alpha at the quadrature points in
 * the layout of K_q, or NULL to remove the term.  Stores the diagonal
 * c_q = alpha_q det J(x_q) of the weighted-quadrature mass matrix
 * M~ = W^(0,0) diag(c) B (Section 3.1, eq. WDB; B = B3 x B2 x B1) in the
 * operator's workspace (FP64, and FP32 when prepared); alpha_q is not kept.
 * From then on wq_apply, wq_apply_T, wq_apply_acc, krylov_solve and ir_solve
 * use K~ + M~.  The paper takes alpha >= 0; other values are used as given.
 * Async on s.  Errors: WQ_EINVAL, WQ_EHIP. */
int wq_set_alpha(wq_op A, const double* alpha_q, wq_stream_t s);

/* Mean over the quadrature points of the reaction diagonal c_q = alpha_q
 * det J(x_q) of the last wq_set_alpha (host output *mean): the representative
 * value sigma that fd_set_shift takes to precondition K~ + M~ (the FD
 * preconditioner of Section 4 with the mass term M3 x M2 x M1 of Section 3.1
 * added, scaled by one constant; the paper's experiments have alpha = 0).
 * Deterministic two-pass FP64 sum on the device; synchronises s.
 * Errors: WQ_EINVAL (null argument, or no reaction coefficient set), WQ_EHIP. */
int wq_alpha_mean(wq_op A, double* mean, wq_stream_t s);

/* w = M~ v alone: the mass product of Algorithm 1 (values of v at the points,
 * times c_q, the W^(0,0) rules), with the c_q of the last wq_set_alpha.  Runs as
 * six banded 1D passes through the operator's scratch (not the fused kernels).
 * Same arguments as wq_apply.  Async on s.  Errors: WQ_EINVAL (also when no
 * alpha is set), WQ_EHIP. */
int wq_apply_mass(wq_op A, int prec, const void* v, void* w, wq_stream_t s);

/* w = K~ v, Algorithm 2: w = sum_{a,b} W^(a,b) D^(a,b) B^(b) v (Section 3.2).
 * prec: WQ_F64 or WQ_F32 (must have been prepared).  v, w device, N entries,
 * must not alias.  With a reaction coefficient set, w = (K~ + M~) v.  Async on s. */
int wq_apply(wq_op A, int prec, const void* v, void* w, wq_stream_t s);

/* w = K~^T v = sum_{a,b} B^(b)T D^(a,b) W^(a,b)T v (transpose of the
 * factorisation of Section 3.2).  Same arguments as wq_apply.  Async. */
int wq_apply_T(wq_op A, int prec, const void* v, void* w, wq_stream_t s);

/* w += K~ v (Algorithm 2, Section 3.2, added to the current contents of w).
 * Same arguments as wq_apply; w is read and updated.  Available for operators
 * that use the fused kernels (p <= 7); WQ_EINVAL otherwise.  Async on s. */
int wq_apply_acc(wq_op A, int prec, const void* v, void* w, wq_stream_t s);

/* Load vector b = W^(0,0) (det J f): the weighted-quadrature mass rule of
 * Section 3.1 (eq. main) applied to f sampled at the quadrature points.
 * f_q device [N_q] FP64, b device [N] FP64.  Async on s. */
int wq_rhs(wq_op A, const double* f_q, double* b, wq_stream_t s);

/* Adjoint gradients of J(u) with K~ u = b (derivative of the factorisation of
 * Section 3.2 in the coefficient values):
 *   dJ/dC_ab(q) = -(W^(a,b)T lam)_q (B^(b) u)_q, chained through eq. C to the
 *   layout of K_q of the current k_kind (WQ_K_SCALAR: [N_q]; WQ_K_SYM6: [6][N_q];
 *   WQ_K_IDENTITY: the six C planes).  gK device, overwritten.  Async. */
int wq_grad_K(wq_op A, const double* lam, const double* u, double* gK, wq_stream_t s);

/* dJ/df_q = det J(q) (W^(0,0)T lam)_q into device [N_q].  Async on s. */
int wq_grad_f(wq_op A, const double* lam, double* gf, wq_stream_t s);

/* wq_grad_K and wq_grad_f together: for operators on the fused kernels
 * (p <= 7) one pass over the quadrature points that reads lam and u and writes
 * both gradients (the adjoint of a solve needs both); otherwise the two calls
 * in turn.  Results equal those of the two calls.  gK, gf device, overwritten.
 * Async on s.  Errors: WQ_EINVAL, WQ_EHIP. */
int wq_grad_Kf(wq_op A, const double* lam, const double* u, double* gK, double* gf, wq_stream_t s);

/* dJ/dalpha_q = -det J(q) (W^(0,0)T lam)_q (B u)_q (M~ is linear in alpha_q,
 * eq. WDB) into device [N_q] FP64; lam, u device [N] FP64.  Async on s.
 * Errors: WQ_EINVAL, WQ_EHIP. */
int wq_grad_alpha(wq_op A, const double* lam, const double* u, double* g, wq_stream_t s);

void wq_destroy(wq_op A);

/* ------------------------------------------------------------------------ *
 * fd_setup -- Fast Diagonalization preconditioner (Section 4; Lynch, Rice and
 * Thomas): P = K3 x M2 x M1 + M3 x K2 x M1 + M3 x M2 x K1 with the exact 1D
 * Galerkin stiffness K_l and mass M_l of the interior B-splines, inverted as
 * P^{-1} = (U3 x U2 x U1) diag(1/(l1_i + l2_j + l3_k)) (U3 x U2 x U1)^T where
 * K_l U_l = M_l U_l diag(l_l), U_l^T M_l U_l = I (eigen-setup in FP64 on the
 * host).  Same knot rules as wq_setup.  prec_mask: WQ_F64 | WQ_F32 | WQ_BF16.
 * ws == NULL: size query.  Synchronises s.
 * Errors: WQ_EINVAL, WQ_ESINGULAR, WQ_ENOMEM, WQ_EHIP.
 * ------------------------------------------------------------------------ */
int fd_setup(int p, const int32_t nknots[3], const double* const knots[3], int prec_mask,
             void* ws, size_t ws_bytes, size_t* ws_needed, wq_stream_t s, fd_pc* out);

/* z = P^{-1} r.  prec WQ_F64: double in/out, FP64 MFMA; WQ_F32: float in/out,
 * FP32 MFMA; WQ_BF16: float in/out, bf16 MFMA products with FP32
 * accumulation.  r, z device (may alias).  Async on s. */
int fd_apply(fd_pc P, int prec, const void* r, void* z, wq_stream_t s);

/* z = P^{-1} r exactly as fd_apply (same kernels, same results bit for bit),
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * intermediate between the mode passes lives in a static device array of
 * WQ_FD_NOALLOC_BYTES (32 MiB) that the library holds on each device it runs on
 * until the process ends, instead of the preconditioner's workspace.  The call
 * allocates nothing; its first call on a device looks up that array's device
 * address (with the device current).  Limit: N <= WQ_FD_NOALLOC_BYTES / 8
 * (4,194,304 unknowns, every precision); larger N returns WQ_ENOMEM.  Every call
 * on one device shares the one array: calls that overlap in time on that device
 * (different streams, or different host threads) race and give wrong results;
 * calls ordered on one stream are safe.  Runs on the current device, which must
 * be the device the preconditioner was set up on.  Arguments as fd_apply.
 * Errors: WQ_EINVAL, WQ_ENOMEM, WQ_EHIP. */
#define WQ_FD_NOALLOC_BYTES (32u << 20)
int fd_apply_noalloc(fd_pc P, int prec, const void* r, void* z, wq_stream_t s);

/* Shift for the reaction term: P becomes P + sigma M3 x M2 x M1, whose inverse
 * has the diagonal 1/(l1_i + l2_j + l3_k + sigma) in the same eigenbasis.
 * sigma is a representative value of alpha det J (e.g. its mean); 0 restores
 * the plain P.  Synchronises s.  Errors: WQ_EINVAL (non-finite sigma, or a
 * non-positive diagonal), WQ_EHIP. */
int fd_set_shift(fd_pc P, double sigma, wq_stream_t s);

/* The 1D factors of the FD preconditioner of Section 4 (fast diagonalization):
 * eigenvalues lam_l (host out, n_l doubles, may be NULL; without the shift) and
 * eigenvectors U_l (host out, row-major n_l x n_l, eigenvector k in column k,
 * may be NULL) of K_l U = M_l U diag(lam), U^T M_l U = I for direction l. */
int fd_factors(fd_pc P, int l, double* lam, double* U);

void fd_destroy(fd_pc P);

/* ------------------------------------------------------------------------ *
 * krylov_solve -- right-preconditioned BiCGStab (van der Vorst) in FP64 for
 * K~ x = b (transpose = 0) or K~^T x = b (transpose = 1), preconditioner
 * P^{-1} (FP64), as in Section 4.  x holds x0 on entry and the solution on
 * exit.  Stops when |b - K~ x|_2 / |b|_2 <= rtol (recurrence residual, then
 * confirmed with the true residual; a failed confirmation restarts the
 * recurrence from the true residual).  ws: device, at least
 * krylov_ws_bytes(A) bytes.  Waits once per iteration for a small scalar
 * block that the device writes into pinned host memory (the calling thread
 * polls it); returns once the stream's work up to the last read-back is done
 * (work enqueued ahead of it, such as the next iteration's first half, may
 * still run on s; it writes only the workspace).  *iters, *relres: host
 * outputs (*relres: the true
 * relative residual on success, the last recurrence value on WQ_ENOCONV).
 * Errors: WQ_EINVAL, WQ_ENOMEM, WQ_ENOCONV, WQ_EBREAKDOWN, WQ_ENONFINITE, WQ_EHIP.
 * ------------------------------------------------------------------------ */
/* krylov_ws_bytes: device workspace bytes krylov_solve needs for A's N (nine
 * FP64 Krylov vectors of the BiCGStab recurrence of Section 4 and the
 * reduction partials); 0 for a null handle. */
size_t krylov_ws_bytes(wq_op A);
int krylov_solve(wq_op A, fd_pc P, int transpose, const double* b, double* x,
                 double rtol, int maxit, void* ws, size_t ws_bytes,
                 int* iters, double* relres, wq_stream_t s);

/* ------------------------------------------------------------------------ *
 * ir_solve -- mixed-precision iterative refinement: outer FP64 residual
 * r = b - K~ x and FP64 update x += d; inner right-preconditioned BiCGStab in
 * FP32 (FP32 apply, FD in `fd_prec` = WQ_F32 or WQ_BF16) on the scaled residual
 * to relative tolerance max(tau_inner, rtol |b|_2 / (2 |r|_2)) (the last inner
 * solve reduces the residual only as far as the outer target needs; an inner
 * solve stops on its recurrence residual, the outer FP64 residual being the
 * check).  Stops when the FP64 residual satisfies |r|_2/|b|_2 <= rtol.
 * x: FP64 in/out.
 * ws: device, at least
 * ir_ws_bytes(A).  *outer, *inner_total, *relres: host outputs.
 * Errors: as krylov_solve.
 * ------------------------------------------------------------------------ */
/* ir_ws_bytes: device workspace bytes ir_solve needs for A's N (the FP64
 * iterate and residual, FP32 copies and the inner BiCGStab workspace); the
 * refinement loop is an addition to the paper's FP64 method.  0 for null. */
size_t ir_ws_bytes(wq_op A);
int ir_solve(wq_op A, fd_pc P, int fd_prec, const double* b, double* x, double rtol,
             double tau_inner, int max_outer, int maxit_inner, void* ws, size_t ws_bytes,
             int* outer, int* inner_total, double* relres, wq_stream_t s);

/* Stagnation fallback of ir_solve: an outer step that does not halve the FP64
 * residual switches the remaining inner solves of that call to FP64 (FP64
 * apply, FP64 FD: the plain method of Section 4 on the residual equation,
 * solved to the accuracy the outer target needs), provided the preconditioner
 * has WQ_F64 prepared; *outer and *inner_total count those steps too.  This
 * returns how many ir_solve calls of the calling thread have switched so far. */
int ir_fallback_count(void);

/* Restarts of krylov_solve's BiCGStab (ir_solve's inner solves stop on the
 * recurrence residual and never restart): when the recurrence residual passes
 * the tolerance but the true
 * residual b - A x does not (reading R8 of the Krylov stopping test, Section 4),
 * the recurrence restarts from the true residual instead of stopping.  This
 * returns how many such restarts the calling thread's solves have made so far. */
int krylov_restart_count(void);

/* ------------------------------------------------------------------------ *
 * Host-only inspection of the set-up (no device work; for checks and tools).
 * ------------------------------------------------------------------------ */

/* One direction's 1D factors (Section 2.2; points and weights as in wq_setup).
 * Pass NULL arrays to get the sizes *n, *nq first.  Outputs are dense,
 * row-major host arrays: xq [nq]; B [2][nq][n] (values, then first derivatives
 * of the interior B-splines b_1 .. b_{m-2} at the points); W [4][n][nq] (weight
 * matrices W^{ab} in the order v = 2a + b, a = test and b = trial derivative).
 * Errors: WQ_EINVAL, WQ_ESINGULAR. */
int wq_space_1d(int p, int nknots, const double* knots, int32_t* n, int32_t* nq, double* xq, double* B,
                double* W);

/* FD factors of one direction: lam [n] and U [n][n] (row-major, eigenvector k
 * in column k) of K U = M U diag(lam), U^T M U = I (the 1D problems behind
 * fd_setup).  Errors: WQ_EINVAL, WQ_ESINGULAR. */
int fd_eig_1d(int p, int nknots, const double* knots, double* lam, double* U);

/* Geometry at the quadrature points of wq_setup, on the host: detJ [N_q],
 * Jinv [9][N_q] (entry (r, c) of J^{-1} in plane 3 r + c) and F [3][N_q];
 * weights NULL for a polynomial map, else the control weights of a rational
 * map as in wq_setup_nurbs.  Errors: WQ_EINVAL, WQ_EGEOM, WQ_ESINGULAR. */
int wq_geometry_host(int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl,
                     const double* weights, double* detJ, double* Jinv, double* F);

/* ------------------------------------------------------------------------ *
 * Evaluation of a discrete solution at tensor Gauss points, for the error
 * measure of the k-refinement study (Section 4, Table 1: relative H1-seminorm
 * error of u_h = sum_j u_j b_j o F^{-1}), in slabs of elements along z so that
 * fine levels (256^3 elements, (p+3)^3 points each) need not be held at once.
 * wq_eval_setup: ng Gauss-Legendre points per element and direction (1..32;
 *   the study takes p + 3) on the knots of wq_setup; ctrl [m3][m2][m1][3] and
 *   weights [m3][m2][m1] (NULL: polynomial map) as in wq_setup_nurbs.  ws
 *   device workspace (NULL: size query into *ws_needed; 256-byte aligned)
 *   holds the tables and the homogeneous control net, 32 bytes per control
 *   point.  Synchronises s.  Errors: WQ_EINVAL, WQ_ENOMEM, WQ_EHIP.
 * wq_eval_dims: elements ne[l] and Gauss points nq[l] = ne[l] ng per direction.
 * wq_eval_slab: for the elements [e3_begin, e3_end) along z and all elements
 *   along x and y, at n = nq1 nq2 (e3_end - e3_begin) ng points ordered
 *   [z][y][x] (x fastest): X [3][n] = F(xi), wdet [n] = w1 w2 w3 |det J|,
 *   uh [n] = u_h and grad [3][n] = J^{-T} grad_xi u_h, from u [N] (device FP64,
 *   interior coefficients as in wq_apply).  All device FP64.  Async on s.
 *   Errors: WQ_EINVAL, WQ_EHIP.
 * ------------------------------------------------------------------------ */
int wq_eval_setup(int p, const int32_t nknots[3], const double* const knots[3], const double* ctrl,
                  const double* weights, int ng, void* ws, size_t ws_bytes, size_t* ws_needed,
                  wq_stream_t s, wq_eval* out);
int wq_eval_dims(wq_eval E, int32_t ne[3], int32_t nq[3]);
int wq_eval_slab(wq_eval E, const double* u, int e3_begin, int e3_end, double* X, double* wdet,
                 double* uh, double* grad, wq_stream_t s);
void wq_eval_destroy(wq_eval E);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* wq_last_error(void);

/* Library version string. */
const char* wq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WQFD_H */
