/*
 * librqrcp -- truncated randomized QR with column pivoting (RQRCP) on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Xiao, Gu, Langou, "Fast Parallel Randomized QR with Column Pivoting
 * Algorithms for Reliable Low-rank Matrix Approximations" (HiPC 2017,
 * arXiv 1804.05138).  The factorization is A Pi = Q R (eq. (1)) truncated at
 * target rank k:
 *
 *     A Pi = Q [R11 R12; 0 R22],   A ~ Q1 [R11 R12] Pi^T     (Section I-A)
 *
 * computed with Alg. 2 (RQRCP): a Gaussian sketch B = Omega A
 * (Omega ~ N(0,1)^{(b+p) x m}), then per block of b columns a partial QRCP of
 * the sketch (Alg. 1) picks b pivots, the pivoted panel of A is factored by
 * Householder QR, the block reflector is applied to the trailing columns, and
 * the sketch is refreshed with update formula (1) of Section III-B.
 *
 * Conventions (all entry points):
 *  - Matrices are column-major with a leading dimension >= the row count.
 *    Indices are 0-based.  Every array argument is DEVICE memory unless its
 *    comment says (host).
 *  - Work is enqueued on the handle's stream and is asynchronous, except
 *    where a comment says the call synchronizes.  The caller owns every
 *    buffer; the library allocates nothing per call (the workspace comes
 *    from rqrcp_workspace_size).  A, B and the workspace must not alias.
 *  - Return value: 0 on success; -i if argument i (1-based) is invalid, in
 *    which case nothing was enqueued; RQRCP_ERR_* otherwise.  Numerical
 *    conditions are reported through the device `info` word.
 *  - One handle per stream; a handle is not thread-safe.
 *
 * Storage of a factorization (LAPACK convention): on exit A holds R in its
 * upper trapezoid (rows 0..k-1), the Householder vectors v_j (v_j[j] = 1
 * implied) below the diagonal of columns 0..k-1, and the trailing block R22
 * in A(k:m, k:n).  tau[j] are the reflector scalars, H_j = I - tau_j v_j v_j^T,
 * Q = H_0 H_1 ... H_{k-1}.  jpvt[j] is the original index of the column at
 * position j.  The reflector convention is LAPACK dlarfg's:
 * beta = -sign(alpha) ||x||, with sign(0) = +.
 */
#ifndef RQRCP_H
#define RQRCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rqrcp_ctx *rqrcp_handle;

/* Status codes (besides 0 and -i). */
#define RQRCP_ERR_HIP 1001         /* a HIP runtime call or launch failed */
#define RQRCP_ERR_WORKSPACE 1002   /* ws_bytes smaller than rqrcp_workspace_size */
#define RQRCP_ERR_UNSUPPORTED 1003 /* dtype combination not supported */
#define RQRCP_ERR_DEVICE 1004      /* the current device is not gfx950 */
#define RQRCP_ERR_LIMIT 1005       /* size beyond what the kernels accept (see rqrcp_limits) */
#define RQRCP_ERR_BARRIER 1006     /* a persistent kernel's grid barrier timed out */
#define RQRCP_ERR_NUMERIC 1007     /* the sketch held a non-finite value: no pivot could be chosen */
#define RQRCP_ERR_PIVOTS 1008      /* a caller's jpvt is not a permutation of 0..n-1 */
#define RQRCP_ERR_SCRATCH 1009     /* rqrcp_factor_noalloc: the sizes need more than
                                      RQRCP_NOALLOC_MAX_BYTES of workspace */

/* Element types.  A may be FP64 or FP32; the sketch B, Omega, tau and all
 * reflector arithmetic are FP64.  The sketch product may run in FP64, BF16 or
 * FP8 (OCP e4m3); with an FP32 A the trailing update runs on FP32 MFMA (the
 * mixed-precision form; the paper itself computes everything in FP64). */
#define RQRCP_F64 0
#define RQRCP_F32 1
#define RQRCP_BF16 2
#define RQRCP_F8E4M3 3

/* rqrcp_params.flags */
#define RQRCP_FROZEN_PIVOTS 1u /* jpvt is an input: factor A(:, jpvt) without pivoting */
#define RQRCP_USER_SKETCH 2u   /* B already holds the sketch Omega A (e.g. from rqrcp_sketch) */
#define RQRCP_HOUSEHOLDER_PANEL 4u /* factor every panel one reflector at a time (Alg. 2's
                                      panel QR as written) instead of by Cholesky-QR2 with
                                      Householder reconstruction; slower, for comparisons */
#define RQRCP_TOURNAMENT 8u  /* choose each block's pivots by QR with tournament pivoting
                                (Section V-C's proposed replacement of the partial QRCP of
                                B; Demmel, Grigori, Gu, Xiang 2015): Alg. 1 on groups of
                                256 sketch columns, nominations merged four sets at a time
                                by Alg. 1 until one set is left, then the sketch block
                                factored with those pivots; b <= 64, b + p <= 80 */

typedef struct {
  int b;           /* block size, 1 <= b <= 128 (the block size of Alg. 2) */
  int p;           /* oversampling, p >= 0, b + p <= 160 (the oversampling of Alg. 2) */
  uint64_t seed;   /* Philox key word 0 of Omega (key word 1 = stream 0) */
  int a_type;      /* storage of A: RQRCP_F64, or RQRCP_F32 (then the trailing update
                      runs in FP32 and R, V are stored in FP32) */
  int sketch_type; /* arithmetic of B = Omega A: RQRCP_F64, RQRCP_BF16 or RQRCP_F8E4M3
                      (FP32 accumulation; FP8 with per-column power-of-two scales) */
  unsigned flags;  /* RQRCP_FROZEN_PIVOTS | RQRCP_USER_SKETCH | RQRCP_HOUSEHOLDER_PANEL |
                      RQRCP_TOURNAMENT */
} rqrcp_params;

/* Create a handle bound to `stream` (a hipStream_t; NULL = default stream)
 * on the current device.  Fails with RQRCP_ERR_DEVICE if that device is not
 * gfx950.  *h (host) receives the handle. */
int rqrcp_create(rqrcp_handle *h, void *stream);
int rqrcp_destroy(rqrcp_handle h);
int rqrcp_set_stream(rqrcp_handle h, void *stream);

/* Workspace in bytes (host output) for rqrcp_factor with these sizes.  A
 * workspace of that size also serves rqrcp_sketch and rqrcp_form_q for the
 * same m, n, k, b, p. */
int rqrcp_workspace_size(int m, int n, int k, const rqrcp_params *prm, size_t *bytes);

/* Largest sizes the kernels accept for sketch row count l = b + p (host
 * outputs): max_b, max_l, and max_n (columns of the sketch QRCP). */
int rqrcp_limits(int l, int *max_b, int *max_l, int *max_n);

/* Omega(0:rows, 0:cols) ~ N(0,1) from the counter-based generator
 * Philox4x64-10 (Salmon et al., SC'11) with key (seed, stream):
 * entry (r, c) is normal number q = c*rows + r, taken from counter
 * (q/4 + 1, 0, 0, 0), word q%4, uniform u = ((x >> 12) + 1/2) 2^-52 and
 * Box-Muller on word pairs (0,1) and (2,3).  Alg. 2 draws the (b+p) x m
 * sketching matrix from stream 0; Alg. 3 draws its probes from stream
 * 2^32 + j.  out: rows x cols, leading dimension ld. */
int rqrcp_gaussian(rqrcp_handle h, int rows, int cols, uint64_t seed, uint64_t stream,
                   double *out, int ld);

/* Sketch B = Omega A (the sketching step of Alg. 2); A is m x n (lda) of
 * a_type (RQRCP_F64 or RQRCP_F32), B is l x n FP64 (ldb).  sketch_type is the
 * product's arithmetic (RQRCP_F64, RQRCP_BF16 or RQRCP_F8E4M3; see
 * rqrcp_params).  Omega: l x m FP64 (ldo) supplied by the caller, or NULL to
 * draw it from Philox(seed, stream 0) into the workspace.  Workspace: that of
 * rqrcp_factor with the same m, n, b + p = l and sketch_type. */
int rqrcp_sketch(rqrcp_handle h, int m, int n, int l, uint64_t seed, int a_type, const void *A,
                 int lda, int sketch_type, const double *Omega, int ldo, double *B, int ldb,
                 void *ws, size_t ws_bytes);

/* Truncated RQRCP (Alg. 2) of the m x n matrix A to rank k, 1 <= k <= min(m, n).
 *  A     (in/out) m x n, lda, of prm->a_type: the factorization in LAPACK
 *        storage (see top).
 *  jpvt  (out) n ints; with RQRCP_FROZEN_PIVOTS an input permutation of
 *        0..n-1, checked on the device before use: an entry outside [0, n)
 *        or a repeated one sets info = -8 and makes rqrcp_check return
 *        RQRCP_ERR_PIVOTS (A then holds no usable factorization).
 *  tau   (out) k doubles.
 *  B     (in/out) (b+p) x n sketch, ldb >= b+p.  Computed from Philox(seed)
 *        unless RQRCP_USER_SKETCH; on exit B(:, k:n) is the sketch of the
 *        trailing block R22 (the input of srqr).  Unused (may be NULL) with
 *        RQRCP_FROZEN_PIVOTS.
 *  info  (out, one int) 0, or s+1 if the largest trailing sketch norm at
 *        global pivot step s was exactly zero (then the sketch is no longer
 *        updated and the remaining steps take the columns in their current
 *        order; the factorization itself is completed).
 * Pivot ties go to the lowest current position. */
int rqrcp_factor(rqrcp_handle h, int m, int n, int k, const rqrcp_params *prm, void *A, int lda,
                 int32_t *jpvt, double *tau, double *B, int ldb, int32_t *info, void *ws,
                 size_t ws_bytes);

/* rqrcp_factor without a workspace argument, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as rqrcp_factor; the
 * workspace is a static device array of RQRCP_NOALLOC_MAX_BYTES bytes inside
 * the library (one per GPU, held until the process ends).  Sizes whose
 * rqrcp_workspace_size exceeds it return RQRCP_ERR_SCRATCH and enqueue
 * nothing (64 MiB covers, e.g., FP64 2048 x 2048 with k = 256, b = 64, p = 8).
 * The call allocates nothing.  Every call on one GPU shares the array, so
 * calls that overlap on one GPU (other streams or threads) race; run them in
 * order.  rqrcp_check(h, NULL) reads the error flags these calls leave. */
#define RQRCP_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int rqrcp_factor_noalloc(rqrcp_handle h, int m, int n, int k, const rqrcp_params *prm, void *A,
                         int lda, int32_t *jpvt, double *tau, double *B, int ldb, int32_t *info);

/* Tolerance-driven RQRCP: Alg. 2 run block by block until the trailing block
 * is small enough (Section III-A notes that the method can be stopped by an
 * error tolerance instead of a target rank).  After each block's sample update
 * the trailing sketch B(:, c:n) equals Omega-hat_2 R22 (Section III-B, formula
 * (1)), so ||B(:, c:n)||_F / sqrt(b+p) estimates ||R22||_F, and the initial
 * sketch likewise estimates ||A||_F.  The loop stops after the first block
 * whose estimate ratio is <= tol (at least one block; at most kmax columns).
 *  tol      0 < tol < 1.
 *  kmax     largest rank; tau holds kmax doubles, the workspace is that of
 *           rqrcp_factor with k = kmax.
 *  k_out    (host) the rank reached: a multiple of b, or kmax.
 *  est_out  (host, may be NULL) the estimate ratio at k_out.
 * Other arguments as rqrcp_factor (RQRCP_FROZEN_PIVOTS is not allowed).
 * Synchronizes the stream once per block (the stopping test is on the host). */
int rqrcp_factor_tol(rqrcp_handle h, int m, int n, int kmax, double tol, const rqrcp_params *prm,
                     void *A, int lda, int32_t *jpvt, double *tau, double *B, int ldb,
                     int32_t *info, int *k_out, double *est_out, void *ws, size_t ws_bytes);

/* Explicit Q1 = H_0 ... H_{k-1} [I_k; 0] (m x k, ldq) from a factorization
 * (A, lda, tau): the orthonormal factor of the rank-k approximation
 * Q1 [R11 R12] Pi^T of Section I-A (eq. (1)), with Q the product of Alg. 2's
 * panel reflectors.  b is the block size used to apply the reflectors; A and Q
 * are of a_type (RQRCP_F64 or RQRCP_F32; FP32 products on FP32 MFMA). */
int rqrcp_form_q(rqrcp_handle h, int m, int k, int b, int a_type, const void *A, int lda,
                 const double *tau, void *Q, int ldq, void *ws, size_t ws_bytes);

/* ---- QR with column pivoting of the whole matrix (the comparator) ----
 * Alg. 1 (Section II): at every step the column of largest trailing norm is
 * brought forward and eliminated by a Householder reflector.  Organized as
 * LAPACK's xGEQP3, the Level-3 form Section II describes: the trailing matrix
 * is updated once per block of nb columns by a GEMM, but every step still reads
 * the whole trailing matrix once (for the reflector's product with it, which
 * the norm downdates need) -- the cost RQRCP avoids.  Trailing norms are
 * downdated (LAPACK's rule) and recomputed exactly when a downdate has lost
 * half the digits.  FP64 only.
 *  A     (in/out) m x n (lda): k steps of the factorization in LAPACK storage.
 *  jpvt  (out) n ints (the identity is the start; ties go to the lowest index).
 *  tau   (out) k doubles.
 * nb: 1..128.  Workspace from rqrcp_qrcp_workspace_size. */
int rqrcp_qrcp_workspace_size(int m, int n, int k, int nb, size_t *bytes);
int rqrcp_qrcp(rqrcp_handle h, int m, int n, int k, int nb, double *A, int lda, int32_t *jpvt,
               double *tau, void *ws, size_t ws_bytes);

/* ---- Spectrum-revealing swaps (Alg. 3, Section IV) ---- */
#define SRQR_EXACT 1u /* g2 from the exact row norms of Rhat^-1 instead of d Gaussian probes */

/* Workspace in bytes (host output) for srqr_swap with these sizes. */
int srqr_workspace_size(int m, int n, int l, const rqrcp_params *prm, int d, unsigned sflags,
                        size_t *bytes);

/* Alg. 3 after an l-step rqrcp_factor (k = l) with the same prm, 1 <= l < min(m, n).
 * FP64 only (prm->a_type = RQRCP_F64; the swap tests are FP64 in every form).
 *  g          tolerance g > 1 of the g2 test (Section IV-C: g2 = |alpha| ||Rhat^-T||_{1,2}).
 *  d          probe count of the g2 estimate g2 ~ |alpha| ||Omega Rhat^-T||_{1,2} / sqrt(d),
 *             Omega (d x (l+1)) from Philox(prm->seed, stream 2^32 + j) at estimate j
 *             (ignored with SRQR_EXACT).
 *  max_swaps  cap on the round-robin swaps (< 0: 2n).
 *  A0         (in) the original m x n matrix (lda0), used to recompute the
 *             factorization after swaps.
 *  A, jpvt, tau (in/out) the factorization from rqrcp_factor (tau has room for
 *             l+1 entries); on exit an (l+1)-step factorization in the same
 *             storage: one more Householder step if no swap was needed, else the
 *             frozen-pivot factorization of A0(:, jpvt) with the final pivots
 *             (Givens rotations cannot be represented by V/tau).
 *  B          (in) the final sketch from rqrcp_factor (its columns l..n-1 give the
 *             initial estimates r_i = ||B(:, i)||^2 / (b+p)).
 *  g2_out     (out, device, may be NULL) the last g2 value.
 *  nswaps_out (out, device, may be NULL) the number of swaps.
 *  info       (out, device) 0, or -max_swaps if the cap was reached with g2 > g.
 * Synchronizes the stream once per g2 evaluation (the loop is host-driven).
 * Limits: l + 1 <= 4096. */
int srqr_swap(rqrcp_handle h, int m, int n, int l, const rqrcp_params *prm, double g, int d,
              int max_swaps, unsigned sflags, const double *A0, int lda0, double *A, int lda,
              int32_t *jpvt, double *tau, const double *B, int ldb, double *g2_out,
              int32_t *nswaps_out, int32_t *info, void *ws, size_t ws_bytes);

/* ---- Uses of a factorization: CX, CUR (Section V-D), SVD compression ----
 * All FP64, from factorizations in LAPACK storage (rqrcp_factor, srqr_swap,
 * rqrcp_qrcp); the library computes every product from the factors, without
 * another pass over A.
 *
 * rqrcp_cx: C = A(:, jpvt[0:k]) (the k leading columns of a k-step or longer
 * factorization AF, jpvt of A) and X = C^+ A (k x n, ldx, original column
 * order), the minimizer of ||C X - A||_F.  From C = Q1 R11 and
 * Q1^T A Pi = [R11 R12]: X Pi = [I | R11^-1 R12].  k <= 1024. */
int rqrcp_cx_workspace_size(int m, int n, int k, size_t *bytes);
int rqrcp_cx(rqrcp_handle h, int m, int n, int k, const double *AF, int ldaf,
             const int32_t *jpvt, double *X, int ldx, void *ws, size_t ws_bytes);

/* rqrcp_cur: C as in rqrcp_cx from the column factorization (AFc, jpvt_c) of
 * the m x n A, R = A(jpvt_r[0:k], :) the rows chosen by the factorization
 * (AFr, tau_r, jpvt_r; block size b) of A^T (n x m), and U = C^+ A R^+
 * (k x k, ldu), the minimizer of ||C U R - A||_F: U = X Q_r1 T11^-T with X of
 * rqrcp_cx, Q_r1 the first k columns of the row factorization's Q and T11 its
 * leading triangle.  k <= 1024. */
int rqrcp_cur_workspace_size(int m, int n, int k, int b, size_t *bytes);
int rqrcp_cur(rqrcp_handle h, int m, int n, int k, int b, const double *AFc, int ldc,
              const int32_t *jpvt_c, const double *AFr, int ldr, const double *tau_r, double *U,
              int ldu, void *ws, size_t ws_bytes);

/* rqrcp_compress: SVD compression of an l-step factorization to rank k <= l
 * (the remark after Alg. 3; useful when SRQR ran with l > k).  With R_l the
 * first l rows of R and U_k the k leading left singular vectors of R_l,
 * A ~ X Y with X = Q_l U_k (m x k, ldx) and Y = U_k^T R_l Pi^T (k x n, ldy);
 * sigma (device, k doubles, may be NULL) receives the k leading singular
 * values of R_l.  U_k comes from the eigenvectors of R_l R_l^T (cyclic Jacobi
 * in one workgroup): l <= 128.  tau holds at least l reflectors. */
int rqrcp_compress_workspace_size(int m, int n, int l, int k, int b, size_t *bytes);
int rqrcp_compress(rqrcp_handle h, int m, int n, int l, int k, int b, const double *AF, int ldaf,
                   const double *tau, const int32_t *jpvt, double *X, int ldx, double *Y,
                   int ldy, double *sigma, void *ws, size_t ws_bytes);

/* ---- Backward of the truncated factorization with frozen pivots ----
 * The paper differentiates nothing; this is the adjoint of the map
 * A -> (Q1, R~), R~ = [R11 R12] (k x n, pivot order), A Pi ~ Q1 R~ (Section I-A),
 * with Pi held fixed.  Its pieces are R12 = Q1^T A2 and the QR A1 = Q1 R11 of
 * the k pivoted columns:
 *   A2_bar = Q1 R12_bar;  Q1_bar' = Q1_bar + A2 R12_bar^T;
 *   M = R11 R11_bar^T - Q1_bar'^T Q1;
 *   A1_bar = (Q1_bar' + Q1 (tril(M) + tril(M,-1)^T)) R11^-T;
 *   A_bar(:, jpvt[j]) = [A1_bar A2_bar](:, j).
 * Q1 and every block's T are recomputed from (V, tau); products on MFMA in
 * the storage precision a_type (RQRCP_F64 or RQRCP_F32).
 *  A      (in) the original m x n matrix (lda), unpivoted.
 *  AF     (in) its factorization from rqrcp_factor (ldaf, same a_type), tau, jpvt.
 *         jpvt is checked on the device: if it is not a permutation of 0..n-1,
 *         rqrcp_check(h, ws) returns RQRCP_ERR_PIVOTS and dA is not usable.
 *  dQ1    (in) m x k cotangent of Q1 (ldq), or NULL for zero.
 *  dR     (in) k x n cotangent of R~ in pivot order (ldr), or NULL for zero.
 *  dA     (out) m x n (ldda), original column order.
 * Limits: k <= 1024. */
int rqrcp_backward_workspace_size(int m, int n, int k, int b, int a_type, size_t *bytes);
int rqrcp_backward(rqrcp_handle h, int m, int n, int k, int b, int a_type, const void *A, int lda,
                   const void *AF, int ldaf, const double *tau, const int32_t *jpvt,
                   const void *dQ1, int ldq, const void *dR, int ldr, void *dA, int ldda,
                   void *ws, size_t ws_bytes);

/* ---- Batched RQRCP of many small, uneven FP32 matrices ----
 * One persistent launch: each workgroup factors one problem at a time (Alg. 2
 * with FP64 sketch, reflectors and sample update, FP32 storage and trailing
 * update) and takes the next problem from a work queue in the workspace, so
 * the call allocates nothing, synchronizes nothing and can be captured in a
 * HIP graph.  Problem j draws its Omega from Philox(prm->seed, stream j + 1).
 * Descriptors are device data; offsets count elements of the pools. */
typedef struct {
  int64_t a_off;    /* A_j at A_pool + a_off: m x n FP32, column-major, leading dim lda */
  int64_t b_off;    /* final sketch at B_pool + b_off: (b+p) x n FP64, leading dim b+p */
  int64_t jpvt_off; /* n ints at jpvt_pool + jpvt_off */
  int64_t tau_off;  /* k doubles at tau_pool + tau_off */
  int32_t m, n, k, lda;
} rqrcp_problem;

/* Limits of the batched kernel (host outputs): m <= max_m, (b+p) n <= max_ln,
 * n <= 1024, b <= max_b, b + p <= max_l; a problem's extent (n-1) lda + m is
 * below 2^31 elements. */
int rqrcp_batched_limits(int *max_m, int *max_ln, int *max_b, int *max_l);
int rqrcp_batched_workspace_size(size_t *bytes);
/* Factor `batch` problems in place (A_j -> R, V, R22 in LAPACK storage).
 * prm: a_type = RQRCP_F32, sketch_type = RQRCP_F64, b, p, seed.  *_elems are the
 * pool sizes in elements; a problem whose descriptor does not fit the kernel's
 * limits or the pools is skipped with info[j] = -1; a sketch with a non-finite
 * value stops that problem's pivoting with info[j] = -2.  info[j] otherwise as in
 * rqrcp_factor.  The kernel variant comes from the library's tuning table
 * (rqrcp_autotune_batched; one per device, shared by all handles of the
 * process), default variant 0. */
int rqrcp_factor_batched(rqrcp_handle h, int batch, const rqrcp_problem *probs,
                         const rqrcp_params *prm, float *A_pool, int64_t a_elems,
                         int32_t *jpvt_pool, int64_t jpvt_elems, double *tau_pool,
                         int64_t tau_elems, double *B_pool, int64_t b_elems, int32_t *info,
                         void *ws, size_t ws_bytes);
/* Autotuner: for every kernel variant, restores A_pool from A_orig (a device
 * copy of the inputs with the same layout, a_elems floats), runs the variant
 * twice and times the second run with HIP events; stores the fastest in the
 * library's table for (device, b, b+p) and finally runs it once more, so the outputs
 * hold its factorization.  Synchronizes.  best_variant and ms_per_variant
 * (host, may be NULL; at most 8 entries) report the measurements. */
int rqrcp_autotune_batched(rqrcp_handle h, int batch, const rqrcp_problem *probs,
                           const rqrcp_params *prm, float *A_pool, int64_t a_elems,
                           int32_t *jpvt_pool, int64_t jpvt_elems, double *tau_pool,
                           int64_t tau_elems, double *B_pool, int64_t b_elems, int32_t *info,
                           void *ws, size_t ws_bytes, const float *A_orig, int *best_variant,
                           float *ms_per_variant);

/* Synchronizes the handle's stream and returns RQRCP_ERR_PIVOTS if a caller's
 * frozen permutation (rqrcp_factor, rqrcp_backward) was invalid,
 * RQRCP_ERR_NUMERIC if the sketch QRCP found no valid pivot (a non-finite
 * sketch; it stops pivoting, and the factorization is not usable),
 * RQRCP_ERR_BARRIER if a persistent kernel reported a barrier timeout since the
 * last check (the flags are cleared), RQRCP_ERR_HIP on a HIP error, else 0.
 * `ws` is the workspace the kernels ran with; NULL after rqrcp_factor_noalloc
 * (its flags are in the static scratch), or to check for HIP errors only.
 *
 * The persistent kernels (sketch QRCP, stepwise panel, batched) need all
 * their workgroups resident at once.  The library checks this with the
 * occupancy API for an otherwise idle device; other work running
 * concurrently on the device (another stream, another process) can keep
 * some workgroups from starting, and the bounded waits then end with
 * RQRCP_ERR_BARRIER instead of hanging.  Run factorizations with the device
 * to themselves. */
int rqrcp_check(rqrcp_handle h, void *ws);

/* Per-phase timing for benchmarks.  While enabled, rqrcp_factor and
 * rqrcp_sketch record a HIP event pair on the handle's stream around every
 * kernel launch, tagged with its phase and the launch's algorithmic work
 * (flops and HBM bytes of the operation it performs, not of padding). */
#define RQRCP_PHASE_SKETCH 0  /* Omega and B = Omega A */
#define RQRCP_PHASE_QRCP 1    /* partial QRCP of the sketch */
#define RQRCP_PHASE_SWAP 2    /* column moves */
#define RQRCP_PHASE_PANEL 3   /* panel QR + T */
#define RQRCP_PHASE_TRAIL 4   /* per-block W = V^T A2 pass */
#define RQRCP_PHASE_BUPDATE 5 /* W and R12 corrections, W' = T^T W, the sample update */
#define RQRCP_PHASE_OTHER 6
#define RQRCP_PHASE_FINAL 7   /* the deferred update A2 -= V W' of an outer block */
#define RQRCP_NPHASES 8
int rqrcp_set_timing(rqrcp_handle h, int enable);
/* Synchronizes the stream, then returns and clears the totals since the last
 * read (host arrays of RQRCP_NPHASES entries, any may be NULL): elapsed
 * milliseconds, number of launches, algorithmic flops and bytes. */
int rqrcp_read_timing(rqrcp_handle h, double *ms, int *count, double *flops, double *bytes);

/* Human-readable text of a status code (static storage). */
const char *rqrcp_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* RQRCP_H */
