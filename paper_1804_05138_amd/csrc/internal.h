// Host-side launchers shared between the kernel translation units and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rqrcp.h"
#include "common.h"

namespace rq {

// Scratch of the persistent sketch-QRCP kernel (lives in the workspace).
struct QrcpScratch {
  GridBarrier bar;
  int npairs;
  int pad[63];
};

// Scratch of the persistent panel kernel: the barrier and its group counters.
struct PanelScratch {
  GridBarrier bar;
  unsigned sub[64 * 32];  // up to 1024 workgroups, one line per group of 16
  int cq_flag[64];        // 1: the Cholesky-QR panel path produced the panel
};

constexpr int MAX_B = 128;      // largest block size b the kernels accept
constexpr int MAX_L = 160;      // largest b + p the kernels accept

// Omega (rows x cols, column-major, leading dimension ld) from Philox(seed, stream).
int launch_gaussian(hipStream_t s, int rows, int cols, uint64_t seed, uint64_t stream,
                    double* out, long long ld);
// The same Omega stored transposed: out[r * ld + c] = Omega(r, c), ld >= cols
// (rows divisible by 4, else RQ_ERR_LIMIT and nothing is enqueued).
int launch_gaussian_t(hipStream_t s, int rows, int cols, uint64_t seed, uint64_t stream,
                      double* out, long long ld);
// B = Omega A in FP64 with Omega given transposed (omt[r * m + i] = Omega(r, i)),
// through the W-pass product (split-K partials in `partial`, then summed in
// order).  Usable (sketch_t_usable) for even m and lda, l divisible by 4 and
// at most 128, and a 16-byte aligned A; otherwise RQ_ERR_LIMIT, nothing enqueued.
bool sketch_t_usable(int m, int l, const double* a, long long lda);
int launch_sketch_t(hipStream_t s, int m, int n, int l, const double* omt, const double* a,
                    long long lda, double* b, long long ldb, double* partial);

// B(0:l, 0:n) = Omega(0:l, 0:m) * A(0:m, 0:n), column-major; A in FP64 or
// FP32, Omega and B in FP64.  stype: SK_F64 (FP64 MFMA), SK_BF16 or SK_FP8
// (low-precision MFMA, FP32 accumulation).  `partial` holds split-K partial
// products (sketch_partial_doubles), `lpbuf` the rounded Omega and the FP8
// column scales (sketch_lp_bytes).
enum { SK_F64 = 0, SK_BF16 = 2, SK_FP8 = 3 };
size_t sketch_partial_doubles(int m, int n, int l);
size_t sketch_lp_bytes(int m, int n, int l, int stype);
template <typename TA>
int launch_sketch(hipStream_t s, int m, int n, int l, int stype, const double* om, long long ldo,
                  const TA* a, long long lda, double* b, long long ldb, double* partial,
                  void* lpbuf);

// Partial QRCP (Alg. 1) on the l x nc block of B starting at column c0.
// On exit B holds the transformed block with its columns in pivot order;
// `pairs` (2 ints per entry: destination position, source position, both
// relative to c0) lists every column that moved, `scr->npairs` their count.
int qrcp_sketch_grid(int l, int nc);
int launch_qrcp_sketch(hipStream_t s, double* b, long long ldb, int l, int c0, int nc,
                       int nsteps, int gstep0, QrcpScratch* scr, double* cand, int* pairs,
                       int* info);
size_t qrcp_cand_doubles(int l, int nc);

// QR with tournament pivoting in place of launch_qrcp_sketch (same outputs):
// b <= tournament_max_b(), l <= tournament_max_l(); ws of tournament_bytes(n).
size_t tournament_bytes(int n);
int tournament_max_b();
int tournament_max_l();
int launch_qrcp_tournament(hipStream_t s, double* b, long long ldb, int l, int c0, int nc,
                           int nsteps, int gstep0, QrcpScratch* scr, int* pairs, int* info,
                           char* ws);

// Column moves from `pairs` (count at *npairs) applied to A(0:m, c0 + .),
// jpvt(c0 + .) and W'(0:wrows, w0 + .) (W' may be null).
template <typename T, typename WT = double>
int launch_apply_pairs(hipStream_t s, int m, T* a, long long lda, int c0, int* jpvt, WT* wp,
                       int wrows, long long ldw, int w0, const int* pairs, const int* npairs,
                       int max_pairs);

// Panel QR of A(i:m, i:i+bb) with the previous block's pending update
// A(ip:m, i:i+bb) -= Vprev * Wp(:, 0:bb) applied first (if bbp > 0, ip = i - bbp).
// Writes V/R in place, tau(i:i+bb) and T (bb x bb, column-major, ld bb).
// T is the storage type of A (double or float); the arithmetic is FP64.
// stepwise_only: one reflector at a time (no Cholesky-QR2).
int panel_grid(int rows, int bb);
template <typename T>
int launch_panel(hipStream_t s, int m, T* a, long long lda, int i, int bb, int bbp,
                 const double* wp, long long ldw, double* tau, double* t, PanelScratch* scr,
                 double* partial, bool stepwise_only);
size_t panel_partial_doubles(int rows, int bb);
// Cholesky-QR2 panel path (k_panel_cq.hip), used by launch_panel for bb <= 64
// and panels at least twice as tall as wide.
bool panel_cq_applicable(int m, int i, int bb);
size_t panel_cq_doubles(int rows);
template <typename T>
int launch_panel_cq(hipStream_t s, int m, T* a, long long lda, int i, int bb, int bbp,
                    const double* wp, long long ldw, double* tau, double* tmat, double* scratch,
                    int* flag);
// Pieces for blocks wider than 64 (two 64-wide halves): the pending update of
// columns i+coff .. i+coff+nc, C = A^T B (CB x CB, fixed-order sum), W' =
// T1^T Y and the T of the whole block.
template <typename T>
int launch_cq_pend(hipStream_t s, int m, T* a, long long lda, int i, int coff, int nc, int bbp,
                   const double* wp, long long ldw);
size_t cq_wide_doubles(int rows);
template <typename T>
int launch_cq_cross(hipStream_t s, int rows, const T* A, long long lda, int na, int adiag,
                    const T* B, long long ldb, int nb, int bdiag, double* part, double* c);
int launch_cq_tty(hipStream_t s, int nb, const double* t1, const double* y, double* w);
int launch_cq_tcombine(hipStream_t s, int nb, const double* t1, const double* t2, const double* z,
                       double* t);

// From the split partials of W = V^T A2 (bb x ncols): W' = T^T W (stored at wp),
// then R12 = A(i:i+bb, c) - V11 W'(:, c), X = R11^-1 R12 and
// B(0:bb, c) -= Rhat11 X for the columns c = c0 .. c0 + ncols - 1 (skipped when
// *info != 0).  Rhat11 = triu(B(0:bb, i:i+bb)).  With r12out (the matrix A
// itself), R12 is also stored to rows i..i+bb of the columns.  Partial z of W
// starts at wpart + z pstride bb (pstride = 0: ncols).
template <typename T>
int launch_bupdate(hipStream_t s, int m, const T* a, long long lda, int i, int bb,
                   const double* t, const T* wpart, int nsplit, double* wp, long long ldw,
                   double* bsk, long long ldb, int c0, int ncols, const int* info,
                   T* r12out = nullptr, long long pstride = 0);

// Batched RQRCP (k_batched.hip): variant v of the persistent kernel.
int batched_variants();
const char* batched_variant_name(int v);
int batched_max(int* max_m, int* max_ln, int* max_b, int* max_l);
int launch_batched(hipStream_t s, int variant, int batch, const rqrcp_problem* probs, int b, int l,
                   uint64_t seed, float* apool, long long a_elems, int* jpool, long long j_elems,
                   double* tpool, long long t_elems, double* bpool, long long b_elems, int* infos,
                   unsigned* queue);

// Level-3 QR with column pivoting of the whole matrix (Alg. 1 organized as
// xGEQP3; k_qrcp_full.hip): k steps, block size nb, FP64.
size_t qrcp_full_workspace(int m, int n, int k, int nb);
int qrcp_full_max_nb();
int launch_qrcp_full(hipStream_t st, int m, int n, int k, int nb, double* a, long long lda,
                     int* jpvt, double* tau, char* ws);

// Explicit Q1 = H_0 ... H_{k-1} [I; 0] (m x k) from LAPACK storage.
int launch_form_q(hipStream_t s, int m, int k, int b, const double* a, long long lda,
                  const double* tau, double* q, long long ldq, double* work);

}  // namespace rq
