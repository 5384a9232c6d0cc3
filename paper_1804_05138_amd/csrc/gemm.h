// Generic MFMA GEMM and explicit-Q helpers (see k_gemm.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace rq {

// ws (ws_elems elements, may be null): room for split-K partials; used when
// the output has few tiles and K is long.
template <typename T>
int gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, T alpha, const T* A, long long lda,
         const T* B, long long ldb, T beta, T* C, long long ldc, T* ws = nullptr,
         size_t ws_elems = 0);

size_t splitk_elems(int m, int n);

// Large-tile GEMM (k_gemm_big.hip): C = alpha op(A) B + beta C, column-major,
// op(A) = A^T when ta.  With ws (ws_elems elements), a shape with few output
// tiles and a long K is split over K, partial sums in ws added in order.
template <typename T>
int gemm_big(hipStream_t s, bool ta, int M, int N, int K, T alpha, const T* A, long long lda,
             const T* B, long long ldb, T beta, T* C, long long ldc, T* ws = nullptr,
             size_t ws_elems = 0);
// The W pass of the left-looking schedule (FP64 or FP32): raw sums over at most
// max_split K ranges, part[z][n][q] = sum_k V(k, q) B(k, n) (leading dimension
// nq <= 128 in FP64, <= 64 in FP32), with B's columns n < n1 from B1 and the
// rest from B2.  Needs even
// K and leading dimensions and bases aligned to two elements (RQ_ERR_LIMIT
// otherwise).
// Columns of B per workgroup of the W pass: a grid of about 512 workgroups
// (two per CU) is one round.
constexpr int kWpassCols = 128;
template <typename T>
int wpass_partials(hipStream_t s, int K, int nq, int N, int n1, const T* V, long long ldv,
                   const T* B1, long long ld1, const T* B2, long long ld2, T* part,
                   int max_split, int* nsplit_out);
// The raw sums op(A) B of at most max_split K ranges (whole 16-steps) into
// part[z][N][M] (leading dimension M); *nsplit_out = ranges written.
template <typename T>
int gemm_big_partials(hipStream_t s, bool ta, int M, int N, int K, const T* A, long long lda,
                      const T* B, long long ldb, T* part, int max_split, int* nsplit_out);

// Dense V (rows x bb), Gram V^T V and T of one reflector block.
template <typename T>
int block_t(hipStream_t s, int rows, int bb, const T* a, long long lda, const double* tau, T* vd,
            T* gram, T* tm, T* ws = nullptr, size_t ws_elems = 0);

size_t form_q_work_elems(int m, int k, int b);

template <typename T>
int form_q(hipStream_t s, int m, int k, int b, const T* a, long long lda, const double* tau, T* q,
           long long ldq, T* work);

// r11 = triu(AF(0:k, 0:k)) and rinv = r11^-1 (both dense k x k, ld k; k <= 1024).
template <typename T>
int upper_inverse(hipStream_t s, int k, const T* af, long long ldaf, T* r11, T* rinv);

// CX, CUR and the SVD compression of a factorization (k_cur.hip), FP64.
size_t cx_workspace(int n, int k);
int launch_cx(hipStream_t s, int m, int n, int k, const double* af, long long ldaf,
              const int* jpvt, double* x, long long ldx, char* ws);
size_t cur_workspace(int m, int n, int k, int b);
int launch_cur(hipStream_t s, int m, int n, int k, int b, const double* afc, long long ldc,
               const int* jpc, const double* afr, long long ldr, const double* taur,
               double* u, long long ldu, char* ws);
int compress_max_l();
size_t compress_workspace(int m, int n, int l, int k, int b);
int launch_compress(hipStream_t s, int m, int n, int l, int k, int b, const double* af,
                    long long ldaf, const double* tau, const int* jpvt, double* x, long long ldx,
                    double* y, long long ldy, double* sigma, char* ws);

// Frozen-pivot adjoint (k_backward.hip): byte offsets of its workspace.
struct BackwardLayout {
  size_t q1, a2, qb, g, r11, rinv, mm, formq, sk, total;
};
BackwardLayout backward_layout(int m, int n, int k, int b, size_t es);
template <typename T>
int backward(hipStream_t s, int m, int n, int k, int b, const T* a, long long lda, const T* af,
             long long ldaf, const double* tau, const int* jpvt, const T* dq1, long long ldq,
             const T* dr, long long ldr, T* da, long long ldda, char* ws);

}  // namespace rq
