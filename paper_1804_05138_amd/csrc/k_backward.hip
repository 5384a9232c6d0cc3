// Adjoint of the truncated factorization with the pivots frozen.
//
// The function differentiated is A -> (Q1, R~), R~ = [R11 R12] = Q1^T (A Pi)(:, 0:n)
// restricted to the first k rows (Section I-A: A Pi ~ Q1 [R11 R12]); its two
// pieces are R12 = Q1^T A2 and the QR factorization A1 = Q1 R11 of the k
// pivoted columns (Alg. 2's panel factorizations, taken together).  Given the
// cotangents Q1_bar (m x k) and R_bar = [R11_bar R12_bar] (k x n, pivot order):
//
//   A2_bar  = Q1 R12_bar                               (through R12 = Q1^T A2)
//   Q1_bar' = Q1_bar + A2 R12_bar^T
//   M       = R11 R11_bar^T - Q1_bar'^T Q1
//   A1_bar  = (Q1_bar' + Q1 copyltu(M)) R11^-T,  copyltu(M) = tril(M) + tril(M, -1)^T
//                                                      (QR adjoint of A1 = Q1 R11)
//   A_bar(:, jpvt[j]) = [A1_bar A2_bar](:, j)
//
// Q1 is recomputed from the stored reflectors (V, tau) block by block, with
// each block's T rebuilt from V^T V (no WY factor is kept from the forward
// pass).  Every product runs on MFMA in the storage precision (FP32 or FP64);
// R11^-1 is formed in FP64 by one wave per column and rounded to the storage
// type.
#include "gemm.h"
#include "internal.h"

namespace rq {
namespace {

constexpr int BT = 256;

unsigned grid_for(long long total) {
  long long g = (total + BT - 1) / BT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// The permutation is validated before the backward runs (an invalid one is
// reported by rqrcp_check); gather and scatter still clamp its entries to
// [0, n) so that no column outside the matrices is ever addressed.
RQ_DEV long long perm_col(const int* perm, int j, int n) {
  return (long long)min(max(perm[j], 0), n - 1);
}

// dst(:, j) = src(:, perm[c0 + j]) for j < ncols (gather of pivoted columns of
// an m x n source).
template <typename T>
__global__ __launch_bounds__(BT) void k_gather(int m, int n, int ncols, const T* __restrict__ src,
                                               long long lds, const int* __restrict__ perm, int c0,
                                               T* __restrict__ dst, long long ldd) {
  const long long total = (long long)m * ncols;
  for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < total;
       e += (long long)gridDim.x * BT) {
    const long long j = e / m, r = e % m;
    dst[j * ldd + r] = src[perm_col(perm, c0 + (int)j, n) * lds + r];
  }
}

// dst(:, perm[j]) = src(:, j) for all n columns.
template <typename T>
__global__ __launch_bounds__(BT) void k_scatter(int m, int n, const T* __restrict__ src,
                                                long long lds, const int* __restrict__ perm,
                                                T* __restrict__ dst, long long ldd) {
  const long long total = (long long)m * n;
  for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < total;
       e += (long long)gridDim.x * BT) {
    const long long j = e / m, r = e % m;
    dst[perm_col(perm, (int)j, n) * ldd + r] = src[j * lds + r];
  }
}

// dst = src (rows x cols), or zero when src is null.
template <typename T>
__global__ __launch_bounds__(BT) void k_copy_or_zero(int rows, int cols, const T* __restrict__ src,
                                                     long long lds, T* __restrict__ dst,
                                                     long long ldd) {
  const long long total = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < total;
       e += (long long)gridDim.x * BT) {
    const long long j = e / rows, r = e % rows;
    dst[j * ldd + r] = src ? src[j * lds + r] : T(0);
  }
}

// M <- tril(M) + tril(M, -1)^T (k x k, in place; one thread per lower entry).
template <typename T>
__global__ __launch_bounds__(BT) void k_copyltu(int k, T* __restrict__ mm, long long ldm) {
  const long long total = (long long)k * k;
  for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < total;
       e += (long long)gridDim.x * BT) {
    const int j = (int)(e / k), r = (int)(e % k);
    if (r > j) mm[(long long)r * ldm + j] = mm[(long long)j * ldm + r];
  }
}

// Column j of R11^-T's transpose, i.e. column j of R11^-1 (upper triangular),
// by back substitution in FP64: one wave per column, lane l holding rows
// l + 64 s.  out is k x k (ld k), zero below the diagonal.
template <typename T, int RS>
__global__ __launch_bounds__(BT) void k_trinv(int k, const T* __restrict__ r, long long ldr,
                                              T* __restrict__ out) {
  const int j = blockIdx.x * (BT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= k) return;
  double x[RS];
#pragma unroll
  for (int s = 0; s < RS; ++s) x[s] = (64 * s + lane == j) ? 1.0 : 0.0;
  // rows above j: x_i = (x_i - sum_{t > i} R(i, t) x_t) / R(i, i), column-oriented
#pragma unroll
  for (int s = RS - 1; s >= 0; --s) {
    for (int ln = 63; ln >= 0; --ln) {
      const int i = 64 * s + ln;
      if (i > j) continue;
      const double rii = (double)r[(long long)i * ldr + i];
      const double xi = __shfl(x[s], ln, 64) / rii;
      if (lane == ln) x[s] = xi;
      // x(0:i) -= R(0:i, i) xi
#pragma unroll
      for (int s2 = 0; s2 <= s; ++s2) {
        const int row = 64 * s2 + lane;
        if (row < i) x[s2] -= (double)r[(long long)i * ldr + row] * xi;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int row = 64 * s + lane;
    if (row < k) out[(long long)j * k + row] = (row <= j) ? (T)x[s] : T(0);
  }
}

// upper triangle of AF(0:k, 0:k) -> dense k x k (zero below the diagonal)
template <typename T>
__global__ __launch_bounds__(BT) void k_triu(int k, const T* __restrict__ af, long long ldaf,
                                             T* __restrict__ out) {
  const long long total = (long long)k * k;
  for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < total;
       e += (long long)gridDim.x * BT) {
    const int j = (int)(e / k), r = (int)(e % k);
    out[e] = (r <= j) ? af[(long long)j * ldaf + r] : T(0);
  }
}

template <typename T>
int launch_trinv(hipStream_t s, int k, const T* r, long long ldr, T* out) {
  const dim3 grid((k + 3) / 4);
  if (k <= 64)
    hipLaunchKernelGGL((k_trinv<T, 1>), grid, dim3(BT), 0, s, k, r, ldr, out);
  else if (k <= 256)
    hipLaunchKernelGGL((k_trinv<T, 4>), grid, dim3(BT), 0, s, k, r, ldr, out);
  else if (k <= 1024)
    hipLaunchKernelGGL((k_trinv<T, 16>), grid, dim3(BT), 0, s, k, r, ldr, out);
  else
    return RQ_ERR_LIMIT;
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace

template <typename T>
int upper_inverse(hipStream_t s, int k, const T* af, long long ldaf, T* r11, T* rinv) {
  hipLaunchKernelGGL(k_triu<T>, dim3(grid_for((long long)k * k)), dim3(BT), 0, s, k, af, ldaf, r11);
  RQ_HIP_CHECK(hipGetLastError());
  return launch_trinv<T>(s, k, r11, k, rinv);
}
template int upper_inverse<double>(hipStream_t, int, const double*, long long, double*, double*);
template int upper_inverse<float>(hipStream_t, int, const float*, long long, float*, float*);

BackwardLayout backward_layout(int m, int n, int k, int b, size_t es) {
  BackwardLayout L;
  size_t off = 0;
  auto take = [&](size_t elems) {
    const size_t o = off;
    off += (elems * es + 255) / 256 * 256;
    return o;
  };
  L.q1 = take((size_t)m * k);
  L.a2 = take((size_t)m * (n - k > 0 ? n - k : 1));
  L.qb = take((size_t)m * k);
  L.g = take((size_t)m * n);
  L.r11 = take((size_t)k * k);
  L.rinv = take((size_t)k * k);
  L.mm = take((size_t)k * k);
  L.formq = take(form_q_work_elems(m, k, b));
  L.sk = take(splitk_elems(k, k));
  L.total = off;
  return L;
}

template <typename T>
int backward(hipStream_t s, int m, int n, int k, int b, const T* a, long long lda, const T* af,
             long long ldaf, const double* tau, const int* jpvt, const T* dq1, long long ldq,
             const T* dr, long long ldr, T* da, long long ldda, char* ws) {
  if (k > 1024) return RQ_ERR_LIMIT;
  const BackwardLayout L = backward_layout(m, n, k, b, sizeof(T));
  T* q1 = (T*)(ws + L.q1);
  T* a2 = (T*)(ws + L.a2);
  T* qb = (T*)(ws + L.qb);
  T* g = (T*)(ws + L.g);
  T* r11 = (T*)(ws + L.r11);
  T* rinv = (T*)(ws + L.rinv);
  T* mm = (T*)(ws + L.mm);
  T* fq = (T*)(ws + L.formq);
  T* sk = (T*)(ws + L.sk);
  const size_t skn = splitk_elems(k, k);
  const int n2 = n - k;
  int rc;
  // Q1 from (V, tau), A2 = (A Pi)(:, k:n), R11
  rc = form_q<T>(s, m, k, b, af, ldaf, tau, q1, m, fq);
  if (rc) return rc;
  if (n2 > 0)
    hipLaunchKernelGGL(k_gather<T>, dim3(grid_for((long long)m * n2)), dim3(BT), 0, s, m, n, n2,
                       a, lda, jpvt, k, a2, (long long)m);
  hipLaunchKernelGGL(k_triu<T>, dim3(grid_for((long long)k * k)), dim3(BT), 0, s, k, af, ldaf, r11);
  RQ_HIP_CHECK(hipGetLastError());
  rc = launch_trinv<T>(s, k, r11, k, rinv);
  if (rc) return rc;
  // Q1_bar' = Q1_bar + A2 R12_bar^T
  hipLaunchKernelGGL(k_copy_or_zero<T>, dim3(grid_for((long long)m * k)), dim3(BT), 0, s, m, k, dq1,
                     ldq, qb, (long long)m);
  RQ_HIP_CHECK(hipGetLastError());
  const T* r12b = dr ? dr + (long long)k * ldr : nullptr;
  if (dr && n2 > 0) {
    rc = gemm<T>(s, false, true, m, k, n2, T(1), a2, m, r12b, ldr, T(1), qb, m);
    if (rc) return rc;
    // A2_bar = Q1 R12_bar -> G(:, k:n)
    rc = gemm<T>(s, false, false, m, n2, k, T(1), q1, m, r12b, ldr, T(0), g + (long long)k * m, m);
    if (rc) return rc;
  } else if (n2 > 0) {
    hipLaunchKernelGGL(k_copy_or_zero<T>, dim3(grid_for((long long)m * n2)), dim3(BT), 0, s, m, n2,
                       (const T*)nullptr, 0LL, g + (long long)k * m, (long long)m);
    RQ_HIP_CHECK(hipGetLastError());
  }
  // M = R11 R11_bar^T - Q1_bar'^T Q1
  if (dr) {
    rc = gemm<T>(s, false, true, k, k, k, T(1), r11, k, dr, ldr, T(0), mm, k);
  } else {
    hipLaunchKernelGGL(k_copy_or_zero<T>, dim3(grid_for((long long)k * k)), dim3(BT), 0, s, k, k,
                       (const T*)nullptr, 0LL, mm, (long long)k);
    rc = RQ_OK;
  }
  if (rc) return rc;
  rc = gemm<T>(s, true, false, k, k, m, T(-1), qb, m, q1, m, T(1), mm, k, sk, skn);
  if (rc) return rc;
  hipLaunchKernelGGL(k_copyltu<T>, dim3(grid_for((long long)k * k)), dim3(BT), 0, s, k, mm,
                     (long long)k);
  RQ_HIP_CHECK(hipGetLastError());
  // Q1_bar' + Q1 copyltu(M), then A1_bar = (.) R11^-T -> G(:, 0:k)
  rc = gemm<T>(s, false, false, m, k, k, T(1), q1, m, mm, k, T(1), qb, m);
  if (rc) return rc;
  rc = gemm<T>(s, false, true, m, k, k, T(1), qb, m, rinv, k, T(0), g, m);
  if (rc) return rc;
  // back to the original column order
  hipLaunchKernelGGL(k_scatter<T>, dim3(grid_for((long long)m * n)), dim3(BT), 0, s, m, n,
                     (const T*)g, (long long)m, jpvt, da, ldda);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int backward<double>(hipStream_t, int, int, int, int, const double*, long long,
                              const double*, long long, const double*, const int*, const double*,
                              long long, const double*, long long, double*, long long, char*);
template int backward<float>(hipStream_t, int, int, int, int, const float*, long long,
                             const float*, long long, const double*, const int*, const float*,
                             long long, const float*, long long, float*, long long, char*);

}  // namespace rq
