// General column-major GEMM on MFMA, C = alpha op(A) op(B) + beta C, for
// FP64 (v_mfma_f64_16x16x4f64) and FP32 (v_mfma_f32_16x16x4f32), plus the
// small helpers that turn LAPACK-stored reflectors into an explicit Q1:
//   Q1 = H_0 H_1 ... H_{k-1} [I; 0], applied block by block in reverse with
//   the compact WY form I - V T V^T, T recomputed from V^T V and tau
//   (forward, columnwise, as PDLARFT forms it).
// 64x64 output tiles, K tiles of 16 staged in LDS, 4 waves of 32x32.
#include "internal.h"
#include "gemm.h"

namespace rq {
namespace {

constexpr int GT = 256;
constexpr int TM = 64, TN = 64, TK = 16;

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static RQ_DEV acc_t run(double a, double b, acc_t c) { return mfma_f64(a, b, c); }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static RQ_DEV acc_t run(float a, float b, acc_t c) { return mfma_f32(a, b, c); }
};

template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(GT) void k_gemm(int M, int N, int K, T alpha, const T* __restrict__ A,
                                             long long lda, const T* __restrict__ B, long long ldb,
                                             T beta, T* __restrict__ C, long long ldc) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T sA[TK][TM + 1];
  __shared__ T sB[TK][TN + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = acc_t{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
    for (int j = 0; j < (TM * TK) / GT; ++j) {
      const int e = tid + GT * j;
      int mi, ki;
      if (!TA) { mi = e % TM; ki = e / TM; } else { ki = e % TK; mi = e / TK; }
      const int gm = m0 + mi, gk = k0 + ki;
      T v = 0;
      if (gm < M && gk < K) v = TA ? A[(long long)gm * lda + gk] : A[(long long)gk * lda + gm];
      sA[ki][mi] = v;
    }
#pragma unroll
    for (int j = 0; j < (TN * TK) / GT; ++j) {
      const int e = tid + GT * j;
      int ni, ki;
      if (!TB) { ki = e % TK; ni = e / TK; } else { ni = e % TN; ki = e / TN; }
      const int gn = n0 + ni, gk = k0 + ki;
      T v = 0;
      if (gn < N && gk < K) v = TB ? B[(long long)gk * ldb + gn] : B[(long long)gn * ldb + gk];
      sB[ki][ni] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < TK / 4; ++kq) {
      T av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = sA[4 * kq + lg][wm + 16 * x + lr16];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = sB[4 * kq + lg][wn + 16 * y + lr16];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<T>::run(av[x], bv[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wm + 16 * x + acc_row<T>(lg, e);
        const int gn = n0 + wn + 16 * y + lr16;
        if (gm < M && gn < N) {
          T* c = C + (long long)gn * ldc + gm;
          const T v = alpha * acc[x][y][e];
          *c = (beta == T(0)) ? v : v + beta * (*c);
        }
      }
}

template <typename T>
__global__ void k_eye(int m, int k, T* __restrict__ q, long long ldq) {
  const long long total = (long long)m * k;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long c = e / m, r = e % m;
    q[c * ldq + r] = (r == c) ? T(1) : T(0);
  }
}

// Dense copy of the unit lower trapezoidal V = A(i:m, i:i+bb) (reflectors).
template <typename T>
__global__ void k_extract_v(int rows, int bb, const T* __restrict__ a, long long lda,
                            T* __restrict__ v) {
  const long long total = (long long)rows * bb;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e / rows), r = (int)(e % rows);
    v[e] = (r > c) ? a[(long long)c * lda + r] : (r == c ? T(1) : T(0));
  }
}

// T (bb x bb, upper, column-major) from the Gram matrix G = V^T V and tau:
// T(t,t) = tau_t, T(0:t, t) = -tau_t T(0:t, 0:t) G(0:t, t).
template <typename T>
__global__ void k_larft(int bb, const T* __restrict__ gm, const double* __restrict__ tau,
                        T* __restrict__ tm) {
  __shared__ double s[MAX_B * MAX_B];
  const int tid = threadIdx.x;
  for (int e = tid; e < bb * bb; e += blockDim.x) s[e] = 0.0;
  __syncthreads();
  for (int t = 0; t < bb; ++t) {
    const double tt = tau[t];
    if (tid < t) {
      double acc = 0.0;
      for (int c = tid; c < t; ++c) acc += s[c * bb + tid] * (double)gm[t * bb + c];
      s[t * bb + tid] = -tt * acc;
    }
    if (tid == t) s[t * bb + t] = tt;
    __syncthreads();
  }
  for (int e = tid; e < bb * bb; e += blockDim.x) tm[e] = (T)s[e];
}

}  // namespace

template <typename T>
int gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, T alpha, const T* A, long long lda,
         const T* B, long long ldb, T beta, T* C, long long ldc) {
  if (M <= 0 || N <= 0) return RQ_OK;
  dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN);
  if (K <= 0) {
    // C = beta C: run with K = 0 (the loop body is skipped)
  }
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, false, false>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, true, false>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<T, false, true>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc);
  else
    hipLaunchKernelGGL((k_gemm<T, true, true>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

template int gemm<double>(hipStream_t, bool, bool, int, int, int, double, const double*, long long,
                          const double*, long long, double, double*, long long);
template int gemm<float>(hipStream_t, bool, bool, int, int, int, float, const float*, long long,
                         const float*, long long, float, float*, long long);

static unsigned grid_for(long long total) {
  long long g = (total + GT - 1) / GT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
int block_t(hipStream_t s, int rows, int bb, const T* a, long long lda, const double* tau, T* vd,
            T* gram, T* tm) {
  hipLaunchKernelGGL(k_extract_v<T>, dim3(grid_for((long long)rows * bb)), dim3(GT), 0, s, rows,
                     bb, a, lda, vd);
  int rc = gemm<T>(s, true, false, bb, bb, rows, T(1), vd, rows, vd, rows, T(0), gram, bb);
  if (rc) return rc;
  hipLaunchKernelGGL(k_larft<T>, dim3(1), dim3(GT), 0, s, bb, gram, tau, tm);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int block_t<double>(hipStream_t, int, int, const double*, long long, const double*,
                             double*, double*, double*);
template int block_t<float>(hipStream_t, int, int, const float*, long long, const double*, float*,
                            float*, float*);

size_t form_q_work_elems(int m, int k, int b) {
  const size_t bb = (size_t)(b < k ? b : k);
  return (size_t)m * bb + 2 * bb * bb + 2 * bb * (size_t)k + 64;
}

template <typename T>
int form_q(hipStream_t s, int m, int k, int b, const T* a, long long lda, const double* tau, T* q,
           long long ldq, T* work) {
  hipLaunchKernelGGL(k_eye<T>, dim3(grid_for((long long)m * k)), dim3(GT), 0, s, m, k, q, ldq);
  RQ_HIP_CHECK(hipGetLastError());
  const int nblk = (k + b - 1) / b;
  const int bbmax = b < k ? b : k;
  T* vd = work;
  T* gram = vd + (size_t)m * bbmax;
  T* tm = gram + (size_t)bbmax * bbmax;
  T* y = tm + (size_t)bbmax * bbmax;
  T* z = y + (size_t)bbmax * k;
  for (int j = nblk - 1; j >= 0; --j) {
    const int ij = j * b;
    const int bb = (k - ij) < b ? (k - ij) : b;
    const int rows = m - ij;
    const int nc = k - ij;
    int rc = block_t<T>(s, rows, bb, a + (long long)ij * lda + ij, lda, tau + ij, vd, gram, tm);
    if (rc) return rc;
    T* qs = q + (long long)ij * ldq + ij;
    rc = gemm<T>(s, true, false, bb, nc, rows, T(1), vd, rows, qs, ldq, T(0), y, bb);
    if (rc) return rc;
    rc = gemm<T>(s, false, false, bb, nc, bb, T(1), tm, bb, y, bb, T(0), z, bb);
    if (rc) return rc;
    rc = gemm<T>(s, false, false, rows, nc, bb, T(-1), vd, rows, z, bb, T(1), qs, ldq);
    if (rc) return rc;
  }
  return RQ_OK;
}
template int form_q<double>(hipStream_t, int, int, int, const double*, long long, const double*,
                            double*, long long, double*);
template int form_q<float>(hipStream_t, int, int, int, const float*, long long, const double*,
                           float*, long long, float*);

int launch_form_q(hipStream_t s, int m, int k, int b, const double* a, long long lda,
                  const double* tau, double* q, long long ldq, double* work) {
  return form_q<double>(s, m, k, b, a, lda, tau, q, ldq, work);
}

}  // namespace rq
