// General column-major GEMM on MFMA, C = alpha op(A) op(B) + beta C, for
// FP64 (v_mfma_f64_16x16x4f64) and FP32 (v_mfma_f32_16x16x4f32), plus the
// small helpers that turn LAPACK-stored reflectors into an explicit Q1:
//   Q1 = H_0 H_1 ... H_{k-1} [I; 0], applied block by block in reverse with
//   the compact WY form I - V T V^T, T recomputed from V^T V and tau
//   (forward, columnwise, as PDLARFT forms it).
// 64x64 output tiles, K steps of 32 double-buffered in LDS, 4 waves of 32x32.
#include "internal.h"
#include "gemm.h"

namespace rq {
namespace {

constexpr int GT = 256;
constexpr int TM = 64, TN = 64, TK = 32;

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

// blockIdx.z selects the K range [z kchunk, (z+1) kchunk); with part != null the
// raw sums go to part[z][N][M] (split K, summed by k_splitk_sum), else to C.
// K steps of TK are double-buffered in LDS: the global loads of step t+1 are
// in flight (in registers) while step t runs on the MFMAs, one barrier per step.
template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(GT, 2) void k_gemm(int M, int N, int K, T alpha,
                                                const T* __restrict__ A, long long lda,
                                                const T* __restrict__ B, long long ldb, T beta,
                                                T* __restrict__ C, long long ldc, int kchunk,
                                                T* __restrict__ part) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NLA = TM * TK / GT, NLB = TN * TK / GT;
  __shared__ T sA[2][TK][TM + 1];
  __shared__ T sB[2][TK][TN + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = acc_t{0, 0, 0, 0};

  T ra[NLA], rb[NLB];
  // coalesced: consecutive threads walk the contiguous index of each operand
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < NLA; ++j) {
      const int e = tid + GT * j;
      int mi, ki;
      if (!TA) { mi = e % TM; ki = e / TM; } else { ki = e % TK; mi = e / TK; }
      const int gm = m0 + mi, gk = k0 + ki;
      const bool ok = gm < M && gk < ke;
      const int gms = ok ? gm : 0, gks = ok ? gk : kb;
      const T v = TA ? A[(long long)gms * lda + gks] : A[(long long)gks * lda + gms];
      ra[j] = ok ? v : T(0);
    }
#pragma unroll
    for (int j = 0; j < NLB; ++j) {
      const int e = tid + GT * j;
      int ni, ki;
      if (!TB) { ki = e % TK; ni = e / TK; } else { ni = e % TN; ki = e / TN; }
      const int gn = n0 + ni, gk = k0 + ki;
      const bool ok = gn < N && gk < ke;
      const int gns = ok ? gn : 0, gks = ok ? gk : kb;
      const T v = TB ? B[(long long)gks * ldb + gns] : B[(long long)gns * ldb + gks];
      rb[j] = ok ? v : T(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NLA; ++j) {
      const int e = tid + GT * j;
      int mi, ki;
      if (!TA) { mi = e % TM; ki = e / TM; } else { ki = e % TK; mi = e / TK; }
      sA[buf][ki][mi] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < NLB; ++j) {
      const int e = tid + GT * j;
      int ni, ki;
      if (!TB) { ki = e % TK; ni = e / TK; } else { ni = e % TN; ki = e / TN; }
      sB[buf][ki][ni] = rb[j];
    }
  };

  if (kb < ke) {
    load(kb);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += TK) {
    const bool more = k0 + TK < ke;
    if (more) load(k0 + TK);
#pragma unroll
    for (int kq = 0; kq < TK / 4; ++kq) {
      T av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = sA[buf][4 * kq + lg][wm + 16 * x + lr16];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = sB[buf][4 * kq + lg][wn + 16 * y + lr16];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<T>::run(av[x], bv[y], acc[x][y]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
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
          if (part) {
            part[((size_t)blockIdx.z * N + gn) * M + gm] = acc[x][y][e];
          } else {
            T* c = C + (long long)gn * ldc + gm;
            const T v = alpha * acc[x][y][e];
            *c = (beta == T(0)) ? v : v + beta * (*c);
          }
        }
      }
}

// C = alpha sum_z part[z] + beta C, the split-K partials added in order.
template <typename T>
__global__ void k_splitk_sum(int M, int N, int S, const T* __restrict__ part, T alpha, T beta,
                             T* __restrict__ C, long long ldc) {
  const long long total = (long long)M * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    T acc = part[e];
    for (int z = 1; z < S; ++z) acc += part[(size_t)z * total + e];
    T* c = C + (e / M) * ldc + e % M;
    const T v = alpha * acc;
    *c = (beta == T(0)) ? v : v + beta * (*c);
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

// T (bb x bb, upper, column-major) from the Gram matrix G = V^T V and tau.
// The forward recurrence T(0:t, t) = -tau_t T(0:t, 0:t) G(0:t, t), T(t, t) =
// tau_t has the closed-form inverse T^-1 = triu(G, 1) + diag(1 / tau) (block
// inversion of one step of the recurrence), so T is one triangular inverse.
// A reflector with tau = 0 is the identity: its row and column of T are zero,
// and dropping its index from M = T^-1 leaves the other entries unchanged.
// One workgroup: row r of [M | I] in lane r of every wave, wave w holding
// columns 16w .. 16w+15 of the inverse; backward elimination with the pivot
// row of each wave's slice taken from lane j by readlane (no barrier per step);
// each lane stores its row once it is final.
// The recurrence itself, for blocks wider than 64 (one workgroup, FP64).
template <typename T>
__global__ void k_larft_seq(int bb, const T* __restrict__ gm, const double* __restrict__ tau,
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

template <typename T>
__global__ __launch_bounds__(256) void k_larft(int bb, const T* __restrict__ gm,
                                               const double* __restrict__ tau,
                                               T* __restrict__ tm) {
  constexpr int P = MAX_B / 2 + 1;   // bb <= 64 here
  __shared__ double sM[(MAX_B / 2) * P];
  __shared__ double sTau[MAX_B / 2];
  const int tid = threadIdx.x;
  for (int e = tid; e < bb; e += 256) sTau[e] = tau[e];
  __syncthreads();
  for (int e = tid; e < bb * bb; e += 256) {
    const int c = e / bb, r = e % bb;
    const bool live = sTau[r] != 0.0 && sTau[c] != 0.0;
    double v = 0.0;
    if (r == c) v = sTau[c] != 0.0 ? 1.0 / sTau[c] : 1.0;
    else if (r < c && live) v = (double)gm[c * bb + r];
    sM[c * P + r] = v;
  }
  __syncthreads();
  const int r = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  double a[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = (r == 16 * w + i) ? 1.0 : 0.0;
  for (int j = bb - 1; j >= 0; --j) {
    const double mult = (r < j) ? sM[j * P + r] / sM[j * P + j] : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = fma(-mult, readlane_f64(a[i], j), a[i]);
  }
  // row r is final since step r (later steps only touch the rows above their pivot)
  if (r < bb) {
    const double inv = 1.0 / sM[r * P + r];
    const bool lr = sTau[r] != 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int c = 16 * w + i;
      if (c < bb) tm[c * bb + r] = (c >= r && lr && sTau[c] != 0.0) ? (T)(a[i] * inv) : T(0);
    }
  }
}

}  // namespace

static unsigned grid_for(long long total) {
  long long g = (total + GT - 1) / GT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
int gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, T alpha, const T* A, long long lda,
         const T* B, long long ldb, T beta, T* C, long long ldc, T* ws, size_t ws_elems) {
  if (M <= 0 || N <= 0) return RQ_OK;
  const int tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  // few output tiles and a long reduction: split K over the z dimension so the
  // grid covers the chip; partials in ws, summed in a fixed order
  int S = 1;
  if (ws && K >= 1024 && tiles < 256) {
    S = (512 + tiles - 1) / tiles;
    S = S < K / 256 ? S : K / 256;
    const size_t fit = ws_elems / ((size_t)M * N);
    S = (size_t)S < fit ? S : (int)fit;
    S = S < 64 ? S : 64;
    if (S < 2) S = 1;
  }
  int kchunk = K > 0 ? K : 1;
  if (S > 1) {
    kchunk = ((K + S - 1) / S + TK - 1) / TK * TK;
    S = (K + kchunk - 1) / kchunk;
  }
  T* part = S > 1 ? ws : nullptr;
  dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN, S);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, false, false>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, kchunk, part);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, true, false>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, kchunk, part);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<T, false, true>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, kchunk, part);
  else
    hipLaunchKernelGGL((k_gemm<T, true, true>), grid, dim3(GT), 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, kchunk, part);
  if (part)
    hipLaunchKernelGGL(k_splitk_sum<T>, dim3(grid_for((long long)M * N)), dim3(GT), 0, s, M, N, S,
                       (const T*)part, alpha, beta, C, ldc);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

template int gemm<double>(hipStream_t, bool, bool, int, int, int, double, const double*, long long,
                          const double*, long long, double, double*, long long, double*, size_t);
template int gemm<float>(hipStream_t, bool, bool, int, int, int, float, const float*, long long,
                         const float*, long long, float, float*, long long, float*, size_t);


template <typename T>
int block_t(hipStream_t s, int rows, int bb, const T* a, long long lda, const double* tau, T* vd,
            T* gram, T* tm, T* ws, size_t ws_elems) {
  hipLaunchKernelGGL(k_extract_v<T>, dim3(grid_for((long long)rows * bb)), dim3(GT), 0, s, rows,
                     bb, a, lda, vd);
  int rc = gemm<T>(s, true, false, bb, bb, rows, T(1), vd, rows, vd, rows, T(0), gram, bb, ws,
                   ws_elems);
  if (rc) return rc;
  if (bb <= 64)
    hipLaunchKernelGGL(k_larft<T>, dim3(1), dim3(256), 0, s, bb, gram, tau, tm);
  else
    hipLaunchKernelGGL(k_larft_seq<T>, dim3(1), dim3(GT), 0, s, bb, gram, tau, tm);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int block_t<double>(hipStream_t, int, int, const double*, long long, const double*,
                             double*, double*, double*, double*, size_t);
template int block_t<float>(hipStream_t, int, int, const float*, long long, const double*, float*,
                            float*, float*, float*, size_t);

// split-K partials of the tall products V^T V and V^T Q (up to 32 splits)
size_t splitk_elems(int m, int n) {
  const size_t e = 32 * (size_t)m * n;
  return e < ((size_t)1 << 22) ? e : ((size_t)1 << 22);
}

size_t form_q_work_elems(int m, int k, int b) {
  const size_t bb = (size_t)(b < k ? b : k);
  return (size_t)m * bb + 2 * bb * bb + 2 * bb * (size_t)k + 64 +
         splitk_elems((int)bb, (int)(bb > (size_t)k ? bb : (size_t)k));
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
  T* sk = z + (size_t)bbmax * k + 64;
  const size_t skn = splitk_elems(bbmax, bbmax > k ? bbmax : k);
  for (int j = nblk - 1; j >= 0; --j) {
    const int ij = j * b;
    const int bb = (k - ij) < b ? (k - ij) : b;
    const int rows = m - ij;
    const int nc = k - ij;
    int rc = block_t<T>(s, rows, bb, a + (long long)ij * lda + ij, lda, tau + ij, vd, gram, tm, sk,
                        skn);
    if (rc) return rc;
    T* qs = q + (long long)ij * ldq + ij;
    rc = gemm<T>(s, true, false, bb, nc, rows, T(1), vd, rows, qs, ldq, T(0), y, bb, sk, skn);
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
