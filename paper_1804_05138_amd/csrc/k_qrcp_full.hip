// QR with column pivoting of the whole matrix A (Alg. 1, Section II), the
// method RQRCP is compared against.  It is organized as LAPACK's xGEQP3
// (Quintana-Orti, Sun and Bischof, 1998), the Level-3 form Section II
// describes: the trailing matrix is updated by one GEMM per block of nb
// columns, while inside a block every step still needs
//
//   * the exact pivot rule of Alg. 1: the largest trailing column norm
//     (kept as downdated estimates, recomputed when a downdate has cancelled
//     too many digits);
//   * the current column brought up to date with the block's earlier
//     reflectors, and its Householder reflector (LAPACK dlarfg convention);
//   * F(:, t) = tau A2^T v over the not-yet-updated trailing matrix -- one
//     pass over the whole trailing matrix per pivot, which is why QRCP is
//     memory-bound and slow (Section II) and what RQRCP removes;
//   * the pivot row of every trailing column, so that its norm can be
//     downdated.
//
// Per step (block start s, step t, column and row c = r = s + t; V(:, j) is
// A(:, s + j) below its diagonal with a unit on it; F is n x nb):
//   k_qp_pivot   p = argmax_{l >= c} vn1[l]; swap columns c, p of A (all rows),
//                rows c, p of F(:, 0:t), vn1, vn2, jpvt
//   k_qp_col     A(r:m, c) -= V(r:m, 0:t) F(c, 0:t)^T; partial sums of squares
//   k_qp_house   beta, tau from the partials (fixed order); v = A(r+1:m, c) / (alpha - beta)
//   k_qp_gemv    y(l) = A(r:m, l)^T v for l in [s, n), l != c
//                (l < c: V(:, l - s)^T v; l > c: the not-yet-updated trailing column)
//   k_qp_upd     F(l, t) = tau (y(l) - F(l, 0:t) y(s:c)); A(r, l) -= V(r, 0:t+1) F(l, 0:t+1)^T;
//                downdate vn1[l] (LAPACK's rule); columns whose estimate lost too
//                much are listed for k_qp_renorm
//   k_qp_renorm  exact norm of the listed columns' trailing part, with the
//                block's pending update applied on the fly
// After the block: A(s+kb:m, s+kb:n) -= V(s+kb:m, 0:kb) F(s+kb:n, 0:kb)^T (MFMA GEMM).
#include "gemm.h"
#include "internal.h"

namespace rq {
namespace {

constexpr int QT = 256;          // threads of the row / column kernels
constexpr int PT = 1024;         // threads of the pivot kernel
constexpr int GV_COLS = 8;       // columns per wave in the GEMV
constexpr int GV_ROWS = 4;       // 64-row chunks per iteration in the GEMV
constexpr int GV_WAVES = QT / 64;
constexpr int RENORM_GRID = 256;
constexpr int MAX_NB = 128;

unsigned grid_of(long long total, int per) {
  long long g = (total + per - 1) / per;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// vn1 = vn2 = ||A(0:m, l)||, one wave per column, fixed summation order.
__global__ __launch_bounds__(QT) void k_qp_norms(int m, int n, const double* __restrict__ a,
                                                 long long lda, double* __restrict__ vn1,
                                                 double* __restrict__ vn2) {
  const int lane = threadIdx.x & 63;
  const long long l = (long long)blockIdx.x * (QT / 64) + (threadIdx.x >> 6);
  if (l >= n) return;
  const double* col = a + l * lda;
  double s = 0.0;
  for (int r = lane; r < m; r += 64) s += col[r] * col[r];
  s = wave_sum_dpp(s);
  if (lane == 0) {
    vn1[l] = sqrt(s);
    vn2[l] = sqrt(s);
  }
}

__global__ void k_qp_iota(int n, int* __restrict__ jpvt, int k, int* __restrict__ fcnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int j = t; j < n; j += gridDim.x * blockDim.x) jpvt[j] = j;
  for (int j = t; j < k; j += gridDim.x * blockDim.x) fcnt[j] = 0;
}

// Pivot of step c: argmax of vn1 over [c, n) (ties to the lowest index), then
// the interchange of columns c and p everywhere.
__global__ __launch_bounds__(PT) void k_qp_pivot(int m, int n, double* __restrict__ a,
                                                 long long lda, int c, int t,
                                                 double* __restrict__ f, long long ldf,
                                                 double* __restrict__ vn1,
                                                 double* __restrict__ vn2,
                                                 int* __restrict__ jpvt) {
  __shared__ double sv[PT / 64];
  __shared__ int sp[PT / 64];
  __shared__ int spiv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double bv = -1.0;
  int bp = 0x7fffffff;
  for (int l = c + tid; l < n; l += PT) {
    const double v = vn1[l];
    if (argbetter(v, l, bv, bp)) {
      bv = v;
      bp = l;
    }
  }
  int dummy = 0;
  wave_argmax(bv, bp, dummy);
  if (lane == 0) {
    sv[wave] = bv;
    sp[wave] = bp;
  }
  __syncthreads();
  if (tid == 0) {
    double v = sv[0];
    int p = sp[0];
    for (int w = 1; w < PT / 64; ++w)
      if (argbetter(sv[w], sp[w], v, p)) {
        v = sv[w];
        p = sp[w];
      }
    // no finite candidate (NaN norms): keep the current column
    spiv = (p >= c && p < n) ? p : c;
  }
  __syncthreads();
  const int p = spiv;
  if (p == c) return;
  double* x0 = a + (long long)c * lda;
  double* x1 = a + (long long)p * lda;
  for (int r = tid; r < m; r += PT) {
    const double u = x0[r];
    x0[r] = x1[r];
    x1[r] = u;
  }
  for (int j = tid; j < t; j += PT) {
    const double u = f[j * ldf + c];
    f[j * ldf + c] = f[j * ldf + p];
    f[j * ldf + p] = u;
  }
  if (tid == 0) {
    double u = vn1[c];
    vn1[c] = vn1[p];
    vn1[p] = u;
    u = vn2[c];
    vn2[c] = vn2[p];
    vn2[p] = u;
    const int q = jpvt[c];
    jpvt[c] = jpvt[p];
    jpvt[p] = q;
  }
}

// Block reduction of one double per thread, fixed order; result in thread 0.
RQ_DEV double block_sum(double v, double* sred) {
  v = wave_sum_dpp(v);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sred[w];
  return s;
}

// A(r:m, c) -= V(r:m, 0:t) F(c, 0:t)^T; part[b] = sum of squares of rows > r.
__global__ __launch_bounds__(QT) void k_qp_col(int m, double* __restrict__ a, long long lda,
                                               int s, int t, const double* __restrict__ f,
                                               long long ldf, double* __restrict__ part) {
  __shared__ double sf[MAX_NB];
  __shared__ double sred[QT / 64];
  const int c = s + t, r = c;
  if (threadIdx.x < t) sf[threadIdx.x] = f[threadIdx.x * ldf + c];
  __syncthreads();
  const int row = r + blockIdx.x * QT + threadIdx.x;
  double x = 0.0;
  if (row < m) {
    x = a[(long long)c * lda + row];
    for (int j = 0; j < t; ++j) x -= a[(long long)(s + j) * lda + row] * sf[j];
    a[(long long)c * lda + row] = x;
  }
  const double sq = (row > r && row < m) ? x * x : 0.0;
  const double tot = block_sum(sq, sred);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Reflector of column c (LAPACK dlarfg): every workgroup sums the partials in
// the same order, scales its rows by 1 / (alpha - beta); workgroup 0 stores
// tau and beta (beta goes into A(r, c) in k_qp_upd, after every workgroup has
// read alpha).
__global__ __launch_bounds__(QT) void k_qp_house(int m, double* __restrict__ a, long long lda,
                                                 int c, const double* __restrict__ part, int np,
                                                 double* __restrict__ tau,
                                                 double* __restrict__ hh) {
  __shared__ double sh[2];
  const int r = c;
  if (threadIdx.x < 64) {
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += 64) v += part[i];
    v = wave_sum_dpp(v);
    if (threadIdx.x == 0) {
      const double alpha = a[(long long)c * lda + r];
      double beta = alpha, tt = 0.0, den = 1.0;
      if (v > 0.0) {
        const double nrm = hypot(alpha, sqrt(v));
        beta = alpha >= 0.0 ? -nrm : nrm;
        tt = (beta - alpha) / beta;
        den = alpha - beta;
      }
      sh[0] = den;
      sh[1] = tt;
      if (blockIdx.x == 0) {
        tau[c] = tt;
        hh[0] = beta;
      }
    }
  }
  __syncthreads();
  const double den = sh[0];
  const int row = r + blockIdx.x * QT + threadIdx.x;
  if (sh[1] != 0.0 && row > r && row < m) a[(long long)c * lda + row] /= den;
}

// y(l) = v^T A(r:m, l), v = [1; A(r+1:m, c)], for l in [s, n) except c.  Each
// wave takes GV_COLS columns, each lane GV_ROWS rows per iteration, so that
// GV_COLS * GV_ROWS loads of a lane are in flight together.
__global__ __launch_bounds__(QT) void k_qp_gemv(int m, int n, const double* __restrict__ a,
                                                long long lda, int s, int c,
                                                double* __restrict__ y) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long l0 = s + ((long long)blockIdx.x * GV_WAVES + wave) * GV_COLS;
  if (l0 >= n) return;
  const int r = c;
  const double* vc = a + (long long)c * lda;
  const double* col[GV_COLS];
#pragma unroll
  for (int q = 0; q < GV_COLS; ++q) {
    const long long l = (l0 + q < n) ? l0 + q : l0;   // clamped: results of l >= n discarded
    col[q] = a + l * lda;
  }
  double acc[GV_COLS];
#pragma unroll
  for (int q = 0; q < GV_COLS; ++q) acc[q] = 0.0;
  for (int r0 = r; r0 < m; r0 += 64 * GV_ROWS) {
    double v[GV_ROWS];
    double x[GV_ROWS][GV_COLS];
#pragma unroll
    for (int u = 0; u < GV_ROWS; ++u) {
      const int row = r0 + 64 * u + lane;
      const int rr = row < m ? row : r;                 // clamped address, masked below
      v[u] = (row == r) ? 1.0 : (row < m ? vc[rr] : 0.0);
#pragma unroll
      for (int q = 0; q < GV_COLS; ++q) x[u][q] = col[q][rr];
    }
#pragma unroll
    for (int u = 0; u < GV_ROWS; ++u)
#pragma unroll
      for (int q = 0; q < GV_COLS; ++q) acc[q] += v[u] * x[u][q];
  }
#pragma unroll
  for (int q = 0; q < GV_COLS; ++q) {
    const double sum = wave_sum_dpp(acc[q]);
    const long long l = l0 + q;
    if (lane == 0 && l < n && l != c) y[l] = sum;
  }
}

// For every trailing column l > c: the new column of F, the pivot row of A and
// the norm downdate (LAPACK's rule, recompute threshold sqrt(eps)).
__global__ __launch_bounds__(QT) void k_qp_upd(int n, double* __restrict__ a, long long lda,
                                               int s, int t, double* __restrict__ f,
                                               long long ldf, const double* __restrict__ y,
                                               const double* __restrict__ tau,
                                               const double* __restrict__ hh,
                                               double* __restrict__ vn1,
                                               double* __restrict__ vn2,
                                               int* __restrict__ flist, int* __restrict__ fcnt) {
  __shared__ double vr[MAX_NB + 1];
  __shared__ double yv[MAX_NB];
  const int c = s + t, r = c;
  if (threadIdx.x < t) {
    vr[threadIdx.x] = a[(long long)(s + threadIdx.x) * lda + r];
    yv[threadIdx.x] = y[s + threadIdx.x];
  }
  if (threadIdx.x == 0) vr[t] = 1.0;
  __syncthreads();
  const double tt = tau[c];
  if (blockIdx.x == 0 && threadIdx.x == 0) a[(long long)c * lda + r] = hh[0];
  const long long l = (long long)c + 1 + (long long)blockIdx.x * QT + threadIdx.x;
  if (l >= n) return;
  double corr = 0.0;
  for (int j = 0; j < t; ++j) corr += f[j * ldf + l] * yv[j];
  const double fl = tt * (y[l] - corr);
  f[t * ldf + l] = fl;
  double x = a[l * lda + r];
  for (int j = 0; j < t; ++j) x -= vr[j] * f[j * ldf + l];
  x -= fl;
  a[l * lda + r] = x;
  const double v1 = vn1[l];
  if (v1 != 0.0) {
    double q = fabs(x) / v1;
    q = fmax(0.0, (1.0 + q) * (1.0 - q));
    const double ratio = v1 / vn2[l];
    const double q2 = q * ratio * ratio;
    if (q2 <= 1.0536712127723509e-08) {   // sqrt(2^-53): the estimate has lost half its digits
      const int slot = atomicAdd(fcnt, 1);
      flist[slot] = (int)l;
    } else {
      vn1[l] = v1 * sqrt(q);
    }
  }
}

// Exact norms of the listed columns: rows r+1..m-1 of
// A(:, l) - V(:, 0:t+1) F(l, 0:t+1)^T (the block's pending update applied on
// the fly).  One workgroup per listed column.
__global__ __launch_bounds__(QT) void k_qp_renorm(int m, const double* __restrict__ a,
                                                  long long lda, int s, int t,
                                                  const double* __restrict__ f, long long ldf,
                                                  const int* __restrict__ flist,
                                                  const int* __restrict__ fcnt,
                                                  double* __restrict__ vn1,
                                                  double* __restrict__ vn2) {
  __shared__ double sf[MAX_NB + 1];
  __shared__ double sred[QT / 64];
  const int cnt = *fcnt;
  const int r = s + t;
  for (int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
    const int l = flist[idx];
    __syncthreads();
    if (threadIdx.x <= t) sf[threadIdx.x] = f[threadIdx.x * ldf + l];
    __syncthreads();
    double sq = 0.0;
    for (int row = r + 1 + threadIdx.x; row < m; row += QT) {
      double x = a[(long long)l * lda + row];
      for (int j = 0; j <= t; ++j) x -= a[(long long)(s + j) * lda + row] * sf[j];
      sq += x * x;
    }
    const double tot = block_sum(sq, sred);
    if (threadIdx.x == 0) {
      vn1[l] = sqrt(tot);
      vn2[l] = sqrt(tot);
    }
  }
}

struct QpLayout {
  size_t f, vn1, vn2, y, part, hh, flist, fcnt, total;
};

QpLayout qp_layout(int m, int n, int k, int nb) {
  QpLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  L.f = take((size_t)n * nb * sizeof(double));
  L.vn1 = take((size_t)n * sizeof(double));
  L.vn2 = take((size_t)n * sizeof(double));
  L.y = take((size_t)n * sizeof(double));
  L.part = take((size_t)grid_of(m, QT) * sizeof(double));
  L.hh = take(4 * sizeof(double));
  L.flist = take((size_t)n * sizeof(int));
  L.fcnt = take((size_t)k * sizeof(int));
  L.total = off;
  return L;
}

}  // namespace

size_t qrcp_full_workspace(int m, int n, int k, int nb) { return qp_layout(m, n, k, nb).total; }

int qrcp_full_max_nb() { return MAX_NB; }

int launch_qrcp_full(hipStream_t st, int m, int n, int k, int nb, double* a, long long lda,
                     int* jpvt, double* tau, char* ws) {
  if (nb < 1 || nb > MAX_NB || k < 1 || k > (m < n ? m : n)) return RQ_ERR_LIMIT;
  const QpLayout L = qp_layout(m, n, k, nb);
  double* f = (double*)(ws + L.f);
  double* vn1 = (double*)(ws + L.vn1);
  double* vn2 = (double*)(ws + L.vn2);
  double* y = (double*)(ws + L.y);
  double* part = (double*)(ws + L.part);
  double* hh = (double*)(ws + L.hh);
  int* flist = (int*)(ws + L.flist);
  int* fcnt = (int*)(ws + L.fcnt);
  const long long ldf = n;
  hipLaunchKernelGGL(k_qp_iota, dim3(grid_of(n > k ? n : k, 256) > 1024 ? 1024 : grid_of(n > k ? n : k, 256)),
                     dim3(256), 0, st, n, jpvt, k, fcnt);
  hipLaunchKernelGGL(k_qp_norms, dim3(grid_of(n, QT / 64)), dim3(QT), 0, st, m, n,
                     (const double*)a, lda, vn1, vn2);
  RQ_HIP_CHECK(hipGetLastError());
  for (int s = 0; s < k; s += nb) {
    const int kb = (k - s < nb) ? k - s : nb;
    for (int t = 0; t < kb; ++t) {
      const int c = s + t, r = c;
      const unsigned rows_grid = grid_of(m - r, QT);
      hipLaunchKernelGGL(k_qp_pivot, dim3(1), dim3(PT), 0, st, m, n, a, lda, c, t, f, ldf, vn1,
                         vn2, jpvt);
      hipLaunchKernelGGL(k_qp_col, dim3(rows_grid), dim3(QT), 0, st, m, a, lda, s, t,
                         (const double*)f, ldf, part);
      hipLaunchKernelGGL(k_qp_house, dim3(rows_grid), dim3(QT), 0, st, m, a, lda, c,
                         (const double*)part, (int)rows_grid, tau, hh);
      if (n - s > 1)
        hipLaunchKernelGGL(k_qp_gemv, dim3(grid_of(n - s, GV_WAVES * GV_COLS)), dim3(QT), 0, st,
                           m, n, (const double*)a, lda, s, c, y);
      if (c + 1 < n) {
        hipLaunchKernelGGL(k_qp_upd, dim3(grid_of(n - c - 1, QT)), dim3(QT), 0, st, n, a, lda, s,
                           t, f, ldf, (const double*)y, (const double*)tau, (const double*)hh,
                           vn1, vn2, flist, fcnt + c);
        hipLaunchKernelGGL(k_qp_renorm, dim3(RENORM_GRID), dim3(QT), 0, st, m, (const double*)a,
                           lda, s, t, (const double*)f, ldf, (const int*)flist,
                           (const int*)(fcnt + c), vn1, vn2);
      } else {
        hipLaunchKernelGGL(k_qp_upd, dim3(1), dim3(QT), 0, st, n, a, lda, s, t, f, ldf,
                           (const double*)y, (const double*)tau, (const double*)hh, vn1, vn2,
                           flist, fcnt + c);
      }
      RQ_HIP_CHECK(hipGetLastError());
    }
    const int e = s + kb;
    if (e < n && e < m) {
      const int rc = gemm<double>(st, false, true, m - e, n - e, kb, -1.0,
                                  a + (long long)s * lda + e, lda, f + e, ldf, 1.0,
                                  a + (long long)e * lda + e, lda);
      if (rc) return rc;
    }
  }
  return RQ_OK;
}

}  // namespace rq
