// Spectrum-revealing swaps (Alg. 3, Section IV-C) after an l-step RQRCP.
//
// State on the device: A holds R in rows 0..l (upper trapezoid) and the
// trailing block in A(l:m, l:n); est[c] are the estimates r_c of the trailing
// column norms squared.  The kernels below are the steps of one pass of the
// Alg. 3 loop; the host repeats them while the g2 estimate exceeds g.
//
//   pick      argmax of est over positions l..n-1 (ties: lowest), swap into l
//   qr step   one Householder reflection on A(l:m, l) applied to A(l:m, l+1:n);
//             est[c] -= A(l, c)^2 (clamped at 0)
//   g2        Y = Rhat^-1 Omega^T for the (l+1) x (l+1) triangle Rhat and a
//             d x (l+1) Gaussian probe (or Omega = I in exact mode); the row
//             norms of Y are the column norms of Omega Rhat^-T, and
//             g2 = |alpha| max_i ||Y(i, :)|| / sqrt(d) (exact: without sqrt(d)),
//             alpha = R(l, l) after the qr step (definition of g2, Section IV-C)
//   rotate    round robin: the column ii with the largest norm moves to
//             position l, columns ii+1..l move one to the left; adjacent-row
//             Givens rotations G(j, j+1), j = ii..l-1, restore the triangle on
//             every column from j on; est[l] = R(l,l)^2, est[c] += R(l,c)^2.
//
// Entries below the diagonal of the first l columns (the Householder vectors
// of the RQRCP) are never read: after a rotation the factorization is
// recomputed with the final pivots frozen, since Givens rotations cannot be
// expressed in the compact form.
#include <limits.h>

#include "srqr.h"

namespace rq {
namespace {

constexpr int ST = 256;

// est[c] = ||B(:, c)||^2 / lsk for c >= l, 0 for c < l.
__global__ __launch_bounds__(ST) void k_srqr_est(int l, int n, int lsk, const double* __restrict__ b,
                                                 long long ldb, double* __restrict__ est) {
  const int c = blockIdx.x * ST + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  if (c >= l) {
    const double* col = b + (long long)c * ldb;
    for (int r = 0; r < lsk; ++r) s += col[r] * col[r];
    s /= lsk;
  }
  est[c] = s;
}

// Workgroup argmax of (value, index) pairs, ties to the lowest index.
template <int NT>
RQ_DEV void block_argmax(double& v, int& p) {
  __shared__ double s_v[NT / 64];
  __shared__ int s_p[NT / 64];
  int dummy = 0;
  wave_argmax(v, p, dummy);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_v[w] = v;
    s_p[w] = p;
  }
  __syncthreads();
  v = s_v[0];
  p = s_p[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q)
    if (argbetter(s_v[q], s_p[q], v, p)) {
      v = s_v[q];
      p = s_p[q];
    }
  __syncthreads();
}

// One workgroup: j = argmax est[l..n-1]; swap columns j and l of A (all rows),
// of jpvt and of est.
constexpr int PT = 1024;
__global__ __launch_bounds__(PT) void k_srqr_pick(int m, int n, int l, double* __restrict__ a,
                                                  long long lda, int* __restrict__ jpvt,
                                                  double* __restrict__ est) {
  double best = -1.0;
  int bp = INT_MAX;
  for (int c = l + threadIdx.x; c < n; c += PT) {
    const double e = est[c];
    if (argbetter(e, c, best, bp)) {
      best = e;
      bp = c;
    }
  }
  block_argmax<PT>(best, bp);
  const int j = bp;
  if (j == l || j >= n) return;
  double* cj = a + (long long)j * lda;
  double* cl = a + (long long)l * lda;
  for (int r = threadIdx.x; r < m; r += PT) {
    const double x = cj[r];
    cj[r] = cl[r];
    cl[r] = x;
  }
  if (threadIdx.x == 0) {
    const int t = jpvt[j];
    jpvt[j] = jpvt[l];
    jpvt[l] = t;
    const double e = est[j];
    est[j] = est[l];
    est[l] = e;
  }
}

// One workgroup: Householder reflection (LAPACK dlarfg convention) of
// A(l:m, l): A(l, l) = beta, v = A(l+1:m, l) / (alpha - beta) stored in place,
// tau[l] = tau; sc[0] = |beta|, sc[1] = tau.
__global__ __launch_bounds__(PT) void k_srqr_house(int m, int l, double* __restrict__ a,
                                                   long long lda, double* __restrict__ tau,
                                                   double* __restrict__ sc) {
  __shared__ double s_part[PT / 64];
  __shared__ double s_h[2];
  double* col = a + (long long)l * lda;
  double x2 = 0.0;
  for (int r = l + 1 + threadIdx.x; r < m; r += PT) x2 += col[r] * col[r];
  x2 = wave_sum_dpp(x2);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = x2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double xn2 = 0.0;
    for (int w = 0; w < PT / 64; ++w) xn2 += s_part[w];
    const double alpha = col[l];
    double beta = alpha, t = 0.0, den = 1.0;
    if (xn2 > 0.0) {
      const double nrm = hypot(alpha, sqrt(xn2));
      beta = (alpha >= 0.0) ? -nrm : nrm;
      t = (beta - alpha) / beta;
      den = alpha - beta;
    }
    s_h[0] = den;
    s_h[1] = t;
    col[l] = beta;
    tau[l] = t;
    sc[0] = fabs(beta);
    sc[1] = t;
  }
  __syncthreads();
  const double den = s_h[0];
  if (s_h[1] != 0.0)
    for (int r = l + 1 + threadIdx.x; r < m; r += PT) col[r] = col[r] / den;
}

// One workgroup per trailing column c > l: A(l:m, c) -= tau v (v^T A(l:m, c)),
// v = [1; A(l+1:m, l)]; then est[c] = max(est[c] - A(l, c)^2, 0).
__global__ __launch_bounds__(ST) void k_srqr_apply(int m, int n, int l, double* __restrict__ a,
                                                   long long lda, const double* __restrict__ sc,
                                                   double* __restrict__ est) {
  __shared__ double s_part[ST / 64];
  const int c = l + 1 + blockIdx.x;
  if (c >= n) return;
  const double t = sc[1];
  double* col = a + (long long)c * lda;
  const double* v = a + (long long)l * lda;
  if (t != 0.0) {
    const double top = col[l];  // read before any thread writes it
    double d = 0.0;
    for (int r = l + 1 + threadIdx.x; r < m; r += ST) d += v[r] * col[r];
    d = wave_sum_dpp(d);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = d;
    __syncthreads();
    d = top;
#pragma unroll
    for (int w = 0; w < ST / 64; ++w) d += s_part[w];
    const double f = t * d;
    for (int r = l + 1 + threadIdx.x; r < m; r += ST) col[r] -= f * v[r];
    if (threadIdx.x == 0) col[l] -= f;
  }
  if (threadIdx.x == 0) {
    const double x = col[l];
    est[c] = fmax(est[c] - x * x, 0.0);
  }
}

// Y = Rhat^-1 Omega^T by back substitution, DW right-hand sides per workgroup
// held in LDS; workgroup w writes part[w * l1 + i] = sum over its columns of
// Y(i, .)^2.  exact: Omega = I (d = l1).
__global__ __launch_bounds__(ST) void k_srqr_trsm(int l1, const double* __restrict__ a, long long lda,
                                                  const double* __restrict__ om, int d, int dw,
                                                  int exact, double* __restrict__ part) {
  extern __shared__ double y[];  // [l1][dw]
  const int r0 = blockIdx.x * dw;
  const int nr = min(dw, d - r0);
  for (int e = threadIdx.x; e < l1 * dw; e += ST) {
    const int i = e / dw, r = e % dw;
    double v = 0.0;
    if (r < nr) v = exact ? ((i == r0 + r) ? 1.0 : 0.0) : om[(long long)i * d + r0 + r];
    y[e] = v;
  }
  __syncthreads();
  for (int i = l1 - 1; i >= 0; --i) {
    const double* ci = a + (long long)i * lda;
    const double rii = ci[i];
    // x_r = y(i, r) / R(i, i); rows j < i: y(j, r) -= R(j, i) x_r
    double ss = 0.0;
    for (int e = threadIdx.x; e < i * dw; e += ST) {
      const int j = e / dw, r = e % dw;
      y[e] -= ci[j] * (y[i * dw + r] / rii);
    }
    if (threadIdx.x == 0) {
      for (int r = 0; r < nr; ++r) {
        const double x = y[i * dw + r] / rii;
        ss += x * x;
      }
      part[(long long)blockIdx.x * l1 + i] = ss;
    }
    __syncthreads();
  }
}

// One workgroup: cn_i = sqrt(sum_w part[w][i]); g2 = alpha max cn / sqrt(d)
// (exact: alpha max cn); ii = first argmax.  out[0] = g2, iout[0] = ii.
__global__ __launch_bounds__(PT) void k_srqr_g2(int l1, int nparts, const double* __restrict__ part,
                                                int d, int exact, const double* __restrict__ sc,
                                                double* __restrict__ g2, int* __restrict__ iout,
                                                double* __restrict__ g2_user) {
  double best = -1.0;
  int bp = INT_MAX;
  for (int i = threadIdx.x; i < l1; i += PT) {
    double s = 0.0;
    for (int w = 0; w < nparts; ++w) s += part[(long long)w * l1 + i];
    const double cn = sqrt(s);
    if (argbetter(cn, i, best, bp)) {
      best = cn;
      bp = i;
    }
  }
  block_argmax<PT>(best, bp);
  if (bp >= l1) bp = l1 - 1;  // no finite norm (singular triangle): rotate nothing
  if (threadIdx.x == 0) {
    const double g = exact ? sc[0] * best : sc[0] * best / sqrt((double)d);
    g2[0] = g;
    iout[0] = bp;
    if (g2_user) g2_user[0] = g;
  }
}

// Round robin: column ii moves to position l, columns ii+1..l move one to the
// left (rows 0..l, and jpvt); rows ii+1..m-1 of the new column l are zero (it
// was already reduced).  est[0..l] = 0.  One thread per row.
__global__ __launch_bounds__(ST) void k_srqr_shift(int m, int l, const int* __restrict__ iip,
                                                   double* __restrict__ a, long long lda,
                                                   int* __restrict__ jpvt, double* __restrict__ est) {
  const int ii = min(max(*iip, 0), l);
  const int r = blockIdx.x * ST + threadIdx.x;
  if (r <= l) {
    const double x = a[(long long)ii * lda + r];
    for (int c = ii; c < l; ++c) a[(long long)c * lda + r] = a[(long long)(c + 1) * lda + r];
    a[(long long)l * lda + r] = (r <= ii) ? x : 0.0;
    est[r] = 0.0;
  } else if (r < m) {
    a[(long long)l * lda + r] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int t = jpvt[ii];
    for (int c = ii; c < l; ++c) jpvt[c] = jpvt[c + 1];
    jpvt[l] = t;
  }
}

// Givens rotations G(j, j+1), j = ii..l-1, on the Hessenberg columns ii..l.
// Column c keeps the running value of its row j (the row the next rotation
// combines with row j+1); rotation j is formed by the thread of column j.
// The (c, s) pairs are written to cs[2 j], cs[2 j + 1] for the trailing columns.
constexpr int GT = 1024;
constexpr int GCPT = 4;  // columns per thread: up to 4096 Hessenberg columns
__global__ __launch_bounds__(GT) void k_srqr_givens(int l, const int* __restrict__ iip,
                                                    double* __restrict__ a, long long lda,
                                                    double* __restrict__ cs,
                                                    double* __restrict__ est) {
  __shared__ double s_cs[2];
  const int ii = min(max(*iip, 0), l);
  double carry[GCPT];
#pragma unroll
  for (int u = 0; u < GCPT; ++u) {
    const int c = ii + threadIdx.x + u * GT;
    carry[u] = (c <= l) ? a[(long long)c * lda + ii] : 0.0;
  }
  for (int j = ii; j < l; ++j) {
    // the owner of column j forms the rotation from (its row j, original row j+1)
    const int q = j - ii;
    if ((q % GT) == (int)threadIdx.x) {
      const int u = q / GT;
      double cj = 0.0;
#pragma unroll
      for (int uu = 0; uu < GCPT; ++uu)
        if (uu == u) cj = carry[uu];
      const double f = cj, g = a[(long long)j * lda + j + 1];
      double c = 1.0, s = 0.0, r = f;
      if (g != 0.0) {
        r = hypot(f, g);
        if (f < 0.0) r = -r;
        c = f / r;
        s = g / r;
      }
      s_cs[0] = c;
      s_cs[1] = s;
      cs[2 * j] = c;
      cs[2 * j + 1] = s;
      a[(long long)j * lda + j] = r;
      a[(long long)j * lda + j + 1] = 0.0;
    }
    __syncthreads();
    const double c = s_cs[0], s = s_cs[1];
#pragma unroll
    for (int u = 0; u < GCPT; ++u) {
      const int col = ii + threadIdx.x + u * GT;
      if (col > j && col <= l) {
        const double g = a[(long long)col * lda + j + 1];
        a[(long long)col * lda + j] = c * carry[u] + s * g;
        carry[u] = -s * carry[u] + c * g;
      }
    }
    __syncthreads();
  }
  // column l ends with its row l in the carry (ii == l: no rotation, row l as is)
#pragma unroll
  for (int u = 0; u < GCPT; ++u) {
    const int col = ii + threadIdx.x + u * GT;
    if (col == l) {
      a[(long long)l * lda + l] = carry[u];
      est[l] = carry[u] * carry[u];
    }
  }
}

// The same rotations on the trailing columns c > l (rows ii..l), one thread
// per column; est[c] += R(l, c)^2.
__global__ __launch_bounds__(ST) void k_srqr_givens_apply(int n, int l, const int* __restrict__ iip,
                                                          double* __restrict__ a, long long lda,
                                                          const double* __restrict__ cs,
                                                          double* __restrict__ est) {
  const int ii = min(max(*iip, 0), l);
  const int c = l + 1 + blockIdx.x * ST + threadIdx.x;
  if (c >= n) return;
  double* col = a + (long long)c * lda;
  double carry = col[ii];
  for (int j = ii; j < l; ++j) {
    const double g = col[j + 1];
    const double cc = cs[2 * j], s = cs[2 * j + 1];
    col[j] = cc * carry + s * g;
    carry = -s * carry + cc * g;
  }
  col[l] = carry;
  est[c] += carry * carry;
}

}  // namespace

SrqrLayout srqr_layout(int m, int n, int l, int d, int exact) {
  SrqrLayout L;
  const int l1 = l + 1;
  const int deff = exact ? l1 : d;
  const int dw = srqr_dw(l1);
  L.nparts = (deff + dw - 1) / dw;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  L.est = take((size_t)n * sizeof(double));
  L.omega = take(exact ? 0 : (size_t)d * l1 * sizeof(double));
  L.part = take((size_t)L.nparts * l1 * sizeof(double));
  L.cs = take((size_t)2 * l1 * sizeof(double));
  L.sc = take(8 * sizeof(double));
  L.iv = take(8 * sizeof(int));
  L.total = off;
  (void)m;
  return L;
}

int srqr_dw(int l1) {
  int dw = 8;
  while (dw > 1 && (size_t)l1 * dw * sizeof(double) > 128 * 1024) dw /= 2;
  return dw;
}

int launch_srqr_init(hipStream_t s, int m, int n, int l, int lsk, double* a, long long lda,
                     int* jpvt, const double* b, long long ldb, double* est) {
  hipLaunchKernelGGL(k_srqr_est, dim3((n + ST - 1) / ST), dim3(ST), 0, s, l, n, lsk, b, ldb, est);
  RQ_HIP_CHECK(hipGetLastError());
  (void)m;
  (void)a;
  (void)lda;
  (void)jpvt;
  return RQ_OK;
}

int launch_srqr_pick_qr(hipStream_t s, int m, int n, int l, double* a, long long lda, int* jpvt,
                        double* est, double* tau, double* sc) {
  hipLaunchKernelGGL(k_srqr_pick, dim3(1), dim3(PT), 0, s, m, n, l, a, lda, jpvt, est);
  RQ_HIP_CHECK(hipGetLastError());
  if (!tau) return RQ_OK;
  hipLaunchKernelGGL(k_srqr_house, dim3(1), dim3(PT), 0, s, m, l, a, lda, tau, sc);
  RQ_HIP_CHECK(hipGetLastError());
  if (n - l - 1 > 0) {
    hipLaunchKernelGGL(k_srqr_apply, dim3(n - l - 1), dim3(ST), 0, s, m, n, l, a, lda, sc, est);
    RQ_HIP_CHECK(hipGetLastError());
  }
  return RQ_OK;
}

int launch_srqr_g2(hipStream_t s, int l, const double* a, long long lda, const double* om, int d,
                   int exact, const SrqrLayout& L, char* ws, double* g2_user) {
  const int l1 = l + 1;
  const int deff = exact ? l1 : d;
  const int dw = srqr_dw(l1);
  if ((size_t)l1 * dw * sizeof(double) > 128 * 1024) return RQ_ERR_LIMIT;
  double* part = (double*)(ws + L.part);
  double* sc = (double*)(ws + L.sc);
  int* iv = (int*)(ws + L.iv);
  const size_t shmem = (size_t)l1 * dw * sizeof(double);
  RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_srqr_trsm),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(k_srqr_trsm, dim3(L.nparts), dim3(ST), shmem, s, l1, a, lda, om, deff, dw,
                     exact, part);
  RQ_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_srqr_g2, dim3(1), dim3(PT), 0, s, l1, L.nparts, (const double*)part, deff,
                     exact, (const double*)sc, sc + 2, iv, g2_user);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

int launch_srqr_rotate(hipStream_t s, int m, int n, int l, double* a, long long lda, int* jpvt,
                       const SrqrLayout& L, char* ws) {
  if (l + 1 > GT * GCPT) return RQ_ERR_LIMIT;
  const int* iip = (const int*)(ws + L.iv);
  double* est = (double*)(ws + L.est);
  double* cs = (double*)(ws + L.cs);
  hipLaunchKernelGGL(k_srqr_shift, dim3((m + ST - 1) / ST), dim3(ST), 0, s, m, l, iip, a, lda, jpvt,
                     est);
  RQ_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_srqr_givens, dim3(1), dim3(GT), 0, s, l, iip, a, lda, cs, est);
  RQ_HIP_CHECK(hipGetLastError());
  if (n - l - 1 > 0) {
    hipLaunchKernelGGL(k_srqr_givens_apply, dim3((n - l - 1 + ST - 1) / ST), dim3(ST), 0, s, n, l,
                       iip, a, lda, (const double*)cs, est);
    RQ_HIP_CHECK(hipGetLastError());
  }
  return RQ_OK;
}

}  // namespace rq
