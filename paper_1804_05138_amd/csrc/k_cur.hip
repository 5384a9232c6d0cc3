// Uses of a (spectrum-revealing) truncated factorization A Pi = Q [R11 R12; 0 R22]:
//
// * CX (Section V-D): C = A(:, jpvt[0:k]) and X = C^+ A.  With C = Q1 R11 and
//   Q1^T A Pi = [R11 R12], X Pi = R11^-1 [R11 R12] = [I | R11^-1 R12]: one
//   triangular inverse, one GEMM and a column scatter -- no pass over A.
// * CUR (Section V-D): with the rows chosen by the factorization of A^T,
//   A^T Pi_r = Q_r [T11 T12; ...], R = A(rows, :) = T11^T Q_r1^T, so
//   R^+ = Q_r1 T11^-T and U = C^+ A R^+ = X Q_r1 T11^-T.
// * SVD compression to rank k (the remark after Alg. 3): with R_l the first l
//   rows of R, A Pi ~ Q_l R_l ~ Q_l U_k U_k^T R_l, U_k the k leading left
//   singular vectors of R_l, i.e. the leading eigenvectors of G = R_l R_l^T.
//   G comes from one MFMA GEMM; its eigenvectors from cyclic two-sided Jacobi
//   (l <= 128: G lives in one workgroup's LDS, l/2 disjoint rotations per round
//   in the round-robin order of a tournament).
#include "gemm.h"
#include "internal.h"

namespace rq {
namespace {

constexpr int CT = 256;
constexpr int JT = 1024;          // threads of the Jacobi workgroup
constexpr int JMAX = 128;         // largest l of the compression
constexpr int JLD = JMAX + 1;     // padded LDS row

unsigned grid_of(long long total) {
  long long g = (total + CT - 1) / CT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

RQ_DEV long long perm_col(const int* perm, int j, int n) {
  return (long long)min(max(perm[j], 0), n - 1);
}

// X(:, jpvt[j]) = [I | Z](:, j) (k x n; Z is k x (n - k), ld k).
__global__ __launch_bounds__(CT) void k_cx_scatter(int k, int n, const double* __restrict__ z,
                                                   const int* __restrict__ jpvt,
                                                   double* __restrict__ x, long long ldx) {
  const long long total = (long long)k * n;
  for (long long e = (long long)blockIdx.x * CT + threadIdx.x; e < total;
       e += (long long)gridDim.x * CT) {
    const int j = (int)(e / k), r = (int)(e % k);
    const double v = (j < k) ? (r == j ? 1.0 : 0.0) : z[(long long)(j - k) * k + r];
    x[perm_col(jpvt, j, n) * ldx + r] = v;
  }
}

// R_l = triu(AF(0:l, 0:n)) as a dense l x n matrix (ld l).
__global__ __launch_bounds__(CT) void k_rl_dense(int l, int n, const double* __restrict__ af,
                                                 long long ldaf, double* __restrict__ rl) {
  const long long total = (long long)l * n;
  for (long long e = (long long)blockIdx.x * CT + threadIdx.x; e < total;
       e += (long long)gridDim.x * CT) {
    const long long j = e / l;
    const int r = (int)(e % l);
    rl[e] = (r <= j) ? af[j * ldaf + r] : 0.0;
  }
}

// Y(:, jpvt[j]) = Yp(:, j) (k x n, Yp ld k).
__global__ __launch_bounds__(CT) void k_scatter_cols(int k, int n, const double* __restrict__ yp,
                                                     const int* __restrict__ jpvt,
                                                     double* __restrict__ y, long long ldy) {
  const long long total = (long long)k * n;
  for (long long e = (long long)blockIdx.x * CT + threadIdx.x; e < total;
       e += (long long)gridDim.x * CT) {
    const int j = (int)(e / k), r = (int)(e % k);
    y[perm_col(jpvt, j, n) * ldy + r] = yp[e];
  }
}

// Eigen-decomposition of the symmetric l x l matrix G (ld l): cyclic Jacobi,
// each round l/2 disjoint rotations (round-robin pairing; an odd l gets a
// dummy partner).  Rotation of (p, q): t = sign(th) / (|th| + sqrt(th^2 + 1)),
// th = (g_qq - g_pp) / (2 g_pq), c = 1 / sqrt(t^2 + 1), s = t c; G <- P^T G P,
// V <- V P with P_pp = P_qq = c, P_pq = s, P_qp = -s.  Sweeps stop when the
// off-diagonal part is below 1e-15 of the whole (in Frobenius norm) or after
// max_sweeps.  evals = diag(G), v (l x l, ld l) the eigenvectors.
__global__ __launch_bounds__(JT) void k_jacobi_eig(int l, const double* __restrict__ g,
                                                   double* __restrict__ v,
                                                   double* __restrict__ evals, int max_sweeps,
                                                   int* __restrict__ sweeps_out) {
  extern __shared__ double sg[];   // l x JLD
  __shared__ double sc[JMAX / 2 + 1], ss[JMAX / 2 + 1];
  __shared__ int sp[JMAX / 2 + 1], sq[JMAX / 2 + 1];
  __shared__ double sred[JT / 64];
  __shared__ int sdone;
  const int tid = threadIdx.x;
  for (int e = tid; e < l * l; e += JT) {
    const int r = e % l, c = e / l;
    sg[r * JLD + c] = g[(long long)c * l + r];
    v[(long long)c * l + r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int le = l + (l & 1);
  const int npair = le / 2;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal mass against the total
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < l * l; e += JT) {
      const int r = e % l, c = e / l;
      const double x = sg[r * JLD + c];
      tot += x * x;
      if (r != c) off += x * x;
    }
    off = wave_sum_dpp(off);
    tot = wave_sum_dpp(tot);
    if ((tid & 63) == 0) sred[tid >> 6] = off;
    __syncthreads();
    if (tid == 0) {
      double o = 0.0;
      for (int w = 0; w < JT / 64; ++w) o += sred[w];
      sred[0] = o;
    }
    __syncthreads();
    const double offs = sred[0];
    __syncthreads();
    if ((tid & 63) == 0) sred[tid >> 6] = tot;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < JT / 64; ++w) t += sred[w];
      sdone = (offs <= 1e-30 * t) ? 1 : 0;
    }
    __syncthreads();
    if (sdone) break;
    for (int round = 0; round < le - 1; ++round) {
      if (tid < npair) {
        auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (le - 1)) + 1; };
        int p = player(tid), q = player(le - 1 - tid);
        if (p > q) {
          const int u = p;
          p = q;
          q = u;
        }
        double c = 1.0, s = 0.0;
        if (q < l) {
          const double apq = sg[p * JLD + q];
          const double app = sg[p * JLD + p], aqq = sg[q * JLD + q];
          if (apq != 0.0 && fabs(apq) > 1e-300) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        } else {
          q = p;   // dummy partner: no rotation
        }
        sp[tid] = p;
        sq[tid] = q;
        sc[tid] = c;
        ss[tid] = s;
      }
      __syncthreads();
      // rows p, q
      for (int e = tid; e < npair * l; e += JT) {
        const int i = e / l, j = e % l;
        const int p = sp[i], q = sq[i];
        if (p == q) continue;
        const double c = sc[i], s = ss[i];
        const double gp = sg[p * JLD + j], gq = sg[q * JLD + j];
        sg[p * JLD + j] = c * gp - s * gq;
        sg[q * JLD + j] = s * gp + c * gq;
      }
      __syncthreads();
      // columns p, q of G and of V
      for (int e = tid; e < npair * l; e += JT) {
        const int i = e / l, r = e % l;
        const int p = sp[i], q = sq[i];
        if (p == q) continue;
        const double c = sc[i], s = ss[i];
        const double gp = sg[r * JLD + p], gq = sg[r * JLD + q];
        sg[r * JLD + p] = c * gp - s * gq;
        sg[r * JLD + q] = s * gp + c * gq;
        const double vp = v[(long long)p * l + r], vq = v[(long long)q * l + r];
        v[(long long)p * l + r] = c * vp - s * vq;
        v[(long long)q * l + r] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < l; i += JT) evals[i] = sg[i * JLD + i];
  if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}

// The k largest eigenvalues (descending, ties to the lower index): uk(:, i) =
// v(:, order[i]), sigma[i] = sqrt(max(eval, 0)).  One workgroup, l <= JMAX.
__global__ __launch_bounds__(CT) void k_topk(int l, int k, const double* __restrict__ evals,
                                             const double* __restrict__ v,
                                             double* __restrict__ uk,
                                             double* __restrict__ sigma) {
  __shared__ int order[JMAX];
  if (threadIdx.x == 0) {
    bool used[JMAX];
    for (int i = 0; i < l; ++i) used[i] = false;
    for (int i = 0; i < k; ++i) {
      int best = -1;
      for (int j = 0; j < l; ++j)
        if (!used[j] && (best < 0 || evals[j] > evals[best])) best = j;
      used[best] = true;
      order[i] = best;
      if (sigma) sigma[i] = sqrt(fmax(evals[best], 0.0));
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < l * k; e += CT) {
    const int i = e / l, r = e % l;
    uk[(long long)i * l + r] = v[(long long)order[i] * l + r];
  }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t cx_workspace(int n, int k) {
  return align256((size_t)k * k * 8) * 2 + align256((size_t)k * (n > k ? n - k : 1) * 8) +
         align256(splitk_elems(k, n) * 8);
}

int launch_cx(hipStream_t s, int m, int n, int k, const double* af, long long ldaf,
              const int* jpvt, double* x, long long ldx, char* ws) {
  (void)m;
  double* r11 = (double*)ws;
  double* rinv = (double*)(ws + align256((size_t)k * k * 8));
  double* z = (double*)(ws + 2 * align256((size_t)k * k * 8));
  int rc = upper_inverse<double>(s, k, af, ldaf, r11, rinv);
  if (rc) return rc;
  if (n > k) {
    rc = gemm<double>(s, false, false, k, n - k, k, 1.0, rinv, k, af + (long long)k * ldaf, ldaf,
                      0.0, z, k);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_cx_scatter, dim3(grid_of((long long)k * n)), dim3(CT), 0, s, k, n,
                     (const double*)z, jpvt, x, ldx);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

size_t cur_workspace(int m, int n, int k, int b) {
  return cx_workspace(n, k) + align256((size_t)k * n * 8) + align256((size_t)n * k * 8) +
         align256(form_q_work_elems(n, k, b) * 8) + 3 * align256((size_t)k * k * 8) +
         align256(splitk_elems(k, k) * 8);
}

int launch_cur(hipStream_t s, int m, int n, int k, int b, const double* afc, long long ldc,
               const int* jpc, const double* afr, long long ldr, const double* taur,
               double* u, long long ldu, char* ws) {
  size_t off = cx_workspace(n, k);
  double* x = (double*)(ws + off);
  off += align256((size_t)k * n * 8);
  double* qr1 = (double*)(ws + off);
  off += align256((size_t)n * k * 8);
  double* fq = (double*)(ws + off);
  off += align256(form_q_work_elems(n, k, b) * 8);
  double* w = (double*)(ws + off);
  off += align256((size_t)k * k * 8);
  double* t11 = (double*)(ws + off);
  off += align256((size_t)k * k * 8);
  double* tinv = (double*)(ws + off);
  off += align256((size_t)k * k * 8);
  double* sk = (double*)(ws + off);
  int rc = launch_cx(s, m, n, k, afc, ldc, jpc, x, k, ws);
  if (rc) return rc;
  // Q_r1: the first k columns of the row factorization's Q (A^T is n x m)
  rc = form_q<double>(s, n, k, b, afr, ldr, taur, qr1, n, fq);
  if (rc) return rc;
  rc = gemm<double>(s, false, false, k, k, n, 1.0, x, k, qr1, n, 0.0, w, k, sk,
                    splitk_elems(k, k));
  if (rc) return rc;
  rc = upper_inverse<double>(s, k, afr, ldr, t11, tinv);
  if (rc) return rc;
  // U = W T11^-T
  return gemm<double>(s, false, true, k, k, k, 1.0, w, k, tinv, k, 0.0, u, ldu);
}

int compress_max_l() { return JMAX; }

size_t compress_workspace(int m, int n, int l, int k, int b) {
  return align256((size_t)l * n * 8) + 3 * align256((size_t)l * l * 8) + align256((size_t)l * 8) +
         align256((size_t)l * k * 8) + align256((size_t)m * l * 8) +
         align256(form_q_work_elems(m, l, b) * 8) + align256((size_t)k * n * 8) +
         align256(splitk_elems(l, l) * 8) + 256;
}

int launch_compress(hipStream_t s, int m, int n, int l, int k, int b, const double* af,
                    long long ldaf, const double* tau, const int* jpvt, double* x, long long ldx,
                    double* y, long long ldy, double* sigma, char* ws) {
  if (l < 1 || l > JMAX || k < 1 || k > l) return RQ_ERR_LIMIT;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = ws + off;
    off += align256(bytes);
    return p;
  };
  double* rl = (double*)take((size_t)l * n * 8);
  double* g = (double*)take((size_t)l * l * 8);
  double* v = (double*)take((size_t)l * l * 8);
  double* spare = (double*)take((size_t)l * l * 8);
  (void)spare;
  double* ev = (double*)take((size_t)l * 8);
  double* uk = (double*)take((size_t)l * k * 8);
  double* ql = (double*)take((size_t)m * l * 8);
  double* fq = (double*)take(form_q_work_elems(m, l, b) * 8);
  double* yp = (double*)take((size_t)k * n * 8);
  double* sk = (double*)take(splitk_elems(l, l) * 8);
  int* sweeps = (int*)take(256);
  hipLaunchKernelGGL(k_rl_dense, dim3(grid_of((long long)l * n)), dim3(CT), 0, s, l, n, af, ldaf,
                     rl);
  RQ_HIP_CHECK(hipGetLastError());
  int rc = gemm<double>(s, false, true, l, l, n, 1.0, rl, l, rl, l, 0.0, g, l, sk,
                        splitk_elems(l, l));
  if (rc) return rc;
  const size_t shmem = (size_t)l * JLD * sizeof(double);
  RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_eig),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(JT), shmem, s, l, (const double*)g, v, ev, 40,
                     sweeps);
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(CT), 0, s, l, k, (const double*)ev, (const double*)v,
                     uk, sigma);
  RQ_HIP_CHECK(hipGetLastError());
  rc = form_q<double>(s, m, l, b, af, ldaf, tau, ql, m, fq);
  if (rc) return rc;
  rc = gemm<double>(s, false, false, m, k, l, 1.0, ql, m, uk, l, 0.0, x, ldx);
  if (rc) return rc;
  rc = gemm<double>(s, true, false, k, n, l, 1.0, uk, l, rl, l, 0.0, yp, k);
  if (rc) return rc;
  hipLaunchKernelGGL(k_scatter_cols, dim3(grid_of((long long)k * n)), dim3(CT), 0, s, k, n,
                     (const double*)yp, jpvt, y, ldy);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace rq
