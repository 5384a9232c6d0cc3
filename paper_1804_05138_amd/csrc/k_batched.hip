// Batched truncated RQRCP (Alg. 2) of many small, uneven matrices in one
// persistent launch: one workgroup factors one problem at a time and takes
// the next problem index from a work queue (an atomic counter) until the
// batch is exhausted, so uneven sizes balance themselves.
//
// Per problem everything but A stays on chip:
//   * the sketch B = Omega A (l x n, FP64) lives in LDS for the whole
//     factorization; Omega (Philox stream problem + 1) is regenerated in
//     64-row chunks while A is streamed once;
//   * the partial QRCP of B (Alg. 1, norms recomputed) runs on LDS;
//   * the panel (rows i..m-1, bb <= 16 columns) is held in registers in FP64,
//     one reduction of 16 dot products per reflector;
//   * the trailing update A2 -= V (T^T (V^T A2)) streams A2 through L2 in FP32
//     (V staged in LDS by row chunks, one thread per column), and formula (1)
//     refreshes that column of B right after its update.
// A is FP32 (the batched form is the mixed-precision one); reflectors, T, the
// sketch and its updates are FP64.
#include <limits.h>

#include "internal.h"

namespace rq {
namespace {

constexpr int BMAX = 16;   // largest block size of the batched kernel
constexpr int LMAX = 32;   // largest b + p
constexpr int MMAX = 1024; // largest row count (panel rows in registers)
constexpr int RC = 64;     // rows per Omega chunk of the sketch
constexpr int SB_DOUBLES = 12288;  // LDS for B: l * n <= 12288

struct BatchedSmem {
  double b[SB_DOUBLES];
  double t[BMAX * BMAX];
  double r11[BMAX * BMAX];
  double gz[BMAX * BMAX];
  double red[16 * BMAX];  // per-wave partial sums (up to 16 waves)
  double row[BMAX];
  double s[BMAX];
  double f[BMAX];
  double g[BMAX];
  double hv[LMAX];        // Householder vector of a sketch step
  double hh[4];
  int jp[1024];
  int pairs[2 * BMAX];
  int npairs;
  int problem;
  int dead;               // a zero sketch pivot was met (no more pivoting or updates)
  int info;
  // sketch phase: Omega chunk (RC x LMAX doubles); trailing phase: V chunk
  // (NT x BMAX floats)
  __attribute__((aligned(16))) char chunk[32768];
};

// Values every thread of the workgroup holds identically (read back from LDS
// after a barrier) are passed through readfirstlane, so the compiler sees the
// loop and branch conditions built from them as uniform and keeps the
// barriers inside them in convergent control flow.
RQ_DEV int uniform_i(int x) { return __builtin_amdgcn_readfirstlane(x); }

template <int NT>
RQ_DEV void block_argmax_pos(double& v, int& p, double* sv, int* sp) {
  int dummy = 0;
  wave_argmax(v, p, dummy);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = v;
    sp[w] = p;
  }
  __syncthreads();
  v = sv[0];
  p = sp[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q)
    if (argbetter(sv[q], sp[q], v, p)) {
      v = sv[q];
      p = sp[q];
    }
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT, 1) void k_rqrcp_batched(
    int batch, const rqrcp_problem* __restrict__ probs, int b, int l, uint64_t seed,
    float* __restrict__ apool, long long a_elems, int* __restrict__ jpool, long long j_elems,
    double* __restrict__ tpool, long long t_elems, double* __restrict__ bpool, long long b_elems,
    int* __restrict__ infos, unsigned* __restrict__ queue) {
  constexpr int RPT = MMAX / NT;
  constexpr int NW = NT / 64;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  BatchedSmem& S = *reinterpret_cast<BatchedSmem*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (;;) {
    if (tid == 0) S.problem = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int pi = uniform_i(S.problem);
    __syncthreads();
    if (pi >= batch) break;  // uniform: every wave leaves

    const rqrcp_problem pr = probs[pi];
    const int m = pr.m, n = pr.n, k = pr.k;
    const long long lda = pr.lda;
    // descriptors are device data: check them here, skip (info = -1) what
    // does not fit the kernel or the pools
    const bool ok = m >= 1 && n >= 1 && k >= 1 && k <= min(m, n) && m <= MMAX && n <= 1024 &&
                    (long long)l * n <= SB_DOUBLES && lda >= m && pr.a_off >= 0 &&
                    pr.a_off + (long long)(n - 1) * lda + m <= a_elems && pr.jpvt_off >= 0 &&
                    pr.jpvt_off + n <= j_elems && pr.tau_off >= 0 && pr.tau_off + k <= t_elems &&
                    pr.b_off >= 0 && pr.b_off + (long long)l * n <= b_elems;
    if (!ok) {
      if (tid == 0) infos[pi] = -1;
    } else {
    float* a = apool + pr.a_off;
    int* jpvt = jpool + pr.jpvt_off;
    double* tau = tpool + pr.tau_off;
    double* bout = bpool + pr.b_off;
    double* sB = S.b;

    // ---- sketch B = Omega A, Omega from Philox(seed, stream pi + 1) ----
    double* som = reinterpret_cast<double*>(S.chunk);  // [rr * l + rho]
    for (int cs = 0; cs < n; cs += NT) {
      const int c = cs + tid;
      const bool cok = c < n;
      const float* acol = a + (long long)(cok ? c : 0) * lda;
      double acc[LMAX];
#pragma unroll
      for (int r = 0; r < LMAX; ++r) acc[r] = 0.0;
      for (int r0 = 0; r0 < m; r0 += RC) {
        // Omega(0:l, r0:r0+RC): normals q = r * l + rho, q in [r0 l, (r0 + RC) l)
        const long long q0 = (long long)r0 * l, q1 = (long long)(r0 + RC) * l;
        __syncthreads();
        for (long long blk = q0 / 4 + tid; blk * 4 < q1; blk += NT) {
          double z[4];
          philox_normals4((uint64_t)blk, seed, (uint64_t)pi + 1, z);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const long long q = 4 * blk + j;
            if (q >= q0 && q < q1) som[q - q0] = (q < (long long)m * l) ? z[j] : 0.0;
          }
        }
        __syncthreads();
        const int rn = min(RC, m - r0);
        // rows in groups so that their loads are in flight together
#pragma unroll 16
        for (int rr = 0; rr < rn; ++rr) {
          const double av = cok ? (double)acol[r0 + rr] : 0.0;
#pragma unroll
          for (int r = 0; r < LMAX; ++r)
            if (r < l) acc[r] += som[rr * l + r] * av;
        }
      }
      if (cok) {
#pragma unroll
        for (int r = 0; r < LMAX; ++r)
          if (r < l) sB[c * l + r] = acc[r];
      }
    }
    for (int c = tid; c < n; c += NT) S.jp[c] = c;
    if (tid == 0) {
      S.dead = 0;
      S.info = 0;
    }
    __syncthreads();

    // ---- block loop ----
    for (int i = 0; i < k; i += b) {
      const int bb = min(b, k - i);
      // (a) partial QRCP of B(:, i:n): bb greedy steps
      if (tid == 0) S.npairs = 0;
      for (int t = 0; t < bb; ++t) {
        const int gpos = i + t;
        __syncthreads();
        if (uniform_i(S.dead)) continue;
        double bn = -1.0;
        int bp = INT_MAX;
        for (int c = gpos + tid; c < n; c += NT) {
          double s2 = 0.0;
          for (int r = t; r < l; ++r) s2 += sB[c * l + r] * sB[c * l + r];
          if (argbetter(s2, c, bn, bp)) {
            bn = s2;
            bp = c;
          }
        }
        block_argmax_pos<NT>(bn, bp, S.red, reinterpret_cast<int*>(S.red + 8 * BMAX));
        // no finite candidate (a NaN in the sketch) or an exact zero sketch: no
        // more pivots, no more sketch updates (info -2 or the rank + 1)
        const bool nonfinite = !(bn >= 0.0) || bp < gpos || bp >= n;
        if (uniform_i((bn == 0.0 || nonfinite) ? 1 : 0)) {
          if (tid == 0) {
            S.dead = 1;
            S.info = nonfinite ? -2 : gpos + 1;
          }
          __syncthreads();
          continue;
        }
        const int js = uniform_i(bp);
        if (js != gpos) {
          for (int r = tid; r < l; r += NT) {
            const double x = sB[js * l + r];
            sB[js * l + r] = sB[gpos * l + r];
            sB[gpos * l + r] = x;
          }
          if (tid == 0) {
            const int tj = S.jp[js];
            S.jp[js] = S.jp[gpos];
            S.jp[gpos] = tj;
            S.pairs[2 * S.npairs] = gpos;
            S.pairs[2 * S.npairs + 1] = js;
            S.npairs = S.npairs + 1;
          }
        }
        __syncthreads();
        // Householder of B(t:l, gpos) (LAPACK dlarfg convention)
        if (wave == 0) {
          double x2 = 0.0;
          for (int r = t + 1 + lane; r < l; r += 64) x2 += sB[gpos * l + r] * sB[gpos * l + r];
          x2 = wave_sum_dpp(x2);
          if (lane == 0) {
            const double alpha = sB[gpos * l + t];
            double beta = alpha, tt = 0.0, den = 1.0;
            if (x2 > 0.0) {
              const double nrm = hypot(alpha, sqrt(x2));
              beta = (alpha >= 0.0) ? -nrm : nrm;
              tt = (beta - alpha) / beta;
              den = alpha - beta;
            }
            S.hh[0] = beta;
            S.hh[1] = tt;
            S.hh[2] = den;
          }
        }
        __syncthreads();
        const double tt = S.hh[1], den = S.hh[2];
        for (int r = tid; r < l; r += NT)
          S.hv[r] = (r == t) ? 1.0 : ((r > t && tt != 0.0) ? sB[gpos * l + r] / den : 0.0);
        __syncthreads();
        if (tid == 0) {
          sB[gpos * l + t] = S.hh[0];
          for (int r = t + 1; r < l; ++r) sB[gpos * l + r] = 0.0;
        }
        if (tt != 0.0) {
          for (int c = gpos + 1 + tid; c < n; c += NT) {
            double d = 0.0;
            for (int r = t; r < l; ++r) d += S.hv[r] * sB[c * l + r];
            const double f = tt * d;
            for (int r = t; r < l; ++r) sB[c * l + r] -= f * S.hv[r];
          }
        }
      }
      __syncthreads();
      // (b) the same transpositions on A (full columns), in order
      const int np = uniform_i(S.npairs);
      for (int e = 0; e < np; ++e) {
        const int c0 = S.pairs[2 * e], c1 = S.pairs[2 * e + 1];
        float* x0 = a + (long long)c0 * lda;
        float* x1 = a + (long long)c1 * lda;
        for (int r = tid; r < m; r += NT) {
          const float v = x0[r];
          x0[r] = x1[r];
          x1[r] = v;
        }
        __syncthreads();
      }

      // (c) panel QR of A(i:m, i:i+bb) in registers (FP64), T from V^T v_t
      double P[RPT][BMAX];
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int r = i + tid + NT * u;
#pragma unroll
        for (int q = 0; q < BMAX; ++q)
          P[u][q] = (r < m && q < bb) ? (double)a[(long long)(i + q) * lda + r] : 0.0;
      }
      for (int t = 0; t < bb; ++t) {
        const int gr = i + t;
        double sp[BMAX];
#pragma unroll
        for (int q = 0; q < BMAX; ++q) sp[q] = 0.0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int r = i + tid + NT * u;
          double xt = 0.0;
#pragma unroll
          for (int q = 0; q < BMAX; ++q)
            if (q == t) xt = P[u][q];
          if (r > gr && r < m) {
#pragma unroll
            for (int q = 0; q < BMAX; ++q) sp[q] += xt * P[u][q];
          }
        }
#pragma unroll
        for (int q = 0; q < BMAX; ++q) {
          const double v = wave_sum_dpp(sp[q]);
          if (lane == 0) S.red[wave * BMAX + q] = v;
        }
        if (tid == t) {
#pragma unroll
          for (int q = 0; q < BMAX; ++q) S.row[q] = P[0][q];
        }
        __syncthreads();
        if (tid < BMAX) {
          double s = 0.0;
          for (int w = 0; w < NW; ++w) s += S.red[w * BMAX + tid];
          S.s[tid] = s;
        }
        __syncthreads();
        if (tid == 0) {
          const double alpha = S.row[t], xn2 = S.s[t];
          double beta = alpha, tt = 0.0, den = 1.0;
          if (xn2 > 0.0) {
            const double nrm = hypot(alpha, sqrt(xn2));
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tt = (beta - alpha) / beta;
            den = alpha - beta;
          }
          S.hh[0] = beta;
          S.hh[1] = tt;
          S.hh[2] = den;
          tau[gr] = tt;
        }
        __syncthreads();
        const double beta = S.hh[0], tt = S.hh[1], den = S.hh[2];
        if (tid < BMAX) {
          const int q = tid;
          S.gz[t * BMAX + q] = (q < t) ? S.row[q] + S.s[q] / den : 0.0;
          const double f = (q > t && q < bb && tt != 0.0) ? tt * (S.row[q] + S.s[q] / den) : 0.0;
          S.f[q] = f;
          S.g[q] = f / den;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int r = i + tid + NT * u;
          double xt = 0.0;
#pragma unroll
          for (int q = 0; q < BMAX; ++q)
            if (q == t) xt = P[u][q];
          if (r > gr && r < m) {
#pragma unroll
            for (int q = 0; q < BMAX; ++q) P[u][q] -= xt * S.g[q];
            if (tt != 0.0) xt = xt / den;
          } else if (r == gr) {
#pragma unroll
            for (int q = 0; q < BMAX; ++q) P[u][q] -= S.f[q];
            xt = beta;
          }
#pragma unroll
          for (int q = 0; q < BMAX; ++q)
            if (q == t) P[u][q] = xt;
        }
      }
      // R11 (FP64) for the sample update; write R and V back (FP32)
      if (tid < bb) {
#pragma unroll
        for (int q = 0; q < BMAX; ++q) S.r11[tid * BMAX + q] = (q >= tid && q < bb) ? P[0][q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int r = i + tid + NT * u;
        if (r < m) {
#pragma unroll
          for (int q = 0; q < BMAX; ++q)
            if (q < bb) a[(long long)(i + q) * lda + r] = (float)P[u][q];
        }
      }
      // T (upper, bb x bb): T(t,t) = tau_t, T(0:t, t) = -tau_t T(0:t, 0:t) gz(t, 0:t)
      __syncthreads();
      for (int e = tid; e < BMAX * BMAX; e += NT) S.t[e] = 0.0;
      __syncthreads();
      for (int t = 0; t < bb; ++t) {
        const double tt = tau[i + t];
        if (tid < t) {
          double acc = 0.0;
          for (int c = tid; c < t; ++c) acc += S.t[tid * BMAX + c] * S.gz[t * BMAX + c];
          S.t[tid * BMAX + t] = -tt * acc;
        }
        if (tid == t) S.t[t * BMAX + t] = tt;
        __syncthreads();
      }

      // (d) trailing update of A(i:m, i+bb:n) and the sample update of B
      float* sv = reinterpret_cast<float*>(S.chunk);  // [rr * BMAX + q]
      const int c0 = i + bb;
      for (int cs = c0; cs < n; cs += NT) {
        const int c = cs + tid;
        const bool cok = c < n;
        float* acol = a + (long long)(cok ? c : 0) * lda;
        float w[BMAX];
#pragma unroll
        for (int q = 0; q < BMAX; ++q) w[q] = 0.0f;
        // W(:, c) = V^T A(i:m, c)
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int r = i + tid + NT * u;
          __syncthreads();
#pragma unroll
          for (int q = 0; q < BMAX; ++q) {
            const int d = r - i;
            float v = (d > q) ? (float)P[u][q] : (d == q ? 1.0f : 0.0f);
            sv[tid * BMAX + q] = (r < m && q < bb) ? v : 0.0f;
          }
          __syncthreads();
          if (cok) {
            const int rb = i + NT * u;
            const int rn = min(NT, m - rb);
#pragma unroll 32
            for (int rr = 0; rr < rn; ++rr) {
              const float av = acol[rb + rr];
#pragma unroll
              for (int q = 0; q < BMAX; ++q) w[q] += sv[rr * BMAX + q] * av;
            }
          }
        }
        // W' = T^T W (FP64)
        float wp[BMAX];
#pragma unroll
        for (int q = 0; q < BMAX; ++q) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j <= q; ++j) s += S.t[j * BMAX + q] * (double)w[j];
          wp[q] = (float)s;
        }
        // A(i:m, c) -= V W'; keep the new rows i..i+bb (R12) in FP64
        double r12[BMAX];
#pragma unroll
        for (int q = 0; q < BMAX; ++q) r12[q] = 0.0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int r = i + tid + NT * u;
          __syncthreads();
#pragma unroll
          for (int q = 0; q < BMAX; ++q) {
            const int d = r - i;
            float v = (d > q) ? (float)P[u][q] : (d == q ? 1.0f : 0.0f);
            sv[tid * BMAX + q] = (r < m && q < bb) ? v : 0.0f;
          }
          __syncthreads();
          if (cok) {
            const int rb = i + NT * u;
            const int rn = min(NT, m - rb);
#pragma unroll 32
            for (int rr = 0; rr < rn; ++rr) {
              float x = acol[rb + rr];
#pragma unroll
              for (int q = 0; q < BMAX; ++q) x -= sv[rr * BMAX + q] * wp[q];
              acol[rb + rr] = x;
              if (u == 0 && rr < BMAX) {
#pragma unroll
                for (int q = 0; q < BMAX; ++q)
                  if (q == rr) r12[q] = (double)x;
              }
            }
          }
        }
        // formula (1): B(0:bb, c) -= Rhat11 R11^-1 R12(:, c)
        if (cok && !uniform_i(S.dead)) {
          double xs[BMAX];
#pragma unroll
          for (int q = BMAX - 1; q >= 0; --q) {
            double s = r12[q];
#pragma unroll
            for (int j = q + 1; j < BMAX; ++j)
              if (j < bb) s -= S.r11[q * BMAX + j] * xs[j];
            xs[q] = (q < bb) ? s / S.r11[q * BMAX + q] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < BMAX; ++q) {
            if (q < bb) {
              double s = 0.0;
#pragma unroll
              for (int j = q; j < BMAX; ++j)
                if (j < bb) s += sB[(i + j) * l + q] * xs[j];
              sB[c * l + q] -= s;
            }
          }
        }
      }
      __syncthreads();
    }

    // ---- outputs: final sketch, permutation, info ----
    for (int e = tid; e < l * n; e += NT) bout[e] = sB[e];
    for (int c = tid; c < n; c += NT) jpvt[c] = S.jp[c];
    if (tid == 0) infos[pi] = S.info;
    }
    __syncthreads();
  }
}

__global__ void k_queue_reset(unsigned* q) { *q = 0u; }

}  // namespace

int batched_variants() { return 2; }
const char* batched_variant_name(int v) { return v == 0 ? "256 threads" : "512 threads"; }

int batched_max(int* max_m, int* max_ln, int* max_b, int* max_l) {
  if (max_m) *max_m = MMAX;
  if (max_ln) *max_ln = SB_DOUBLES;
  if (max_b) *max_b = BMAX;
  if (max_l) *max_l = LMAX;
  return 0;
}

int launch_batched(hipStream_t s, int variant, int batch, const rqrcp_problem* probs, int b, int l,
                   uint64_t seed, float* apool, long long a_elems, int* jpool, long long j_elems,
                   double* tpool, long long t_elems, double* bpool, long long b_elems, int* infos,
                   unsigned* queue) {
  if (b < 1 || b > BMAX || l < 1 || l > LMAX) return RQ_ERR_LIMIT;
  int dev = 0, ncu = 0;
  RQ_HIP_CHECK(hipGetDevice(&dev));
  RQ_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const size_t shmem = sizeof(BatchedSmem);
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, queue);
  RQ_HIP_CHECK(hipGetLastError());
  int grid = ncu;  // one problem-sized LDS footprint per compute unit
  if (grid > batch) grid = batch;
  if (grid < 1) return RQ_OK;
  if (variant == 0) {
    auto kern = &k_rqrcp_batched<256>;
    RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), shmem, s, batch, probs, b, l, seed, apool,
                       a_elems, jpool, j_elems, tpool, t_elems, bpool, b_elems, infos, queue);
  } else {
    auto kern = &k_rqrcp_batched<512>;
    RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(512), shmem, s, batch, probs, b, l, seed, apool,
                       a_elems, jpool, j_elems, tpool, t_elems, bpool, b_elems, infos, queue);
  }
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace rq
