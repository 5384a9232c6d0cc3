// Batched truncated RQRCP (Alg. 2) of many small, uneven matrices in one
// persistent launch: one workgroup factors one problem at a time and takes
// the next problem index from a work queue (an atomic counter) until the
// batch is exhausted, so uneven sizes balance themselves.
//
// Per problem everything but A stays on chip:
//   * the sketch B = Omega A (l x n, FP64) lives in LDS for the whole
//     factorization; it is formed on FP64 MFMA (16x16x4) with Omega (Philox
//     stream problem + 1) regenerated in 64-row chunks while A is streamed once;
//   * the partial QRCP of B (Alg. 1, norms recomputed) runs on LDS;
//   * the panel (rows i..m-1, bb <= 16 columns) is held in registers in FP64,
//     one reduction of 16 dot products per reflector;
//   * the trailing update A2 -= V (T^T (V^T A2)) runs on FP32 MFMA, one wave
//     per 16-column tile with its row loads double-buffered in registers;
//     T^T W and formula (1) (B(0:bb, tile) -= Rhat11 R11^-1 R12) are FP64 MFMA
//     products on the tile's registers.
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
constexpr int SB_DOUBLES = 12288;  // largest l * n (the LDS copy holds (l | 1) * n)

struct BatchedSmem {
  double b[SB_DOUBLES + 1024];  // (l | 1) n <= l n + n, n <= 1024
  double t[BMAX * BMAX];
  double r11[BMAX * BMAX];
  double gz[BMAX * BMAX];
  double mm[BMAX * BMAX];  // M = Rhat11 R11^-1 of formula (1), row-major
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
  // sketch phase: Omega chunk (RC x LMAX doubles)
  __attribute__((aligned(16))) char chunk[RC * LMAX * 8];
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
  constexpr int SKT = 4;                  // 16-column tiles per wave in the sketch
  constexpr int TG = NT >= 512 ? 1 : 2;   // 16-row steps per load group (trailing update)
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
                    (long long)(n - 1) * lda + m <= (long long)INT_MAX &&
                    pr.a_off + (long long)(n - 1) * lda + m <= a_elems && pr.jpvt_off >= 0 &&
                    pr.jpvt_off + n <= j_elems && pr.tau_off >= 0 && pr.tau_off + k <= t_elems &&
                    pr.b_off >= 0 && pr.b_off + (long long)l * n <= b_elems;
    if (!ok) {
      if (tid == 0) infos[pi] = -1;
    } else {
    float* a = apool + pr.a_off;
    const unsigned ulda = (unsigned)lda;  // (n - 1) lda + m < 2^31: 32-bit offsets
    int* jpvt = jpool + pr.jpvt_off;
    double* tau = tpool + pr.tau_off;
    double* bout = bpool + pr.b_off;
    double* sB = S.b;
    // column stride of the sketch in LDS: odd, so that the lanes of a wave that
    // walk consecutive columns hit different banks
    const int lb = l | 1;

    // ---- sketch B = Omega A on FP64 MFMA, Omega from Philox(seed, stream pi + 1) ----
    // Each wave owns SKT 16-column tiles of B per pass; the K loop runs over A's
    // rows in Omega chunks of RC rows generated into LDS.  Operands (16x16x4
    // FP64): Omega(16 rows of l, 4 rows of A) from LDS, A(4 rows, 16 columns)
    // from global memory -- a wave's load covers four consecutive rows of 16
    // columns, so a cache line serves eight k-steps.
    double* som = reinterpret_cast<double*>(S.chunk);  // [rr * l + rho]
    const int lr16 = lane & 15, lg = lane >> 4;
    for (int cs = 0; cs < n; cs += 16 * SKT * NW) {
      v4d acc[SKT][2];
#pragma unroll
      for (int j = 0; j < SKT; ++j) acc[j][0] = acc[j][1] = v4d{0, 0, 0, 0};
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
#pragma unroll 4
        for (int kk = 0; kk < RC / 4; ++kk) {
          const int kr = 4 * kk + lg;             // row of the chunk this lane feeds
          const int krow = r0 + kr;
          const double o0 = (lr16 < l) ? som[kr * l + (lr16 < l ? lr16 : 0)] : 0.0;
          const double o1 = (16 + lr16 < l) ? som[kr * l + (16 + lr16 < l ? 16 + lr16 : 0)] : 0.0;
          double bv[SKT];
#pragma unroll
          for (int j = 0; j < SKT; ++j) {
            const int col = cs + 16 * (wave + j * NW) + lr16;
            const float x = a[(unsigned)(col < n ? col : 0) * ulda + (unsigned)(krow < m ? krow : 0)];
            bv[j] = (col < n && krow < m) ? (double)x : 0.0;
          }
#pragma unroll
          for (int j = 0; j < SKT; ++j) {
            acc[j][0] = mfma_f64(o0, bv[j], acc[j][0]);
            acc[j][1] = mfma_f64(o1, bv[j], acc[j][1]);
          }
        }
      }
      // FP64 accumulator layout: lane l, element e holds row l/16 + 4e, column l%16
#pragma unroll
      for (int j = 0; j < SKT; ++j) {
        const int col = cs + 16 * (wave + j * NW) + lr16;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = 16 * rt + lg + 4 * e;
            if (col < n && r < l) sB[col * lb + r] = acc[j][rt][e];
          }
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
          for (int r = t; r < l; ++r) s2 += sB[c * lb + r] * sB[c * lb + r];
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
            const double x = sB[js * lb + r];
            sB[js * lb + r] = sB[gpos * lb + r];
            sB[gpos * lb + r] = x;
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
          for (int r = t + 1 + lane; r < l; r += 64)
            x2 += sB[gpos * lb + r] * sB[gpos * lb + r];
          x2 = wave_sum_dpp(x2);
          if (lane == 0) {
            const double alpha = sB[gpos * lb + t];
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
          S.hv[r] = (r == t) ? 1.0 : ((r > t && tt != 0.0) ? sB[gpos * lb + r] / den : 0.0);
        __syncthreads();
        if (tid == 0) {
          sB[gpos * lb + t] = S.hh[0];
          for (int r = t + 1; r < l; ++r) sB[gpos * lb + r] = 0.0;
        }
        if (tt != 0.0) {
          for (int c = gpos + 1 + tid; c < n; c += NT) {
            double d = 0.0;
            for (int r = t; r < l; ++r) d += S.hv[r] * sB[c * lb + r];
            const double f = tt * d;
            for (int r = t; r < l; ++r) sB[c * lb + r] -= f * S.hv[r];
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
      // M = Rhat11 R11^-1 (upper, bb x bb; zero outside): row q solves M(q, :) R11 =
      // Rhat11(q, :), Rhat11(q, j) = B(q, i + j) the sketch's R after its QRCP
      if (tid < BMAX) {
        const int q = tid;
        double mrow[BMAX];
#pragma unroll
        for (int j = 0; j < BMAX; ++j) {
          double x = 0.0;
          if (q < bb && j < bb && j >= q) {
            x = sB[(i + j) * lb + q];
#pragma unroll
            for (int p = 0; p < j; ++p)
              if (p >= q) x -= mrow[p] * S.r11[p * BMAX + j];
            x /= S.r11[j * BMAX + j];
          }
          mrow[j] = x;
        }
#pragma unroll
        for (int j = 0; j < BMAX; ++j) S.mm[q * BMAX + j] = mrow[j];
      }
      __syncthreads();

      // (d) trailing update of A(i:m, i+bb:n) on FP32 MFMA (16x16x4) and the sample
      // update of B.  A wave owns whole 16-column tiles: W = V^T A2 (K = the rows),
      // W' = T^T W per column in FP64, A2 -= V W' (K = bb), then formula (1) for
      // the tile's sketch columns from its R12 rows -- no workgroup barrier.  V is
      // read from A itself (written back above in FP32): V(r, q) = A(r, i+q) below
      // the unit diagonal.  Rows go in groups of TG (16-row steps); the next
      // group's loads are issued before the current group is used, so two groups
      // of loads are in flight per wave.
      {
        const int c0 = i + bb;
        const int ntile = (n - c0 + 15) / 16;
        const int qv = (lr16 < bb) ? lr16 : 0;
        const unsigned vcol = (unsigned)(i + qv) * ulda;              // V(:, lane % 16)
        unsigned vq[4];                                                // V(:, 4 kk + lane / 16)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) vq[kk] = (unsigned)(i + (4 * kk + lg < bb ? 4 * kk + lg : 0)) * ulda;
        for (int tt = wave; tt < ntile; tt += NW) {
          const int col = c0 + 16 * tt + lr16;
          const bool cok = col < n;
          const unsigned acol = (unsigned)(cok ? col : c0) * ulda;
          // W: lane (lg, lr16) takes rows r0 + 16u + 4 lg + e for both operands
          v4f w4 = v4f{0, 0, 0, 0};
          {
            float xa0[4 * TG], xv0[4 * TG], xa1[4 * TG], xv1[4 * TG];
            auto wload = [&](float (&xa)[4 * TG], float (&xv)[4 * TG], int r0) {
#pragma unroll
              for (int u = 0; u < TG; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int row = r0 + 16 * u + 4 * lg + e;
                  const unsigned rc = (unsigned)(row < m ? row : m - 1);
                  xa[4 * u + e] = a[acol + rc];
                  xv[4 * u + e] = a[vcol + rc];
                }
            };
            auto wmma = [&](const float (&xa)[4 * TG], const float (&xv)[4 * TG], int r0) {
#pragma unroll
              for (int u = 0; u < TG; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int row = r0 + 16 * u + 4 * lg + e;
                  const int d = row - i;
                  float v = (d > lr16) ? xv[4 * u + e] : (d == lr16 ? 1.0f : 0.0f);
                  v = (row < m && lr16 < bb) ? v : 0.0f;
                  const float x = (row < m && cok) ? xa[4 * u + e] : 0.0f;
                  w4 = mfma_f32(v, x, w4);
                }
            };
            // the exit test comes before a group's loads, so no load is dead on a
            // path (the compiler would sink it behind the use of the previous group)
            int r0 = i;
            wload(xa0, xv0, r0);
            for (;;) {
              if (r0 + 16 * TG >= m) {
                wmma(xa0, xv0, r0);
                break;
              }
              wload(xa1, xv1, r0 + 16 * TG);
              wmma(xa0, xv0, r0);
              r0 += 16 * TG;
              if (r0 + 16 * TG >= m) {
                wmma(xa1, xv1, r0);
                break;
              }
              wload(xa0, xv0, r0 + 16 * TG);
              wmma(xa1, xv1, r0);
              r0 += 16 * TG;
            }
          }
          // W' = T^T W on FP64 MFMA.  W's accumulator layout gives lane (lg, lr16)
          // W(4 lg + e, lr16); the K index of product e is j = 4 lg + e, so the A
          // operand is T^T(lr16, 4 lg + e) = T(4 lg + e, lr16).  The FP64 result
          // holds W'(lg + 4 e, lr16): element kk is the B operand -W'(4 kk + lg, lr16)
          // of the update's product kk.
          float wq[4];
          {
            v4d wp = v4d{0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) wp = mfma_f64(S.t[(4 * lg + e) * BMAX + lr16], (double)w4[e], wp);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) wq[kk] = (float)(-wp[kk]);
          }
          // A2 -= V W': C tile rows r0 + 16u + 4 lg + e, column lr16 (accumulator layout);
          // A operand V(r0 + 16u + lr16, 4 kk + lg)
          float r12v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
          {
            float xc0[4 * TG], xw0[4 * TG], xc1[4 * TG], xw1[4 * TG];
            auto uload = [&](float (&xc)[4 * TG], float (&xw)[4 * TG], int r0) {
#pragma unroll
              for (int u = 0; u < TG; ++u) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int row = r0 + 16 * u + 4 * lg + e;
                  xc[4 * u + e] = a[acol + (unsigned)(row < m ? row : m - 1)];
                }
                const int vr = r0 + 16 * u + lr16;
                const unsigned vrc = (unsigned)(vr < m ? vr : m - 1);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) xw[4 * u + kk] = a[vq[kk] + vrc];
              }
            };
            auto ucomp = [&](const float (&xc)[4 * TG], const float (&xw)[4 * TG], int r0) {
#pragma unroll
              for (int u = 0; u < TG; ++u) {
                const int rb = r0 + 16 * u;
                v4f c = v4f{xc[4 * u], xc[4 * u + 1], xc[4 * u + 2], xc[4 * u + 3]};
                const int vr = rb + lr16;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                  const int q = 4 * kk + lg;
                  const int d = vr - i;
                  float v = (d > q) ? xw[4 * u + kk] : (d == q ? 1.0f : 0.0f);
                  v = (vr < m && q < bb) ? v : 0.0f;
                  c = mfma_f32(v, wq[kk], c);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int row = rb + 4 * lg + e;
                  if (cok && row < m) a[acol + (unsigned)row] = c[e];
                  if (rb == i) r12v[e] = c[e];   // R12(4 lg + e, lr16)
                }
              }
            };
            // a group's loads are issued before the previous group's stores
            int r0 = i;
            uload(xc0, xw0, r0);
            for (;;) {
              if (r0 + 16 * TG >= m) {
                ucomp(xc0, xw0, r0);
                break;
              }
              uload(xc1, xw1, r0 + 16 * TG);
              ucomp(xc0, xw0, r0);
              r0 += 16 * TG;
              if (r0 + 16 * TG >= m) {
                ucomp(xc1, xw1, r0);
                break;
              }
              uload(xc0, xw0, r0 + 16 * TG);
              ucomp(xc1, xw1, r0);
              r0 += 16 * TG;
            }
          }
          // formula (1) for this tile's columns: B(0:bb, c) -= M R12(:, c) on FP64
          // MFMA, K index 4 lg + e as for W' (lane (lg, lr16) holds R12(4 lg + e, lr16));
          // the result holds the update of B(lg + 4 e, lr16)
          if (!uniform_i(S.dead)) {
            v4d bu = v4d{0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) bu = mfma_f64(S.mm[lr16 * BMAX + 4 * lg + e], (double)r12v[e], bu);
            if (cok) {
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int q = lg + 4 * e;
                if (q < bb) sB[col * lb + q] -= bu[e];
              }
            }
          }
        }
      }
      __syncthreads();
    }

    // ---- outputs: final sketch, permutation, info ----
    for (int e = tid; e < l * n; e += NT) bout[e] = sB[(e / l) * lb + e % l];
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
  auto launch = [&](auto kern, int nt) -> int {
    RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), shmem, s, batch, probs, b, l, seed, apool,
                       a_elems, jpool, j_elems, tpool, t_elems, bpool, b_elems, infos, queue);
    return RQ_OK;
  };
  int rc = RQ_OK;
  if (variant == 0)
    rc = launch(&k_rqrcp_batched<256>, 256);
  else
    rc = launch(&k_rqrcp_batched<512>, 512);
  if (rc != RQ_OK) return rc;
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace rq
