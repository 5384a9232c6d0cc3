// Householder QR of the pivoted panel (the panel factorization without
// pivoting in Alg. 2; PDGEQRF in Alg. 4) and its compact-WY factor T (PDLARFT).
// The arithmetic is FP64 for both storage types of A: an FP32 panel is
// widened on load and R, V are rounded to FP32 on the way back.
//
// One persistent, co-resident grid; each workgroup keeps a contiguous slab of
// panel rows in LDS for the whole call.  Reflector t needs one global
// reduction: every workgroup sums, over its rows below the diagonal, the
// products of column t with every panel column c (c > t: the dot products of
// the reflector with the remaining columns; c < t: the dot products with the
// earlier Householder vectors, which give column t of T; c = t: the norm).
// The last workgroup to arrive adds the partials in a fixed order, so the
// result is deterministic.  Each workgroup then forms the same reflector
// (LAPACK dlarfg convention) and updates its own rows.
//
// Before factoring, the panel columns receive the previous block's pending
// update A(ip:m, panel) -= V_prev W'(:, panel) (rows from the previous
// block's first row ip), which the fused trailing pass leaves out.
#include "internal.h"

namespace rq {
namespace {

constexpr int PT = 256;
constexpr int VCH = 16;  // rows per chunk of the pending-update pass

template <typename T>
__global__ __launch_bounds__(PT, 1) void k_panel(int m, T* __restrict__ a, long long lda,
                                                 int i, int bb, int bbp,
                                                 const double* __restrict__ wp, long long ldw,
                                                 double* __restrict__ tau, double* __restrict__ tmat,
                                                 GridBarrier* bar, double* __restrict__ gpart,
                                                 int R, const int* __restrict__ skip) {
  if (skip && *skip) return;  // the panel was already factored by another path
  extern __shared__ double lds[];
  const int ldp = bb + 1;
  double* P = lds;                      // R x bb panel slab, row stride ldp
  double* Vc = lds + (size_t)R * ldp;   // VCH x bbp chunk of previous reflectors
  __shared__ double s_red[PT];
  __shared__ double s_row[MAX_B];
  __shared__ double s_S[MAX_B];
  __shared__ double s_f[MAX_B];
  __shared__ double s_g[MAX_B];
  (void)s_f;
  __shared__ double s_hh[3];
  __shared__ BarrierLocal bl;

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int rp = i - bbp;
  const int rs = rp + g * R;
  const int re = min(m, rs + R);
  const int nr = max(0, re - rs);
  double* growbuf = gpart + 2 * (size_t)G * bb;  // [2][bb] pivot rows
  double* gz = growbuf + 2 * bb;                 // [bb][bb] columns V^T v_t for T
  grid_sync_init(bar, &bl);

  // ---- load the slab ----
  for (int e = tid; e < nr * bb; e += PT) {
    const int c = e / nr, r = e % nr;
    P[r * ldp + c] = (double)a[(long long)(i + c) * lda + rs + r];
  }
  __syncthreads();

  // ---- pending update of the previous block ----
  if (bbp > 0) {
    for (int ch = 0; ch < nr; ch += VCH) {
      for (int e = tid; e < VCH * bbp; e += PT) {
        const int q = e / VCH, rr = e % VCH;
        const int r = rs + ch + rr;
        double v = 0.0;
        if (ch + rr < nr) {
          const int d = r - rp;
          v = (d > q) ? (double)a[(long long)(rp + q) * lda + r] : (d == q ? 1.0 : 0.0);
        }
        Vc[rr * bbp + q] = v;
      }
      __syncthreads();
      for (int e = tid; e < VCH * bb; e += PT) {
        const int c = e % bb, rr = e / bb;
        if (ch + rr < nr) {
          const double* w = wp + (long long)c * ldw;
          double acc = 0.0;
          for (int q = 0; q < bbp; ++q) acc += Vc[rr * bbp + q] * w[q];
          P[(ch + rr) * ldp + c] -= acc;
        }
      }
      __syncthreads();
    }
  }

  const int ng = PT / bb;  // row groups: thread (c, q) works on column c, rows q, q+ng, ...
  const int cc = tid % bb, qq0 = tid / bb;
  for (int t = 0; t < bb; ++t) {
    const int gr = i + t;
    // first local row strictly below the diagonal row, in my row group
    const int lo = max(0, gr - rs + 1);
    const int lr0 = lo + (((qq0 - lo) % ng) + ng) % ng;
    double* gp = gpart + (size_t)(t & 1) * G * bb;  // partials of this step
    // ---- partial dot products over my rows below the diagonal ----
    {
      double acc = 0.0;
      if (qq0 < ng) {
        for (int lr = lr0; lr < nr; lr += ng) acc += P[lr * ldp + t] * P[lr * ldp + cc];
      }
      s_red[tid] = acc;
      __syncthreads();
      if (tid < bb) {
        double sum = 0.0;
        for (int qq = 0; qq < ng; ++qq) sum += s_red[qq * bb + tid];
        gp[(size_t)g * bb + tid] = sum;
      }
      if (gr >= rs && gr < re && tid < bb) growbuf[(t & 1) * bb + tid] = P[(gr - rs) * ldp + tid];
    }
    grid_barrier(bar, G, &bl);
    // ---- every workgroup adds all partials in the same fixed order ----
    {
      double acc = 0.0;
      if (qq0 < ng) {
        int gg = qq0;
        for (; gg + 15 * ng < G; gg += 16 * ng) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = gp[(size_t)(gg + u * ng) * bb + cc];
#pragma unroll
          for (int u = 0; u < 16; ++u) acc += v[u];
        }
        for (; gg < G; gg += ng) acc += gp[(size_t)gg * bb + cc];
      }
      s_red[tid] = acc;
      if (tid < bb) s_row[tid] = growbuf[(t & 1) * bb + tid];
      __syncthreads();
      if (tid < bb) {
        double sum = 0.0;
        for (int qq = 0; qq < ng; ++qq) sum += s_red[qq * bb + tid];
        s_S[tid] = sum;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const double alpha = s_row[t], xn2 = s_S[t];
      double beta = alpha, tt = 0.0, den = 1.0;
      if (xn2 > 0.0) {
        const double nrm = hypot(alpha, sqrt(xn2));
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tt = (beta - alpha) / beta;
        den = alpha - beta;
      }
      s_hh[0] = beta;
      s_hh[1] = tt;
      s_hh[2] = den;
      if (g == 0) tau[i + t] = tt;
    }
    __syncthreads();
    const double beta = s_hh[0], tt = s_hh[1], den = s_hh[2];
    if (g == 0 && tid < bb) gz[t * bb + tid] = (tid < t) ? (s_row[tid] + s_S[tid] / den) : 0.0;
    // s_f[c] = tau * (v^T a_c) for c > t; s_g[c] = s_f[c] / (alpha - beta)
    if (tid < bb) {
      const double f = (tid > t && tt != 0.0) ? tt * (s_row[tid] + s_S[tid] / den) : 0.0;
      s_f[tid] = f;
      s_g[tid] = f / den;
    }
    __syncthreads();
    if (tt != 0.0) {
      if (qq0 < ng && cc > t) {
        const double g = s_g[cc];
        for (int lr = lr0; lr < nr; lr += ng) P[lr * ldp + cc] -= P[lr * ldp + t] * g;
        if (gr >= rs && gr < re && qq0 == 0) P[(gr - rs) * ldp + cc] -= s_f[cc];
      }
      __syncthreads();
    }
    for (int lr = tid; lr < nr; lr += PT) {
      const int gro = rs + lr;
      if (gro == gr)
        P[lr * ldp + t] = beta;
      else if (gro > gr && tt != 0.0)
        P[lr * ldp + t] = P[lr * ldp + t] / den;
    }
    __syncthreads();
  }

  // ---- write the slab back ----
  for (int e = tid; e < nr * bb; e += PT) {
    const int c = e / nr, r = e % nr;
    a[(long long)(i + c) * lda + rs + r] = (T)P[r * ldp + c];
  }

  // ---- T from the stored (V^T v_t) columns (forward, columnwise); workgroup 0
  // wrote every tau and gz entry itself ----
  if (g == 0) {
    __syncthreads();
    double* Tm = P;  // bb x bb: the panel slab is free by now
    for (int e = tid; e < bb * bb; e += PT) Tm[e] = 0.0;
    __syncthreads();
    for (int t = 0; t < bb; ++t) {
      const double tt = tau[i + t];
      if (tid < t) {
        double acc = 0.0;
        for (int c = tid; c < t; ++c) acc += Tm[c * bb + tid] * gz[t * bb + c];
        Tm[t * bb + tid] = -tt * acc;
      }
      if (tid == t) Tm[t * bb + t] = tt;
      __syncthreads();
    }
    for (int e = tid; e < bb * bb; e += PT) tmat[e] = Tm[e];
  }
}


// ---------------------------------------------------------------------------
// Register-resident form of the same algorithm (the default).  Thread
// (cc, grp) = (tid % BBM, tid / BBM) holds column cc of the panel for the rows
// rs + grp + NG j, j < RPT, of its workgroup's slab in registers (FP64), so a
// reflector step is: broadcast column t through LDS, RPT fused multiply-adds
// of partial dot products, a reduction over the NG row groups, the grid-wide
// sum, and RPT multiply-adds of update -- all unrolled.  Columns past bb are
// zero padding up to the compile-time width BBM.
// ---------------------------------------------------------------------------
constexpr int RPT = 32;  // panel rows per thread

template <typename T, int BBM>
__global__ __launch_bounds__(PT, 2) void k_panel_r(int m, T* __restrict__ a, long long lda, int i,
                                                    int bb, int bbp,
                                                    const double* __restrict__ wp, long long ldw,
                                                    double* __restrict__ tau,
                                                    double* __restrict__ tmat, GridBarrier* bar,
                                                    unsigned* __restrict__ bsub,
                                                    double* __restrict__ gpart,
                                                    const int* __restrict__ skip) {
  if (skip && *skip) return;  // the panel was already factored by another path
  constexpr int NG = PT / BBM;       // row groups
  constexpr int R = NG * RPT;        // slab rows per workgroup
  constexpr int QC = 4096 / R;       // reflector columns per staging chunk (32 KB)
  __shared__ double s_col[R];        // column t of the step, by local row
  __shared__ double s_v[QC * R];     // previous block's reflectors, [q][local row]
  __shared__ double s_red[NG * BBM];
  __shared__ double s_row[2][BBM];   // pivot row, by step parity
  __shared__ double s_S[2][BBM];     // grid-wide dot products, by step parity
  __shared__ double s_t[MAX_B * MAX_B / 4];  // T of widths <= 64 (wider: in global)
  __shared__ unsigned s_flag;
  __shared__ BarrierLocal bl;

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int cc = tid % BBM, grp = tid / BBM;
  const int rp = i - bbp;
  const int rs = rp + g * R;
  const int ngrp = (G + GRID_GROUP - 1) / GRID_GROUP;  // barrier groups of workgroups
  const int mygrp = g / GRID_GROUP;
  const int gfirst = mygrp * GRID_GROUP, gsize = min(GRID_GROUP, G - gfirst);
  double* growbuf = gpart + 2 * (size_t)G * BBM;  // [2][BBM] pivot rows
  double* gsum = growbuf + 2 * BBM;               // [2][BBM] grid-wide sums
  double* ggrp = gsum + 2 * BBM;                  // [2][64][BBM] group sums
  double* gz = ggrp + 2 * 64 * BBM;               // [bb][bb] columns V^T v_t for T
  grid_sync_init(bar, &bl);

  // ---- load my rows of column cc (zero outside the panel and past m) ----
  double x[RPT];
  {
    const T* col = a + (long long)(i + (cc < bb ? cc : 0)) * lda;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = rs + grp + NG * j;
      const T v = col[r < m ? r : m - 1];
      x[j] = (cc < bb && r < m) ? (double)v : 0.0;
    }
  }

  // ---- pending update of the previous block: x -= V_prev(rows, :) W'(:, cc) ----
  for (int q0 = 0; q0 < bbp; q0 += QC) {
    __syncthreads();
    for (int e = tid; e < QC * R; e += PT) {
      const int q = q0 + e / R, lr = e % R;
      const int r = rs + lr;
      const int d = r - rp;
      double v = 0.0;
      if (q < bbp && r < m)
        v = (d > q) ? (double)a[(long long)(rp + q) * lda + r] : (d == q ? 1.0 : 0.0);
      s_v[(e / R) * R + lr] = v;
    }
    __syncthreads();
    const double* wcol = wp + (long long)(cc < bb ? cc : 0) * ldw;
    for (int qq = 0; qq < QC && q0 + qq < bbp; ++qq) {
      const double w = (cc < bb) ? wcol[q0 + qq] : 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) x[j] -= s_v[qq * R + grp + NG * j] * w;
    }
  }

  for (int t = 0; t < bb; ++t) {
    const int gr = i + t;
    const int lgr = gr - rs;  // local index of the pivot row (may be outside the slab)
    const int par = t & 1;
    double* gp = gpart + (size_t)par * G * BBM;
    double* gg = ggrp + (size_t)par * 64 * BBM;
    // ---- broadcast column t and the pivot row ----
    if (cc == t) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) s_col[grp + NG * j] = x[j];
    }
    if (lgr >= 0 && lgr < R && grp == lgr % NG) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) v = (grp + NG * j == lgr) ? x[j] : v;
      growbuf[par * BBM + cc] = v;
    }
    __syncthreads();
    double xt[RPT];
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      xt[j] = s_col[grp + NG * j];
      d += (grp + NG * j > lgr) ? xt[j] * x[j] : 0.0;
    }
    s_red[grp * BBM + cc] = d;
    __syncthreads();
    if (grp == 0) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < NG; ++q) sum += s_red[q * BBM + cc];
      gp[(size_t)g * BBM + cc] = sum;
    }
    // ---- two-level reduction over the grid (fixed order, so the result does
    // not depend on which workgroups finish last):
    //   the last workgroup of each group of GRID_GROUP adds its group's rows,
    //   the last group adds the group sums, publishes them and releases ----
    __syncthreads();
    if (tid == 0) {
      unsigned* c = bsub + mygrp * GRID_SUB_STRIDE;
      const unsigned a0 = __hip_atomic_fetch_add(c, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      s_flag = (a0 == (unsigned)gsize - 1) ? 1u : 0u;
      if (s_flag) __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    bool released = false;
    if (__builtin_amdgcn_readfirstlane(s_flag)) {
      // group rows gfirst .. gfirst + gsize - 1 (at most GRID_GROUP / NG per thread)
      double sum = 0.0;
      {
        double v[GRID_GROUP / NG > 0 ? GRID_GROUP / NG : 1];
#pragma unroll
        for (int u = 0; u < (GRID_GROUP / NG > 0 ? GRID_GROUP / NG : 1); ++u) {
          const int q = grp + NG * u;
          v[u] = (q < gsize) ? gp[(size_t)(gfirst + q) * BBM + cc] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < (GRID_GROUP / NG > 0 ? GRID_GROUP / NG : 1); ++u) sum += v[u];
      }
      s_red[grp * BBM + cc] = sum;
      __syncthreads();
      if (grp == 0) {
        double tot = 0.0;
#pragma unroll
        for (int q = 0; q < NG; ++q) tot += s_red[q * BBM + cc];
        gg[(size_t)mygrp * BBM + cc] = tot;
      }
      __syncthreads();
      if (tid == 0) {
        const unsigned b0 =
            __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_flag = (b0 == (unsigned)ngrp - 1) ? 1u : 0u;
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(s_flag)) {
        // the group sums, in group order (at most 64 / NG per thread)
        double sum2 = 0.0;
        {
          constexpr int U = (64 + NG - 1) / NG;
          double v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int q = grp + NG * u;
            v[u] = (q < ngrp) ? gg[(size_t)q * BBM + cc] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) sum2 += v[u];
        }
        s_red[grp * BBM + cc] = sum2;
        __syncthreads();
        if (grp == 0) {
          double tot = 0.0;
#pragma unroll
          for (int q = 0; q < NG; ++q) tot += s_red[q * BBM + cc];
          s_S[par][cc] = tot;
          gsum[par * BBM + cc] = tot;
        }
        grid_release(bar, &bl);
        released = true;
      }
    }
    if (!released) {
      grid_wait(bar, &bl);
      if (grp == 0) s_S[par][cc] = gsum[par * BBM + cc];
    }
    if (grp == 0) s_row[par][cc] = growbuf[par * BBM + cc];
    __syncthreads();
    // ---- the reflector (dlarfg) and its update, computed by every thread ----
    const double alpha = s_row[par][t], xn2 = s_S[par][t];
    double beta = alpha, tt = 0.0, den = 1.0;
    if (xn2 > 0.0) {
      const double nrm = hypot(alpha, sqrt(xn2));
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tt = (beta - alpha) / beta;
      den = alpha - beta;
    }
    if (g == 0 && tid == 0) tau[i + t] = tt;
    const double vta = s_row[par][cc] + s_S[par][cc] / den;  // v_t^T a_cc
    if (g == 0 && grp == 0 && cc < bb) gz[t * bb + cc] = (cc < t) ? vta : 0.0;
    // f = tau (v^T a_cc) for cc > t; g = f / (alpha - beta)
    const double fc = (cc > t && cc < bb && tt != 0.0) ? tt * vta : 0.0;
    const double gc = fc / den;
    // column t itself: rows below the pivot become v = x / (alpha - beta)
    const bool ist = cc == t;
    const double sc = (ist && tt != 0.0) ? 1.0 / den : 1.0;
    // selects only: no branches in the unrolled loop
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int lr = grp + NG * j;
      const double v = x[j];
      const double below = ist ? xt[j] * sc : v - xt[j] * gc;
      const double piv = ist ? beta : v - fc;
      x[j] = (lr > lgr) ? below : ((lr == lgr) ? piv : v);
    }
  }

  // ---- write my rows back ----
  if (cc < bb) {
    T* col = a + (long long)(i + cc) * lda;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = rs + grp + NG * j;
      if (r < m) col[r] = (T)x[j];
    }
  }

  // ---- T from the stored (V^T v_t) columns; workgroup 0 wrote every tau and gz ----
  if (g == 0) {
    __syncthreads();
    double* Tm = (bb * bb <= MAX_B * MAX_B / 4) ? s_t : tmat;
    for (int e = tid; e < bb * bb; e += PT) Tm[e] = 0.0;
    __syncthreads();
    for (int t = 0; t < bb; ++t) {
      const double tt = tau[i + t];
      if (tid < t) {
        double acc = 0.0;
        for (int c = tid; c < t; ++c) acc += Tm[c * bb + tid] * gz[t * bb + c];
        Tm[t * bb + tid] = -tt * acc;
      }
      if (tid == t) Tm[t * bb + t] = tt;
      __syncthreads();
    }
    if (Tm == s_t)
      for (int e = tid; e < bb * bb; e += PT) tmat[e] = Tm[e];
  }
}

}  // namespace

static int panel_rows_per_wg(int bb, int bbp) {
  const int budget = 150 * 1024 - VCH * bbp * 8;
  int R = budget / ((bb + 1) * 8);
  R = R / 16 * 16;
  if (R > 256) R = 256;
  return R < 16 ? 16 : R;
}

static int panel_bbm(int bb) { return bb <= 16 ? 16 : bb <= 32 ? 32 : bb <= 64 ? 64 : 128; }

static size_t stepwise_partial_doubles(int rows, int bb) {
  const int R = panel_rows_per_wg(bb, MAX_B);
  const size_t G = (size_t)(rows + R - 1) / R;
  const int bbm = panel_bbm(bb);
  const size_t Rr = (size_t)(PT / bbm) * RPT;
  const size_t Gr = (rows + Rr - 1) / Rr;
  const size_t old_need = 2 * G * bb + 2 * (size_t)bb + (size_t)bb * bb + 64;
  const size_t reg_need = 2 * Gr * bbm + 4 * (size_t)bbm + 2 * 64 * (size_t)bbm +
                          (size_t)bb * bb + 64;
  return old_need > reg_need ? old_need : reg_need;
}

size_t panel_partial_doubles(int rows, int bb) {
  return stepwise_partial_doubles(rows, bb) + panel_cq_doubles(rows) +
         (bb > 64 ? cq_wide_doubles(rows) : 0);
}

int panel_grid(int rows, int bb) {
  const int R = panel_rows_per_wg(bb, MAX_B);
  return (rows + R - 1) / R;
}

template <typename T, int BBM>
static int launch_panel_r(hipStream_t s, int m, T* a, long long lda, int i, int bb, int bbp,
                          const double* wp, long long ldw, double* tau, double* t,
                          PanelScratch* scr, double* partial, bool* launched,
                          const int* skip) {
  *launched = false;
  const int rows = m - (i - bbp);
  constexpr int R = (PT / BBM) * RPT;
  const int G = (rows + R - 1) / R;
  auto kern = &k_panel_r<T, BBM>;
  int dev = 0, ncu = 0, per_cu = 0;
  RQ_HIP_CHECK(hipGetDevice(&dev));
  RQ_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  RQ_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(kern), PT, 0));
  // the grid barrier needs every workgroup resident at once
  if (G > ncu * per_cu) return RQ_OK;
  if (G > 64 * GRID_GROUP) return RQ_OK;
  hipLaunchKernelGGL(kern, dim3(G), dim3(PT), 0, s, m, a, lda, i, bb, bbp, wp, ldw, tau, t,
                     &scr->bar, scr->sub, partial, skip);
  RQ_HIP_CHECK(hipGetLastError());
  *launched = true;
  return RQ_OK;
}

template <typename T>
static int launch_stepwise(hipStream_t s, int m, T* a, long long lda, int i, int bb, int bbp,
                           const double* wp, long long ldw, double* tau, double* t,
                           PanelScratch* scr, double* partial, const int* skip) {
  {
    bool done = false;
    int rc = RQ_OK;
    switch (panel_bbm(bb)) {
      case 16: rc = launch_panel_r<T, 16>(s, m, a, lda, i, bb, bbp, wp, ldw, tau, t, scr, partial, &done, skip); break;
      case 32: rc = launch_panel_r<T, 32>(s, m, a, lda, i, bb, bbp, wp, ldw, tau, t, scr, partial, &done, skip); break;
      case 64: rc = launch_panel_r<T, 64>(s, m, a, lda, i, bb, bbp, wp, ldw, tau, t, scr, partial, &done, skip); break;
      default: rc = launch_panel_r<T, 128>(s, m, a, lda, i, bb, bbp, wp, ldw, tau, t, scr, partial, &done, skip); break;
    }
    if (rc || done) return rc;
  }
  // too many rows for one resident grid of the register form: LDS-slab form
  const int rows = m - (i - bbp);
  const int R = panel_rows_per_wg(bb, MAX_B);
  const int G = (rows + R - 1) / R;
  if ((size_t)R * (bb + 1) < (size_t)bb * bb) return RQ_ERR_LIMIT;  // room for T in WG 0
  const size_t shmem = ((size_t)R * (bb + 1) + (size_t)VCH * bbp) * sizeof(double);
  int dev = 0, ncu = 0, per_cu = 0;
  RQ_HIP_CHECK(hipGetDevice(&dev));
  RQ_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_panel<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  RQ_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(&k_panel<T>), PT, shmem));
  // the grid barrier needs every workgroup resident at once
  if (G > ncu * per_cu) return RQ_ERR_LIMIT;
  hipLaunchKernelGGL(k_panel<T>, dim3(G), dim3(PT), shmem, s, m, a, lda, i, bb, bbp, wp, ldw, tau, t,
                     &scr->bar, partial, R, skip);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

template <typename T>
int launch_panel(hipStream_t s, int m, T* a, long long lda, int i, int bb, int bbp,
                 const double* wp, long long ldw, double* tau, double* t, PanelScratch* scr,
                 double* partial, bool stepwise_only) {
  if (bb < 1 || bb > MAX_B || bbp < 0 || bbp > MAX_B) return RQ_ERR_LIMIT;
  if (stepwise_only)
    return launch_stepwise<T>(s, m, a, lda, i, bb, bbp, wp, ldw, tau, t, scr, partial, nullptr);
  // The previous block's pending update of columns i+coff .. i+coff+nc,
  // A -= V_prev W', in rank-64 pieces: piece q0 is V_prev(:, q0:q0+qb), unit
  // lower from row rp + q0, against rows q0.. of W'.
  auto pend_all = [&](int coff, int nc) -> int {
    const int rp = i - bbp;
    for (int q0 = 0; q0 < bbp; q0 += 64) {
      const int qb = bbp - q0 < 64 ? bbp - q0 : 64;
      const int ie = rp + q0 + qb;      // the kernel's "panel start" for this piece
      const int ce = i + coff - ie;     // target columns i + coff + c
      const double* we = wp + q0 + (long long)(ie - i) * ldw;   // we[(ce + c) ldw + q] = W'(q0 + q, coff + c)
      const int rc = launch_cq_pend<T>(s, m, a, lda, ie, ce, nc, qb, we, ldw);
      if (rc) return rc;
    }
    return RQ_OK;
  };
  if (bb > 64 && panel_cq_applicable(m, i, 64) && panel_cq_applicable(m, i + 64, bb - 64)) {
    // Two 64-wide halves by Cholesky-QR2 (each with the stepwise kernel as its
    // fallback): factor the first, apply its reflectors to the second
    // (X2 -= V1 T1^T V1^T X2), factor the second, and join the T factors,
    // T = [[T1, -T1 (V1^T V2) T2], [0, T2]], for Q = Q1 Q2.
    const int b2 = bb - 64;
    double* cqs = partial + stepwise_partial_doubles(m - (i - bbp), bb);
    double* wide = cqs + panel_cq_doubles(m - i);
    double* part = wide;
    double* t1 = part + cq_wide_doubles(m - i) - 5 * 64 * 64;
    double* t2 = t1 + 64 * 64;
    double* y = t2 + 64 * 64;
    double* wq = y + 64 * 64;
    double* z = wq + 64 * 64;
    int rc;
    if (bbp > 0) {
      if ((rc = pend_all(0, 64))) return rc;
      if ((rc = pend_all(64, b2))) return rc;
    }
    // first half
    if ((rc = launch_panel_cq<T>(s, m, a, lda, i, 64, 0, nullptr, 0, tau, t1, cqs, scr->cq_flag)))
      return rc;
    if ((rc = launch_stepwise<T>(s, m, a, lda, i, 64, 0, nullptr, 0, tau, t1, scr, partial,
                                 scr->cq_flag)))
      return rc;
    // X2 -= V1 (T1^T (V1^T X2)) over rows i .. m-1
    const T* v1 = a + (long long)i * lda + i;
    const T* x2 = a + (long long)(i + 64) * lda + i;
    if ((rc = launch_cq_cross<T>(s, m - i, v1, lda, 64, 0, x2, lda, b2, -1, part, y))) return rc;
    if ((rc = launch_cq_tty(s, b2, t1, y, wq))) return rc;
    if ((rc = launch_cq_pend<T>(s, m, a, lda, i + 64, 0, b2, 64, wq, 64))) return rc;
    // second half
    if ((rc = launch_panel_cq<T>(s, m, a, lda, i + 64, b2, 0, nullptr, 0, tau, t2, cqs,
                                 scr->cq_flag)))
      return rc;
    if ((rc = launch_stepwise<T>(s, m, a, lda, i + 64, b2, 0, nullptr, 0, tau, t2, scr, partial,
                                 scr->cq_flag)))
      return rc;
    // Z = V1^T V2 over rows i+64 .. m-1, then T
    const T* v1b = a + (long long)i * lda + i + 64;
    const T* v2 = a + (long long)(i + 64) * lda + i + 64;
    if ((rc = launch_cq_cross<T>(s, m - i - 64, v1b, lda, 64, -1, v2, lda, b2, 0, part, z)))
      return rc;
    return launch_cq_tcombine(s, b2, t1, t2, z, t);
  }
  if (panel_cq_applicable(m, i, bb)) {
    // Cholesky-QR2 panel; the stepwise kernel runs only if that path declined
    double* cqs = partial + stepwise_partial_doubles(m - (i - bbp), bb);
    int rc;
    if (bbp > 0 && (rc = pend_all(0, bb))) return rc;
    rc = launch_panel_cq<T>(s, m, a, lda, i, bb, 0, nullptr, 0, tau, t, cqs, scr->cq_flag);
    if (rc) return rc;
    return launch_stepwise<T>(s, m, a, lda, i, bb, 0, nullptr, 0, tau, t, scr, partial,
                              scr->cq_flag);
  }
  return launch_stepwise<T>(s, m, a, lda, i, bb, bbp, wp, ldw, tau, t, scr, partial, nullptr);
}
template int launch_panel<double>(hipStream_t, int, double*, long long, int, int, int,
                                  const double*, long long, double*, double*, PanelScratch*,
                                  double*, bool);
template int launch_panel<float>(hipStream_t, int, float*, long long, int, int, int,
                                 const double*, long long, double*, double*, PanelScratch*,
                                 double*, bool);

}  // namespace rq
