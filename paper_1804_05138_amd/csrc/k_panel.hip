// Householder QR of the pivoted panel (Alg. 2 "unpivoted QR on
// A(i:m, i:i+b-1)"; PDGEQRF in Alg. 4) and its compact-WY factor T (PDLARFT).
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
                                                 int R) {
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

}  // namespace

static int panel_rows_per_wg(int bb, int bbp) {
  const int budget = 150 * 1024 - VCH * bbp * 8;
  int R = budget / ((bb + 1) * 8);
  R = R / 16 * 16;
  if (R > 256) R = 256;
  return R < 16 ? 16 : R;
}

size_t panel_partial_doubles(int rows, int bb) {
  const int R = panel_rows_per_wg(bb, MAX_B);
  const size_t G = (size_t)(rows + R - 1) / R;
  return 2 * G * bb + 2 * (size_t)bb + (size_t)bb * bb + 64;
}

int panel_grid(int rows, int bb) {
  const int R = panel_rows_per_wg(bb, MAX_B);
  return (rows + R - 1) / R;
}

template <typename T>
int launch_panel(hipStream_t s, int m, T* a, long long lda, int i, int bb, int bbp,
                 const double* wp, long long ldw, double* tau, double* t, PanelScratch* scr,
                 double* partial) {
  if (bb < 1 || bb > MAX_B || bbp < 0 || bbp > MAX_B) return RQ_ERR_LIMIT;
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
                     &scr->bar, partial, R);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_panel<double>(hipStream_t, int, double*, long long, int, int, int,
                                  const double*, long long, double*, double*, PanelScratch*,
                                  double*);
template int launch_panel<float>(hipStream_t, int, float*, long long, int, int, int,
                                 const double*, long long, double*, double*, PanelScratch*,
                                 double*);

}  // namespace rq
