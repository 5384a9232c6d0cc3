// Partial QRCP on the sketch (Alg. 1 applied to B(:, i:n) inside Alg. 2).
//
// One persistent, co-resident grid.  Every thread owns one sketch column (or
// one half of it, TPC = 2) in registers for the whole call, so the only
// global traffic per pivot step is one small candidate record per workgroup
// and one read of the winning column: each step is
//   local argmax of the trailing norms -> publish candidate -> grid barrier
//   -> global argmax (ties: lowest position) -> Householder vector (LAPACK
//   dlarfg convention) -> apply it to every active column -> exact new norms.
// The norms are recomputed from the column each step (the definition of r_s
// in Alg. 1), not downdated, so there is no cancellation to guard against.
// Columns never move during the call; positions are tracked logically and
// the columns are written back to their final positions at the end, with
// the list of moved columns for the matching moves in A.
#include <limits.h>

#include "internal.h"

namespace rq {
namespace {

RQ_DEV bool better(double n1, int p1, double n2, int p2) {
  return n1 > n2 || (n1 == n2 && p1 < p2);
}

RQ_DEV void wave_best(double& n, int& p, int& s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double n2 = __shfl_xor(n, off, 64);
    const int p2 = __shfl_xor(p, off, 64);
    const int s2 = __shfl_xor(s, off, 64);
    if (better(n2, p2, n, p)) {
      n = n2;
      p = p2;
      s = s2;
    }
  }
}

template <int TPC>
RQ_DEV double tpc_sum(double v) {
  if constexpr (TPC == 2) v += __shfl_xor(v, 1, 64);
  return v;
}

// QT threads per workgroup; every workgroup holds CPW = QT / TPC = 256 columns.
template <int RPT, int TPC, int QT>
__global__ __launch_bounds__(QT, 1) void k_qrcp_sketch(
    double* __restrict__ bsk, long long ldb, int l, int nc, int nsteps, int gstep0,
    GridBarrier* bar, double* __restrict__ cand, int cs, int* __restrict__ pairs,
    int* __restrict__ npairs, int* __restrict__ info) {
  constexpr int CPW = QT / TPC;
  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int sub = tid % TPC;
  const int slot = g * CPW + tid / TPC;
  const bool valid = slot < nc;
  bool active = valid;
  int my_pos = slot;

  __shared__ double s_col[RPT * TPC];
  __shared__ double s_v[RPT * TPC];
  __shared__ int s_p2s[MAX_B];
  __shared__ double s_wn[QT / 64];
  __shared__ int s_wp[QT / 64];
  __shared__ int s_ws[QT / 64];
  __shared__ double s_bn;
  __shared__ int s_bp, s_bs;
  __shared__ double s_beta, s_tau, s_den;
  __shared__ int s_wslot, s_qslot, s_jpos;
  __shared__ double s_gn;
  __shared__ BarrierLocal bl;

  // A zero sketch pivot in an earlier block: no more pivoting (identity).
  if (*info != 0) {
    if (g == 0 && tid == 0) *npairs = 0;
    return;
  }

  double x[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = j * TPC + sub;
    x[j] = (valid && r < l) ? bsk[(long long)slot * ldb + r] : 0.0;
  }
  if (tid < nsteps) s_p2s[tid] = tid;
  if (g == 0 && tid == 0) *npairs = 0;

  double nrm2 = 0.0;
#pragma unroll
  for (int j = 0; j < RPT; ++j) nrm2 += x[j] * x[j];
  nrm2 = tpc_sum<TPC>(nrm2);

  for (int t = 0; t < nsteps; ++t) {
    // ---- (a) best trailing column of this workgroup ----
    double bn = (active && sub == 0) ? nrm2 : -1.0;
    int bp = (active && sub == 0) ? my_pos : INT_MAX;
    int bs = slot;
    wave_best(bn, bp, bs);
    if ((tid & 63) == 0) {
      s_wn[tid >> 6] = bn;
      s_wp[tid >> 6] = bp;
      s_ws[tid >> 6] = bs;
    }
    __syncthreads();
    if (tid == 0) {
      double n = s_wn[0];
      int p = s_wp[0], s = s_ws[0];
      for (int w = 1; w < QT / 64; ++w)
        if (better(s_wn[w], s_wp[w], n, p)) {
          n = s_wn[w];
          p = s_wp[w];
          s = s_ws[w];
        }
      s_bn = n;
      s_bp = p;
      s_bs = s;
    }
    __syncthreads();

    // ---- (b) publish the candidate record ----
    double* rec = cand + ((long long)(t & 1) * G + g) * cs;
    if (tid == 0) {
      rec[0] = s_bn;
      rec[1] = (double)s_bp;
      rec[2] = (double)s_bs;
    }
    if (valid && active && slot == s_bs) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = j * TPC + sub;
        if (r < l) rec[4 + r] = x[j];
      }
    }

    // ---- (c) all candidates are published ----
    grid_barrier(bar, G, &bl);

    // ---- (d) global winner ----
    {
      double wn = -2.0;
      int wp = INT_MAX, ww = 0;
      for (int q = tid; q < G; q += QT) {
        const double* r = cand + ((long long)(t & 1) * G + q) * cs;
        const double n = r[0];
        const int p = (n >= 0.0) ? (int)r[1] : INT_MAX;
        if (better(n, p, wn, wp)) {
          wn = n;
          wp = p;
          ww = q;
        }
      }
      wave_best(wn, wp, ww);
      if ((tid & 63) == 0) {
        s_wn[tid >> 6] = wn;
        s_wp[tid >> 6] = wp;
        s_ws[tid >> 6] = ww;
      }
      __syncthreads();
      if (tid == 0) {
        double n = s_wn[0];
        int p = s_wp[0], w = s_ws[0];
        for (int k = 1; k < QT / 64; ++k)
          if (better(s_wn[k], s_wp[k], n, p)) {
            n = s_wn[k];
            p = s_wp[k];
            w = s_ws[k];
          }
        s_gn = n;
        s_jpos = p;
        s_wslot = (int)cand[((long long)(t & 1) * G + w) * cs + 2];
        s_ws[0] = w;
      }
      __syncthreads();
    }
    const int wwg = s_ws[0];
    const double* wrec = cand + ((long long)(t & 1) * G + wwg) * cs;
    for (int r = tid; r < l; r += QT) s_col[r] = (r >= t) ? wrec[4 + r] : 0.0;
    __syncthreads();

    // ---- (e) Householder reflector of the winning column (dlarfg) ----
    if (tid < 64) {
      double acc = 0.0;
      for (int r = t + 1 + tid; r < l; r += 64) acc += s_col[r] * s_col[r];
      acc = wave_sum(acc);
      if (tid == 0) {
        const double alpha = s_col[t];
        double beta = alpha, tau = 0.0, den = 1.0;
        if (acc > 0.0) {
          const double nrm = hypot(alpha, sqrt(acc));
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          den = alpha - beta;
        }
        s_beta = beta;
        s_tau = tau;
        s_den = den;
        const int q = s_p2s[t];
        s_qslot = q;
        s_p2s[t] = s_wslot;
        if (s_jpos < nsteps && s_jpos != t) s_p2s[s_jpos] = q;
        if (g == 0 && s_gn == 0.0 && *info == 0) *info = gstep0 + t + 1;
      }
    }
    __syncthreads();
    for (int r = tid; r < l; r += QT)
      s_v[r] = (r == t) ? 1.0 : ((r > t && s_tau != 0.0) ? s_col[r] / s_den : 0.0);
    __syncthreads();

    const double beta = s_beta, tau = s_tau;
    const int wsl = s_wslot, qsl = s_qslot, jpos = s_jpos;

    // ---- (f) bookkeeping of positions ----
    if (valid) {
      if (slot == wsl) {
        my_pos = t;
        active = false;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int r = j * TPC + sub;
          if (r == t) x[j] = beta;
          else if (r > t) x[j] = 0.0;
        }
      } else if (slot == qsl) {
        my_pos = jpos;
      }
    }

    // ---- (g) apply H to the active columns, new trailing norms ----
    if (active) {
      if (tau != 0.0) {
        double d = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int r = j * TPC + sub;
          if (r >= t && r < l) d += s_v[r] * x[j];
        }
        d = tpc_sum<TPC>(d);
        const double f = tau * d;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int r = j * TPC + sub;
          if (r >= t && r < l) x[j] -= f * s_v[r];
        }
      }
      double nn = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = j * TPC + sub;
        if (r > t && r < l) nn += x[j] * x[j];
      }
      nrm2 = tpc_sum<TPC>(nn);
    }
  }

  // ---- write the block back in pivot order; list the moved columns ----
  if (valid) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = j * TPC + sub;
      if (r < l) bsk[(long long)my_pos * ldb + r] = x[j];
    }
    if (sub == 0 && my_pos != slot) {
      const int e = atomicAdd(npairs, 1);
      pairs[2 * e] = my_pos;
      pairs[2 * e + 1] = slot;
    }
  }
}

template <int RPT, int TPC>
int launch_t(hipStream_t s, double* b, long long ldb, int l, int nc, int nsteps, int gstep0,
             QrcpScratch* scr, double* cand, int* pairs, int* info) {
  constexpr int QT = 256 * TPC;
  constexpr int CPW = QT / TPC;
  auto kern = &k_qrcp_sketch<RPT, TPC, QT>;
  const int G = (nc + CPW - 1) / CPW;
  const int cs = ((l + 4) + 7) / 8 * 8;
  int dev = 0, ncu = 0, per_cu = 0;
  RQ_HIP_CHECK(hipGetDevice(&dev));
  RQ_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  RQ_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(kern), QT, 0));
  // the grid barrier needs every workgroup resident at once
  if (G > ncu * per_cu) return RQ_ERR_LIMIT;
  hipLaunchKernelGGL(kern, dim3(G), dim3(QT), 0, s, b, ldb, l, nc, nsteps, gstep0, &scr->bar, cand,
                     cs, pairs, &scr->npairs, info);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace

size_t qrcp_cand_doubles(int l, int nc) {
  const int cpw = 256;
  const size_t G = (size_t)(nc + cpw - 1) / cpw;
  const size_t cs = ((l + 4) + 7) / 8 * 8;
  return 2 * G * cs;
}

int qrcp_sketch_grid(int l, int nc) {
  const int cpw = 256;
  return (nc + cpw - 1) / cpw;
}

int launch_qrcp_sketch(hipStream_t s, double* b, long long ldb, int l, int c0, int nc, int nsteps,
                       int gstep0, QrcpScratch* scr, double* cand, int* pairs, int* info) {
  if (nsteps < 1 || nsteps > MAX_B || l > MAX_L || nsteps > l) return RQ_ERR_LIMIT;
  double* bb = b + (long long)c0 * ldb;
  if (l <= 16) return launch_t<16, 1>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  if (l <= 32) return launch_t<32, 1>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  if (l <= 48) return launch_t<48, 1>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  if (l <= 80) return launch_t<40, 2>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  return launch_t<80, 2>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
}

}  // namespace rq
