// Partial QRCP on the sketch (Alg. 1 applied to B(:, i:n) inside Alg. 2).
//
// One persistent, co-resident grid.  Every column of the sketch block lives
// in registers of TPC threads for the whole call, so the only global traffic
// per pivot step is one candidate record per workgroup:
//   1. each workgroup finds its best trailing column (largest norm, ties to
//      the lowest position) and publishes a record {norm^2, position, slot,
//      sequence number, column};
//   2. every workgroup waits until all records carry this step's sequence
//      number (the global pivot step + 1), which doubles as the grid barrier;
//   3. every workgroup reads the G record headers, picks the same global
//      winner, reads the winner's column and forms the same Householder
//      reflector (LAPACK dlarfg convention) from it;
//   4. every workgroup applies it to its own active columns and recomputes
//      their trailing norms exactly (the definition of r_s in Alg. 1; no
//      downdating, so no cancellation to guard against).
// Columns never move during the call; positions are tracked logically and
// the block is written back in pivot order at the end, together with the
// list of moved columns for the matching column moves in A.
#include <limits.h>

#include "internal.h"

namespace rq {
namespace {

template <int TPC>
RQ_DEV double tpc_sum(double v) {
  if constexpr (TPC == 2) v = pair_sum_dpp(v);
  if constexpr (TPC == 4) v = quad_sum_dpp(v);
  return v;
}

// QT threads per workgroup; every workgroup holds CPW = QT / TPC columns (256,
// or 128 for the tallest sketches), each column split over TPC threads (rows
// sub, sub + TPC, ...).
template <int RPT, int TPC, int QT>
__global__ __launch_bounds__(QT, 1) void k_qrcp_sketch(
    double* __restrict__ bsk, long long ldb, int l, int nc, int nsteps, int gstep0,
    GridBarrier* bar, double* __restrict__ cand, int cs, int* __restrict__ pairs,
    int* __restrict__ npairs, int* __restrict__ info) {
  constexpr int CPW = QT / TPC;
  constexpr int NW = QT / 64;
  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int sub = tid % TPC;
  const int slot = g * CPW + tid / TPC;
  const bool valid = slot < nc;
  bool active = valid;
  int my_pos = slot;

  __shared__ int s_p2s[MAX_B];
  __shared__ double s_v[MAX_L];  // scaled Householder vector of the step
  __shared__ double s_wn[NW];
  __shared__ int s_wp[NW];
  __shared__ int s_ws[NW];
  // the winner's column of the step
  extern __shared__ double s_rec[];

  // A zero sketch pivot in an earlier block: no more pivoting (identity).
  if (*info != 0) {
    if (g == 0 && tid == 0) *npairs = 0;
    return;
  }

  double x[RPT];
  {
    const double* col = bsk + (long long)(valid ? slot : 0) * ldb;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = j * TPC + sub;
      const double v = col[r < l ? r : 0];
      x[j] = (valid && r < l) ? v : 0.0;
    }
  }
  if (tid < nsteps) s_p2s[tid] = tid;
  if (tid == 0) s_v[MAX_L - 1] = 0.0;
  if (g == 0 && tid == 0) *npairs = 0;

  double nrm2 = 0.0;
#pragma unroll
  for (int j = 0; j < RPT; ++j) nrm2 += x[j] * x[j];
  nrm2 = tpc_sum<TPC>(nrm2);

  for (int t = 0; t < nsteps; ++t) {
    // ---- (1) best trailing column of this workgroup ----
    {
      double bn = (active && sub == 0) ? nrm2 : -1.0;
      int bp = (active && sub == 0) ? my_pos : INT_MAX;
      int bs = slot;
      wave_argmax(bn, bp, bs);
      if (lane == 0) {
        s_wn[wave] = bn;
        s_wp[wave] = bp;
        s_ws[wave] = bs;
      }
    }
    __syncthreads();
    // slot now at position t (thread 0 last wrote s_p2s before this sync)
    const int q_at_t = s_p2s[t];
    double bn = s_wn[0];
    int bp = s_wp[0], bs = s_ws[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (argbetter(s_wn[w], s_wp[w], bn, bp)) {
        bn = s_wn[w];
        bp = s_wp[w];
        bs = s_ws[w];
      }

    // ---- publish the candidate record ----
    double* rec = cand + ((long long)(t & 1) * G + g) * cs;
    const unsigned seq = (unsigned)(gstep0 + t + 1);
    if (tid == 0) {
      rec[0] = bn;
      rec[1] = (double)bp;
      rec[2] = (double)bs;
    }
    if (active && slot == bs) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = j * TPC + sub;
        if (r < l) rec[4 + r] = x[j];
      }
    }
    __syncthreads();
    if (tid == 0) publish_seq(reinterpret_cast<unsigned*>(rec + 3), seq);

    // ---- (2) wait until every workgroup has published this step ----
    wait_all_seq(reinterpret_cast<const unsigned*>(cand + (long long)(t & 1) * G * cs + 3),
                 2LL * cs, G, seq, bar);

    // ---- (3) global winner and its reflector, computed by every workgroup ----
    // every wave reads the headers itself (lane q: records q, q + 64, ...)
    // and reduces with DPP; then the winner's column (rows 0..l-1) into LDS
    const double* recs = cand + (long long)(t & 1) * G * cs;
    double gn = -2.0;
    int jpos = INT_MAX;
    int ww = 0;
    for (int q = lane; q < G; q += 64) {
      const double n = recs[(long long)q * cs];
      const double pd = recs[(long long)q * cs + 1];
      const int p = (n >= 0.0) ? (int)pd : INT_MAX;
      if (argbetter(n, p, gn, jpos)) {
        gn = n;
        jpos = p;
        ww = q;
      }
    }
    wave_argmax(gn, jpos, ww);
    int wslot = (int)recs[(long long)ww * cs + 2];
    double* wcol = s_rec;
    for (int r = tid; r < l; r += QT) wcol[r] = recs[(long long)ww * cs + 4 + r];
    __syncthreads();
    // A winner that is not a column of this block (no candidate norm is a
    // finite nonnegative number, e.g. a NaN in the sketch) must not steer the
    // bookkeeping or the write-back: flag it and keep the column already at
    // position t (no move); the factorization is then reported unusable.
    if (!(gn >= 0.0) || jpos < 0 || jpos >= nc || wslot < 0 || wslot >= nc) {
      if (g == 0 && tid == 0) atomicOr(&bar->err, 2u);
      jpos = t;
      wslot = q_at_t;
    }
    // dlarfg on the winner's rows t..l-1 (every wave, same order, same result)
    double xn2 = 0.0;
    for (int r = t + 1 + lane; r < l; r += 64) xn2 += wcol[r] * wcol[r];
    xn2 = wave_sum_dpp(xn2);
    const double alpha = wcol[t];
    double beta = alpha, tau = 0.0, den = 1.0;
    if (xn2 > 0.0) {
      const double nrm = hypot(alpha, sqrt(xn2));
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      den = alpha - beta;
    }
    if (g == 0 && tid == 0 && gn == 0.0 && *info == 0) *info = gstep0 + t + 1;
    // v_t = 1, v_r = wcol[r] / (alpha - beta) for r > t, zero above t
    {
      const double inv = 1.0 / den;
      for (int r = tid; r < l; r += QT)
        s_v[r] = (r == t) ? 1.0 : ((r > t && tau != 0.0) ? wcol[r] * inv : 0.0);
    }
    __syncthreads();

    // ---- position bookkeeping (identical in every workgroup) ----
    if (tid == 0) {
      s_p2s[t] = wslot;
      if (jpos < nsteps && jpos != t) s_p2s[jpos] = q_at_t;
    }
    if (valid) {
      if (slot == wslot) {
        my_pos = t;
        active = false;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int r = j * TPC + sub;
          x[j] = (r == t) ? beta : ((r > t) ? 0.0 : x[j]);
        }
      } else if (slot == q_at_t) {
        my_pos = jpos;
      }
    }

    // ---- (4) apply H = I - tau v v^T to the active columns, new norms ----
    // (branch-free: finished columns take f = 0 and their norms are unused)
    {
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = j * TPC + sub;
        d += s_v[r < l ? r : MAX_L - 1] * x[j];  // rows past l hold x = 0
      }
      d = tpc_sum<TPC>(d);
      const double f = active ? tau * d : 0.0;
      double nn = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = j * TPC + sub;
        x[j] -= f * s_v[r < l ? r : MAX_L - 1];
        nn += (r > t) ? x[j] * x[j] : 0.0;
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
  constexpr int QT = TPC == 4 ? 512 : 256 * TPC;   // at most 512 threads: room for x[RPT]
  constexpr int CPW = QT / TPC;
  auto kern = &k_qrcp_sketch<RPT, TPC, QT>;
  const int G = (nc + CPW - 1) / CPW;
  const int cs = ((l + 4) + 7) / 8 * 8;
  int dev = 0, ncu = 0, per_cu = 0;
  RQ_HIP_CHECK(hipGetDevice(&dev));
  RQ_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  // LDS: the winner's column.  (Reading every record, columns included, in
  // one round trip measured 11% slower than two short round trips, headers
  // then the winner's column, at every width from 4 to 128 workgroups.)
  const size_t shmem = (size_t)cs * sizeof(double);
  RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  RQ_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(kern), QT, shmem));
  // the exchange waits on every workgroup: all must be resident at once
  if (G > ncu * per_cu) return RQ_ERR_LIMIT;
  hipLaunchKernelGGL(kern, dim3(G), dim3(QT), shmem, s, b, ldb, l, nc, nsteps, gstep0, &scr->bar,
                     cand, cs, pairs, &scr->npairs, info);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace

size_t qrcp_cand_doubles(int l, int nc) {
  const size_t cpw = l > 80 ? 128 : 256;
  const size_t G = ((size_t)nc + cpw - 1) / cpw;
  const size_t cs = ((l + 4) + 7) / 8 * 8;
  return 2 * G * cs;
}

int qrcp_sketch_grid(int l, int nc) {
  const int cpw = l > 80 ? 128 : 256;
  return (nc + cpw - 1) / cpw;
}

int launch_qrcp_sketch(hipStream_t s, double* b, long long ldb, int l, int c0, int nc, int nsteps,
                       int gstep0, QrcpScratch* scr, double* cand, int* pairs, int* info) {
  if (nsteps < 1 || nsteps > MAX_B || l > MAX_L || nsteps > l) return RQ_ERR_LIMIT;
  double* bb = b + (long long)c0 * ldb;
  if (l <= 16) return launch_t<16, 1>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  if (l <= 32) return launch_t<32, 1>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  if (l <= 48) return launch_t<48, 1>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  if (l <= 72) return launch_t<36, 2>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  if (l <= 80) return launch_t<40, 2>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
  return launch_t<40, 4>(s, bb, ldb, l, nc, nsteps, gstep0, scr, cand, pairs, info);
}

}  // namespace rq
