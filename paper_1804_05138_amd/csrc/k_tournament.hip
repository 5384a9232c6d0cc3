// QR with tournament pivoting on the sketch, in place of the partial QRCP of
// B(:, c0:n) (the first improvement Section V-C proposes for the distributed
// method; Demmel, Grigori, Gu and Xiang, "Communication avoiding rank
// revealing QR factorization with column pivoting", 2015).
//
// The b pivots of a block are chosen by a reduction tree instead of b
// grid-wide argmaxes: every workgroup runs b steps of Alg. 1 on its own group
// of 256 sketch columns (norms recomputed, ties to the lowest position), and
// the nominated columns are merged four sets at a time, each merged set again
// reduced to b columns by Alg. 1 on the original sketch columns, until one set
// is left.  No workgroup ever waits for another inside a launch.  The winners
// are then moved to the front in their final order (LAPACK-style sequential
// transpositions, folded into one permutation), and the sketch block is
// factored with those pivots fixed: Householder QR of its b leading columns,
// the reflectors applied to the rest.  The outputs are those of the partial
// QRCP kernel: B in pivot order and transformed, the moved-column list for A,
// jpvt and W', and info.
#include <limits.h>

#include "internal.h"

namespace rq {
namespace {

constexpr int TQ = 512;        // threads of a selection workgroup
constexpr int TPC = 2;         // threads per column
constexpr int TS = TQ / TPC;   // columns per leaf group
constexpr int TRPT = 40;       // rows per thread (l <= 80)
constexpr int TLMAX = TPC * TRPT;
constexpr int TFAN = 4;        // sets merged by one workgroup above the leaves
constexpr int TMAXB = TS / TFAN;

// One selection subproblem per workgroup.  Level 0: columns g*TS .. of the
// block; level > 0: the concatenation of sets g*TFAN .. g*TFAN + TFAN - 1 of
// the previous level (a chunk holding one set is copied through).
__global__ __launch_bounds__(TQ, 1) void k_tp_select(
    const double* __restrict__ bsk, long long ldb, int l, int nc, int nsteps, int level,
    const int* __restrict__ in_sets, const int* __restrict__ in_cnt, int nsets_in,
    int* __restrict__ out_sets, int* __restrict__ out_cnt, const int* __restrict__ info,
    unsigned* __restrict__ err, double* __restrict__ vref, double* __restrict__ tref,
    double* __restrict__ rhat) {
  // vref != null on the root: the run that picks the final winners also
  // factors them (its reflectors are those of the sketch block's QR with the
  // winners as pivots), so it stores the reflectors (TLMAX rows each, zero
  // outside t..l-1), tau and the factored winner columns (R-hat, TLMAX rows).
  constexpr int NW = TQ / 64;
  __shared__ int s_cand[TS];
  __shared__ int s_ncand;
  __shared__ int s_p2s[TMAXB];
  __shared__ int s_chosen[TMAXB];
  __shared__ double s_w[TLMAX];
  __shared__ double s_v[TLMAX];
  __shared__ double s_wn[NW];
  __shared__ int s_wp[NW];
  __shared__ int s_ws[NW];
  const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sub = tid % TPC, slot = tid / TPC;
  if (*info != 0) {   // an earlier block met a zero sketch pivot: no more pivoting
    if (tid == 0) out_cnt[g] = 0;
    return;
  }
  if (tid == 0) {
    int nc_ = 0;
    if (level == 0) {
      const int c_begin = g * TS;
      nc_ = min(TS, nc - c_begin);
      for (int j = 0; j < nc_; ++j) s_cand[j] = c_begin + j;
    } else {
      const int s0 = g * TFAN, s1 = min(nsets_in, s0 + TFAN);
      for (int st = s0; st < s1; ++st)
        for (int j = 0; j < in_cnt[st]; ++j) s_cand[nc_++] = in_sets[st * TMAXB + j];
      if (s1 - s0 == 1) {   // a lone set passes through unchanged
        for (int j = 0; j < nc_; ++j) out_sets[g * TMAXB + j] = s_cand[j];
        out_cnt[g] = nc_;
        nc_ = -1;
      }
    }
    s_ncand = nc_;
  }
  __syncthreads();
  const int ncand = s_ncand;
  if (ncand < 0) return;
  const bool valid = slot < ncand;
  bool active = valid;
  int my_pos = slot;
  double x[TRPT];
  {
    const double* col = bsk + (long long)(valid ? s_cand[slot] : 0) * ldb;
#pragma unroll
    for (int j = 0; j < TRPT; ++j) {
      const int r = j * TPC + sub;
      const double v = col[r < l ? r : 0];
      x[j] = (valid && r < l) ? v : 0.0;
    }
  }
  if (tid < nsteps) s_p2s[tid] = tid;
  double nrm2 = 0.0;
#pragma unroll
  for (int j = 0; j < TRPT; ++j) nrm2 += x[j] * x[j];
  nrm2 = pair_sum_dpp(nrm2);
  const int steps = min(nsteps, ncand);
  int nchosen = 0;
  for (int t = 0; t < steps; ++t) {
    double bn = (active && sub == 0) ? nrm2 : -1.0;
    int bp = (active && sub == 0) ? my_pos : INT_MAX;
    int bs = slot;
    wave_argmax(bn, bp, bs);
    if (lane == 0) {
      s_wn[wave] = bn;
      s_wp[wave] = bp;
      s_ws[wave] = bs;
    }
    __syncthreads();
    const int q_at_t = s_p2s[t];
    bn = s_wn[0];
    bp = s_wp[0];
    bs = s_ws[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (argbetter(s_wn[w], s_wp[w], bn, bp)) {
        bn = s_wn[w];
        bp = s_wp[w];
        bs = s_ws[w];
      }
    // every remaining column exactly zero, or no finite norm: stop here
    if (!(bn > 0.0) || bs < 0 || bs >= ncand) {
      if (!(bn >= 0.0) && tid == 0) atomicOr(err, 2u);
      break;
    }
    if (active && slot == bs) {
#pragma unroll
      for (int j = 0; j < TRPT; ++j) {
        const int r = j * TPC + sub;
        if (r < l) s_w[r] = x[j];
      }
    }
    __syncthreads();
    double xn2 = 0.0;
    for (int r = t + 1 + lane; r < l; r += 64) xn2 += s_w[r] * s_w[r];
    xn2 = wave_sum_dpp(xn2);
    const double alpha = s_w[t];
    double tau = 0.0, den = 1.0, beta = alpha;
    if (xn2 > 0.0) {
      const double nrm = hypot(alpha, sqrt(xn2));
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      den = alpha - beta;
    }
    {
      const double inv = 1.0 / den;
      for (int r = tid; r < TLMAX; r += TQ)
        s_v[r] = (r == t) ? 1.0 : ((r > t && r < l && tau != 0.0) ? s_w[r] * inv : 0.0);
    }
    if (tid == 0) {
      s_chosen[t] = s_cand[bs];
      s_p2s[t] = bs;
      if (bp < nsteps && bp != t) s_p2s[bp] = q_at_t;
    }
    __syncthreads();
    if (vref != nullptr) {
      for (int r = tid; r < TLMAX; r += TQ) vref[(long long)t * TLMAX + r] = s_v[r];
      if (tid == 0) tref[t] = tau;
      if (valid && slot == bs) {
#pragma unroll
        for (int j = 0; j < TRPT; ++j) {
          const int r = j * TPC + sub;
          rhat[(long long)t * TLMAX + r] = (r < t) ? x[j] : ((r == t) ? beta : 0.0);
        }
      }
    }
    if (valid) {
      if (slot == bs) {
        active = false;
        my_pos = t;
      } else if (slot == q_at_t) {
        my_pos = bp;
      }
    }
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < TRPT; ++j) d += s_v[j * TPC + sub] * x[j];
    d = pair_sum_dpp(d);
    const double f = active ? tau * d : 0.0;
    double nn = 0.0;
#pragma unroll
    for (int j = 0; j < TRPT; ++j) {
      const int r = j * TPC + sub;
      x[j] -= f * s_v[r];
      nn += (r > t) ? x[j] * x[j] : 0.0;
    }
    nrm2 = pair_sum_dpp(nn);
    nchosen = t + 1;
  }
  __syncthreads();
  for (int j = tid; j < nchosen; j += TQ) out_sets[g * TMAXB + j] = s_chosen[j];
  if (tid == 0) out_cnt[g] = nchosen;
}

// The root set -> the column moves (dest, src) of the sequential transpositions
// that bring winners[0], winners[1], ... to positions 0, 1, ...; the number of
// steps the block factorization takes; info for a rank stop.  One wave: the
// touched positions (the c front positions and the winners' own positions
// beyond them) are entries in LDS, and step t finds the entry holding winner t
// with one ballot over the wave.
__global__ __launch_bounds__(64) void k_tp_finish(int nsteps, int gstep0,
                                                  const int* __restrict__ root,
                                                  const int* __restrict__ root_cnt,
                                                  int* __restrict__ pairs, int* __restrict__ npairs,
                                                  int* __restrict__ tp_count,
                                                  int* __restrict__ info) {
  __shared__ int key[2 * TMAXB], val[2 * TMAXB];
  __shared__ int s_nk;
  const int lane = threadIdx.x;
  if (*info != 0) {
    if (lane == 0) {
      *npairs = 0;
      *tp_count = 0;
    }
    return;
  }
  const int c = *root_cnt;
  if (lane == 0) {
    int nk = c;
    for (int e = 0; e < c; ++e) key[e] = val[e] = e;
    for (int t = 0; t < c; ++t) {
      const int w = root[t];
      if (w >= c) {
        key[nk] = val[nk] = w;
        ++nk;
      }
    }
    s_nk = nk;
  }
  __syncthreads();
  const int nk = s_nk;
  for (int t = 0; t < c; ++t) {
    const int w = root[t];
    // the entry holding column w (exactly one)
    int hit = -1;
    for (int e = lane; e < nk; e += 64)
      if (val[e] == w) hit = e;
    const unsigned long long bal = __ballot(hit >= 0);
    const int src_lane = bal ? (int)__builtin_ctzll(bal) : 0;
    const int ep = __shfl(hit, src_lane, 64);
    if (lane == 0 && ep != t && ep >= 0) {
      const int ct = val[t];
      val[t] = w;
      val[ep] = ct;
    }
    __syncthreads();
  }
  // the moves: every touched position whose final column differs
  if (lane == 0) {
    int np = 0;
    for (int e = 0; e < nk; ++e)
      if (val[e] != key[e]) {
        pairs[2 * np] = key[e];
        pairs[2 * np + 1] = val[e];
        ++np;
      }
    *npairs = np;
    *tp_count = c;
    if (c < nsteps) *info = gstep0 + c + 1;
  }
}

// The block's reflectors applied to the sketch columns count .. nc-1 (one
// thread per column, the column in registers); the winners' columns
// 0 .. count-1 take the factored columns R-hat.
__global__ __launch_bounds__(256) void k_tp_apply(double* __restrict__ bsk, long long ldb, int l,
                                                  int nc, const int* __restrict__ tp_count,
                                                  const double* __restrict__ vref,
                                                  const double* __restrict__ tref,
                                                  const double* __restrict__ rhat) {
  __shared__ double s_v[TLMAX * TMAXB];
  __shared__ double s_t[TMAXB];
  const int cnt = *tp_count;
  if (cnt == 0) return;
  for (int e = threadIdx.x; e < TLMAX * cnt; e += 256) s_v[e] = vref[e];
  for (int e = threadIdx.x; e < cnt; e += 256) s_t[e] = tref[e];
  __syncthreads();
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  double* col = bsk + (long long)c * ldb;
  if (c < cnt) {
    for (int r = 0; r < l; ++r) col[r] = rhat[(long long)c * TLMAX + r];
    return;
  }
  double x[TLMAX];
#pragma unroll
  for (int r = 0; r < TLMAX; ++r) x[r] = (r < l) ? col[r < l ? r : 0] : 0.0;
  for (int t = 0; t < cnt; ++t) {
    const double* v = s_v + t * TLMAX;
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < TLMAX; ++r) d += v[r] * x[r];   // v is zero above t and past l
    const double f = s_t[t] * d;
#pragma unroll
    for (int r = 0; r < TLMAX; ++r) x[r] -= f * v[r];
  }
#pragma unroll
  for (int r = 0; r < TLMAX; ++r)
    if (r < l) col[r] = x[r];
}

}  // namespace

size_t tournament_bytes(int n) {
  const size_t g0 = ((size_t)n + TS - 1) / TS;
  return 2 * g0 * TMAXB * sizeof(int) + 2 * g0 * sizeof(int) +
         2 * TLMAX * TMAXB * sizeof(double) + TMAXB * sizeof(double) + 4096;
}

int tournament_max_b() { return TMAXB; }
int tournament_max_l() { return TLMAX; }

int launch_qrcp_tournament(hipStream_t s, double* b, long long ldb, int l, int c0, int nc,
                           int nsteps, int gstep0, QrcpScratch* scr, int* pairs, int* info,
                           char* ws) {
  if (nsteps < 1 || nsteps > TMAXB || l > TLMAX || nsteps > l) return RQ_ERR_LIMIT;
  double* bb = b + (long long)c0 * ldb;
  const int g0 = (nc + TS - 1) / TS;
  int* sets[2] = {(int*)ws, (int*)ws + (size_t)g0 * TMAXB};
  int* cnts[2] = {(int*)ws + 2 * (size_t)g0 * TMAXB, (int*)ws + 2 * (size_t)g0 * TMAXB + g0};
  char* tail = ws + 2 * g0 * TMAXB * sizeof(int) + 2 * g0 * sizeof(int);
  tail = (char*)(((uintptr_t)tail + 255) / 256 * 256);
  double* vref = (double*)tail;
  double* rhat = vref + TLMAX * TMAXB;
  double* tref = rhat + TLMAX * TMAXB;
  int* tp_count = (int*)(tref + TMAXB);
  unsigned* err = &scr->bar.err;
  int ng = g0, cur = 0;
  // the leaves; they are the root when one group holds the whole block
  const bool leaf_root = (g0 == 1);
  hipLaunchKernelGGL(k_tp_select, dim3(ng), dim3(TQ), 0, s, (const double*)bb, ldb, l, nc, nsteps,
                     0, (const int*)nullptr, (const int*)nullptr, 0, sets[cur], cnts[cur],
                     (const int*)info, err, leaf_root ? vref : nullptr,
                     leaf_root ? tref : nullptr, leaf_root ? rhat : nullptr);
  while (ng > 1) {
    const int nn = (ng + TFAN - 1) / TFAN;
    const bool root = (nn == 1);
    hipLaunchKernelGGL(k_tp_select, dim3(nn), dim3(TQ), 0, s, (const double*)bb, ldb, l, nc,
                       nsteps, 1, (const int*)sets[cur], (const int*)cnts[cur], ng, sets[cur ^ 1],
                       cnts[cur ^ 1], (const int*)info, err, root ? vref : nullptr,
                       root ? tref : nullptr, root ? rhat : nullptr);
    cur ^= 1;
    ng = nn;
  }
  hipLaunchKernelGGL(k_tp_finish, dim3(1), dim3(64), 0, s, nsteps, gstep0, (const int*)sets[cur],
                     (const int*)cnts[cur], pairs, &scr->npairs, tp_count, info);
  RQ_HIP_CHECK(hipGetLastError());
  // the sketch columns move like A's; the winners take R-hat, the rest the
  // root's reflectors
  int rc = launch_apply_pairs<double>(s, l, b, ldb, c0, nullptr, (double*)nullptr, 0, 0, 0,
                                      pairs,
                                      &scr->npairs, 2 * nsteps);
  if (rc) return rc;
  hipLaunchKernelGGL(k_tp_apply, dim3((nc + 255) / 256), dim3(256), 0, s, bb, ldb, l, nc,
                     (const int*)tp_count, (const double*)vref, (const double*)tref,
                     (const double*)rhat);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace rq
