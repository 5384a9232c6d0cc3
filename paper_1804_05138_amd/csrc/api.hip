// C ABI of librqrcp: argument checks, workspace layout and the block loop of
// Alg. 2 (RQRCP), reorganized so that each block needs one pass over the
// trailing matrix:
//
//   B = Omega A;  QRCP(B) -> pivots of block 0;  move columns;  panel 0;
//   W_0 = V_0^T A2 (one read of A2)
//   for each block i:
//     W'_i = T_i^T W_i;  R12;  sample update of B (formula (1))
//     if another block follows:
//        QRCP(B) -> its pivots; move columns of A, jpvt and W'_i
//        panel i+1 (after applying block i's update to its own columns)
//        fused pass: A2 -= V_i W'_i  and  W_{i+1} = V_{i+1}^T A2
//     else: last pass A2 -= V_i W'_i
//
// The arithmetic is that of Alg. 2; only the order of independent work
// changes: the next block's pivots depend on the sketch, which needs only W_i
// (through R12), not on the rest of the trailing update.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/rqrcp.h"
#include "gemm.h"
#include "internal.h"
#include "srqr.h"

struct rqrcp_ctx {
  hipStream_t stream;
  int device;
  // device address of this GPU's static scratch array (rqrcp_factor_noalloc),
  // and whether a call on this handle has used it (rqrcp_check reads its flags)
  void* scratch = nullptr;
  bool used_scratch = false;
  // per-phase timing (benchmarks only)
  struct Mark {
    int phase;
    hipEvent_t a, b;
    double flops, bytes;
  };
  bool timing = false;
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  double ms[RQRCP_NPHASES] = {};
  int count[RQRCP_NPHASES] = {};
  double flops[RQRCP_NPHASES] = {};
  double bytes[RQRCP_NPHASES] = {};

  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

namespace {
// Records an event pair around the launches issued during its lifetime.
struct PhaseTimer {
  rqrcp_ctx* h;
  rqrcp_ctx::Mark mk;
  bool on;
  PhaseTimer(rqrcp_ctx* h_, int phase, double flops, double bytes) : h(h_), on(h_->timing) {
    if (!on) return;
    mk.phase = phase;
    mk.flops = flops;
    mk.bytes = bytes;
    mk.a = h->event();
    mk.b = h->event();
    if (!mk.a || !mk.b) {
      on = false;
      return;
    }
    hipEventRecord(mk.a, h->stream);
  }
  ~PhaseTimer() {
    if (!on) return;
    hipEventRecord(mk.b, h->stream);
    h->marks.push_back(mk);
  }
};
}  // namespace

namespace {

using namespace rq;

constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t omega, sketch_part, sketch_lp, qscr, cand, pairs, pscr, ppart, tmat, wpart, wp, copy,
      mark, formq, est, tourn, vall, wpall, gmat, gpart, total;
  int ko;              // columns of an outer block of the left-looking schedule
  int wsplit;          // most row splits of a W pass
  long long ldv, ldwa; // leading dimensions of the dense V (m x ko) and of W' (ko x n)
};

// Left-looking schedule: partial sums of the per-block W pass (one more slot
// for the correction term), and of the small Gram products V_j^T V.
constexpr int kLLSplit = 8;
// Outer block of the left-looking schedule when k > n/2: the reflectors of at
// most this many columns are kept, and A2 -= V W' is applied whenever they are
// full, so the Gram corrections (about m kO per column) stay bounded.
constexpr int kLLOuter = 512;
// Row splits of a W pass with outer blocks: the trailing width shrinks to a few
// column tiles late in a full-rank factorization, so more splits keep the grid full.
constexpr int kLLSplitWide = 32;
size_t ll_split_elems(int m, int n, int k, int b) {
  return (size_t)b * std::max({(size_t)8 * m, (size_t)16 * n, (size_t)64 * k});
}

size_t elem_size(int t) { return t == RQRCP_F32 ? sizeof(float) : sizeof(double); }

// Every workspace starts with the scratch words of the persistent kernels, so
// that rqrcp_check can find their error flags without the call's sizes.
constexpr size_t QSCR_OFF = 0;
const size_t PSCR_OFF = (sizeof(rq::QrcpScratch) + 255) / 256 * 256;
const size_t HEADER = PSCR_OFF + (sizeof(rq::PanelScratch) + 255) / 256 * 256;

Layout layout(int m, int n, int k, const rqrcp_params& prm) {
  Layout L;
  const int b = prm.b, p = prm.p, l = b + p;
  const unsigned flags = prm.flags;
  const size_t es = elem_size(prm.a_type);
  size_t off = HEADER;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.omega = take((size_t)l * m * sizeof(double));
  L.sketch_part = take(sketch_partial_doubles(m, n, l) * sizeof(double));
  L.sketch_lp = take(sketch_lp_bytes(m, n, l, prm.sketch_type));
  L.qscr = QSCR_OFF;
  L.cand = take(qrcp_cand_doubles(l, n) * sizeof(double));
  L.pairs = take(4 * MAX_B * sizeof(int));
  L.pscr = PSCR_OFF;
  L.ppart = take(panel_partial_doubles(m, std::min(b, k)) * sizeof(double));
  L.tmat = take((size_t)MAX_B * MAX_B * sizeof(double));
  // left-looking: one outer block when the rank is at most half the width (its
  // Gram blocks V_j^T V_<j add about m k^2 flops to the 4 m n k of the
  // updates), else outer blocks of kLLOuter columns
  L.ko = (2LL * k <= n) ? k : std::min(k, kLLOuter);
  L.ldv = m + (m & 1);
  L.ldwa = L.ko + (L.ko & 1);
  L.wsplit = (L.ko < k) ? kLLSplitWide : kLLSplit;
  L.wpart = take((size_t)(L.wsplit + 1) * n * b * es);
  L.wp = take((size_t)b * n * sizeof(double));
  L.vall = take((size_t)L.ldv * L.ko * es);
  L.wpall = take((size_t)L.ldwa * n * es);
  L.gmat = take((size_t)2 * b * L.ko * es);
  L.gpart = take(ll_split_elems(m, n, L.ko, b) * es);
  L.copy = take((flags & RQRCP_FROZEN_PIVOTS) ? (size_t)m * n * es : 0);
  L.mark = take((flags & RQRCP_FROZEN_PIVOTS) ? (size_t)n * sizeof(int) : 0);
  L.formq = take(form_q_work_elems(m, k, b) * es);
  L.est = take(4 * sizeof(double));
  L.tourn = take((flags & RQRCP_TOURNAMENT) ? tournament_bytes(n) : 0);
  L.total = off;
  return L;
}

// Clears the scratch words of one factorization.  The candidate records of the
// sketch QRCP carry a sequence number (the global pivot step + 1) that tells
// readers a record is current; zeroing them keeps a record left by an earlier
// call on the same workspace from passing for one of this call.
__global__ void k_init(QrcpScratch* q, PanelScratch* p, int* info, int* jpvt, int n, int iota,
                       double* cand, long long ncand) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  for (long long e = t; e < ncand; e += (long long)gridDim.x * blockDim.x) cand[e] = 0.0;
  for (int e = t; e < (int)(sizeof(p->sub) / sizeof(unsigned)); e += gridDim.x * blockDim.x)
    p->sub[e] = 0u;
  if (t == 0) {
    q->bar.count = 0;
    q->bar.err = 0;
    q->npairs = 0;
    p->bar.count = 0;
    p->bar.err = 0;
    *info = 0;
  }
  if (iota)
    for (int j = t; j < n; j += gridDim.x * blockDim.x) jpvt[j] = j;
}

// dst(:, c) = src(:, perm[c]) (src(:, c) without perm), c < n.  A caller's
// permutation is validated by k_perm_check before this runs; indices are still
// clamped to [0, n) so that an invalid one can never address outside src.
template <typename T>
__global__ void k_copy_cols(int m, int n, const T* __restrict__ src, long long lds,
                            T* __restrict__ dst, long long ldd, const int* __restrict__ perm) {
  const long long total = (long long)m * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long c = e / m, r = e % m;
    const long long sc = perm ? (long long)min(max(perm[c], 0), n - 1) : c;
    dst[c * ldd + r] = src[sc * lds + r];
  }
}

// Validation of a caller-supplied permutation (frozen pivots, backward):
// k_perm_clear zeroes the n marks (and the two error words rqrcp_check reads,
// if given), then
// k_perm_check counts every entry; an entry outside [0, n) or one seen twice
// sets bit 2 of the error word (rqrcp_check then returns RQRCP_ERR_PIVOTS)
// and, if info is given, *info = info_code.
__global__ void k_perm_clear(int n, int* __restrict__ mark, unsigned* err0, unsigned* err1) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int j = t; j < n; j += gridDim.x * blockDim.x) mark[j] = 0;
  if (t == 0) {
    if (err0) *err0 = 0u;
    if (err1) *err1 = 0u;
  }
}

__global__ void k_perm_check(int n, const int* __restrict__ perm, int* __restrict__ mark,
                             unsigned* err, int* info, int info_code) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int j = t; j < n; j += gridDim.x * blockDim.x) {
    const int v = perm[j];
    bool bad = v < 0 || v >= n;
    if (!bad) bad = atomicAdd(&mark[v], 1) != 0;
    if (bad) {
      atomicOr(err, 4u);
      if (info) *info = info_code;
    }
  }
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// L (2w x c, leading dimension 2w) of the stacked correction product: rows
// 0..w-1 are V(c0 + r, 0:c) (the block's own rows of the earlier reflectors),
// rows w..2w-1 the Gram block G = sum of the nparts partials of G (each at
// stride gstride), or left as they are when nparts = 0.
template <typename T>
__global__ void k_build_l(int w, int c, int c0, const T* __restrict__ v, long long ldv,
                          int nparts, long long gstride, const T* __restrict__ gp,
                          T* __restrict__ l) {
  const long long total = 2LL * w * c;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % (2 * w)), col = (int)(e / (2 * w));
    if (r < w) {
      l[e] = v[(long long)col * ldv + c0 + r];
    } else if (nparts > 0) {
      const long long g = (long long)col * w + (r - w);
      T acc = gp[g];
      for (int z = 1; z < nparts; ++z) acc += gp[(long long)z * gstride + g];
      l[e] = acc;
    }
  }
}

// The stacked correction P = L W' (partials, 2w x nc each): rows 0..w-1 are
// subtracted from A(c0 .. c0+w-1, cols), rows w..2w-1 negated into the W
// correction partial (leading dimension w).
template <typename T>
__global__ void k_apply_corr(int w, int nc, int nparts, const T* __restrict__ p,
                             T* __restrict__ a, long long lda, T* __restrict__ wslot) {
  const long long total = 2LL * w * nc;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    T acc = p[e];
    for (int z = 1; z < nparts; ++z) acc += p[(long long)z * total + e];
    const int r = (int)(e % (2 * w)), col = (int)(e / (2 * w));
    if (r < w)
      a[(long long)col * lda + r] -= acc;
    else
      wslot[(long long)col * w + (r - w)] = -acc;
  }
}

// Dense copy of the reflectors of columns c .. c+w-1 over all m rows:
// v(r, c + q - ob) = A(r, c + q) below row c + q, 1 on it, 0 above (the unit
// lower trapezoidal V of Alg. 2's block, kept for the left-looking products;
// ob is the first column of the current outer block).
template <typename T>
__global__ void k_copy_v(int m, int c, int w, int ob, const T* __restrict__ a, long long lda,
                         T* __restrict__ v, long long ldv) {
  const long long total = (long long)m * w;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(e / m), r = (int)(e % m);
    const int d = r - (c + q);
    v[(long long)(c + q - ob) * ldv + r] = d > 0 ? a[(long long)(c + q) * lda + r] : T(d == 0 ? 1 : 0);
  }
}

// W'(i:i+w, c0 + c) = wp(0:w, c) in the storage type, c < nc (FP32 storage:
// the sample-update kernel forms W' in FP64; the left-looking products apply
// it in FP32, as the fused pass does)
template <typename T>
__global__ void k_store_w(int w, int nc, const double* __restrict__ wp, long long ldw,
                          T* __restrict__ dst, long long ldd) {
  const long long total = (long long)w * nc;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e / w), r = (int)(e % w);
    dst[(long long)c * ldd + r] = (T)wp[(long long)c * ldw + r];
  }
}

// *out = ||B(0:l, c0:n)||_F^2 (one workgroup, fixed summation order).
__global__ __launch_bounds__(1024) void k_sketch_fro2(const double* __restrict__ b, long long ldb,
                                                      int l, int c0, int n, double* out) {
  __shared__ double sred[16];
  double s = 0.0;
  const long long total = (long long)l * (n - c0);
  for (long long e = threadIdx.x; e < total; e += 1024) {
    const double x = b[(c0 + e / l) * ldb + e % l];
    s += x * x;
  }
  s = wave_sum_dpp(s);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sred[w];
    *out = t;
  }
}

unsigned grid_for(long long total) {
  long long g = (total + 255) / 256;
  return (unsigned)std::max<long long>(1, std::min<long long>(g, 65536));
}

bool valid_params(const rqrcp_params* prm) {
  return prm && prm->b >= 1 && prm->p >= 0 &&
         (prm->a_type == RQRCP_F64 || prm->a_type == RQRCP_F32) &&
         (prm->sketch_type == RQRCP_F64 || prm->sketch_type == RQRCP_BF16 ||
          prm->sketch_type == RQRCP_F8E4M3);
}

}  // namespace

namespace {

// The block loop of Alg. 2 for storage type T of A (see the top of the file).
// Sketch estimate of ||A(c0:m, c0:n)'s trailing block||_F: ||B(:, c0:n)||_F / sqrt(l)
// (formula (1) keeps B(:, c0:n) = Omega-hat_2 R22 with l Gaussian rows).
// Synchronizes the stream.
int sketch_estimate(hipStream_t s, const double* B, int ldb, int l, int c0, int n, double* dev,
                    double* est) {
  hipLaunchKernelGGL(k_sketch_fro2, dim3(1), dim3(1024), 0, s, B, (long long)ldb, l, c0, n, dev);
  RQ_HIP_CHECK(hipGetLastError());
  double v = 0.0;
  RQ_HIP_CHECK(hipMemcpyAsync(&v, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  RQ_HIP_CHECK(hipStreamSynchronize(s));
  *est = sqrt(v / l);
  return 0;
}

// tol > 0: stop after the first block whose trailing sketch estimate is at
// most tol times the estimate of ||A||_F (both from the sketch); *k_done (host)
// receives the rank reached, *est_out (host) the last estimate ratio.
template <typename T>
int factor_impl(rqrcp_ctx* h, int m, int n, int k, const rqrcp_params* prm, const Layout& L,
                T* A, int lda, int32_t* jpvt, double* tau, double* B, int ldb, int32_t* info,
                void* ws, double tol = 0.0, int* k_done = nullptr, double* est_out = nullptr) {
  const int b = prm->b, p = prm->p, l = b + p;
  (void)p;
  const bool frozen = (prm->flags & RQRCP_FROZEN_PIVOTS) != 0;
  const bool stepwise = (prm->flags & RQRCP_HOUSEHOLDER_PANEL) != 0;
  hipStream_t s = h->stream;
  char* w = (char*)ws;
  double* om = (double*)(w + L.omega);
  void* sklp = w + L.sketch_lp;
  double* spart = (double*)(w + L.sketch_part);
  QrcpScratch* qscr = (QrcpScratch*)(w + L.qscr);
  double* cand = (double*)(w + L.cand);
  int* pairs = (int*)(w + L.pairs);
  PanelScratch* pscr = (PanelScratch*)(w + L.pscr);
  double* ppart = (double*)(w + L.ppart);
  double* tmat = (double*)(w + L.tmat);
  T* wpart = (T*)(w + L.wpart);
  double* wp = (double*)(w + L.wp);
  const long long ldw = b;
  int rc;
  // Left-looking schedule: A2 is not written per block.  Within an outer block
  // (columns ob .. ob+ko-1, one block of all k columns when k <= n/2) each
  // block keeps its reflectors in the dense V (m x ko, column c at c - ob) and
  // its W' rows in W' (ko x n, row c at c - ob); the rows R12 are finished in
  // place by the sample-update kernel, a panel takes the pending update of the
  // outer block's earlier blocks before it is factored, the per-block product
  // W_j = V_j^T A2 reads A2 as the outer block found it and subtracts
  // (V_j^T V_<j) W'_<j, and A2 -= V W' runs when the outer block is full and
  // at the end.
  const int ko = L.ko;
  int ob = 0;
  T* vall = (T*)(w + L.vall);
  T* wpall = (T*)(w + L.wpall);
  T* gmat = (T*)(w + L.gmat);
  T* gpart = (T*)(w + L.gpart);
  const long long ldv = L.ldv, ldwa = L.ldwa;
  const size_t gpart_elems = ll_split_elems(m, n, ko, b);
  auto copy_v = [&](int c, int wd) -> int {
    hipLaunchKernelGGL(k_copy_v<T>, dim3(grid_for((long long)m * wd)), dim3(256), 0, s, m, c, wd,
                       ob, (const T*)A, (long long)lda, vall, ldv);
    RQ_HIP_CHECK(hipGetLastError());
    return 0;
  };
  // Corrections of block (c, wd) from the outer block's earlier blocks, one
  // product with L = [V(c:c+wd, ob:c); G] (in gmat, 2 wd x (c - ob)): the
  // block's rows of the trailing columns, A(c:c+wd, c+wd:n) -= V(c:c+wd, ob:c)
  // W'(ob:c, .), and the W partial -G W'(ob:c, .) at wslot.
  auto stacked_corr = [&](int c, int wd, T* wslot) -> int {
    const int cb = c + wd, nc = n - cb, kc = c - ob;
    PhaseTimer pt(h, RQRCP_PHASE_BUPDATE, 4.0 * wd * (double)kc * nc, 8.0 * (double)kc * nc);
    // (64 x 64 output tiles for the 2 wd <= 128 rows of these products)
    const int tiles = ((2 * wd + 63) / 64) * ((nc + 63) / 64);
    int sp = (512 + tiles - 1) / tiles;   // about one round of two workgroups per CU
    sp = std::min(sp, std::max(1, kc / 32));
    sp = (int)std::min<long long>(sp, (long long)(gpart_elems / ((size_t)2 * wd * nc)));
    sp = std::max(sp, 1);
    int got = 0;
    int r = gemm_big_partials<T>(s, false, 2 * wd, nc, kc, gmat, 2 * wd,
                                 wpall + (long long)cb * ldwa, ldwa, gpart, sp, &got);
    if (r) return r;
    hipLaunchKernelGGL(k_apply_corr<T>, dim3(grid_for(2LL * wd * nc)), dim3(256), 0, s, wd, nc,
                       got, (const T*)gpart, A + c + (long long)cb * lda, (long long)lda, wslot);
    RQ_HIP_CHECK(hipGetLastError());
    return 0;
  };
  // W partials of block (c, wd) over the trailing columns c+wd .. n: the read
  // pass V^T A2 (split over rows) and, after the outer block's first block, the
  // correction -(V^T V(:, ob:c)) W'(ob:c, .) as one more partial.  *nsp_out =
  // partials written; partial z of W starts at wpw + z pstr wd (pstr = 0:
  // n - c - wd columns).
  T* wpw = wpart;
  long long pstr = 0;
  auto w_pass = [&](int c, int wd, int* nsp_out) -> int {
    const int cb = c + wd, nc = n - cb;
    *nsp_out = 0;
    wpw = wpart;
    pstr = 0;
    if (nc <= 0) return 0;
    T* part = wpart;
    const int kc = c - ob;                          // earlier reflectors of the outer block
    const T* vc = vall + c + (long long)kc * ldv;  // V_c, rows c .. m
    int got = 0, r = 0;
    // one pass over [V(c:m, ob:c) | A(c:m, cb:n)]: the Gram block G = V_c^T V(:, ob:c)
    // rides along with W = V_c^T A2
    const int nt = kc + nc;
    {
      const int tiles = (nt + kWpassCols - 1) / kWpassCols;
      int sp = (512 + tiles - 1) / tiles;
      sp = std::max(1, std::min(sp, std::min(L.wsplit, (m - c) / 256)));
      PhaseTimer pt(h, RQRCP_PHASE_TRAIL, 2.0 * (m - c) * (double)wd * nt,
                    8.0 * (m - c) * (double)nt);
      r = wpass_partials<T>(s, m - c, wd, nt, kc, vc, ldv, vall + c, ldv,
                            (const T*)A + c + (long long)cb * lda, lda, part, sp, &got);
      if (r && r != RQ_ERR_LIMIT) return r;
    }
    if (r == 0) {
      wpw = part + (long long)kc * wd;
      pstr = nt;
      if (kc > 0) {
        hipLaunchKernelGGL(k_build_l<T>, dim3(grid_for(2LL * wd * kc)), dim3(256), 0, s, wd, kc, c,
                           (const T*)vall, ldv, got, (long long)nt * wd, (const T*)part, gmat);
        RQ_HIP_CHECK(hipGetLastError());
        if ((r = stacked_corr(c, wd, part + ((long long)got * nt + kc) * wd))) return r;
        ++got;
      }
      *nsp_out = got;
      return 0;
    }
    // shapes the streaming pass does not take (odd sizes): the general GEMM
    {
      const int tiles = (nc + 255) / 256;
      int sp = (512 + tiles - 1) / tiles;
      sp = std::max(1, std::min(sp, std::min(L.wsplit, (m - c) / 256)));
      PhaseTimer pt(h, RQRCP_PHASE_TRAIL, 2.0 * (m - c) * (double)wd * nc,
                    8.0 * (m - c) * (double)nc);
      r = gemm_big_partials<T>(s, true, wd, nc, m - c, vc, ldv,
                               (const T*)A + c + (long long)cb * lda, lda, part, sp, &got);
      if (r) return r;
    }
    if (kc > 0) {
      {
        PhaseTimer pt(h, RQRCP_PHASE_BUPDATE, 2.0 * wd * (double)kc * (m - c),
                      8.0 * (double)kc * (m - c));
        r = gemm_big<T>(s, true, wd, kc, m - c, T(1), vc, ldv, vall + c, ldv, T(0), gmat + wd,
                        2 * wd, gpart, gpart_elems);
        if (r) return r;
      }
      hipLaunchKernelGGL(k_build_l<T>, dim3(grid_for(2LL * wd * kc)), dim3(256), 0, s, wd, kc, c,
                         (const T*)vall, ldv, 0, 0LL, (const T*)nullptr, gmat);
      RQ_HIP_CHECK(hipGetLastError());
      if ((r = stacked_corr(c, wd, part + (long long)got * nc * wd))) return r;
      ++got;
    }
    *nsp_out = got;
    return 0;
  };

  hipLaunchKernelGGL(k_init, dim3(grid_for(n)), dim3(256), 0, s, qscr, pscr, info, jpvt, n,
                     frozen ? 0 : 1, cand, frozen ? 0LL : (long long)qrcp_cand_doubles(l, n));
  RQ_HIP_CHECK(hipGetLastError());

  if (frozen) {
    T* cp = (T*)(w + L.copy);
    int* mark = (int*)(w + L.mark);
    hipLaunchKernelGGL(k_perm_clear, dim3(grid_for(n)), dim3(256), 0, s, n, mark,
                       (unsigned*)nullptr, (unsigned*)nullptr);
    hipLaunchKernelGGL(k_perm_check, dim3(grid_for(n)), dim3(256), 0, s, n, (const int*)jpvt,
                       mark, &qscr->bar.err, (int*)info, -8);
    hipLaunchKernelGGL(k_copy_cols<T>, dim3(grid_for((long long)m * n)), dim3(256), 0, s, m, n,
                       (const T*)A, (long long)lda, cp, (long long)m, (const int*)nullptr);
    hipLaunchKernelGGL(k_copy_cols<T>, dim3(grid_for((long long)m * n)), dim3(256), 0, s, m, n,
                       (const T*)cp, (long long)m, A, (long long)lda, (const int*)jpvt);
    RQ_HIP_CHECK(hipGetLastError());
  } else if (!(prm->flags & RQRCP_USER_SKETCH)) {
    PhaseTimer pt(h, RQRCP_PHASE_SKETCH, 2.0 * l * (double)m * n,
                  8.0 * ((double)m * n + (double)l * n));
    bool done = false;
    if constexpr (std::is_same<T, double>::value) {
      if (prm->sketch_type == SK_F64 && sketch_t_usable(m, l, A, lda)) {
        // Omega drawn transposed, so that B = Omega A runs as the W-pass product
        rc = launch_gaussian_t(s, l, m, prm->seed, 0, om, m);
        if (rc) return rc;
        rc = launch_sketch_t(s, m, n, l, om, A, lda, B, ldb, spart);
        if (rc) return rc;
        done = true;
      }
    }
    if (!done) {
      rc = launch_gaussian(s, l, m, prm->seed, 0, om, l);
      if (rc) return rc;
      rc = launch_sketch<T>(s, m, n, l, prm->sketch_type, om, l, A, lda, B, ldb, spart, sklp);
      if (rc) return rc;
    }
  }

  // algorithmic work of one launch of each phase
  auto qrcp_flops = [&](int nc, int steps) {
    double f = 0.0;
    for (int t = 0; t < steps; ++t) f += 4.0 * (l - t) * (double)(nc - t);
    return f;
  };
  auto panel_flops = [&](int rows, int w, int wprev) {
    return 3.0 * rows * (double)w * w + 2.0 * (rows + wprev) * (double)wprev * w;
  };
  double* estd = (double*)(w + L.est);
  // partial QRCP of B(:, c0:c0+nc) for nsteps pivots: the grid-wide greedy
  // kernel, or tournament pivoting
  auto qrcp_block = [&](int c0q, int ncq, int nsteps, int gstep0) -> int {
    if (prm->flags & RQRCP_TOURNAMENT)
      return launch_qrcp_tournament(s, B, ldb, l, c0q, ncq, nsteps, gstep0, qscr, pairs, info,
                                    w + L.tourn);
    return launch_qrcp_sketch(s, B, ldb, l, c0q, ncq, nsteps, gstep0, qscr, cand, pairs, info);
  };
  double norm_a = 0.0, ratio = 1.0;
  if (tol > 0.0) {
    rc = sketch_estimate(s, B, ldb, l, 0, n, estd, &norm_a);
    if (rc) return rc;
  }

  int i = 0;
  int bb = std::min(b, k);
  int nsp = 0;
  if (!frozen) {
    {
      PhaseTimer pt(h, RQRCP_PHASE_QRCP, qrcp_flops(n, bb), 16.0 * l * (double)n);
      rc = qrcp_block(0, n, bb, 0);
      if (rc) return rc;
    }
    PhaseTimer pt(h, RQRCP_PHASE_SWAP, 0.0, 0.0);
    rc = launch_apply_pairs<T>(s, m, A, lda, 0, jpvt, (double*)nullptr, 0, 0, 0, pairs,
                               &qscr->npairs,
                               2 * bb);
    if (rc) return rc;
  }
  {
    PhaseTimer pt(h, RQRCP_PHASE_PANEL, panel_flops(m, bb, 0), 16.0 * m * (double)bb);
    rc = launch_panel<T>(s, m, A, lda, 0, bb, 0, nullptr, 0, tau, tmat, pscr, ppart, stepwise);
    if (rc) return rc;
    if ((rc = copy_v(0, bb))) return rc;
  }
  if (n - bb > 0 && (rc = w_pass(0, bb, &nsp))) return rc;
  for (;;) {
    const int c0 = i + bb;
    const int ncols = n - c0;
    if (ncols > 0) {
      PhaseTimer pt(h, RQRCP_PHASE_BUPDATE, 4.0 * bb * (double)bb * ncols,
                    8.0 * ncols * (double)bb * (nsp + 4));
      // W' in FP64 goes straight into the W' rows; in FP32 storage through wp
      double* wout = wp;
      long long ldwo = ldw;
      if constexpr (std::is_same<T, double>::value) {
        wout = wpall + (long long)c0 * ldwa + (i - ob);
        ldwo = ldwa;
      }
      rc = launch_bupdate<T>(s, m, A, lda, i, bb, tmat, (const T*)wpw, nsp, wout, ldwo,
                             frozen ? nullptr : B, ldb, c0, ncols, info, A, pstr);
      if (rc) return rc;
      if (!std::is_same<T, double>::value) {
        hipLaunchKernelGGL(k_store_w<T>, dim3(grid_for((long long)bb * ncols)), dim3(256), 0, s,
                           bb, ncols, (const double*)wp, ldw,
                           wpall + (long long)c0 * ldwa + (i - ob), ldwa);
        RQ_HIP_CHECK(hipGetLastError());
      }
    }
    bool stop = false;
    if (tol > 0.0 && ncols > 0) {
      double e = 0.0;
      rc = sketch_estimate(s, B, ldb, l, c0, n, estd, &e);
      if (rc) return rc;
      ratio = norm_a > 0.0 ? e / norm_a : 0.0;
      stop = ratio <= tol;
    }
    if (c0 < k && !stop && c0 - ob + std::min(b, k - c0) > ko) {
      // the outer block is full: A2 -= V W' for its blocks (rows ob..c0 are
      // final already), and the next block starts a new outer block
      PhaseTimer pt(h, RQRCP_PHASE_FINAL, 2.0 * (m - c0) * (double)(c0 - ob) * ncols,
                    16.0 * (m - c0) * (double)ncols);
      rc = gemm_big<T>(s, false, m - c0, ncols, c0 - ob, T(-1), vall + c0, ldv,
                       wpall + (long long)c0 * ldwa, ldwa, T(1), A + c0 + (long long)c0 * lda,
                       lda);
      if (rc) return rc;
      ob = c0;
    }
    if (c0 < k && !stop) {
      const int bbn = std::min(b, k - c0);
      if (!frozen) {
        {
          PhaseTimer pt(h, RQRCP_PHASE_QRCP, qrcp_flops(ncols, bbn), 16.0 * l * (double)ncols);
          rc = qrcp_block(c0, ncols, bbn, c0);
          if (rc) return rc;
        }
        PhaseTimer pt(h, RQRCP_PHASE_SWAP, 0.0, 0.0);
        rc = launch_apply_pairs<T, T>(s, m, A, lda, c0, jpvt, wpall + (long long)c0 * ldwa,
                                      c0 - ob, ldwa, 0, pairs, &qscr->npairs, 2 * bbn);
        if (rc) return rc;
      }
      {
        PhaseTimer pt(h, RQRCP_PHASE_PANEL,
                      panel_flops(m - c0, bbn, 0) + 2.0 * (m - c0) * (double)(c0 - ob) * bbn,
                      16.0 * (m - c0) * (double)bbn);
        // the panel's pending update from the outer block's earlier blocks, then its QR
        if (c0 > ob) {
          rc = gemm_big<T>(s, false, m - c0, bbn, c0 - ob, T(-1), vall + c0, ldv,
                           wpall + (long long)c0 * ldwa, ldwa, T(1),
                           A + c0 + (long long)c0 * lda, lda, gpart, gpart_elems);
          if (rc) return rc;
        }
        rc = launch_panel<T>(s, m, A, lda, c0, bbn, 0, nullptr, 0, tau, tmat, pscr, ppart,
                             stepwise);
        if (rc) return rc;
        if ((rc = copy_v(c0, bbn))) return rc;
      }
      const int nrest = n - (c0 + bbn);
      if (nrest > 0) {
        if ((rc = w_pass(c0, bbn, &nsp))) return rc;
      } else {
        nsp = 0;
      }
      i = c0;
      bb = bbn;
    } else {
      if (ncols > 0 && c0 > ob) {
        // A2 -= V W' for the outer block's blocks at once (rows 0..c0 are final already)
        PhaseTimer pt(h, RQRCP_PHASE_FINAL, 2.0 * (m - c0) * (double)(c0 - ob) * ncols,
                      16.0 * (m - c0) * (double)ncols);
        rc = gemm_big<T>(s, false, m - c0, ncols, c0 - ob, T(-1), vall + c0, ldv,
                         wpall + (long long)c0 * ldwa, ldwa, T(1), A + c0 + (long long)c0 * lda,
                         lda);
        if (rc) return rc;
      }
      if (k_done) *k_done = c0;
      if (est_out) *est_out = (tol > 0.0 && ncols > 0) ? ratio : 0.0;
      break;
    }
  }
  return 0;
}

}  // namespace

// ---- Static scratch of the allocation-free entry point ----
// rqrcp_factor_noalloc takes its workspace from this file-scope device array
// instead of a caller's buffer.  Each GPU the library runs on holds its own
// copy until the process ends; host code must never pass the array's name to a
// kernel (on the host it is only a stand-in): its device address is looked up
// once per device, with that device current, when a handle is created, and
// only that address is used.  Every call on one GPU shares the array, so calls
// that overlap on one GPU (other streams, other threads) race.
constexpr size_t kStaticScratchBytes = RQRCP_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= 64) return RQRCP_ERR_LIMIT;
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return RQRCP_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

// The argument checks rqrcp_factor and rqrcp_factor_noalloc share (all but the
// workspace).
int factor_checks(rqrcp_handle h, int m, int n, int k, const rqrcp_params* prm, void* A, int lda,
                  int32_t* jpvt, double* tau, double* B, int ldb, int32_t* info) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (k < 1 || k > std::min(m, n)) return -4;
  if (!valid_params(prm)) return -5;
  const int b = prm->b, p = prm->p, l = b + p;
  const bool frozen = (prm->flags & RQRCP_FROZEN_PIVOTS) != 0;
  if (b > MAX_B || l > MAX_L) return RQRCP_ERR_LIMIT;
  if (!A) return -6;
  if (lda < m) return -7;
  if (!jpvt) return -8;
  if (!tau) return -9;
  if (!frozen && !B) return -10;
  if (!frozen && ldb < l) return -11;
  if (!info) return -12;
  if (!frozen) {
    int maxn = 0;
    rqrcp_limits(l, nullptr, nullptr, &maxn);
    if (n > maxn) return RQRCP_ERR_LIMIT;
  }
  if ((prm->flags & RQRCP_TOURNAMENT) && (b > tournament_max_b() || l > tournament_max_l()))
    return RQRCP_ERR_LIMIT;
  return 0;
}
}  // namespace

extern "C" {

int rqrcp_create(rqrcp_handle* h, void* stream) {
  if (!h) return -1;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RQRCP_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return RQRCP_ERR_HIP;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return RQRCP_ERR_DEVICE;
  // this device's copy of the static scratch (rqrcp_factor_noalloc)
  void* sp = nullptr;
  const int src = scratch_address(dev, &sp);
  if (src) return src;
  rqrcp_ctx* c = new (std::nothrow) rqrcp_ctx;
  if (!c) return RQRCP_ERR_HIP;
  c->stream = (hipStream_t)stream;
  c->device = dev;
  c->scratch = sp;
  *h = c;
  return 0;
}

int rqrcp_destroy(rqrcp_handle h) {
  if (!h) return -1;
  for (auto& mk : h->marks) {
    hipEventDestroy(mk.a);
    hipEventDestroy(mk.b);
  }
  for (auto e : h->pool) hipEventDestroy(e);
  delete h;
  return 0;
}

int rqrcp_set_stream(rqrcp_handle h, void* stream) {
  if (!h) return -1;
  h->stream = (hipStream_t)stream;
  return 0;
}

int rqrcp_limits(int l, int* max_b, int* max_l, int* max_n) {
  if (max_b) *max_b = MAX_B;
  if (max_l) *max_l = MAX_L;
  // the sketch QRCP's grid (256 columns per workgroup, 128 for l > 80) at
  // one workgroup per compute unit
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (max_n) *max_n = (l > 80 ? 128 : 256) * ncu;
  return 0;
}

int rqrcp_workspace_size(int m, int n, int k, const rqrcp_params* prm, size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (k < 1 || k > std::min(m, n)) return -3;
  if (!valid_params(prm)) return -4;
  if (!bytes) return -5;
  *bytes = layout(m, n, k, *prm).total;
  return 0;
}

int rqrcp_gaussian(rqrcp_handle h, int rows, int cols, uint64_t seed, uint64_t stream, double* out,
                   int ld) {
  if (!h) return -1;
  if (rows < 0) return -2;
  if (cols < 0) return -3;
  if (!out && rows * (long long)cols > 0) return -6;
  if (ld < std::max(1, rows)) return -7;
  return launch_gaussian(h->stream, rows, cols, seed, stream, out, ld);
}

int rqrcp_sketch(rqrcp_handle h, int m, int n, int l, uint64_t seed, int a_type, const void* A,
                 int lda, int sketch_type, const double* Omega, int ldo, double* B, int ldb,
                 void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (l < 1 || l > MAX_L) return -4;
  if (a_type != RQRCP_F64 && a_type != RQRCP_F32) return -6;
  if (!A) return -7;
  if (lda < m) return -8;
  if (sketch_type != RQRCP_F64 && sketch_type != RQRCP_BF16 && sketch_type != RQRCP_F8E4M3)
    return -9;
  if (Omega && ldo < l) return -11;
  if (!B) return -12;
  if (ldb < l) return -13;
  const size_t om_b = align_up((size_t)l * m * sizeof(double));
  const size_t part_b = align_up(sketch_partial_doubles(m, n, l) * sizeof(double));
  const size_t need = HEADER + om_b + part_b + sketch_lp_bytes(m, n, l, sketch_type);
  if (!ws || ws_bytes < need) return RQRCP_ERR_WORKSPACE;
  char* w = (char*)ws + HEADER;
  double* om = (double*)w;
  double* part = (double*)(w + om_b);
  void* lp = w + om_b + part_b;
  long long ldo_eff = ldo;
  if (!Omega && a_type == RQRCP_F64 && sketch_type == RQRCP_F64 &&
      sketch_t_usable(m, l, (const double*)A, lda)) {
    // Omega drawn transposed, so that B = Omega A runs as the W-pass product
    int rc = launch_gaussian_t(h->stream, l, m, seed, 0, om, m);
    if (rc) return rc;
    return launch_sketch_t(h->stream, m, n, l, om, (const double*)A, lda, B, ldb, part);
  }
  if (!Omega) {
    int rc = launch_gaussian(h->stream, l, m, seed, 0, om, l);
    if (rc) return rc;
    Omega = om;
    ldo_eff = l;
  }
  if (a_type == RQRCP_F64)
    return launch_sketch<double>(h->stream, m, n, l, sketch_type, Omega, ldo_eff,
                                 (const double*)A, lda, B, ldb, part, lp);
  return launch_sketch<float>(h->stream, m, n, l, sketch_type, Omega, ldo_eff, (const float*)A,
                              lda, B, ldb, part, lp);
}

int rqrcp_factor(rqrcp_handle h, int m, int n, int k, const rqrcp_params* prm, void* A, int lda,
                 int32_t* jpvt, double* tau, double* B, int ldb, int32_t* info, void* ws,
                 size_t ws_bytes) {
  const int rc = factor_checks(h, m, n, k, prm, A, lda, jpvt, tau, B, ldb, info);
  if (rc) return rc;
  const Layout L = layout(m, n, k, *prm);
  if (!ws || ws_bytes < L.total) return RQRCP_ERR_WORKSPACE;
  if (prm->a_type == RQRCP_F32)
    return factor_impl<float>(h, m, n, k, prm, L, (float*)A, lda, jpvt, tau, B, ldb, info, ws);
  return factor_impl<double>(h, m, n, k, prm, L, (double*)A, lda, jpvt, tau, B, ldb, info, ws);
}

int rqrcp_factor_noalloc(rqrcp_handle h, int m, int n, int k, const rqrcp_params* prm, void* A,
                         int lda, int32_t* jpvt, double* tau, double* B, int ldb,
                         int32_t* info) {
  const int rc = factor_checks(h, m, n, k, prm, A, lda, jpvt, tau, B, ldb, info);
  if (rc) return rc;
  const Layout L = layout(m, n, k, *prm);
  if (L.total > kStaticScratchBytes) return RQRCP_ERR_SCRATCH;
  if (!h->scratch) return RQRCP_ERR_HIP;
  h->used_scratch = true;
  // the same kernels as rqrcp_factor, on this device's static array (its
  // scratch words are cleared by the first kernel of every call)
  if (prm->a_type == RQRCP_F32)
    return factor_impl<float>(h, m, n, k, prm, L, (float*)A, lda, jpvt, tau, B, ldb, info,
                              h->scratch);
  return factor_impl<double>(h, m, n, k, prm, L, (double*)A, lda, jpvt, tau, B, ldb, info,
                             h->scratch);
}

int rqrcp_factor_tol(rqrcp_handle h, int m, int n, int kmax, double tol, const rqrcp_params* prm,
                     void* A, int lda, int32_t* jpvt, double* tau, double* B, int ldb,
                     int32_t* info, int* k_out, double* est_out, void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (kmax < 1 || kmax > std::min(m, n)) return -4;
  if (!(tol > 0.0 && tol < 1.0)) return -5;
  if (!valid_params(prm) || (prm->flags & RQRCP_FROZEN_PIVOTS)) return -6;
  const int b = prm->b, p = prm->p, l = b + p;
  if (b > MAX_B || l > MAX_L) return RQRCP_ERR_LIMIT;
  if (!A) return -7;
  if (lda < m) return -8;
  if (!jpvt) return -9;
  if (!tau) return -10;
  if (!B) return -11;
  if (ldb < l) return -12;
  if (!info) return -13;
  if (!k_out) return -14;
  const Layout L = layout(m, n, kmax, *prm);
  if (!ws || ws_bytes < L.total) return RQRCP_ERR_WORKSPACE;
  int maxn = 0;
  rqrcp_limits(l, nullptr, nullptr, &maxn);
  if (n > maxn) return RQRCP_ERR_LIMIT;
  if ((prm->flags & RQRCP_TOURNAMENT) && (b > tournament_max_b() || l > tournament_max_l()))
    return RQRCP_ERR_LIMIT;
  double ratio = 0.0;
  int rc;
  if (prm->a_type == RQRCP_F32)
    rc = factor_impl<float>(h, m, n, kmax, prm, L, (float*)A, lda, jpvt, tau, B, ldb, info, ws,
                            tol, k_out, &ratio);
  else
    rc = factor_impl<double>(h, m, n, kmax, prm, L, (double*)A, lda, jpvt, tau, B, ldb, info, ws,
                             tol, k_out, &ratio);
  if (est_out) *est_out = ratio;
  return rc;
}

int srqr_workspace_size(int m, int n, int l, const rqrcp_params* prm, int d, unsigned sflags,
                        size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (l < 1 || l >= std::min(m, n)) return -3;
  if (!valid_params(prm)) return -4;
  if (d < 1 && !(sflags & SRQR_EXACT)) return -5;
  if (!bytes) return -7;
  rqrcp_params fprm = *prm;
  fprm.flags = RQRCP_FROZEN_PIVOTS;
  const size_t fac = align_up(layout(m, n, l + 1, fprm).total);
  *bytes = fac + srqr_layout(m, n, l, d, (sflags & SRQR_EXACT) ? 1 : 0).total;
  return 0;
}

int srqr_swap(rqrcp_handle h, int m, int n, int l, const rqrcp_params* prm, double g, int d,
              int max_swaps, unsigned sflags, const double* A0, int lda0, double* A, int lda,
              int32_t* jpvt, double* tau, const double* B, int ldb, double* g2_out,
              int32_t* nswaps_out, int32_t* info, void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (l < 1 || l >= std::min(m, n)) return -4;
  if (!valid_params(prm) || prm->b > MAX_B) return -5;
  if (prm->a_type != RQRCP_F64) return RQRCP_ERR_UNSUPPORTED;
  if (!(g > 1.0)) return -6;
  const int exact = (sflags & SRQR_EXACT) ? 1 : 0;
  if (!exact && d < 1) return -7;
  if (!A0) return -10;
  if (lda0 < m) return -11;
  if (!A) return -12;
  if (lda < m) return -13;
  if (!jpvt) return -14;
  if (!tau) return -15;
  if (!B) return -16;
  if (ldb < prm->b + prm->p) return -17;
  if (!info) return -20;
  if (l + 1 > 4096) return RQRCP_ERR_LIMIT;
  size_t need = 0;
  int rc = srqr_workspace_size(m, n, l, prm, d, sflags, &need);
  if (rc) return rc;
  if (!ws || ws_bytes < need) return RQRCP_ERR_WORKSPACE;
  if (max_swaps < 0) max_swaps = 2 * n;
  hipStream_t s = h->stream;
  rqrcp_params fprm = *prm;
  fprm.flags = RQRCP_FROZEN_PIVOTS;
  const size_t fac = align_up(layout(m, n, l + 1, fprm).total);
  char* sw = (char*)ws + fac;
  const SrqrLayout L = srqr_layout(m, n, l, d, exact);
  double* est = (double*)(sw + L.est);
  double* om = (double*)(sw + L.omega);
  double* sc = (double*)(sw + L.sc);
  const int deff = exact ? l + 1 : d;
  // the scratch words rqrcp_check reads start cleared, whether or not a
  // refactorization runs
  hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, (QrcpScratch*)((char*)ws + QSCR_OFF),
                     (PanelScratch*)((char*)ws + PSCR_OFF), info, nullptr, 0, 0, nullptr, 0LL);
  RQ_HIP_CHECK(hipGetLastError());

  auto g2_round = [&](int it) -> int {
    if (!exact) {
      int r = launch_gaussian(s, d, l + 1, prm->seed, (1ull << 32) + (uint64_t)it, om, d);
      if (r) return r;
    }
    return launch_srqr_g2(s, l, A, lda, om, deff, exact, L, sw, g2_out);
  };
  auto read_g2 = [&](double* v) -> int {
    if (hipMemcpyAsync(v, sc + 2, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
      return RQRCP_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RQRCP_ERR_HIP;
    return 0;
  };

  // r_i from the final sketch, the first pick, one QR step, g2
  rc = launch_srqr_init(s, m, n, l, prm->b + prm->p, A, lda, jpvt, B, ldb, est);
  if (rc) return rc;
  rc = launch_srqr_pick_qr(s, m, n, l, A, lda, jpvt, est, tau, sc);
  if (rc) return rc;
  rc = g2_round(0);
  if (rc) return rc;
  double g2 = 0.0;
  rc = read_g2(&g2);
  if (rc) return rc;
  int nswaps = 0;
  while (g2 > g && nswaps < max_swaps) {
    rc = launch_srqr_rotate(s, m, n, l, A, lda, jpvt, L, sw);
    if (rc) return rc;
    rc = launch_srqr_pick_qr(s, m, n, l, A, lda, jpvt, est, tau, sc);
    if (rc) return rc;
    ++nswaps;
    rc = g2_round(nswaps);
    if (rc) return rc;
    rc = read_g2(&g2);
    if (rc) return rc;
  }
  if (nswaps > 0) {
    // Givens rotations are not representable by (V, tau): refactor A0(:, jpvt)
    hipLaunchKernelGGL(k_copy_cols<double>, dim3(grid_for((long long)m * n)), dim3(256), 0, s, m, n, A0,
                       (long long)lda0, A, (long long)lda, (const int*)nullptr);
    RQ_HIP_CHECK(hipGetLastError());
    rc = rqrcp_factor(h, m, n, l + 1, &fprm, A, lda, jpvt, tau, nullptr, 0, info, ws, fac);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, info, (g2 > g) ? -max_swaps : 0);
  if (nswaps_out) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, nswaps_out, nswaps);
  RQ_HIP_CHECK(hipGetLastError());
  return 0;
}

int rqrcp_qrcp_workspace_size(int m, int n, int k, int nb, size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (k < 1 || k > std::min(m, n)) return -3;
  if (nb < 1 || nb > qrcp_full_max_nb()) return -4;
  if (!bytes) return -5;
  *bytes = qrcp_full_workspace(m, n, k, nb);
  return 0;
}

int rqrcp_qrcp(rqrcp_handle h, int m, int n, int k, int nb, double* A, int lda, int32_t* jpvt,
               double* tau, void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (k < 1 || k > std::min(m, n)) return -4;
  if (nb < 1 || nb > qrcp_full_max_nb()) return -5;
  if (!A) return -6;
  if (lda < m) return -7;
  if (!jpvt) return -8;
  if (!tau) return -9;
  if (!ws || ws_bytes < qrcp_full_workspace(m, n, k, nb)) return RQRCP_ERR_WORKSPACE;
  PhaseTimer pt(h, RQRCP_PHASE_OTHER, 0.0, 0.0);
  return launch_qrcp_full(h->stream, m, n, k, nb, A, lda, (int*)jpvt, tau, (char*)ws);
}

int rqrcp_cx_workspace_size(int m, int n, int k, size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (k < 1 || k > std::min(m, n)) return -3;
  if (!bytes) return -4;
  *bytes = HEADER + cx_workspace(n, k);
  return 0;
}

int rqrcp_cx(rqrcp_handle h, int m, int n, int k, const double* AF, int ldaf,
             const int32_t* jpvt, double* X, int ldx, void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (k < 1 || k > std::min(m, n)) return -4;
  if (!AF) return -5;
  if (ldaf < m) return -6;
  if (!jpvt) return -7;
  if (!X) return -8;
  if (ldx < k) return -9;
  if (k > 1024) return RQRCP_ERR_LIMIT;
  if (!ws || ws_bytes < HEADER + cx_workspace(n, k)) return RQRCP_ERR_WORKSPACE;
  return launch_cx(h->stream, m, n, k, AF, ldaf, (const int*)jpvt, X, ldx, (char*)ws + HEADER);
}

int rqrcp_cur_workspace_size(int m, int n, int k, int b, size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (k < 1 || k > std::min(m, n)) return -3;
  if (b < 1 || b > MAX_B) return -4;
  if (!bytes) return -5;
  *bytes = HEADER + cur_workspace(m, n, k, b);
  return 0;
}

int rqrcp_cur(rqrcp_handle h, int m, int n, int k, int b, const double* AFc, int ldc,
              const int32_t* jpvt_c, const double* AFr, int ldr, const double* tau_r, double* U,
              int ldu, void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (k < 1 || k > std::min(m, n)) return -4;
  if (b < 1 || b > MAX_B) return -5;
  if (!AFc) return -6;
  if (ldc < m) return -7;
  if (!jpvt_c) return -8;
  if (!AFr) return -9;
  if (ldr < n) return -10;
  if (!tau_r) return -11;
  if (!U) return -12;
  if (ldu < k) return -13;
  if (k > 1024) return RQRCP_ERR_LIMIT;
  if (!ws || ws_bytes < HEADER + cur_workspace(m, n, k, b)) return RQRCP_ERR_WORKSPACE;
  return launch_cur(h->stream, m, n, k, b, AFc, ldc, (const int*)jpvt_c, AFr, ldr, tau_r, U, ldu,
                    (char*)ws + HEADER);
}

int rqrcp_compress_workspace_size(int m, int n, int l, int k, int b, size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (l < 1 || l > std::min(m, n)) return -3;
  if (k < 1 || k > l) return -4;
  if (b < 1 || b > MAX_B) return -5;
  if (!bytes) return -6;
  *bytes = HEADER + compress_workspace(m, n, l, k, b);
  return 0;
}

int rqrcp_compress(rqrcp_handle h, int m, int n, int l, int k, int b, const double* AF, int ldaf,
                   const double* tau, const int32_t* jpvt, double* X, int ldx, double* Y,
                   int ldy, double* sigma, void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (l < 1 || l > std::min(m, n)) return -4;
  if (k < 1 || k > l) return -5;
  if (b < 1 || b > MAX_B) return -6;
  if (!AF) return -7;
  if (ldaf < m) return -8;
  if (!tau) return -9;
  if (!jpvt) return -10;
  if (!X) return -11;
  if (ldx < m) return -12;
  if (!Y) return -13;
  if (ldy < k) return -14;
  if (l > compress_max_l()) return RQRCP_ERR_LIMIT;
  if (!ws || ws_bytes < HEADER + compress_workspace(m, n, l, k, b)) return RQRCP_ERR_WORKSPACE;
  return launch_compress(h->stream, m, n, l, k, b, AF, ldaf, tau, (const int*)jpvt, X, ldx, Y,
                         ldy, sigma, (char*)ws + HEADER);
}

int rqrcp_form_q(rqrcp_handle h, int m, int k, int b, int a_type, const void* A, int lda,
                 const double* tau, void* Q, int ldq, void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (k < 1 || k > m) return -3;
  if (b < 1 || b > MAX_B) return -4;
  if (a_type != RQRCP_F64 && a_type != RQRCP_F32) return -5;
  if (!A) return -6;
  if (lda < m) return -7;
  if (!tau) return -8;
  if (!Q) return -9;
  if (ldq < m) return -10;
  if (!ws || ws_bytes < HEADER + form_q_work_elems(m, k, b) * elem_size(a_type))
    return RQRCP_ERR_WORKSPACE;
  void* work = (char*)ws + HEADER;
  if (a_type == RQRCP_F32)
    return form_q<float>(h->stream, m, k, b, (const float*)A, lda, tau, (float*)Q, ldq,
                         (float*)work);
  return form_q<double>(h->stream, m, k, b, (const double*)A, lda, tau, (double*)Q, ldq,
                        (double*)work);
}

int rqrcp_backward_workspace_size(int m, int n, int k, int b, int a_type, size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (k < 1 || k > std::min(m, n)) return -3;
  if (b < 1 || b > MAX_B) return -4;
  if (a_type != RQRCP_F64 && a_type != RQRCP_F32) return -5;
  if (!bytes) return -6;
  *bytes = HEADER + align_up((size_t)n * sizeof(int)) +
           backward_layout(m, n, k, b, elem_size(a_type)).total;
  return 0;
}

int rqrcp_backward(rqrcp_handle h, int m, int n, int k, int b, int a_type, const void* A, int lda,
                   const void* AF, int ldaf, const double* tau, const int32_t* jpvt,
                   const void* dQ1, int ldq, const void* dR, int ldr, void* dA, int ldda,
                   void* ws, size_t ws_bytes) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (k < 1 || k > std::min(m, n)) return -4;
  if (b < 1 || b > MAX_B) return -5;
  if (a_type != RQRCP_F64 && a_type != RQRCP_F32) return -6;
  if (!A) return -7;
  if (lda < m) return -8;
  if (!AF) return -9;
  if (ldaf < m) return -10;
  if (!tau) return -11;
  if (!jpvt) return -12;
  if (dQ1 && ldq < m) return -14;
  if (dR && ldr < k) return -16;
  if (!dA) return -17;
  if (ldda < m) return -18;
  if (k > 1024) return RQRCP_ERR_LIMIT;
  size_t need = 0;
  int rc = rqrcp_backward_workspace_size(m, n, k, b, a_type, &need);
  if (rc) return rc;
  if (!ws || ws_bytes < need) return RQRCP_ERR_WORKSPACE;
  {
    int* mark = (int*)((char*)ws + HEADER);
    // both error words rqrcp_check reads start cleared
    unsigned* err = &((QrcpScratch*)((char*)ws + QSCR_OFF))->bar.err;
    unsigned* err1 = &((PanelScratch*)((char*)ws + PSCR_OFF))->bar.err;
    hipLaunchKernelGGL(k_perm_clear, dim3(grid_for(n)), dim3(256), 0, h->stream, n, mark, err,
                       err1);
    hipLaunchKernelGGL(k_perm_check, dim3(grid_for(n)), dim3(256), 0, h->stream, n,
                       (const int*)jpvt, mark, err, (int*)nullptr, 0);
    RQ_HIP_CHECK(hipGetLastError());
  }
  char* w = (char*)ws + HEADER + align_up((size_t)n * sizeof(int));
  if (a_type == RQRCP_F32)
    return backward<float>(h->stream, m, n, k, b, (const float*)A, lda, (const float*)AF, ldaf,
                           tau, jpvt, (const float*)dQ1, ldq, (const float*)dR, ldr, (float*)dA,
                           ldda, w);
  return backward<double>(h->stream, m, n, k, b, (const double*)A, lda, (const double*)AF, ldaf,
                          tau, jpvt, (const double*)dQ1, ldq, (const double*)dR, ldr, (double*)dA,
                          ldda, w);
}

// The autotuner's table: batched kernel variant per (device, b, b + p), shared
// by every handle of the process (a graph captured on another stream's handle
// uses the tuned variant too); -1 = not tuned.
static std::mutex g_tune_mu;
static int g_tune[64][17][33];
static bool g_tune_init = false;

static int tuned_variant(int dev, int b, int l) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_init || dev < 0 || dev >= 64) return -1;
  return g_tune[dev][b][l];
}

static void set_tuned_variant(int dev, int b, int l, int v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_init) {
    for (auto& d : g_tune)
      for (auto& r : d)
        for (int& x : r) x = -1;
    g_tune_init = true;
  }
  if (dev >= 0 && dev < 64) g_tune[dev][b][l] = v;
}

int rqrcp_batched_limits(int* max_m, int* max_ln, int* max_b, int* max_l) {
  return batched_max(max_m, max_ln, max_b, max_l);
}

int rqrcp_batched_workspace_size(size_t* bytes) {
  if (!bytes) return -1;
  *bytes = 256;
  return 0;
}

static int batched_checks(rqrcp_handle h, int batch, const rqrcp_problem* probs,
                          const rqrcp_params* prm, float* A_pool, int32_t* jpvt_pool,
                          double* tau_pool, double* B_pool, int32_t* info, void* ws,
                          size_t ws_bytes) {
  if (!h) return -1;
  if (batch < 0) return -2;
  if (!probs && batch > 0) return -3;
  int mb = 0, ml = 0;
  batched_max(nullptr, nullptr, &mb, &ml);
  if (!prm || prm->b < 1 || prm->b > mb || prm->p < 0 || prm->b + prm->p > ml) return -4;
  if (prm->a_type != RQRCP_F32 || prm->sketch_type != RQRCP_F64) return RQRCP_ERR_UNSUPPORTED;
  if (!A_pool) return -5;
  if (!jpvt_pool) return -7;
  if (!tau_pool) return -9;
  if (!B_pool) return -11;
  if (!info) return -13;
  if (!ws || ws_bytes < 256) return RQRCP_ERR_WORKSPACE;
  return 0;
}

int rqrcp_factor_batched(rqrcp_handle h, int batch, const rqrcp_problem* probs,
                         const rqrcp_params* prm, float* A_pool, int64_t a_elems,
                         int32_t* jpvt_pool, int64_t jpvt_elems, double* tau_pool,
                         int64_t tau_elems, double* B_pool, int64_t b_elems, int32_t* info,
                         void* ws, size_t ws_bytes) {
  int rc = batched_checks(h, batch, probs, prm, A_pool, jpvt_pool, tau_pool, B_pool, info, ws,
                          ws_bytes);
  if (rc) return rc;
  if (batch == 0) return 0;
  const int l = prm->b + prm->p;
  int v = tuned_variant(h->device, prm->b, l);
  if (v < 0) v = 0;
  return launch_batched(h->stream, v, batch, probs, prm->b, l, prm->seed, A_pool, a_elems,
                        jpvt_pool, jpvt_elems, tau_pool, tau_elems, B_pool, b_elems, info,
                        (unsigned*)ws);
}

int rqrcp_autotune_batched(rqrcp_handle h, int batch, const rqrcp_problem* probs,
                           const rqrcp_params* prm, float* A_pool, int64_t a_elems,
                           int32_t* jpvt_pool, int64_t jpvt_elems, double* tau_pool,
                           int64_t tau_elems, double* B_pool, int64_t b_elems, int32_t* info,
                           void* ws, size_t ws_bytes, const float* A_orig, int* best_variant,
                           float* ms_per_variant) {
  int rc = batched_checks(h, batch, probs, prm, A_pool, jpvt_pool, tau_pool, B_pool, info, ws,
                          ws_bytes);
  if (rc) return rc;
  if (!A_orig) return -16;
  if (batch == 0 || a_elems <= 0) return 0;
  const int l = prm->b + prm->p;
  const int nv = batched_variants();
  hipEvent_t e0 = h->event(), e1 = h->event();
  if (!e0 || !e1) return RQRCP_ERR_HIP;
  int best = 0;
  float best_ms = 0.0f;
  for (int v = 0; v < nv; ++v) {
    float ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {  // the first run warms up
      RQ_HIP_CHECK(hipMemcpyAsync(A_pool, A_orig, (size_t)a_elems * sizeof(float),
                                  hipMemcpyDeviceToDevice, h->stream));
      RQ_HIP_CHECK(hipEventRecord(e0, h->stream));
      rc = launch_batched(h->stream, v, batch, probs, prm->b, l, prm->seed, A_pool, a_elems,
                          jpvt_pool, jpvt_elems, tau_pool, tau_elems, B_pool, b_elems, info,
                          (unsigned*)ws);
      if (rc) return rc;
      RQ_HIP_CHECK(hipEventRecord(e1, h->stream));
      RQ_HIP_CHECK(hipEventSynchronize(e1));
      RQ_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    }
    if (ms_per_variant && v < 8) ms_per_variant[v] = ms;
    if (v == 0 || ms < best_ms) {
      best = v;
      best_ms = ms;
    }
  }
  h->pool.push_back(e0);
  h->pool.push_back(e1);
  set_tuned_variant(h->device, prm->b, l, best);
  if (best_variant) *best_variant = best;
  // leave the outputs of the chosen variant
  RQ_HIP_CHECK(hipMemcpyAsync(A_pool, A_orig, (size_t)a_elems * sizeof(float),
                              hipMemcpyDeviceToDevice, h->stream));
  return launch_batched(h->stream, best, batch, probs, prm->b, l, prm->seed, A_pool, a_elems,
                        jpvt_pool, jpvt_elems, tau_pool, tau_elems, B_pool, b_elems, info,
                        (unsigned*)ws);
}

int rqrcp_check(rqrcp_handle h, void* ws) {
  if (!h) return -1;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return RQRCP_ERR_HIP;
  if (hipGetLastError() != hipSuccess) return RQRCP_ERR_HIP;
  if (!ws) {
    // after rqrcp_factor_noalloc the flags live in the device's static scratch
    if (!h->used_scratch || !h->scratch) return 0;
    ws = h->scratch;
  }
  char* w = (char*)ws;
  GridBarrier bars[2];
  if (hipMemcpy(&bars[0], w + QSCR_OFF, sizeof(GridBarrier), hipMemcpyDeviceToHost) != hipSuccess)
    return RQRCP_ERR_HIP;
  if (hipMemcpy(&bars[1], w + PSCR_OFF, sizeof(GridBarrier), hipMemcpyDeviceToHost) != hipSuccess)
    return RQRCP_ERR_HIP;
  if (bars[0].err || bars[1].err) {
    const unsigned zero[3] = {0, 0, 0};
    hipMemcpy(w + QSCR_OFF, zero, sizeof(zero), hipMemcpyHostToDevice);
    hipMemcpy(w + PSCR_OFF, zero, sizeof(zero), hipMemcpyHostToDevice);
    // bit 2 of the first word: a caller's permutation was invalid; bit 1: the
    // sketch QRCP found no valid pivot (a non-finite sketch)
    if (bars[0].err & 4u) return RQRCP_ERR_PIVOTS;
    return (bars[0].err & 2u) ? RQRCP_ERR_NUMERIC : RQRCP_ERR_BARRIER;
  }
  return 0;
}

int rqrcp_set_timing(rqrcp_handle h, int enable) {
  if (!h) return -1;
  h->timing = enable != 0;
  return 0;
}

int rqrcp_read_timing(rqrcp_handle h, double* ms, int* count, double* flops, double* bytes) {
  if (!h) return -1;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return RQRCP_ERR_HIP;
  for (auto& mk : h->marks) {
    float e = 0.0f;
    if (hipEventElapsedTime(&e, mk.a, mk.b) == hipSuccess) {
      h->ms[mk.phase] += e;
      h->count[mk.phase] += 1;
      h->flops[mk.phase] += mk.flops;
      h->bytes[mk.phase] += mk.bytes;
    }
    h->pool.push_back(mk.a);
    h->pool.push_back(mk.b);
  }
  h->marks.clear();
  for (int p = 0; p < RQRCP_NPHASES; ++p) {
    if (ms) ms[p] = h->ms[p];
    if (count) count[p] = h->count[p];
    if (flops) flops[p] = h->flops[p];
    if (bytes) bytes[p] = h->bytes[p];
    h->ms[p] = 0.0;
    h->count[p] = 0;
    h->flops[p] = 0.0;
    h->bytes[p] = 0.0;
  }
  return 0;
}

const char* rqrcp_status_string(int status) {
  if (status == 0) return "success";
  if (status < 0) return "invalid argument";
  switch (status) {
    case RQRCP_ERR_HIP: return "HIP runtime error";
    case RQRCP_ERR_WORKSPACE: return "workspace too small";
    case RQRCP_ERR_UNSUPPORTED: return "unsupported data type combination";
    case RQRCP_ERR_DEVICE: return "device is not gfx950";
    case RQRCP_ERR_LIMIT: return "size beyond the kernels' limits";
    case RQRCP_ERR_BARRIER: return "grid barrier timed out";
    case RQRCP_ERR_NUMERIC: return "non-finite value in the sketch (no pivot could be chosen)";
    case RQRCP_ERR_PIVOTS: return "jpvt is not a permutation of 0..n-1";
    case RQRCP_ERR_SCRATCH:
      return "the factorization needs more workspace than the static scratch of "
             "rqrcp_factor_noalloc holds (RQRCP_NOALLOC_MAX_BYTES)";
    default: return "unknown status";
  }
}

}  // extern "C"
