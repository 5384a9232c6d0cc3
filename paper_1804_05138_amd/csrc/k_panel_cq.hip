// Panel QR of Alg. 2 (PDGEQRF + PDLARFT in Alg. 4) with few grid-wide
// reductions: CholeskyQR2 followed by Householder reconstruction.
//
// The stepwise panel needs one grid-wide reduction per reflector.  Here the
// panel X = A(i:m, i:i+bb) (bb <= 64, after the previous block's pending
// update) is orthogonalized with two Cholesky QR passes,
//     G1 = X^T X = R1^T R1,   Q1 = X R1^-1,   G2 = Q1^T Q1 = R2^T R2,   Q = Q1 R2^-1,
// and the compact-WY Householder form of the same factorization is rebuilt
// from Q (Ballard et al., "Reconstructing Householder vectors from tall-skinny
// QR", 2014): with S = diag(s), the LU factorization without pivoting
//     Q - [S; 0] = Y U,   s_t = -sign(of the eliminated diagonal entry, sign(0) = +),
// gives the unit lower trapezoidal reflectors Y (= V), T = -U S Y1^-T and
// R = S R2 R1.  In exact arithmetic this is the factorization the LAPACK
// dlarfg convention produces: H_0 ... H_{bb-1} [R; 0] = X with tau_t = T(t, t)
// in [1, 2] and R(t, t) = -sign(alpha_t) ||x_t||.  (Its rounding differs from
// the stepwise reflectors by O(kappa(X) eps).)
//
// Kernels (one launch each, no persistent grid): pending update, Gram
// partials + a fixed-order sum, one-wave Cholesky and inverse, Q1 with the
// second Gram, the small-matrix step (Cholesky, modified LU, T, R), and the
// write-back of V and R.  A flag in the scratch records whether the
// factorization can be trusted (every Cholesky pivot positive and finite,
// diag(R1) within a factor kCqMaxSpread, the pivots of the second Gram matrix within
// [1/4, 4]); if not, every later kernel of this path
// returns at once and the stepwise kernel, which reads the same flag, factors
// the (already updated) panel instead.
#include "internal.h"

namespace rq {
namespace {

// Largest ratio between diagonal entries of R1 (the Cholesky factor of the
// panel's Gram matrix) for which the Cholesky-QR2 result is used.  Measured
// against stepwise Householder reflectors on panels graded inside one block,
// the columnwise difference of V grows as about 3e-16 times this ratio (R and
// tau about half that): at 1e3 it stays below 3e-13, inside the 1e-12 parity
// bar; wider spreads go to the stepwise kernel.
constexpr double kCqMaxSpread = 1e3;

constexpr int CB = 64;        // largest panel width of this path
constexpr int CP = CB + 1;    // LDS pitch
constexpr int CR = 64;        // rows per workgroup of the row-parallel kernels
constexpr int RT = CR / 64;   // 16-row tiles per wave in them (four waves)
constexpr int CT = 256;

// ---- pending update A(rp:m, i+coff : i+coff+bb) -= V_prev W'(:, coff : coff+bb)
// (V_prev unit lower at column rp = i - bbp) ----
// One row per lane (coalesced column accesses): each thread holds its row of
// V_prev in registers and updates a quarter of the bb columns; W' is staged
// in LDS and read by wave-uniform (broadcast) loads.  Each entry is
// a - sum_q V(r, q) W'(q, c), the sum taken over q = 0, 1, ... in order.
constexpr int PR = 64;  // rows per workgroup of the pending update
template <typename T>
__global__ __launch_bounds__(CT) void k_cq_pend(int m, T* __restrict__ a, long long lda, int i,
                                                int coff, int bb, int bbp,
                                                const double* __restrict__ wp, long long ldw) {
  __shared__ double sw[CB * CB];  // W'(q, c) at sw[c * CB + q], zero for q >= bbp
  const int rp = i - bbp;
  const int tid = threadIdx.x;
  const int rr = tid % PR;
  const int part = __builtin_amdgcn_readfirstlane(tid / PR);  // one part per wave
  const int r = rp + blockIdx.x * PR + rr;
  for (int e = tid; e < bb * CB; e += CT) {
    const int c = e / CB, q = e % CB;
    sw[e] = q < bbp ? wp[(long long)(coff + c) * ldw + q] : 0.0;
  }
  // this thread's row of V_prev (loads from clamped addresses, masked after)
  const int rs = r < m ? r : m - 1;
  const int d = r - rp;
  double v[CB];
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    const double x = (double)a[(long long)(rp + (q < bbp ? q : 0)) * lda + rs];
    v[q] = (q < bbp && d > q) ? x : ((q < bbp && d == q) ? 1.0 : 0.0);
  }
  __syncthreads();
  if (r >= m) return;
  for (int c = part; c < bb; c += CT / PR) {
    const double* w = sw + c * CB;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < CB; ++q) s += v[q] * w[q];
    T* col = a + (long long)(i + coff + c) * lda;
    col[r] = (T)((double)col[r] - s);
  }
}

// Stage rows [r0, r0 + CR) of a column-major matrix (bb <= CB columns, zero
// padded, rows past `rows` zero) into sx[row * CP + col]: all loads of a
// thread are issued before any LDS store.
template <typename S>
RQ_DEV void stage_chunk(const S* __restrict__ x, long long ldx, int rows, int r0, int bb,
                        double* sx) {
  constexpr int NL = CR * CB / CT;
  double v[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = threadIdx.x + u * CT;
    const int c = e / CR, rr = e % CR;
    const int r = r0 + rr;
    const int rs = r < rows ? r : rows - 1;
    const int cs = c < bb ? c : 0;
    v[u] = (double)x[(long long)cs * ldx + rs];
  }
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = threadIdx.x + u * CT;
    const int c = e / CR, rr = e % CR;
    sx[rr * CP + c] = (c < bb && r0 + rr < rows) ? v[u] : 0.0;
  }
}

// ---- Gram partial of a CR-row chunk on FP64 MFMA: part[g] = Xc^T Xc (CB x CB) ----
// Source rows [0, rows) of a column-major matrix with bb columns (zero padded
// to CB).  Each wave owns 16 output rows (c1) and all 4 column tiles.
template <typename S>
RQ_DEV void gram_chunk(const double* sx, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int tcol = 0; tcol < 4; ++tcol) acc[tcol] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < CR / 4; ++kk) {
    const int r = 4 * kk + lg;
    const double av = sx[r * CP + 16 * wave + l16];
#pragma unroll
    for (int tcol = 0; tcol < 4; ++tcol) acc[tcol] = mfma_f64(av, sx[r * CP + 16 * tcol + l16], acc[tcol]);
  }
#pragma unroll
  for (int tcol = 0; tcol < 4; ++tcol)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c1 = 16 * wave + acc_row<double>(lg, e), c2 = 16 * tcol + l16;
      out[c1 * CB + c2] = acc[tcol][e];
    }
}

template <typename S>
__global__ __launch_bounds__(CT) void k_cq_gram(int rows, const S* __restrict__ x, long long ldx,
                                                int bb, double* __restrict__ part,
                                                const int* __restrict__ flag) {
  __shared__ double sx[CR * CP];
  if (flag && *flag == 0) return;
  stage_chunk<S>(x, ldx, rows, blockIdx.x * CR, bb, sx);
  __syncthreads();
  gram_chunk<S>(sx, part + (size_t)blockIdx.x * CB * CB);
}

// out[e] = sum over p of part[p][e] (deterministic): a workgroup takes 64
// entries, each summed over four consecutive ranges of p by four waves (in
// order within a range), and the four range sums are added in range order.
constexpr int SUMW = CT / 64;  // ranges of p per entry
__global__ __launch_bounds__(CT) void k_cq_sum(int nparts, const double* __restrict__ part,
                                               double* __restrict__ out,
                                               const int* __restrict__ flag) {
  __shared__ double ss[SUMW][64];
  if (flag && *flag == 0) return;
  const int el = threadIdx.x & 63, k = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;     // CB * CB is a multiple of 64
  const int per = (nparts + SUMW - 1) / SUMW;
  const int p1 = min(nparts, (k + 1) * per);
  constexpr int U = 16;  // loads in flight per batch; the sum keeps the order within the range
  double s = 0.0;
  int p = k * per;
  for (; p + U <= p1; p += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[(size_t)(p + u) * CB * CB + e];
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; p < p1; ++p) s += part[(size_t)p * CB * CB + e];
  ss[k][el] = s;
  __syncthreads();
  if (k == 0) {
    double t = ss[0][el];
#pragma unroll
    for (int j = 1; j < SUMW; ++j) t += ss[j][el];
    out[e] = t;
  }
}

// ---- small dense steps on CB x CB matrices (LDS by columns, pitch CP) ----
// One workgroup of ST threads.  The eliminations keep row r of an augmented
// matrix in lane r of every wave, wave w holding a slice of its columns in
// registers; each wave takes pivot rows of its own slice from lane j with
// readlane, and only multipliers cross waves, through LDS.

constexpr int ST = 1024;      // threads of the small-matrix kernels
constexpr int SW = ST / 64;   // their waves

RQ_DEV int wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// 1 / d for a normal, nonzero d: hardware reciprocal and two Newton steps
// (within about 1 ulp); fewer dependent operations than a full division.
RQ_DEV double recip(double d) {
  double x = __builtin_amdgcn_rcp(d);
  double e = fma(-d, x, 1.0);
  x = fma(x, e, x);
  e = fma(-d, x, 1.0);
  return fma(x, e, x);
}

// Identity outside the leading bb x bb block (entries inside are left alone).
RQ_DEV void pad_identity(double* m, int bb) {
  for (int e = threadIdx.x; e < CB * CB; e += ST) {
    const int c = e / CB, r = e % CB;
    if (r >= bb || c >= bb) m[c * CP + r] = (r == c) ? 1.0 : 0.0;
  }
}

// The eliminations below run in blocks of CW steps, the CW columns of one
// wave: that wave factors its own columns in registers (the multipliers of a
// step are its own column over the pivot, the pivot row comes from lane j by
// readlane), publishes the CW multiplier columns in LDS, and after one block
// barrier every other wave applies the CW steps to its columns in order.  One
// barrier per CW steps; the multiplier buffer alternates between two halves.
constexpr int EW = 2 * CB / SW;   // columns of an augmented [M | I] per wave

// Cholesky G = R^T R of the symmetric g (bb x bb) and R^-1 in one symmetric
// elimination of [G | I]: row j of the left half over sqrt(pivot) is row j of
// R, row j of the right half over sqrt(pivot) is row j of R^-T.  rout and
// rinv get identity padding; rinv may be g.  Returns false if a pivot is not
// positive and finite; dmin/dmax are the extreme pivots (diag(R)^2).
// LDS: smult 2 EW 64 doubles, sd and sraw CB each.
RQ_DEV bool chol_inv_pass(const double* g, double* rout, double* rinv, int bb, double* smult,
                          double* sd, double* sraw, double& dmin, double& dmax) {
  constexpr int CW = EW;
  const int r = threadIdx.x & 63, w = wave_index();
  double a[CW];
#pragma unroll
  for (int i = 0; i < CW; ++i) {
    const int c = CW * w + i, cl = c & (CB - 1);
    const bool in = c < CB && r < bb && cl < bb;
    a[i] = in ? g[cl * CP + r] : (r == cl ? 1.0 : 0.0);
  }
  pad_identity(rout, bb);
  pad_identity(rinv, bb);
  __syncthreads();
  for (int jb = 0; jb < bb; jb += CW) {
    const int owner = jb / CW;
    double* sm = smult + (owner & 1) * CW * 64;
    if (w == owner) {
#pragma unroll
      for (int s = 0; s < CW; ++s) {
        const int j = jb + s;
        if (j < bb) {
          const double d = readlane_f64(a[s], j);
          const bool good = (d > 1e-300) && (d < 1e300);
          const double dd = good ? d : 1.0;
          const double mult = (r > j && r < bb) ? a[s] * recip(dd) : 0.0;
          sm[s * 64 + r] = mult;
          if (r == 0) {
            sd[j] = dd;
            sraw[j] = d;
          }
#pragma unroll
          for (int i = s + 1; i < CW; ++i) a[i] = fma(-mult, readlane_f64(a[i], j), a[i]);
        }
      }
    }
    __syncthreads();
    if (w != owner) {
#pragma unroll
      for (int s = 0; s < CW; ++s) {
        const int j = jb + s;
        if (j < bb) {
          const double mult = sm[s * 64 + r];
#pragma unroll
          for (int i = 0; i < CW; ++i) a[i] = fma(-mult, readlane_f64(a[i], j), a[i]);
        }
      }
    }
  }
  // row r stopped changing at step r (later steps only touch rows below their
  // pivot): store the rows unscaled
  if (r < bb) {
#pragma unroll
    for (int i = 0; i < CW; ++i) {
      const int c = CW * w + i, cl = c & (CB - 1);
      if (cl < bb) {
        if (c < CB) rout[cl * CP + r] = a[i];
        else rinv[r * CP + cl] = a[i];   // R^-T(r, cl) = R^-1(cl, r)
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < bb * bb; e += ST) {
    const int c = e / bb, q = e % bb;
    const double s = 1.0 / sqrt(sd[q]);
    rout[c * CP + q] = (c >= q) ? rout[c * CP + q] * s : 0.0;   // R(q, c)
    rinv[q * CP + c] = (c <= q) ? rinv[q * CP + c] * s : 0.0;   // R^-1(c, q)
  }
  bool ok = true;
  dmin = 1e300;
  dmax = 0.0;
  for (int j = 0; j < bb; ++j) {
    const double d = sraw[j];
    ok = ok && (d > 1e-300) && (d < 1e300);
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
  }
  return ok;
}

// Elimination without pivoting of A - S = L U with s_j = -sign(pivot), sign(0)
// = + (the pivot is the current diagonal entry before s_j is taken off), run
// on [A | I]: uout = U, linv = L^-1 (both identity padded), L's strict lower
// part to l1g (global, CB x CB by columns; the caller zeroes the rest), s_j to
// s_s.  Blocked as chol_inv_pass.  LDS: smult 2 EW 64 doubles, udg CB.
RQ_DEV void lu_pass(const double* am, double* uout, double* linv, double* __restrict__ l1g,
                    int bb, double* smult, double* s_s, double* udg) {
  constexpr int CW = EW;
  const int r = threadIdx.x & 63, w = wave_index();
  double a[CW];
#pragma unroll
  for (int i = 0; i < CW; ++i) {
    const int c = CW * w + i, cl = c & (CB - 1);
    const bool in = c < CB && r < bb && cl < bb;
    a[i] = in ? am[cl * CP + r] : (r == cl ? 1.0 : 0.0);
  }
  pad_identity(uout, bb);
  pad_identity(linv, bb);
  __syncthreads();
  for (int jb = 0; jb < bb; jb += CW) {
    const int owner = jb / CW;
    double* sm = smult + (owner & 1) * CW * 64;
    if (w == owner) {
#pragma unroll
      for (int s = 0; s < CW; ++s) {
        const int j = jb + s;
        if (j < bb) {
          const double p = readlane_f64(a[s], j);
          const double st = (p >= 0.0) ? -1.0 : 1.0;
          const double utt = p - st;   // |utt| >= 1
          const double mult = (r > j && r < bb) ? a[s] * recip(utt) : 0.0;
          sm[s * 64 + r] = mult;
          if (r > j && r < bb) l1g[j * CB + r] = mult;
          if (r == 0) {
            s_s[j] = st;
            udg[j] = utt;
          }
#pragma unroll
          for (int i = s + 1; i < CW; ++i) a[i] = fma(-mult, readlane_f64(a[i], j), a[i]);
        }
      }
    }
    __syncthreads();
    if (w != owner) {
#pragma unroll
      for (int s = 0; s < CW; ++s) {
        const int j = jb + s;
        if (j < bb) {
          const double mult = sm[s * 64 + r];
#pragma unroll
          for (int i = 0; i < CW; ++i) a[i] = fma(-mult, readlane_f64(a[i], j), a[i]);
        }
      }
    }
  }
  if (r < bb) {   // final rows (as in chol_inv_pass)
#pragma unroll
    for (int i = 0; i < CW; ++i) {
      const int c = CW * w + i, cl = c & (CB - 1);
      if (cl < bb) {
        if (c < CB) uout[cl * CP + r] = a[i];
        else linv[cl * CP + r] = a[i];   // L^-1(r, cl)
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < bb * bb; e += ST) {
    const int c = e / bb, q = e % bb;
    uout[c * CP + q] = (c > q) ? uout[c * CP + q] : (c == q ? udg[q] : 0.0);   // U(q, c)
    linv[c * CP + q] = (c <= q) ? linv[c * CP + q] : 0.0;                       // L^-1(q, c)
  }
}

// X = U^-1 (identity padded) by backward elimination of [U | I]: the
// multipliers U(r, j) / U(j, j) are read from um and only the right half is
// kept, so the waves need no barrier.  The caller synchronizes afterwards.
RQ_DEV void upper_inv_pass(const double* um, double* xout, int bb) {
  constexpr int CW = CB / SW;   // columns per wave
  const int r = threadIdx.x & 63, w = wave_index();
  double a[CW];
#pragma unroll
  for (int i = 0; i < CW; ++i) a[i] = (r == CW * w + i) ? 1.0 : 0.0;
  pad_identity(xout, bb);
  for (int j = bb - 1; j >= 0; --j) {
    const double inv = recip(um[j * CP + j]);
    const double mult = (r < j) ? um[j * CP + r] * inv : 0.0;
#pragma unroll
    for (int i = 0; i < CW; ++i) a[i] = fma(-mult, readlane_f64(a[i], j), a[i]);
  }
  // row r is final since step r (later steps touch rows above their pivot only)
  if (r < bb) {
    const double inv = recip(um[r * CP + r]);
#pragma unroll
    for (int i = 0; i < CW; ++i) {
      const int c = CW * w + i;
      if (c < bb) xout[c * CP + r] = a[i] * inv;   // U^-1(r, c), zero for c < r
    }
  }
}

// One 16 x 16 tile per wave of C = A B on FP64 MFMA, A and B CB x CB (A in LDS
// by columns, B through bel(k, c) = B(k, c)).  Wave w owns rows 16 (w % 4) ..
// and columns 16 (w / 4) ..: acc[e] = C(16 (w % 4) + acc_row(lane / 16, e),
// 16 (w / 4) + lane % 16).
template <typename F>
RQ_DEV v4d mm_tile(const double* A, F bel) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int l16 = lane & 15, lg = lane >> 4, rb = w & 3, cb = w >> 2;
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < CB / 4; ++kk) {
    const int k = 4 * kk + lg;
    acc = mfma_f64(A[k * CP + 16 * rb + l16], bel(k, 16 * cb + l16), acc);
  }
  return acc;
}

// Stage a CB x CB column-major (or symmetric) matrix from global src[col * CB + row]
// into dst[col * CP + row] with NT threads, every load in flight at once.
template <int NT>
RQ_DEV void stage_small(const double* __restrict__ src, double* dst) {
  constexpr int NL = CB * CB / NT;
  double v[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) v[u] = src[threadIdx.x + u * NT];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = threadIdx.x + u * NT;
    dst[(e / CB) * CP + (e % CB)] = v[u];
  }
}

// ---- Cholesky of G1 and R1^-1; flag = 1 if usable ----
__global__ __launch_bounds__(ST) void k_cq_chol1(int bb, const double* __restrict__ g1,
                                                 double* __restrict__ r1,
                                                 double* __restrict__ r1inv,
                                                 int* __restrict__ flag) {
  __shared__ double smult[2 * EW * 64];
  __shared__ double sd[CB];
  __shared__ double sraw[CB];
  __shared__ double sG[CB * CP];   // G1, then R1^-1
  __shared__ double sR[CB * CP];
  stage_small<ST>(g1, sG);   // G1 is symmetric: its rows are its columns
  __syncthreads();
  double dmin, dmax;
  const bool ok = chol_inv_pass(sG, sR, sG, bb, smult, sd, sraw, dmin, dmax);
  __syncthreads();
  // usable if every pivot is positive and finite and diag(R1) spreads less
  // than kCqMaxSpread
  if (threadIdx.x == 0) *flag = (ok && dmin * kCqMaxSpread * kCqMaxSpread > dmax) ? 1 : 0;
  for (int e = threadIdx.x; e < CB * CB; e += ST) {
    r1[e] = sR[(e / CB) * CP + (e % CB)];
    r1inv[e] = sG[(e / CB) * CP + (e % CB)];
  }
}

// ---- Q1 = X R1^-1 for a CR-row chunk (MFMA), stored, and its Gram partial ----
template <typename T>
__global__ __launch_bounds__(CT) void k_cq_q1(int rows, const T* __restrict__ x, long long ldx,
                                              int bb, const double* __restrict__ r1inv,
                                              double* __restrict__ q1, long long ldq,
                                              double* __restrict__ part,
                                              const int* __restrict__ flag) {
  __shared__ double sx[CR * CP];
  __shared__ double sm[CB * CP];   // R1^-1(k, c) at sm[k * CP + c]
  if (*flag == 0) return;
  const int r0 = blockIdx.x * CR;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  {
    double v[CB * CB / CT];
#pragma unroll
    for (int u = 0; u < CB * CB / CT; ++u) v[u] = r1inv[tid + u * CT];
    stage_chunk<T>(x, ldx, rows, r0, bb, sx);
#pragma unroll
    for (int u = 0; u < CB * CB / CT; ++u) {
      const int e = tid + u * CT, c = e / CB, k = e % CB;
      sm[k * CP + c] = v[u];
    }
  }
  __syncthreads();
  // wave w: rows 16 RT w .. (RT row tiles) x 4 column tiles
  v4d acc[RT][4];
#pragma unroll
  for (int b = 0; b < RT; ++b)
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) acc[b][tc] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < CB / 4; ++kk) {
    const int k = 4 * kk + lg;
    double av[RT];
#pragma unroll
    for (int b = 0; b < RT; ++b) av[b] = sx[(16 * RT * wave + 16 * b + l16) * CP + k];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
      const double bv = sm[k * CP + 16 * tc + l16];
#pragma unroll
      for (int b = 0; b < RT; ++b) acc[b][tc] = mfma_f64(av[b], bv, acc[b][tc]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < RT; ++b)
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = 16 * RT * wave + 16 * b + acc_row<double>(lg, e);
        const int c = 16 * tc + l16;
        const double v = (r0 + rr < rows) ? acc[b][tc][e] : 0.0;
        sx[rr * CP + c] = v;
      }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < CR * CB / CT; ++u) {
    const int e = tid + u * CT;
    const int c = e / CR, rr = e % CR;
    const int r = r0 + rr;
    if (r < rows && c < bb) q1[(long long)c * ldq + r] = sx[rr * CP + c];
  }
  gram_chunk<double>(sx, part + (size_t)blockIdx.x * CB * CB);
}

// ---- the small-matrix step ----
// In: G2, R1, the top bb rows of Q1.  Out: M2 = R2^-1 U^-1, Rh = S R2 R1
// (upper), L1 (strict lower: the top block of V), T (bb x bb) and tau.
// LDS buffers P0..P3 (CB x CB by columns) are reused along the way:
//   P0 G2 -> R2^-1;  P1 R1 -> Qtop -> U^-1;  P2 Q1top -> U;  P3 R2 -> L1^-1.
__global__ __launch_bounds__(ST) void k_cq_small(int bb, const double* __restrict__ g2,
                                                 const double* __restrict__ r1,
                                                 const double* __restrict__ q1, long long ldq,
                                                 double* __restrict__ m2,
                                                 double* __restrict__ rh,
                                                 double* __restrict__ l1out,
                                                 double* __restrict__ tmat,
                                                 double* __restrict__ tau,
                                                 int* __restrict__ flag) {
  __shared__ double smult[2 * EW * 64];
  __shared__ double s_s[CB];
  __shared__ double sd[CB];
  __shared__ double sraw[CB];
  __shared__ double P0[CB * CP];
  __shared__ double P1[CB * CP];
  __shared__ double P2[CB * CP];
  __shared__ double P3[CB * CP];
  if (*flag == 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, l16 = lane & 15, lg = lane >> 4;
  const int rb = w & 3, cb = w >> 2;
  {
    constexpr int NL = CB * CB / ST;
    double v[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = tid + u * ST, k = e / CB, r = e % CB;
      v[u] = (k < bb && r < bb) ? q1[(long long)k * ldq + r] : 0.0;
    }
    stage_small<ST>(g2, P0);
    stage_small<ST>(r1, P1);
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = tid + u * ST;
      P2[(e / CB) * CP + (e % CB)] = v[u];
    }
    // L1's entries outside the strict lower bb x bb part are zero
    for (int e = tid; e < CB * CB; e += ST) {
      const int c = e / CB, r = e % CB;
      if (!(r > c && r < bb)) l1out[e] = 0.0;
    }
  }
  __syncthreads();
  double dmin, dmax;
  const bool ok = chol_inv_pass(P0, P3, P0, bb, smult, sd, sraw, dmin, dmax);   // R2 -> P3, R2^-1 -> P0
  __syncthreads();
  const v4d rh0 = mm_tile(P3, [&](int k, int c) { return P1[c * CP + k]; });   // R2 R1
  const v4d qt = mm_tile(P2, [&](int k, int c) { return P0[c * CP + k]; });    // Q1top R2^-1
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) P1[(16 * cb + l16) * CP + 16 * rb + acc_row<double>(lg, e)] = qt[e];
  __syncthreads();
  lu_pass(P1, P2, P3, l1out, bb, smult, s_s, sd);   // U -> P2, L1^-1 -> P3
  __syncthreads();
  upper_inv_pass(P2, P1, bb);                     // U^-1 -> P1
  __syncthreads();
  const v4d mv = mm_tile(P0, [&](int k, int c) { return P1[c * CP + k]; });   // R2^-1 U^-1
  // T = -U S L1^-T: B(k, c) = s_k L1^-1(c, k)
  const v4d tv = mm_tile(P2, [&](int k, int c) { return (k < bb ? s_s[k] : 0.0) * P3[k * CP + c]; });
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = 16 * rb + acc_row<double>(lg, e), c = 16 * cb + l16;
    m2[c * CB + r] = (r < bb && c < bb) ? mv[e] : 0.0;
    if (r < bb && c < bb) {
      tmat[c * bb + r] = (r <= c) ? -tv[e] : 0.0;
      if (r == c) tau[c] = -tv[e];
    }
    const double sr = (r < bb) ? s_s[r] : 0.0;
    rh[c * CB + r] = (r <= c && c < bb) ? sr * rh0[e] : 0.0;
  }
  // the first pass left Q1 close to orthonormal: every pivot of G2 = Q1^T Q1 near 1
  if (tid == 0 && !(ok && dmin > 0.25 && dmax < 4.0)) *flag = 0;
}

// ---- write V (rows below the top block: Q1 M2) and the top block (Rh / L1) ----
template <typename T>
__global__ __launch_bounds__(CT) void k_cq_y(int rows, T* __restrict__ x, long long ldx, int bb,
                                             const double* __restrict__ q1, long long ldq,
                                             const double* __restrict__ m2,
                                             const double* __restrict__ rh,
                                             const double* __restrict__ l1,
                                             const int* __restrict__ flag) {
  __shared__ double sx[CR * CP];
  __shared__ double sm[CB * CP];
  if (*flag == 0) return;
  const int r0 = blockIdx.x * CR;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  {
    double v[CB * CB / CT];
#pragma unroll
    for (int u = 0; u < CB * CB / CT; ++u) v[u] = m2[tid + u * CT];
    stage_chunk<double>(q1, ldq, rows, r0, bb, sx);
#pragma unroll
    for (int u = 0; u < CB * CB / CT; ++u) {
      const int e = tid + u * CT, c = e / CB, k = e % CB;
      sm[k * CP + c] = v[u];
    }
  }
  __syncthreads();
  v4d acc[RT][4];
#pragma unroll
  for (int b = 0; b < RT; ++b)
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) acc[b][tc] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < CB / 4; ++kk) {
    const int k = 4 * kk + lg;
    double av[RT];
#pragma unroll
    for (int b = 0; b < RT; ++b) av[b] = sx[(16 * RT * wave + 16 * b + l16) * CP + k];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
      const double bv = sm[k * CP + 16 * tc + l16];
#pragma unroll
      for (int b = 0; b < RT; ++b) acc[b][tc] = mfma_f64(av[b], bv, acc[b][tc]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < RT; ++b)
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = 16 * RT * wave + 16 * b + acc_row<double>(lg, e);
        sx[rr * CP + 16 * tc + l16] = acc[b][tc][e];
      }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < CR * CB / CT; ++u) {
    const int e = tid + u * CT;
    const int c = e / CR, rr = e % CR;
    const int r = r0 + rr;
    if (r < rows && c < bb) {
      double v;
      if (r >= bb)
        v = sx[rr * CP + c];
      else
        v = (r <= c) ? rh[c * CB + r] : l1[c * CB + r];
      x[(long long)c * ldx + r] = (T)v;
    }
  }
}

// ---- blocks wider than CB: two CB-wide halves and the T of the whole block ----

// Partial C = A^T B (CB x CB) of a CR-row chunk on FP64 MFMA.  A and B have
// na, nb <= CB columns; a nonnegative adiag/bdiag makes that operand the unit
// lower trapezoid whose diagonal starts at that row (entries above it zero).
template <typename T>
__global__ __launch_bounds__(CT) void k_cq_cross(int rows, const T* __restrict__ A, long long lda,
                                                 int na, int adiag, const T* __restrict__ B,
                                                 long long ldb, int nb, int bdiag,
                                                 double* __restrict__ part) {
  __shared__ double sa[CR * CP];
  __shared__ double sb[CR * CP];
  const int r0 = blockIdx.x * CR;
  for (int e = threadIdx.x; e < CR * CB; e += CT) {
    const int c = e / CR, rr = e % CR, r = r0 + rr;
    const bool in = r < rows;
    double va = 0.0, vb = 0.0;
    if (in && c < na) {
      const double v = (double)A[(long long)c * lda + r];
      va = (adiag < 0 || r - adiag > c) ? v : (r - adiag == c ? 1.0 : 0.0);
    }
    if (in && c < nb) {
      const double v = (double)B[(long long)c * ldb + r];
      vb = (bdiag < 0 || r - bdiag > c) ? v : (r - bdiag == c ? 1.0 : 0.0);
    }
    sa[rr * CP + c] = va;
    sb[rr * CP + c] = vb;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < CR / 4; ++kk) {
    const int r = 4 * kk + lg;
    const double av = sa[r * CP + 16 * wave + l16];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = mfma_f64(av, sb[r * CP + 16 * t + l16], acc[t]);
  }
  double* out = part + (size_t)blockIdx.x * CB * CB;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      out[(16 * t + l16) * CB + 16 * wave + acc_row<double>(lg, e)] = acc[t][e];
}

// W' = T1^T Y (T1: CB x CB upper, ld CB; Y: CB x nb, ld CB; W': ld CB).
__global__ __launch_bounds__(CT) void k_cq_tty(int nb, const double* __restrict__ t1,
                                               const double* __restrict__ y,
                                               double* __restrict__ w) {
  for (int e = threadIdx.x; e < CB * nb; e += CT) {
    const int c = e / CB, q = e % CB;
    double acc = 0.0;
    for (int p = 0; p <= q; ++p) acc += t1[q * CB + p] * y[c * CB + p];
    w[c * CB + q] = acc;
  }
}

// T of the whole block (bb = CB + nb, ld bb): [[T1, -T1 Z T2], [0, T2]] with
// Z = V1^T V2 (CB x nb, ld CB), T1 (ld CB), T2 (nb x nb, ld nb).
__global__ __launch_bounds__(CT) void k_cq_tcombine(int nb, const double* __restrict__ t1,
                                                    const double* __restrict__ t2,
                                                    const double* __restrict__ z,
                                                    double* __restrict__ t) {
  __shared__ double sm[CB * CB];   // Z T2
  const int bb = CB + nb;
  for (int e = threadIdx.x; e < CB * nb; e += CT) {
    const int c = e / CB, p = e % CB;
    double acc = 0.0;
    for (int q = 0; q <= c; ++q) acc += z[q * CB + p] * t2[c * nb + q];
    sm[c * CB + p] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < bb * bb; e += CT) {
    const int c = e / bb, r = e % bb;
    double v = 0.0;
    if (c < CB) {
      v = (r < CB) ? t1[c * CB + r] : 0.0;
    } else if (r >= CB) {
      v = t2[(c - CB) * nb + (r - CB)];
    } else {
      double acc = 0.0;
      for (int s2 = r; s2 < CB; ++s2) acc += t1[s2 * CB + r] * sm[(c - CB) * CB + s2];
      v = -acc;
    }
    t[e] = v;
  }
}

}  // namespace

size_t panel_cq_doubles(int rows) {
  const size_t nchunk = (size_t)(rows + CR - 1) / CR;
  return (size_t)rows * CB + nchunk * CB * CB + 8 * (size_t)CB * CB + 64;
}

bool panel_cq_applicable(int m, int i, int bb) {
  return bb >= 1 && bb <= CB && (m - i) >= 2 * bb;
}

// Runs the CholeskyQR2 path; *flag (device) ends 1 if it produced the
// factorization, 0 if the stepwise kernel must factor the updated panel.
template <typename T>
int launch_panel_cq(hipStream_t s, int m, T* a, long long lda, int i, int bb, int bbp,
                    const double* wp, long long ldw, double* tau, double* tmat, double* scratch,
                    int* flag) {
  const int rows = m - i;
  const int nchunk = (rows + CR - 1) / CR;
  double* q1 = scratch;
  double* part = q1 + (size_t)rows * CB;
  double* g = part + (size_t)nchunk * CB * CB;
  double* r1 = g + CB * CB;
  double* r1inv = r1 + CB * CB;
  double* m2 = r1inv + CB * CB;
  double* rh = m2 + CB * CB;
  double* l1 = rh + CB * CB;
  T* x = a + (long long)i * lda + i;
  if (bbp > 0) {
    const int prow = m - (i - bbp);
    hipLaunchKernelGGL(k_cq_pend<T>, dim3((prow + PR - 1) / PR), dim3(CT), 0, s, m, a, lda, i, 0,
                       bb, bbp, wp, ldw);
  }
  hipLaunchKernelGGL(k_cq_gram<T>, dim3(nchunk), dim3(CT), 0, s, rows, (const T*)x, lda, bb, part,
                     (const int*)nullptr);
  hipLaunchKernelGGL(k_cq_sum, dim3(CB * CB / 64), dim3(CT), 0, s, nchunk, (const double*)part, g,
                     (const int*)nullptr);
  hipLaunchKernelGGL(k_cq_chol1, dim3(1), dim3(ST), 0, s, bb, (const double*)g, r1, r1inv, flag);
  hipLaunchKernelGGL(k_cq_q1<T>, dim3(nchunk), dim3(CT), 0, s, rows, (const T*)x, lda, bb,
                     (const double*)r1inv, q1, (long long)rows, part, (const int*)flag);
  hipLaunchKernelGGL(k_cq_sum, dim3(CB * CB / 64), dim3(CT), 0, s, nchunk, (const double*)part, g,
                     (const int*)flag);
  hipLaunchKernelGGL(k_cq_small, dim3(1), dim3(ST), 0, s, bb, (const double*)g,
                     (const double*)r1, (const double*)q1, (long long)rows, m2, rh, l1, tmat,
                     tau + i, flag);
  hipLaunchKernelGGL(k_cq_y<T>, dim3(nchunk), dim3(CT), 0, s, rows, x, lda, bb,
                     (const double*)q1, (long long)rows, (const double*)m2, (const double*)rh,
                     (const double*)l1, (const int*)flag);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_panel_cq<double>(hipStream_t, int, double*, long long, int, int, int,
                                     const double*, long long, double*, double*, double*, int*);
template int launch_panel_cq<float>(hipStream_t, int, float*, long long, int, int, int,
                                    const double*, long long, double*, double*, double*, int*);

template <typename T>
int launch_cq_pend(hipStream_t s, int m, T* a, long long lda, int i, int coff, int nc, int bbp,
                   const double* wp, long long ldw) {
  if (nc < 1 || nc > CB || bbp < 1 || bbp > CB) return RQ_ERR_LIMIT;
  const int prow = m - (i - bbp);
  hipLaunchKernelGGL(k_cq_pend<T>, dim3((prow + PR - 1) / PR), dim3(CT), 0, s, m, a, lda, i, coff,
                     nc, bbp, wp, ldw);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_cq_pend<double>(hipStream_t, int, double*, long long, int, int, int, int,
                                    const double*, long long);
template int launch_cq_pend<float>(hipStream_t, int, float*, long long, int, int, int, int,
                                   const double*, long long);

size_t cq_wide_doubles(int rows) {
  const size_t nchunk = (size_t)(rows + CR - 1) / CR;
  return nchunk * CB * CB + 5 * (size_t)CB * CB;
}

// C = A^T B over `rows` rows (see k_cq_cross), summed in a fixed order into c
// (CB x CB doubles, ld CB); part: cq_wide scratch.
template <typename T>
int launch_cq_cross(hipStream_t s, int rows, const T* A, long long lda, int na, int adiag,
                    const T* B, long long ldb, int nb, int bdiag, double* part, double* c) {
  const int nchunk = (rows + CR - 1) / CR;
  hipLaunchKernelGGL(k_cq_cross<T>, dim3(nchunk), dim3(CT), 0, s, rows, A, lda, na, adiag, B, ldb,
                     nb, bdiag, part);
  hipLaunchKernelGGL(k_cq_sum, dim3(CB * CB / 64), dim3(CT), 0, s, nchunk, (const double*)part, c,
                     (const int*)nullptr);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_cq_cross<double>(hipStream_t, int, const double*, long long, int, int,
                                     const double*, long long, int, int, double*, double*);
template int launch_cq_cross<float>(hipStream_t, int, const float*, long long, int, int,
                                    const float*, long long, int, int, double*, double*);

int launch_cq_tty(hipStream_t s, int nb, const double* t1, const double* y, double* w) {
  hipLaunchKernelGGL(k_cq_tty, dim3(1), dim3(CT), 0, s, nb, t1, y, w);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

int launch_cq_tcombine(hipStream_t s, int nb, const double* t1, const double* t2, const double* z,
                       double* t) {
  hipLaunchKernelGGL(k_cq_tcombine, dim3(1), dim3(CT), 0, s, nb, t1, t2, z, t);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

}  // namespace rq
