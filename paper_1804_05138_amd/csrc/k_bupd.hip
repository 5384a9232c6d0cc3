// Sample update of Alg. 2 with updating formula (1) of Section III-B:
//     B(0:b, c) <- B(0:b, c) - Rhat11 R11^{-1} R12(:, c)
// for every trailing column c, where Rhat11 = triu(B(0:b, i:i+b)) is the top
// of the QRCP-transformed sketch and R11, R12 are the new rows of R.
//
// The kernel also finishes the block-reflector factor for the trailing pass:
// from the split partial sums of W = V^T A2 it forms W' = T^T W (stored for
// the next pass and the next panel), and R12 = A2(0:b, c) - V11 W'(:, c) is
// obtained from W' directly (V11 = unit lower top block of V), so the sample
// update does not wait for the trailing pass.
//
// Two forms: blocks up to 64 wide (one workgroup per 64 columns) and blocks
// 65..128 wide (2 x 2 quadrants, one workgroup per 32 columns).
#include "internal.h"

namespace rq {
namespace {

constexpr int BT = 256;    // threads of the quadrant form
constexpr int BTS = 512;   // threads of the staged form (eight waves: two per SIMD)

// Staged form for block widths up to 64 (the default): every global access is
// coalesced (column-major tiles move through LDS with a padded row pitch); the
// three 64 x 64 x 64 products (W' = T^T W, V11 W', Rhat11 X) run on FP64 MFMA
// from LDS (each of eight waves a 16 x 32 tile of the result), and the
// triangular solve X = R11^-1 R12 keeps each column in registers of eight
// lanes of one wave (8 columns per wave), so its dependent chain never waits
// on memory.
constexpr int SB = 64;        // largest block width of the staged form
constexpr int CW = 64;        // columns per workgroup
constexpr int SP = CW + 1;    // LDS row pitch of the column tiles
constexpr int AP = SB + 1;    // LDS pitch of the bb x bb blocks

template <typename T>
__global__ __launch_bounds__(BTS) void k_bupdate_s(int m, const T* a, long long lda,
                                                  int i, int bb, const double* __restrict__ tm,
                                                  const T* __restrict__ wpart, int nsplit,
                                                  double* __restrict__ wp, long long ldw,
                                                  double* __restrict__ bsk, long long ldb,
                                                  int c0, int ncols, const int* __restrict__ info,
                                                  T* r12out, long long pstride) {
  extern __shared__ double smem[];
  double* sT = smem;                 // T(q, r) at sT[r * AP + q]; later Rhat11(q, r)
  double* sA = sT + SB * AP;         // A(i + r, i + c) at sA[c * AP + r]
  double* sW = sA + SB * AP;         // [q][col]: W, then R12, then the B delta
  double* sX = sW + SB * SP;         // [q][col]: W', then X
  double* sInv = sX + SB * SP;       // 1 / R11(r, r)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, l16 = lane & 15, lg = lane >> 4;
  const int cb = blockIdx.x * CW;                 // first column (relative to c0)
  const int nc = min(CW, ncols - cb);             // columns of this workgroup

  // C(m, n) = sum_k L(m, k) R(k, n) for this wave's rows mr .. mr + 15 and
  // columns nb .. nb + 31 (eight waves: four row strips times two column
  // halves): acc[t][e] = C(mr + acc_row(lg, e), nb + 16 t + l16)
  const int mr = 16 * (wave & 3), nb = 32 * (wave >> 2);
  auto mm = [&](auto lel, const double* rm, v4d (&acc)[2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < SB / 4; ++kk) {
      const int k = 4 * kk + lg;
      const double av = lel(mr + l16, k);
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[t] = mfma_f64(av, rm[k * SP + nb + 16 * t + l16], acc[t]);
    }
  };

  // (column, row) of element e of a bb-row column tile: shifts for the usual
  // bb = 64 (a uniform branch), a division otherwise
  auto split_e = [&](int e, int& c, int& r) {
    if (bb == SB) {
      c = e >> 6;
      r = e & (SB - 1);
    } else {
      c = e / bb;
      r = e % bb;
    }
  };
  // Every global read of the kernel is issued up front from clamped (always
  // valid) addresses and masked afterwards, so the reads cost one memory round
  // trip per split of W instead of one per element.
  constexpr int NE = SB * SB / BTS;   // elements of a bb x bb block per thread
  constexpr int NC = SB * CW / BTS;   // elements of a bb x CW column tile per thread
  static_assert(NE * BTS == SB * SB && NC * BTS == SB * CW, "tiles split evenly over the threads");
  const bool upd = bsk != nullptr;   // uniform: the sample update runs (not frozen pivots)
  double tv[NE], av[NE], rv[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * BTS, r = e / SB, q = e % SB;   // column r, row q
    const bool in = r < bb && q < bb;
    const int rs = in ? r : 0, qs = in ? q : 0;
    tv[u] = tm[rs * bb + qs];
    av[u] = (double)a[(long long)(i + rs) * lda + i + qs];
    rv[u] = upd ? bsk[(long long)(i + rs) * ldb + qs] : 0.0;
  }
  double a12[NC], bo[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int e = tid + u * BTS;
    const int c = e / SB, r = e % SB;     // R12 start: A(i + r, c0 + cb + c)
    const bool ok = c < nc && r < bb;
    a12[u] = (double)a[(long long)(c0 + cb + (ok ? c : 0)) * lda + i + (ok ? r : 0)];
    int c2, r2;                           // B(r2, c0 + cb + c2), updated at the end
    split_e(e, c2, r2);
    const bool ok2 = e < nc * bb;
    bo[u] = upd ? bsk[(long long)(c0 + cb + (ok2 ? c2 : 0)) * ldb + (ok2 ? r2 : 0)] : 0.0;
  }
  // W(:, cb + c) = sum of the split partials, in split order
  double ws[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) ws[u] = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) {
    double pv[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int e = tid + u * BTS, c = e / SB, q = e % SB;
      const bool ok = c < nc && q < bb;
      pv[u] = (double)wpart[((long long)sp * pstride + cb + (ok ? c : 0)) * bb + (ok ? q : 0)];
    }
#pragma unroll
    for (int u = 0; u < NC; ++u) ws[u] += pv[u];
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * BTS, r = e / SB, q = e % SB;
    const bool in = r < bb && q < bb;
    sT[r * AP + q] = in ? tv[u] : 0.0;
    sA[r * AP + q] = in ? av[u] : 0.0;  // column r, row q
  }
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int e = tid + u * BTS, c = e / SB, q = e % SB;
    sW[q * SP + c] = (c < nc && q < bb) ? ws[u] : 0.0;
  }
  __syncthreads();
  v4d acc[2];
  // W' = T^T W
  mm([&](int r, int k) { return sT[r * AP + k]; }, sW, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) sX[(mr + acc_row<double>(lg, e)) * SP + nb + 16 * t + l16] = acc[t][e];
  __syncthreads();
  for (int e = tid; e < nc * bb; e += BTS) {
    int c, r;
    split_e(e, c, r);
    wp[(long long)(cb + c) * ldw + r] = sX[r * SP + c];
  }
  // uniform: the sample update runs (sketch given, pivoting not stopped)
  const bool sample = upd && *info == 0;
  if (!sample && r12out == nullptr) return;
  // Rhat11 = triu(B(0:bb, i:i+bb)) into sT; R12 starts as A(i:i+bb, col)
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * BTS, r = e / SB, q = e % SB;   // column r, row q
    sT[r * AP + q] = (q <= r && r < bb) ? rv[u] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int e = tid + u * BTS, c = e / SB, r = e % SB;
    sW[r * SP + c] = (c < nc && r < bb) ? a12[u] : 0.0;
  }
  if (tid < SB) sInv[tid] = (tid < bb) ? 1.0 / sA[tid * AP + tid] : 1.0;
  __syncthreads();
  // R12 = A(i:i+bb, col) - V11 W'   (V11 unit lower: A(i + r, i + q), q < r)
  mm([&](int r, int k) { return (k < r) ? sA[k * AP + r] : 0.0; }, sX, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = mr + acc_row<double>(lg, e), c = nb + 16 * t + l16;
      sW[r * SP + c] = sW[r * SP + c] - sX[r * SP + c] - acc[t][e];
    }
  __syncthreads();
  // the final rows R12 = A(i:i+bb, col) (left-looking schedule: A2 itself is
  // not updated until the end)
  if (r12out != nullptr)
    for (int e = tid; e < nc * bb; e += BTS) {
      int c, r;
      split_e(e, c, r);
      r12out[(long long)(c0 + cb + c) * lda + i + r] = (T)sW[r * SP + c];
    }
  if (!sample) return;
  // X = R11^{-1} R12: back substitution.  Wave w solves columns 8w .. 8w+7;
  // lane (g, c) holds rows g, g + 8, ..., g + 56 of column 8w + c in
  // registers.  Step r: the lanes holding row r form x_r = y_r / R11(r, r),
  // pass it to the other seven lanes of their column, and every lane takes
  // R11(q, r) x_r off its rows q < r (each entry sees the same operations in
  // the same order as a column solved by one lane).
  {
    const int c8 = lane & 7, g8 = lane >> 3;
    const int c = 8 * wave + c8;
    double y[SB / 8];
#pragma unroll
    for (int u = 0; u < SB / 8; ++u) y[u] = sW[(8 * u + g8) * SP + c];
#pragma unroll
    for (int r = SB - 1; r >= 0; --r) {
      if (r < bb) {
        const int gr = r & 7, ur = r >> 3;
        const double xo = y[ur] * sInv[r];
        const double x = __shfl(xo, c8 + 8 * gr, 64);
        y[ur] = (g8 == gr) ? x : y[ur];
#pragma unroll
        for (int u = 0; u <= ur; ++u) {
          const int q = 8 * u + g8;
          const double rq = sA[r * AP + (q < r ? q : 0)];
          y[u] = (q < r) ? fma(-rq, x, y[u]) : y[u];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SB / 8; ++u) {
      const int q = 8 * u + g8;
      sX[q * SP + c] = (q < bb) ? y[u] : 0.0;
    }
  }
  __syncthreads();
  // delta = Rhat11 X, then B(0:bb, col) -= delta
  mm([&](int r, int k) { return (k >= r) ? sT[k * AP + r] : 0.0; }, sX, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) sW[(mr + acc_row<double>(lg, e)) * SP + nb + 16 * t + l16] = acc[t][e];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int e = tid + u * BTS;
    int c, r;
    split_e(e, c, r);
    if (e < nc * bb) bsk[(long long)(c0 + cb + c) * ldb + r] = bo[u] - sW[r * SP + c];
  }
  (void)m;
}


// Quadrant form for block widths 65..128: the bb x bb blocks (T, V11, R11,
// Rhat11) are split into 64 x 64 quadrants staged in LDS one or two at a
// time, so every product is a sum of 64 x 64 x 32 MFMA products and the
// triangular solve runs as two 64-row solves in registers joined by one
// product:  X1 = R11[1,1]^-1 R12[1],  X0 = R11[0,0]^-1 (R12[0] - R11[0,1] X1).
// 32 columns per workgroup keep the two quadrants and the two column tiles
// within one CU's LDS.
constexpr int QB = 64;         // quadrant size
constexpr int QW = 32;         // columns per workgroup
constexpr int QP = QW + 1;     // LDS row pitch of the column tiles
constexpr int QAP = QB + 1;    // LDS pitch of a quadrant

template <typename T>
__global__ __launch_bounds__(BT) void k_bupdate_q(int m, const T* a, long long lda,
                                                  int i, int bb, const double* __restrict__ tm,
                                                  const T* __restrict__ wpart, int nsplit,
                                                  double* __restrict__ wp, long long ldw,
                                                  double* __restrict__ bsk, long long ldb,
                                                  int c0, int ncols, const int* __restrict__ info,
                                                  T* r12out, long long pstride) {
  extern __shared__ double smem[];
  double* sQ = smem;                 // quadrant: element (row r, column k) at sQ[k * QAP + r]
  double* sQ2 = sQ + QB * QAP;       // second quadrant, same layout
  double* sW = sQ2 + QB * QAP;       // [q][col], 128 rows: W, then R12, then the B delta
  double* sX = sW + 2 * QB * QP;     // [q][col], 128 rows: W', then X
  double* sInv = sX + 2 * QB * QP;   // 1 / R11(r, r), 128 entries
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, l16 = lane & 15, lg = lane >> 4;
  const int cb = blockIdx.x * QW;                 // first column (relative to c0)
  const int nc = min(QW, ncols - cb);             // columns of this workgroup

  // Stage quadrant (gr, gc) of a bb x bb matrix: element (r, k) is
  // get(64 gr + r, 64 gc + k), zero outside the block width.
  // All reads of a thread are issued before any LDS store (clamped addresses,
  // masked afterwards), so a stage costs one memory round trip.
  constexpr int NS = QB * QB / BT;
  static_assert(NS * BT == QB * QB, "quadrant splits evenly over the threads");
  auto stage = [&](double* dst, int gr, int gc, auto get) {
    double v[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + u * BT, k = e / QB, r = e % QB;
      const int gi = QB * gr + r, gj = QB * gc + k;
      const bool ok = gi < bb && gj < bb;
      v[u] = get(ok ? gi : 0, ok ? gj : 0);
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + u * BT, k = e / QB, r = e % QB;
      const int gi = QB * gr + r, gj = QB * gc + k;
      dst[k * QAP + r] = (gi < bb && gj < bb) ? v[u] : 0.0;
    }
  };
  // acc += L(16 wave + row, :) x rm(0:64, 0:32) for a quadrant L in LDS;
  // acc[t][e] = C(16 wave + acc_row(lg, e), 16 t + l16); `keep(r, k)` masks L.
  auto mmq = [&](const double* q, auto keep, const double* rm, v4d (&acc)[2]) {
#pragma unroll 4
    for (int kk = 0; kk < QB / 4; ++kk) {
      const int k = 4 * kk + lg, r = 16 * wave + l16;
      const double av = keep(r, k) ? q[k * QAP + r] : 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[t] = mfma_f64(av, rm[k * QP + 16 * t + l16], acc[t]);
    }
  };
  auto all = [](int, int) { return true; };
  auto zero = [](v4d (&acc)[2]) {
    acc[0] = v4d{0.0, 0.0, 0.0, 0.0};
    acc[1] = v4d{0.0, 0.0, 0.0, 0.0};
  };
  auto tget = [&](int r, int k) { return tm[r * bb + k]; };  // T^T(r, k) = T(k, r)

  // W(:, cb + c) = sum of the split partials, in split order (every read of a
  // split in flight together)
  constexpr int NCQ = 2 * QB * QW / BT;
  static_assert(NCQ * BT == 2 * QB * QW, "column tile splits evenly over the threads");
  {
    double ws[NCQ];
#pragma unroll
    for (int u = 0; u < NCQ; ++u) ws[u] = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) {
      double pv[NCQ];
#pragma unroll
      for (int u = 0; u < NCQ; ++u) {
        const int e = tid + u * BT, c = e / (2 * QB), q = e % (2 * QB);
        const bool ok = c < nc && q < bb;
        pv[u] = (double)wpart[((long long)sp * pstride + cb + (ok ? c : 0)) * bb + (ok ? q : 0)];
      }
#pragma unroll
      for (int u = 0; u < NCQ; ++u) ws[u] += pv[u];
    }
#pragma unroll
    for (int u = 0; u < NCQ; ++u) {
      const int e = tid + u * BT, c = e / (2 * QB), q = e % (2 * QB);
      sW[q * QP + c] = (c < nc && q < bb) ? ws[u] : 0.0;
    }
  }
  // W' = T^T W (T^T lower triangular): W'[0] = T00^T W[0],
  // W'[1] = T01^T W[0] + T11^T W[1]
  stage(sQ, 0, 0, tget);
  __syncthreads();
  v4d acc[2];
  zero(acc);
  mmq(sQ, [](int r, int k) { return k <= r; }, sW, acc);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) sX[(16 * wave + acc_row<double>(lg, e)) * QP + 16 * t + l16] = acc[t][e];
  stage(sQ, 1, 0, tget);
  stage(sQ2, 1, 1, tget);
  __syncthreads();
  zero(acc);
  mmq(sQ, all, sW, acc);
  mmq(sQ2, [](int r, int k) { return k <= r; }, sW + QB * QP, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      sX[(QB + 16 * wave + acc_row<double>(lg, e)) * QP + 16 * t + l16] = acc[t][e];
  __syncthreads();
  for (int e = tid; e < nc * bb; e += BT) {
    const int c = e / bb, r = e % bb;
    wp[(long long)(cb + c) * ldw + r] = sX[r * QP + c];
  }
  const bool sample = bsk != nullptr && *info == 0;  // uniform
  if (!sample && r12out == nullptr) return;

  // R12 = A(i:i+bb, col) - V11 W'  (V11 unit lower: A(i + r, i + q), q < r)
  auto aget = [&](int r, int k) { return (double)a[(long long)(i + k) * lda + i + r]; };
  {
    double v[NCQ];
#pragma unroll
    for (int u = 0; u < NCQ; ++u) {
      const int e = tid + u * BT, c = e / (2 * QB), r = e % (2 * QB);
      const bool ok = c < nc && r < bb;
      v[u] = (double)a[(long long)(c0 + cb + (ok ? c : 0)) * lda + i + (ok ? r : 0)];
    }
#pragma unroll
    for (int u = 0; u < NCQ; ++u) {
      const int e = tid + u * BT, c = e / (2 * QB), r = e % (2 * QB);
      sW[r * QP + c] = (c < nc && r < bb) ? v[u] : 0.0;
    }
  }
  if (tid < 2 * QB) sInv[tid] = (tid < bb) ? 1.0 / aget(tid, tid) : 1.0;
  stage(sQ, 0, 0, aget);
  __syncthreads();
  // rows 0..63: V00 W'[0]
  zero(acc);
  mmq(sQ, [](int r, int k) { return k < r; }, sX, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * wave + acc_row<double>(lg, e), c = 16 * t + l16;
      sW[r * QP + c] = sW[r * QP + c] - sX[r * QP + c] - acc[t][e];
    }
  __syncthreads();
  // rows 64..127: V10 W'[0] + V11 W'[1]
  stage(sQ, 1, 0, aget);
  stage(sQ2, 1, 1, aget);
  __syncthreads();
  zero(acc);
  mmq(sQ, all, sX, acc);
  mmq(sQ2, [](int r, int k) { return k < r; }, sX + QB * QP, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = QB + 16 * wave + acc_row<double>(lg, e), c = 16 * t + l16;
      sW[r * QP + c] = sW[r * QP + c] - sX[r * QP + c] - acc[t][e];
    }
  __syncthreads();
  if (r12out != nullptr)
    for (int e = tid; e < nc * bb; e += BT) {
      const int c = e / bb, r = e % bb;
      r12out[(long long)(c0 + cb + c) * lda + i + r] = (T)sW[r * QP + c];
    }
  if (!sample) return;

  // 64-row back substitution of the rows h*64.. against the quadrant in sQ
  // (R11(64h + q, 64h + r) at sQ[r * QAP + q]), column `lane` in registers.
  auto solve = [&](int h) {
    if (wave == 0 && lane < QW) {
      const int nb = min(QB, bb - QB * h);
      double y[QB];
#pragma unroll
      for (int r = 0; r < QB; ++r) y[r] = sW[(QB * h + r) * QP + lane];
#pragma unroll
      for (int r = QB - 1; r >= 0; --r) {
        if (r < nb) {
          const double x = y[r] * sInv[QB * h + r];
          y[r] = x;
#pragma unroll
          for (int q = 0; q < r; ++q) y[q] -= sQ[r * QAP + q] * x;
        }
      }
#pragma unroll
      for (int r = 0; r < QB; ++r) sX[(QB * h + r) * QP + lane] = (r < nb) ? y[r] : 0.0;
    }
  };
  // X1 = R11[1,1]^-1 R12[1]
  stage(sQ, 1, 1, aget);
  stage(sQ2, 0, 1, aget);  // R11[0,1] for the join
  __syncthreads();
  solve(1);
  __syncthreads();
  // R12[0] -= R11[0,1] X1
  zero(acc);
  mmq(sQ2, all, sX + QB * QP, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * wave + acc_row<double>(lg, e), c = 16 * t + l16;
      sW[r * QP + c] -= acc[t][e];
    }
  __syncthreads();
  // X0 = R11[0,0]^-1 R12[0]
  stage(sQ, 0, 0, aget);
  __syncthreads();
  solve(0);
  __syncthreads();

  // delta = Rhat11 X (Rhat11 = triu(B(0:bb, i:i+bb))): rows 0..63 take
  // quadrants (0,0) and (0,1), rows 64..127 quadrant (1,1)
  auto bget = [&](int r, int k) { return bsk[(long long)(i + k) * ldb + r]; };
  stage(sQ, 0, 0, bget);
  stage(sQ2, 0, 1, bget);
  __syncthreads();
  zero(acc);
  mmq(sQ, [](int r, int k) { return k >= r; }, sX, acc);
  mmq(sQ2, all, sX + QB * QP, acc);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) sW[(16 * wave + acc_row<double>(lg, e)) * QP + 16 * t + l16] = acc[t][e];
  stage(sQ, 1, 1, bget);
  __syncthreads();
  zero(acc);
  mmq(sQ, [](int r, int k) { return k >= r; }, sX + QB * QP, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      sW[(QB + 16 * wave + acc_row<double>(lg, e)) * QP + 16 * t + l16] = acc[t][e];
  __syncthreads();
  for (int e = tid; e < nc * bb; e += BT) {
    const int c = e / bb, r = e % bb;
    bsk[(long long)(c0 + cb + c) * ldb + r] -= sW[r * QP + c];
  }
  (void)m;
}

}  // namespace

template <typename T>
int launch_bupdate(hipStream_t s, int m, const T* a, long long lda, int i, int bb,
                   const double* t, const T* wpart, int nsplit, double* wp, long long ldw,
                   double* bsk, long long ldb, int c0, int ncols, const int* info, T* r12out,
                   long long pstride) {
  if (ncols <= 0) return RQ_OK;
  if (pstride <= 0) pstride = ncols;
  if (bb > MAX_B) return RQ_ERR_LIMIT;
  if (bb <= SB) {
    const size_t shmem = (2 * (size_t)SB * AP + 2 * (size_t)SB * SP + SB) * sizeof(double);
    RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bupdate_s<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    hipLaunchKernelGGL(k_bupdate_s<T>, dim3((ncols + CW - 1) / CW), dim3(BTS), shmem, s, m, a, lda,
                       i, bb, t, wpart, nsplit, wp, ldw, bsk, ldb, c0, ncols, info, r12out, pstride);
    RQ_HIP_CHECK(hipGetLastError());
    return RQ_OK;
  }
  static_assert(2 * QB >= MAX_B, "the quadrant form covers every block width");
  const size_t shmem = (2 * (size_t)QB * QAP + 4 * (size_t)QB * QP + 2 * QB) * sizeof(double);
  RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bupdate_q<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(k_bupdate_q<T>, dim3((ncols + QW - 1) / QW), dim3(BT), shmem, s, m, a, lda, i,
                     bb, t, wpart, nsplit, wp, ldw, bsk, ldb, c0, ncols, info, r12out, pstride);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_bupdate<double>(hipStream_t, int, const double*, long long, int, int,
                                    const double*, const double*, int, double*, long long,
                                    double*, long long, int, int, const int*, double*, long long);
template int launch_bupdate<float>(hipStream_t, int, const float*, long long, int, int,
                                   const double*, const float*, int, double*, long long, double*,
                                   long long, int, int, const int*, float*, long long);

}  // namespace rq
