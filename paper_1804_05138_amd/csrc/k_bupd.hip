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
// One workgroup per 64 columns.  The generic form (blocks wider than 64): lane
// = column, the four waves split the rows of every triangular product, the
// triangular solve runs in wave 0.
#include "internal.h"

namespace rq {
namespace {

constexpr int BT = 256;

template <typename T>
__global__ __launch_bounds__(BT) void k_bupdate(int m, const T* __restrict__ a, long long lda,
                                                int i, int bb, const double* __restrict__ tm,
                                                const T* __restrict__ wpart, int nsplit,
                                                double* __restrict__ wp, long long ldw,
                                                double* __restrict__ bsk, long long ldb, int c0,
                                                int ncols, const int* __restrict__ info) {
  __shared__ double v0[MAX_B * 64];
  __shared__ double v1[MAX_B * 64];
  const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int cl = blockIdx.x * 64 + lane;  // column index relative to c0
  const bool ok = cl < ncols;
  const int col = c0 + cl;

  // W(:, c) = sum of the split partials
  for (int q = part; q < bb; q += 4) {
    double s = 0.0;
    if (ok)
      for (int sp = 0; sp < nsplit; ++sp) s += (double)wpart[((long long)sp * ncols + cl) * bb + q];
    v0[q * 64 + lane] = s;
  }
  __syncthreads();
  // W' = T^T W   (T upper triangular, column-major bb x bb)
  for (int r = part; r < bb; r += 4) {
    double s = 0.0;
    for (int q = 0; q <= r; ++q) s += tm[r * bb + q] * v0[q * 64 + lane];
    v1[r * 64 + lane] = s;
    if (ok) wp[(long long)cl * ldw + r] = s;
  }
  __syncthreads();
  // no sketch (frozen pivots), or no more sketch updates after a zero pivot
  if (bsk == nullptr || *info != 0) return;
  // R12 = A(i:i+bb, col) - V11 W'
  for (int r = part; r < bb; r += 4) {
    double s = ok ? (double)a[(long long)col * lda + i + r] - v1[r * 64 + lane] : 0.0;
    for (int q = 0; q < r; ++q) s -= (double)a[(long long)(i + q) * lda + i + r] * v1[q * 64 + lane];
    v0[r * 64 + lane] = s;
  }
  __syncthreads();
  // X = R11^{-1} R12 (back substitution), into v1
  if (part == 0) {
    for (int r = bb - 1; r >= 0; --r) {
      double s = v0[r * 64 + lane];
      for (int q = r + 1; q < bb; ++q)
        s -= (double)a[(long long)(i + q) * lda + i + r] * v1[q * 64 + lane];
      v1[r * 64 + lane] = s / (double)a[(long long)(i + r) * lda + i + r];
    }
  }
  __syncthreads();
  // B(0:bb, col) -= Rhat11 X
  if (ok) {
    for (int r = part; r < bb; r += 4) {
      double s = 0.0;
      for (int q = r; q < bb; ++q) s += bsk[(long long)(i + q) * ldb + r] * v1[q * 64 + lane];
      bsk[(long long)col * ldb + r] -= s;
    }
  }
}


// Staged form for block widths up to 64 (the default): every global access is
// coalesced (column-major tiles move through LDS with a padded row pitch); the
// three 64 x 64 x 64 products (W' = T^T W, V11 W', Rhat11 X) run on FP64 MFMA
// from LDS (each wave a 16-row strip of the result), and the triangular solve
// X = R11^-1 R12 keeps each column in registers of one lane of wave 0, so its
// dependent chain never waits on memory.
constexpr int SB = 64;        // largest block width of the staged form
constexpr int CW = 64;        // columns per workgroup
constexpr int SP = CW + 1;    // LDS row pitch of the column tiles
constexpr int AP = SB + 1;    // LDS pitch of the bb x bb blocks

template <typename T>
__global__ __launch_bounds__(BT) void k_bupdate_s(int m, const T* __restrict__ a, long long lda,
                                                  int i, int bb, const double* __restrict__ tm,
                                                  const T* __restrict__ wpart, int nsplit,
                                                  double* __restrict__ wp, long long ldw,
                                                  double* __restrict__ bsk, long long ldb,
                                                  int c0, int ncols, const int* __restrict__ info) {
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

  // C(m, n) = sum_k L(m, k) R(k, n) for this wave's rows 16 wave .. +15 and all
  // 64 columns: acc[t][e] = C(16 wave + acc_row(lg, e), 16 t + l16)
  auto mm = [&](auto lel, const double* rm, v4d (&acc)[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < SB / 4; ++kk) {
      const int k = 4 * kk + lg;
      const double av = lel(16 * wave + l16, k);
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = mfma_f64(av, rm[k * SP + 16 * t + l16], acc[t]);
    }
  };

  for (int e = tid; e < SB * SB; e += BT) {
    const int r = e / SB, q = e % SB;
    const bool in = r < bb && q < bb;
    sT[r * AP + q] = in ? tm[r * bb + q] : 0.0;
    sA[r * AP + q] = in ? (double)a[(long long)(i + r) * lda + i + q] : 0.0;  // column r, row q
  }
  // W(:, cb + c) = sum of the split partials (contiguous per column)
  for (int e = tid; e < SB * CW; e += BT) {
    const int c = e / SB, q = e % SB;
    double s = 0.0;
    if (c < nc && q < bb)
      for (int sp = 0; sp < nsplit; ++sp)
        s += (double)wpart[((long long)sp * ncols + cb + c) * bb + q];
    sW[q * SP + c] = s;
  }
  __syncthreads();
  v4d acc[4];
  // W' = T^T W
  mm([&](int r, int k) { return sT[r * AP + k]; }, sW, acc);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) sX[(16 * wave + acc_row<double>(lg, e)) * SP + 16 * t + l16] = acc[t][e];
  __syncthreads();
  for (int e = tid; e < nc * bb; e += BT) {
    const int c = e / bb, r = e % bb;
    wp[(long long)(cb + c) * ldw + r] = sX[r * SP + c];
  }
  if (bsk == nullptr || *info != 0) return;
  // Rhat11 = triu(B(0:bb, i:i+bb)) into sT; R12 starts as A(i:i+bb, col)
  for (int e = tid; e < SB * SB; e += BT) {
    const int r = e / SB, q = e % SB;   // column r, row q
    sT[r * AP + q] = (q <= r && r < bb) ? bsk[(long long)(i + r) * ldb + q] : 0.0;
  }
  for (int e = tid; e < SB * CW; e += BT) {
    const int c = e / SB, r = e % SB;
    sW[r * SP + c] = (c < nc && r < bb) ? (double)a[(long long)(c0 + cb + c) * lda + i + r] : 0.0;
  }
  if (tid < SB) sInv[tid] = (tid < bb) ? 1.0 / sA[tid * AP + tid] : 1.0;
  __syncthreads();
  // R12 = A(i:i+bb, col) - V11 W'   (V11 unit lower: A(i + r, i + q), q < r)
  mm([&](int r, int k) { return (k < r) ? sA[k * AP + r] : 0.0; }, sX, acc);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * wave + acc_row<double>(lg, e), c = 16 * t + l16;
      sW[r * SP + c] = sW[r * SP + c] - sX[r * SP + c] - acc[t][e];
    }
  __syncthreads();
  // X = R11^{-1} R12: back substitution, column `lane` in registers of wave 0
  if (wave == 0) {
    double y[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) y[r] = sW[r * SP + lane];
#pragma unroll
    for (int r = SB - 1; r >= 0; --r) {
      if (r < bb) {
        const double x = y[r] * sInv[r];
        y[r] = x;
#pragma unroll
        for (int q = 0; q < r; ++q) y[q] -= sA[r * AP + q] * x;
      }
    }
#pragma unroll
    for (int r = 0; r < SB; ++r) sX[r * SP + lane] = (r < bb) ? y[r] : 0.0;
  }
  __syncthreads();
  // delta = Rhat11 X, then B(0:bb, col) -= delta
  mm([&](int r, int k) { return (k >= r) ? sT[k * AP + r] : 0.0; }, sX, acc);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) sW[(16 * wave + acc_row<double>(lg, e)) * SP + 16 * t + l16] = acc[t][e];
  __syncthreads();
  for (int e = tid; e < nc * bb; e += BT) {
    const int c = e / bb, r = e % bb;
    bsk[(long long)(c0 + cb + c) * ldb + r] -= sW[r * SP + c];
  }
  (void)m;
}

}  // namespace

template <typename T>
int launch_bupdate(hipStream_t s, int m, const T* a, long long lda, int i, int bb,
                   const double* t, const T* wpart, int nsplit, double* wp, long long ldw,
                   double* bsk, long long ldb, int c0, int ncols, const int* info) {
  if (ncols <= 0) return RQ_OK;
  if (bb > MAX_B) return RQ_ERR_LIMIT;
  if (bb <= SB) {
    const size_t shmem = (2 * (size_t)SB * AP + 2 * (size_t)SB * SP + SB) * sizeof(double);
    RQ_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bupdate_s<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    hipLaunchKernelGGL(k_bupdate_s<T>, dim3((ncols + CW - 1) / CW), dim3(BT), shmem, s, m, a, lda,
                       i, bb, t, wpart, nsplit, wp, ldw, bsk, ldb, c0, ncols, info);
    RQ_HIP_CHECK(hipGetLastError());
    return RQ_OK;
  }
  hipLaunchKernelGGL(k_bupdate<T>, dim3((ncols + 63) / 64), dim3(BT), 0, s, m, a, lda, i, bb, t,
                     wpart, nsplit, wp, ldw, bsk, ldb, c0, ncols, info);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_bupdate<double>(hipStream_t, int, const double*, long long, int, int,
                                    const double*, const double*, int, double*, long long,
                                    double*, long long, int, int, const int*);
template int launch_bupdate<float>(hipStream_t, int, const float*, long long, int, int,
                                   const double*, const float*, int, double*, long long, double*,
                                   long long, int, int, const int*);

}  // namespace rq
