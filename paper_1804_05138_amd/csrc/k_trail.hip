// Trailing-matrix update of Alg. 2 ("A(i:m, i+b:n) <- Q~^T A(i:m, i+b:n)",
// PDLARFB in Alg. 4), fused with the first product of the next block's
// update, on FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// With the compact WY form Q~ = I - V T V^T the update is A2 -= V (T^T V^T A2).
// The factor W' = T^T V^T A2 of block i is known before this pass (it was
// accumulated by the previous pass, and it is also what the sample update
// needs), so one pass over A2 does
//     tile  <- tile - V_i W'_i(:, tile columns)            (K = b)
//     W_{i+1}(:, tile columns) += V_{i+1}^T tile            (K = tile rows)
// where V_{i+1} are the next panel's reflectors (factored before this pass).
// Each element of A2 is read and written once per block.  The updated tile
// stays in the MFMA accumulator layout (lane l, element e: row l/16 + 4e),
// which is exactly the B-operand layout the second product needs when the
// reduction index of the 4-wide chunk e is taken as rows {g + 4e} (g = l/16),
// so no data moves between the two products.
//
// Grid: x = 64-column strips (one 16-column slab per wave), y = row splits;
// each workgroup walks its rows in 64-row tiles and keeps its W_{i+1} slab in
// registers; row splits write separate partial sums.
#include "internal.h"

namespace rq {
namespace {

constexpr int TT = 256;
constexpr int TR = 64;  // rows per tile

template <int BBM>
__global__ __launch_bounds__(TT, 2) void k_trail_f64(
    int m, double* __restrict__ a, long long lda, int i, int bbu, int bbn,
    const double* __restrict__ wp, long long ldw, int w0, int c_begin, int c_end,
    double* __restrict__ wpart, int rows_per_split) {
  constexpr int LDV = BBM + 2;
  __shared__ double sVu[TR * LDV];
  __shared__ double sVn[TR * LDV];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;
  const int col = c_begin + blockIdx.x * 64 + wave * 16 + lr16;
  const bool colok = col < c_end;
  const int ri0 = i + blockIdx.y * rows_per_split;
  const int ri1 = min(m, ri0 + rows_per_split);
  const int in = i + bbu;  // first row of the next reflectors

  double bw[BBM / 4];
#pragma unroll
  for (int kq = 0; kq < BBM / 4; ++kq) {
    const int q = 4 * kq + lg;
    bw[kq] = (colok && q < bbu) ? -wp[(long long)(col - w0) * ldw + q] : 0.0;
  }
  v4d acc[BBM / 16];
#pragma unroll
  for (int qb = 0; qb < BBM / 16; ++qb) acc[qb] = v4d{0.0, 0.0, 0.0, 0.0};

  double* acol = a + (long long)col * lda;
  for (int r0 = ri0; r0 < ri1; r0 += TR) {
    // ---- stage the reflector rows of this tile (unit lower trapezoidal) ----
    {
      const int rr = tid & 63;
      const int r = r0 + rr;
      for (int q = tid >> 6; q < BBM; q += TT / 64) {
        double vu = 0.0, vn = 0.0;
        if (r < m) {
          if (q < bbu) {
            const int d = r - i;
            vu = (d > q) ? a[(long long)(i + q) * lda + r] : (d == q ? 1.0 : 0.0);
          }
          if (q < bbn) {
            const int d = r - in;
            vn = (d > q) ? a[(long long)(in + q) * lda + r] : (d == q ? 1.0 : 0.0);
          }
        }
        sVu[rr * LDV + q] = vu;
        sVn[rr * LDV + q] = vn;
      }
    }
    // ---- the tile slab of this wave, in accumulator layout ----
    v4d d[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = r0 + 16 * b + acc_row<double>(lg, e);
        d[b][e] = (colok && row < ri1) ? acol[row] : 0.0;
      }
    __syncthreads();

    if (bbu > 0) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int kq = 0; kq < BBM / 4; ++kq) {
          if (4 * kq < bbu) {
            const double av = sVu[(16 * b + lr16) * LDV + 4 * kq + lg];
            d[b] = mfma_f64(av, bw[kq], d[b]);
          }
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + 16 * b + acc_row<double>(lg, e);
          if (colok && row < ri1) acol[row] = d[b][e];
        }
    }
    if (bbn > 0) {
#pragma unroll
      for (int qb = 0; qb < BBM / 16; ++qb) {
        if (16 * qb < bbn) {
#pragma unroll
          for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const double av = sVn[(16 * b + acc_row<double>(lg, e)) * LDV + 16 * qb + lr16];
              acc[qb] = mfma_f64(av, d[b][e], acc[qb]);
            }
        }
      }
    }
    __syncthreads();
  }

  if (bbn > 0 && colok) {
    double* out = wpart + ((long long)blockIdx.y * (c_end - c_begin) + (col - c_begin)) * bbn;
#pragma unroll
    for (int qb = 0; qb < BBM / 16; ++qb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = 16 * qb + acc_row<double>(lg, e);
        if (q < bbn) out[q] = acc[qb][e];
      }
  }
}

}  // namespace

TrailPlan trail_plan(int m_rows, int ncols) {
  TrailPlan p;
  p.ntiles = (ncols + 63) / 64;
  int ns = 1;
  // aim for at least two workgroups per compute unit; keep >= 256 rows per split
  while (p.ntiles * ns < 512 && (m_rows / (ns * 2)) >= 256) ns *= 2;
  p.nsplit = ns;
  return p;
}

int launch_trail_f64(hipStream_t s, int m, double* a, long long lda, int i, int bbu, int bbn,
                     const double* wp, long long ldw, int w0, int c_begin, int c_end,
                     double* wpart, int nsplit, int* nsp_out) {
  const int ncols = c_end - c_begin;
  *nsp_out = 0;
  if (ncols <= 0 || (bbu <= 0 && bbn <= 0)) return RQ_OK;
  const int rows = m - i;
  int rps = (rows + nsplit - 1) / nsplit;
  rps = (rps + TR - 1) / TR * TR;
  const int nsp = (rows + rps - 1) / rps;
  dim3 grid((ncols + 63) / 64, nsp);
  const int bbm = bbu > bbn ? bbu : bbn;
  if (bbm <= 32)
    hipLaunchKernelGGL(k_trail_f64<32>, grid, dim3(TT), 0, s, m, a, lda, i, bbu, bbn, wp, ldw, w0,
                       c_begin, c_end, wpart, rps);
  else if (bbm <= 64)
    hipLaunchKernelGGL(k_trail_f64<64>, grid, dim3(TT), 0, s, m, a, lda, i, bbu, bbn, wp, ldw, w0,
                       c_begin, c_end, wpart, rps);
  else if (bbm <= 128)
    hipLaunchKernelGGL(k_trail_f64<128>, grid, dim3(TT), 0, s, m, a, lda, i, bbu, bbn, wp, ldw,
                       w0, c_begin, c_end, wpart, rps);
  else
    return RQ_ERR_LIMIT;
  RQ_HIP_CHECK(hipGetLastError());
  *nsp_out = nsp;  // number of partial sums written
  return RQ_OK;
}

}  // namespace rq
