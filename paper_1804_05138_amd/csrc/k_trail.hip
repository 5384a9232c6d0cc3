// Trailing-matrix update of Alg. 2 (the block reflector's transpose applied
// to the trailing columns, PDLARFB in Alg. 4) in the right-looking order, used
// when k > n/2 (otherwise the left-looking schedule of k_gemm_big.hip runs),
// fused with the first product of the next block's update, on FP64 MFMA
// (v_mfma_f64_16x16x4f64) for an FP64 matrix and on FP32 MFMA
// (v_mfma_f32_16x16x4f32) for an FP32 matrix (the mixed-precision form:
// reflectors formed in FP64, stored and applied in FP32).
//
// With the compact WY form Q~ = I - V T V^T the update is A2 -= V (T^T V^T A2).
// The factor W' = T^T V^T A2 of block i is known before this pass (it was
// accumulated by the previous pass, and it is also what the sample update
// needs), so one pass over A2 does
//     tile  <- tile - V_i W'_i(:, tile columns)            (K = b)
//     W_{i+1}(:, tile columns) += V_{i+1}^T tile            (K = tile rows)
// where V_{i+1} are the next panel's reflectors (factored before this pass).
// Each element of A2 is read and written once per block.  The updated tile
// stays in the MFMA accumulator layout (lane l, element e: row acc_row(l/16, e),
// l/16 + 4e for FP64, 4(l/16) + e for FP32), which is exactly the B-operand
// layout the second product needs when the reduction index of the 4-wide
// chunk e is taken as the rows {acc_row(g, e) : g = 0..3}, so no data moves
// between the two products.
//
// Grid: x = column strips (NW waves of 16 columns each), y = row splits;
// each workgroup walks its rows in 32-row tiles and keeps its W_{i+1} slab in
// registers; row splits write separate partial sums.  Every wave of a
// workgroup reads the reflector rows the workgroup staged in LDS, so wider
// strips stage less per unit of work; the register budget decides how wide.
#include "internal.h"

namespace rq {
namespace {

constexpr int TR = 32;  // rows per tile

// LDS layouts (no padding; the XOR swizzles make both the row-contiguous
// staging stores and the MFMA operand reads free of bank conflicts per
// half-wave):
//   V_i   staged transposed, element (r, q) at q*TR + (r ^ 16*(q & 1))
//   V_i+1 staged by rows,    element (r, q) at r*BBM + (q ^ swz(r)),
//         swz(r) = ((r >> 1) & 15) | ((r & 1) << 4)
RQ_DEV int swz_n(int r) { return ((r >> 1) & 15) | ((r & 1) << 4); }

template <typename T>
struct TrailMfma;
template <>
struct TrailMfma<double> {
  typedef v4d acc_t;
  static RQ_DEV acc_t run(double a, double b, acc_t c) { return mfma_f64(a, b, c); }
};
template <>
struct TrailMfma<float> {
  typedef v4f acc_t;
  static RQ_DEV acc_t run(float a, float b, acc_t c) { return mfma_f32(a, b, c); }
};

// NW waves per workgroup, compiled for WPS waves per SIMD (512 / WPS
// registers per lane).
template <typename T, int BBM, int NW, int WPS>
__global__ __launch_bounds__(64 * NW, WPS) void k_trail(
    int m, T* __restrict__ a, long long lda, int i, int bbu, int bbn,
    const double* __restrict__ wp, long long ldw, int w0, int c_begin, int c_end,
    T* __restrict__ wpart, int rows_per_split) {
  static_assert(BBM % 32 == 0, "block width must be a multiple of 32");
  typedef typename TrailMfma<T>::acc_t acc_t;
  constexpr int TT = 64 * NW;
  constexpr int QS = TT / TR;       // reflector columns staged per pass of the block
  constexpr int NQ = BBM / QS;      // reflector values staged per thread and matrix
  __shared__ T sVuT[BBM * TR];
  __shared__ T sVn[TR * BBM];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;
  const int col = c_begin + blockIdx.x * (16 * NW) + wave * 16 + lr16;
  const bool colok = col < c_end;
  const int ri0 = i + blockIdx.y * rows_per_split;
  const int ri1 = min(m, ri0 + rows_per_split);
  const int in = i + bbu;  // first row of the next reflectors

  // Loads below are unconditional from clamped (always valid) addresses and
  // masked afterwards: a load under a branch costs a full memory round trip.
  const int cols = colok ? col : c_begin;  // a valid column for masked lanes
  T bw[BBM / 4];
#pragma unroll
  for (int kq = 0; kq < BBM / 4; ++kq) {
    const int q = 4 * kq + lg;
    const double v = (bbu > 0) ? wp[(long long)(cols - w0) * ldw + (q < bbu ? q : 0)] : 0.0;
    bw[kq] = (colok && q < bbu) ? (T)(-v) : T(0);
  }
  acc_t acc[BBM / 16];
#pragma unroll
  for (int qb = 0; qb < BBM / 16; ++qb) acc[qb] = acc_t{0, 0, 0, 0};

  T* acol = a + (long long)cols * lda;
  // this thread's share of a tile's reflector rows: row rr, columns q0 + QS*j
  const int rr = tid % TR, q0 = tid / TR;
  T pu[NQ], pn[NQ];
  // raw values only; the unit-lower-trapezoidal mask is applied when staging
  auto fetch_v = [&](int r0) {
    const int r = r0 + rr;
    const int rsafe = r < m ? r : m - 1;
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int q = q0 + QS * j;
      pu[j] = a[(long long)(i + (q < bbu ? q : 0)) * lda + rsafe];
      pn[j] = a[(long long)(q < bbn ? in + q : i) * lda + rsafe];
    }
  };
  // This wave's 16 columns of a tile, in accumulator layout.  Row splits are
  // multiples of the tile height, so rows past ri1 only occur past m, where
  // the staged reflector rows are zero; those rows (clamped to m-1) and the
  // columns past c_end (clamped to c_begin) only feed results that are never
  // stored, so no masking is needed.
  auto fetch_a = [&](int r0, acc_t* dd) {
#pragma unroll
    for (int b = 0; b < TR / 16; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = r0 + 16 * b + acc_row<T>(lg, e);
        dd[b][e] = acol[row < m ? row : m - 1];
      }
  };

  acc_t d[TR / 16], dn[TR / 16];
  fetch_v(ri0);
  fetch_a(ri0, d);
  for (int r0 = ri0; r0 < ri1; r0 += TR) {
    // ---- stage this tile's reflector rows (fetched one tile ahead) ----
    // Tiles below both diagonal blocks, inside the matrix and with full-width
    // blocks need no masking (the common case, a uniform branch).
    if (r0 >= in + bbn && r0 + TR <= m && bbu == BBM && bbn == BBM) {
#pragma unroll
      for (int j = 0; j < NQ; ++j) {
        const int q = q0 + QS * j;
        sVuT[q * TR + (rr ^ ((q & 1) << 4))] = pu[j];
        sVn[rr * BBM + (q ^ swz_n(rr))] = pn[j];
      }
    } else {
      // flat selects (no branches): zero outside the block width and past row m,
      // so partial blocks run the full-width MFMA loop on zero padding
      const int r = r0 + rr;
      const int du = r - i, dv = r - in;
      const bool rin = r < m;
#pragma unroll
      for (int j = 0; j < NQ; ++j) {
        const int q = q0 + QS * j;
        T vu = (du == q) ? T(1) : T(0);
        vu = (du > q) ? pu[j] : vu;
        vu = (rin & (q < bbu)) ? vu : T(0);
        T vn = (dv == q) ? T(1) : T(0);
        vn = (dv > q) ? pn[j] : vn;
        vn = (rin & (q < bbn)) ? vn : T(0);
        sVuT[q * TR + (rr ^ ((q & 1) << 4))] = vu;
        sVn[rr * BBM + (q ^ swz_n(rr))] = vn;
      }
    }
    __syncthreads();
    // ---- fetch the next tile while this one is on the MFMAs ----
    // Unconditional: after the last tile the clamped addresses stay valid and
    // the values go unused.  (Under a branch, the wait analysis at the join
    // made the MFMAs below wait for these loads.)
    fetch_v(r0 + TR);
    fetch_a(r0 + TR, dn);

    if (bbu > 0) {
#pragma unroll
      for (int kq = 0; kq < BBM / 4; ++kq) {
        const int q = 4 * kq + lg;
#pragma unroll
        for (int b = 0; b < TR / 16; ++b) {
          const T av = sVuT[q * TR + ((16 * b + lr16) ^ ((q & 1) << 4))];
          d[b] = TrailMfma<T>::run(av, bw[kq], d[b]);
        }
      }
#pragma unroll
      for (int b = 0; b < TR / 16; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + 16 * b + acc_row<T>(lg, e);
          if (colok & (row < ri1)) acol[row] = d[b][e];
        }
    }
    if (bbn > 0) {
#pragma unroll
      for (int b = 0; b < TR / 16; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 16 * b + acc_row<T>(lg, e);
          // all operands of this row first, then the MFMAs (one LDS wait)
          T av[BBM / 16];
#pragma unroll
          for (int qb = 0; qb < BBM / 16; ++qb) av[qb] = sVn[r * BBM + ((16 * qb + lr16) ^ swz_n(r))];
#pragma unroll
          for (int qb = 0; qb < BBM / 16; ++qb) acc[qb] = TrailMfma<T>::run(av[qb], d[b][e], acc[qb]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < TR / 16; ++b) d[b] = dn[b];
  }

  if (bbn > 0 && colok) {
    T* out = wpart + ((long long)blockIdx.y * (c_end - c_begin) + (col - c_begin)) * bbn;
#pragma unroll
    for (int qb = 0; qb < BBM / 16; ++qb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = 16 * qb + acc_row<T>(lg, e);
        if (q < bbn) out[q] = acc[qb][e];
      }
  }
}

}  // namespace

TrailPlan trail_plan(int m_rows, int ncols, int strip) {
  TrailPlan p;
  p.ntiles = (ncols + strip - 1) / strip;
  int ns = 1;
  // aim for at least two workgroups per compute unit; keep >= 256 rows per split
  while (p.ntiles * ns < 512 && (m_rows / (ns * 2)) >= 256) ns *= 2;
  p.nsplit = ns;
  return p;
}

// Launch shape: four waves per workgroup at two waves per SIMD for blocks up
// to 64 wide; for wider blocks the FP64 form needs a whole SIMD per wave
// (472 registers), while the FP32 form fits eight-wave workgroups at two
// waves per SIMD (246 registers), which halves its reflector staging.
template <typename T>
static int trail_waves(int bbm) {
  return (bbm > 64 && sizeof(T) == 4) ? 8 : 4;
}

template <typename T>
int trail_strip(int bbm) {
  return 16 * trail_waves<T>(bbm);
}
static_assert(16 * 8 <= kTrailMaxStrip, "workspace sizing assumes the widest strip");
template int trail_strip<double>(int);
template int trail_strip<float>(int);

template <typename T>
int launch_trail(hipStream_t s, int m, T* a, long long lda, int i, int bbu, int bbn,
                 const double* wp, long long ldw, int w0, int c_begin, int c_end, T* wpart,
                 int nsplit, int* nsp_out) {
  const int ncols = c_end - c_begin;
  *nsp_out = 0;
  if (ncols <= 0 || (bbu <= 0 && bbn <= 0)) return RQ_OK;
  const int rows = m - i;
  int rps = (rows + nsplit - 1) / nsplit;
  rps = (rps + TR - 1) / TR * TR;
  const int nsp = (rows + rps - 1) / rps;
  const int bbm = bbu > bbn ? bbu : bbn;
  if (bbm > 128) return RQ_ERR_LIMIT;
  const int nw = trail_waves<T>(bbm), strip = 16 * nw;
  const dim3 grid((ncols + strip - 1) / strip, nsp), block(64 * nw);
  if (bbm <= 32)
    hipLaunchKernelGGL((k_trail<T, 32, 4, 2>), grid, block, 0, s, m, a, lda, i, bbu, bbn, wp, ldw,
                       w0, c_begin, c_end, wpart, rps);
  else if (bbm <= 64)
    hipLaunchKernelGGL((k_trail<T, 64, 4, 2>), grid, block, 0, s, m, a, lda, i, bbu, bbn, wp, ldw,
                       w0, c_begin, c_end, wpart, rps);
  else if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL((k_trail<T, 128, 8, 2>), grid, block, 0, s, m, a, lda, i, bbu, bbn, wp,
                       ldw, w0, c_begin, c_end, wpart, rps);
  else
    hipLaunchKernelGGL((k_trail<T, 128, 4, 1>), grid, block, 0, s, m, a, lda, i, bbu, bbn, wp,
                       ldw, w0, c_begin, c_end, wpart, rps);
  RQ_HIP_CHECK(hipGetLastError());
  *nsp_out = nsp;  // number of partial sums written
  return RQ_OK;
}
template int launch_trail<double>(hipStream_t, int, double*, long long, int, int, int,
                                  const double*, long long, int, int, int, double*, int, int*);
template int launch_trail<float>(hipStream_t, int, float*, long long, int, int, int,
                                 const double*, long long, int, int, int, float*, int, int*);

}  // namespace rq
