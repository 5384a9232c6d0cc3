// Column moves of Alg. 2 (the block's pivots are moved to the front of the
// trailing columns of A and of the permutation): the sketch kernel lists every
// (destination, source) position pair of the block's sequential
// transpositions; here they are applied to A (full height, so rows of R
// already computed move too), to the permutation vector and to the rows of W'
// computed so far (the pending block's, or every block's in the left-looking
// schedule).  Each workgroup owns a slab of rows and first
// gathers every source column of its slab into registers, then scatters, so
// the move is a race-free permutation without a global temporary.
#include "internal.h"

namespace rq {
namespace {

constexpr int ST = 256;
constexpr int SLAB = 32;  // rows per workgroup

// Moves the listed columns of rows [r0, r0 + nrow) of x (leading dimension
// ldx, column offset c0): the pair list goes to LDS, every source element of
// the thread is read into registers with all loads in flight (clamped
// addresses, masked afterwards), and after one barrier every destination is
// written, so the move is a race-free permutation without a temporary array.
constexpr int NPT = 2 * MAX_B * SLAB / ST;  // elements per thread at most
template <typename S>
RQ_DEV void move_slab(S* __restrict__ x, long long ldx, int c0, int r0, int nrow,
                      const int* __restrict__ pairs, int np, int* spairs) {
  for (int e = threadIdx.x; e < 2 * np; e += ST) spairs[e] = pairs[e];
  __syncthreads();
  S v[NPT];
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    const int e = threadIdx.x + u * ST, p = e / SLAB, r = e % SLAB;
    const bool ok = e < np * SLAB && r < nrow;
    v[u] = x[(long long)(c0 + spairs[2 * (ok ? p : 0) + 1]) * ldx + r0 + (ok ? r : 0)];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    const int e = threadIdx.x + u * ST, p = e / SLAB, r = e % SLAB;
    if (e < np * SLAB && r < nrow) x[(long long)(c0 + spairs[2 * p]) * ldx + r0 + r] = v[u];
  }
}

// One launch for the three moves of a block: the first na workgroups take
// SLAB-row slabs of A, the next nw slabs of the pending W' block (wrows rows,
// no column offset), and the last one (when jpvt is given) the permutation
// vector.  Each workgroup touches only its own rows, so the roles never race.
template <typename T, typename WT>
__global__ __launch_bounds__(ST) void k_apply_pairs(int rows, T* __restrict__ a, long long lda,
                                                    int c0, int na, WT* __restrict__ wp,
                                                    int wrows, long long ldw, int nw,
                                                    int* __restrict__ jpvt,
                                                    const int* __restrict__ pairs,
                                                    const int* __restrict__ npairs) {
  __shared__ int spairs[2 * 2 * MAX_B];
  const int np = *npairs;
  if (np <= 0 || np > 2 * MAX_B) return;
  const int g = blockIdx.x;
  if (g < na) {
    const int r0 = g * SLAB;
    move_slab<T>(a, lda, c0, r0, min(SLAB, rows - r0), pairs, np, spairs);
  } else if (g < na + nw) {
    const int r0 = (g - na) * SLAB;
    move_slab<WT>(wp, ldw, 0, r0, min(SLAB, wrows - r0), pairs, np, spairs);
  } else if (jpvt != nullptr) {
    move_slab<int>(jpvt, 1LL, c0, 0, 1, pairs, np, spairs);
  }
}

}  // namespace

template <typename T, typename WT>
int launch_apply_pairs(hipStream_t s, int m, T* a, long long lda, int c0, int* jpvt, WT* wp,
                       int wrows, long long ldw, int w0, const int* pairs, const int* npairs,
                       int max_pairs) {
  if (max_pairs > 2 * MAX_B) return RQ_ERR_LIMIT;
  const int na = m > 0 ? (m + SLAB - 1) / SLAB : 0;
  const int nw = (wp != nullptr && wrows > 0) ? (wrows + SLAB - 1) / SLAB : 0;
  const int nj = jpvt != nullptr ? 1 : 0;
  if (na + nw + nj > 0)
    hipLaunchKernelGGL((k_apply_pairs<T, WT>), dim3(na + nw + nj), dim3(ST), 0, s, m, a, lda, c0,
                       na, wp,
                       wrows, ldw, nw, jpvt, pairs, npairs);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_apply_pairs<double, double>(hipStream_t, int, double*, long long, int, int*,
                                                double*, int, long long, int, const int*,
                                                const int*, int);
template int launch_apply_pairs<float, double>(hipStream_t, int, float*, long long, int, int*,
                                               double*, int, long long, int, const int*,
                                               const int*, int);
template int launch_apply_pairs<float, float>(hipStream_t, int, float*, long long, int, int*,
                                              float*, int, long long, int, const int*, const int*,
                                              int);

}  // namespace rq
