// Column moves of Alg. 2 ("swap the pivots into positions i..i+b-1 in A and
// Pi"): the sketch kernel lists every (destination, source) position pair of
// the block's sequential transpositions; here they are applied to A (full
// height, so rows of R already computed move too), to the permutation vector
// and to the pending W' block.  Each workgroup owns a slab of rows and first
// gathers every source column of its slab into LDS, then scatters, so the
// move is a race-free permutation without a global temporary.
#include "internal.h"

namespace rq {
namespace {

constexpr int ST = 256;
constexpr int SLAB = 32;  // rows per workgroup

template <typename T>
__global__ __launch_bounds__(ST) void k_apply_pairs(int rows, T* __restrict__ a, long long lda,
                                                    int c0, const int* __restrict__ pairs,
                                                    const int* __restrict__ npairs) {
  __shared__ T buf[2 * MAX_B * SLAB];
  const int np = *npairs;
  const int r0 = blockIdx.x * SLAB;
  const int nrow = min(SLAB, rows - r0);
  if (nrow <= 0 || np <= 0) return;
  for (int e = threadIdx.x; e < np * SLAB; e += ST) {
    const int p = e / SLAB, r = e % SLAB;
    if (r < nrow) buf[e] = a[(long long)(c0 + pairs[2 * p + 1]) * lda + r0 + r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < np * SLAB; e += ST) {
    const int p = e / SLAB, r = e % SLAB;
    if (r < nrow) a[(long long)(c0 + pairs[2 * p]) * lda + r0 + r] = buf[e];
  }
}

}  // namespace

template <typename T>
int launch_apply_pairs(hipStream_t s, int m, T* a, long long lda, int c0, int* jpvt, double* wp,
                       int wrows, long long ldw, int w0, const int* pairs, const int* npairs,
                       int max_pairs) {
  if (max_pairs > 2 * MAX_B) return RQ_ERR_LIMIT;
  if (m > 0)
    hipLaunchKernelGGL(k_apply_pairs<T>, dim3((m + SLAB - 1) / SLAB), dim3(ST), 0, s, m, a,
                       lda, c0, pairs, npairs);
  if (wp != nullptr && wrows > 0)
    hipLaunchKernelGGL(k_apply_pairs<double>, dim3((wrows + SLAB - 1) / SLAB), dim3(ST), 0, s,
                       wrows, wp, ldw, 0, pairs, npairs);
  if (jpvt != nullptr)
    hipLaunchKernelGGL(k_apply_pairs<int>, dim3(1), dim3(ST), 0, s, 1, jpvt, 1LL, c0, pairs,
                       npairs);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}
template int launch_apply_pairs<double>(hipStream_t, int, double*, long long, int, int*, double*,
                                        int, long long, int, const int*, const int*, int);
template int launch_apply_pairs<float>(hipStream_t, int, float*, long long, int, int*, double*,
                                       int, long long, int, const int*, const int*, int);

}  // namespace rq
