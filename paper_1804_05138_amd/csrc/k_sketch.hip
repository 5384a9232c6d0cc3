// Gaussian sketch of Alg. 2: Omega ~ N(0,1)^{(b+p) x m} and B = Omega A.
//
// Omega is drawn once per call from the counter-based Philox4x64-10 stream
// (seed, stream) and kept in the workspace (l x m doubles; it is re-read from
// L2 by every column strip of the product).  B = Omega A runs on FP64 MFMA:
// each workgroup owns a 64-column strip of A (one 16-column slab per wave) and
// a K range; Omega tiles are staged in LDS, A is read once from HBM straight
// into the B-operand layout (4 consecutive rows x 16 columns per instruction;
// four consecutive instructions cover whole 128-byte column segments).
#include "internal.h"

namespace rq {
namespace {

constexpr int GT = 256;

__global__ __launch_bounds__(GT) void k_gaussian(int rows, int cols, uint64_t seed,
                                                 uint64_t stream, double* __restrict__ out,
                                                 long long ld) {
  const long long total = (long long)rows * cols;
  const long long nblk = (total + 3) / 4;
  for (long long blk = (long long)blockIdx.x * GT + threadIdx.x; blk < nblk;
       blk += (long long)gridDim.x * GT) {
    double z[4];
    philox_normals4((uint64_t)blk, seed, stream, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long q = 4 * blk + j;
      if (q < total) {
        const long long c = q / rows, r = q % rows;
        out[c * ld + r] = z[j];
      }
    }
  }
}

constexpr int KT = 64;  // K rows per LDS tile

template <int MB>
__global__ __launch_bounds__(GT, 2) void k_sketch_f64(int m, int n, int l,
                                                     const double* __restrict__ om, long long ldo,
                                                     const double* __restrict__ a, long long lda,
                                                     double* __restrict__ out, long long ldout,
                                                     long long split_stride, int k_per_split) {
  constexpr int LDS_L = MB * 16 + 1;
  __shared__ double sO[KT * LDS_L];  // [k][row]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;
  const int col = blockIdx.x * 64 + wave * 16 + lr16;
  const bool colok = col < n;
  const int k0 = blockIdx.y * k_per_split;
  const int k1 = min(m, k0 + k_per_split);
  v4d acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = v4d{0.0, 0.0, 0.0, 0.0};
  // Loads are unconditional from clamped (valid) addresses and masked
  // afterwards, so they are all in flight together.
  const double* acol = a + (long long)(colok ? col : 0) * lda;

  for (int kt = k0; kt < k1; kt += KT) {
    // stage Omega(0:l, kt:kt+KT) as [k][row]
    constexpr int NS = (KT * MB * 16 + GT - 1) / GT;
    double ov[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + u * GT;
      const int r = e % (MB * 16), kk = e / (MB * 16);
      const int k = kt + kk;
      ov[u] = om[(long long)(k < k1 ? k : k1 - 1) * ldo + (r < l ? r : 0)];
    }
    // rows k >= k1 of this tile meet zero Omega columns, so clamped reads of A
    // need no mask; columns past n are never stored
    double bv[KT / 4];
#pragma unroll
    for (int kq = 0; kq < KT / 4; ++kq) {
      const int k = kt + 4 * kq + lg;
      bv[kq] = acol[k < k1 ? k : k1 - 1];
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + u * GT;
      const int r = e % (MB * 16), kk = e / (MB * 16);
      if (e < KT * MB * 16) sO[kk * LDS_L + r] = (r < l && kt + kk < k1) ? ov[u] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < KT / 4; ++kq) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const double av = sO[(4 * kq + lg) * LDS_L + 16 * mb + lr16];
        acc[mb] = mfma_f64(av, bv[kq], acc[mb]);
      }
    }
    __syncthreads();
  }
  if (colok) {
    double* o = out + (long long)blockIdx.y * split_stride + (long long)col * ldout;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * mb + acc_row<double>(lg, e);
        if (r < l) o[r] = acc[mb][e];
      }
  }
}

__global__ __launch_bounds__(GT) void k_sum_splits(int l, int n, const double* __restrict__ part,
                                                   long long split_stride, int nsplit,
                                                   double* __restrict__ b, long long ldb) {
  const long long total = (long long)l * n;
  for (long long e = (long long)blockIdx.x * GT + threadIdx.x; e < total;
       e += (long long)gridDim.x * GT) {
    const long long c = e / l, r = e % l;
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += part[sp * split_stride + c * l + r];
    b[c * ldb + r] = s;
  }
}

void sketch_split(int m, int n, int* nsplit, int* kps) {
  const int ntiles = (n + 63) / 64;
  int ns = 1;
  while (ntiles * ns < 512 && m / (ns * 2) >= 512) ns *= 2;
  int k = (m + ns - 1) / ns;
  k = (k + KT - 1) / KT * KT;
  *nsplit = (m + k - 1) / k;
  *kps = k;
}

}  // namespace

int launch_gaussian(hipStream_t s, int rows, int cols, uint64_t seed, uint64_t stream,
                    double* out, long long ld) {
  if (rows <= 0 || cols <= 0) return RQ_OK;
  const long long nblk = ((long long)rows * cols + 3) / 4;
  long long grid = (nblk + GT - 1) / GT;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)grid), dim3(GT), 0, s, rows, cols, seed, stream,
                     out, ld);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

size_t sketch_partial_doubles(int m, int n, int l) {
  int ns, kps;
  sketch_split(m, n, &ns, &kps);
  return ns > 1 ? (size_t)ns * l * n : 0;
}

template <int MB>
static void launch_mb(hipStream_t s, dim3 grid, int m, int n, int l, const double* om,
                      long long ldo, const double* a, long long lda, double* out, long long ldout,
                      long long stride, int kps) {
  hipLaunchKernelGGL(k_sketch_f64<MB>, grid, dim3(GT), 0, s, m, n, l, om, ldo, a, lda, out, ldout,
                     stride, kps);
}

int launch_sketch_f64(hipStream_t s, int m, int n, int l, const double* om, long long ldo,
                      const double* a, long long lda, double* b, long long ldb, double* partial) {
  if (l > MAX_L) return RQ_ERR_LIMIT;
  int ns, kps;
  sketch_split(m, n, &ns, &kps);
  double* out = ns > 1 ? partial : b;
  const long long ldout = ns > 1 ? l : ldb;
  const long long stride = (long long)l * n;
  dim3 grid((n + 63) / 64, ns);
  const int mb = (l + 15) / 16;
  switch (mb) {
    case 1: launch_mb<1>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 2: launch_mb<2>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 3: launch_mb<3>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 4: launch_mb<4>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 5: launch_mb<5>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 6: launch_mb<6>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 7: launch_mb<7>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 8: launch_mb<8>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 9: launch_mb<9>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    case 10: launch_mb<10>(s, grid, m, n, l, om, ldo, a, lda, out, ldout, stride, kps); break;
    default: return RQ_ERR_LIMIT;
  }
  RQ_HIP_CHECK(hipGetLastError());
  if (ns > 1) {
    long long total = (long long)l * n;
    long long grid2 = (total + GT - 1) / GT;
    if (grid2 > 65536) grid2 = 65536;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)grid2), dim3(GT), 0, s, l, n, partial, stride,
                       ns, b, ldb);
    RQ_HIP_CHECK(hipGetLastError());
  }
  return RQ_OK;
}

}  // namespace rq
