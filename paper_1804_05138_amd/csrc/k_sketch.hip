// Gaussian sketch of Alg. 2: Omega ~ N(0,1)^{(b+p) x m} and B = Omega A.
//
// Three arithmetic forms (the paper's is FP64; the other two are the
// mixed-precision sketch, whose result B is still kept in FP64):
//  * FP64 MFMA (v_mfma_f64_16x16x4f64), A in FP64 or FP32 (widened on load);
//  * BF16 MFMA (v_mfma_f32_16x16x32_bf16): Omega and A rounded to bfloat16
//    (round to nearest even), FP32 accumulation;
//  * FP8 MFMA (v_mfma_f32_16x16x32_fp8_fp8, OCP e4m3): column j of A is scaled
//    by the power of two s_j = 2^floor(log2(448 / max_i |A(i,j)|)) so that its
//    largest entry lands at most at the format's largest finite value, rounded
//    to e4m3, and B(:, j) is the FP32-accumulated product times 1/s_j (exact);
//    Omega is rounded without a scale (|N(0,1)| samples stay far below 448).
//
// Omega is drawn once per call from the counter-based Philox4x64-10 stream
// (seed, stream) and kept in the workspace (l x m doubles; it is re-read from
// L2 by every column strip of the product).  B = Omega A runs on FP64 MFMA:
// each workgroup owns a 64-column strip of A (one 16-column slab per wave) and
// a K range; Omega tiles are staged in LDS, A is read once from HBM straight
// into the B-operand layout (4 consecutive rows x 16 columns per instruction;
// four consecutive instructions cover whole 128-byte column segments).
#include <algorithm>

#include "internal.h"
#include "gemm.h"

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

// The same Omega stored transposed (out[r * ld + c] = Omega(r, c)), for rows
// divisible by 4: a Philox block holds Omega(4 rb .. 4 rb + 3, c), and
// consecutive threads take consecutive c so that every store is coalesced.
__global__ __launch_bounds__(GT) void k_gaussian_t(int rows, int cols, uint64_t seed,
                                                   uint64_t stream, double* __restrict__ out,
                                                   long long ld) {
  const int rb4 = rows / 4;
  const long long nblk = (long long)rb4 * cols;
  for (long long t = (long long)blockIdx.x * GT + threadIdx.x; t < nblk;
       t += (long long)gridDim.x * GT) {
    const long long c = t % cols, rb = t / cols;
    double z[4];
    philox_normals4((uint64_t)(c * rb4 + rb), seed, stream, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) out[(4 * rb + j) * ld + c] = z[j];
  }
}

constexpr int KT = 64;  // K rows per LDS tile

template <int MB, typename TA>
__global__ __launch_bounds__(GT, 2) void k_sketch_f64(int m, int n, int l,
                                                     const double* __restrict__ om, long long ldo,
                                                     const TA* __restrict__ a, long long lda,
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
  const TA* acol = a + (long long)(colok ? col : 0) * lda;

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
      bv[kq] = (double)acol[k < k1 ? k : k1 - 1];
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


// ---- low-precision sketch ----
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 v8bf;

constexpr int LKT = 128;  // K rows per LDS stage of the low-precision kernels

// Omega (l x m FP64, ld l) rounded to the low-precision format, stored by rows
// (row r at r * ldq) with zero padding up to lpad rows and mpad columns.
template <int FMT>
__global__ __launch_bounds__(GT) void k_omega_lp(int l, int m, const double* __restrict__ om,
                                                 long long ldo, void* __restrict__ out,
                                                 long long ldq, int lpad, int mpad) {
  const long long total = (long long)lpad * mpad;
  for (long long e = (long long)blockIdx.x * GT + threadIdx.x; e < total;
       e += (long long)gridDim.x * GT) {
    const long long r = e / mpad, k = e % mpad;
    const double v = (r < l && k < m) ? om[k * ldo + r] : 0.0;
    if constexpr (FMT == 0) {
      ((__bf16*)out)[r * ldq + k] = (__bf16)(float)v;
    } else {
      const int w = __builtin_amdgcn_cvt_pk_fp8_f32((float)v, 0.0f, 0, false);
      ((unsigned char*)out)[r * ldq + k] = (unsigned char)(w & 0xff);
    }
  }
}

// s_j = 2^floor(log2(448 / max_i |A(i, j)|)) (1 for a zero column); one wave per column.
template <typename TA>
__global__ __launch_bounds__(GT) void k_colscale(int m, int n, const TA* __restrict__ a,
                                                 long long lda, float* __restrict__ scale) {
  const int col = blockIdx.x * (GT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= n) return;
  const TA* c = a + (long long)col * lda;
  double mx = 0.0;
  for (int r = lane; r < m; r += 64) mx = fmax(mx, fabs((double)c[r]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) scale[col] = (mx > 0.0) ? (float)ldexp(1.0, ilogb(448.0 / mx)) : 1.0f;
}

// B(:, strip) partial over a K range = Omega_lp A_lp.  Each wave owns 16
// columns; each lane loads 8 consecutive rows of its column per K chunk of 32
// (the B-operand layout of the 16x16x32 instructions: lane group g holds the
// chunk's rows 8g..8g+7), rounds them and feeds the MFMA directly; the Omega
// tile is staged in LDS by rows.
template <int MB, int FMT, typename TA>
__global__ __launch_bounds__(GT, 2) void k_sketch_lp(int m, int n, int l, const void* __restrict__ oq,
                                                     long long ldq, const TA* __restrict__ a,
                                                     long long lda, const float* __restrict__ scale,
                                                     double* __restrict__ out, long long ldout,
                                                     long long split_stride, int k_per_split) {
  constexpr int ES = (FMT == 0) ? 2 : 1;          // bytes per element
  constexpr int ROWB = LKT * ES + 16;             // LDS row pitch in bytes (16-byte pad)
  __shared__ __attribute__((aligned(16))) unsigned char sO[MB * 16 * ROWB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;
  const int col = blockIdx.x * 64 + wave * 16 + lr16;
  const bool colok = col < n;
  const int k0 = blockIdx.y * k_per_split;
  const int k1 = min(m, k0 + k_per_split);
  const TA* acol = a + (long long)(colok ? col : 0) * lda;
  const float sc = (FMT == 1 && colok) ? scale[col] : 1.0f;
  v4f acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int kt = k0; kt < k1; kt += LKT) {
    // stage Omega_lp(0:16MB, kt:kt+LKT): 16-byte pieces, rows contiguous in k
    constexpr int PPR = LKT * ES / 16;            // pieces per row
    constexpr int NP = (MB * 16 * PPR + GT - 1) / GT;
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + u * GT;
      if (e < MB * 16 * PPR) {
        const int r = e / PPR, pc = e % PPR;
        const uint4 v = *reinterpret_cast<const uint4*>(
            reinterpret_cast<const unsigned char*>(oq) + (long long)r * ldq * ES +
            (long long)kt * ES + pc * 16);
        *reinterpret_cast<uint4*>(sO + r * ROWB + pc * 16) = v;
      }
    }
    // this lane's A rows of the stage: chunk c, rows kt + 32c + 8lg .. +7
    // (rows past k1 meet zero Omega columns or belong to the next split's
    // range, whose Omega columns this split does not stage: mask them)
    float av[LKT / 32][8];
#pragma unroll
    for (int c = 0; c < LKT / 32; ++c)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kt + 32 * c + 8 * lg + j;
        const float v = (float)acol[k < k1 ? k : k1 - 1];
        av[c][j] = (k < k1) ? v * sc : 0.0f;
      }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < LKT / 32; ++c) {
      if constexpr (FMT == 0) {
        v8bf bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = (__bf16)av[c][j];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const v8bf ov = *reinterpret_cast<const v8bf*>(sO + (16 * mb + lr16) * ROWB +
                                                          (32 * c + 8 * lg) * ES);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ov, bv, acc[mb], 0, 0, 0);
        }
      } else {
        int w0 = 0, w1 = 0;
        w0 = __builtin_amdgcn_cvt_pk_fp8_f32(av[c][0], av[c][1], w0, false);
        w0 = __builtin_amdgcn_cvt_pk_fp8_f32(av[c][2], av[c][3], w0, true);
        w1 = __builtin_amdgcn_cvt_pk_fp8_f32(av[c][4], av[c][5], w1, false);
        w1 = __builtin_amdgcn_cvt_pk_fp8_f32(av[c][6], av[c][7], w1, true);
        const long bv = (long)(((unsigned long)(unsigned)w1 << 32) | (unsigned)w0);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const long ov = *reinterpret_cast<const long*>(sO + (16 * mb + lr16) * ROWB +
                                                          (32 * c + 8 * lg) * ES);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ov, bv, acc[mb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (colok) {
    const double inv = 1.0 / (double)sc;
    double* o = out + (long long)blockIdx.y * split_stride + (long long)col * ldout;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * mb + acc_row<float>(lg, e);
        if (r < l) o[r] = (double)acc[mb][e] * inv;
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

// K ranges of the sketch through the W-pass product: about 512 workgroups
// (two per CU) in one round, at most 4 ranges of at least 256 rows.
int sketch_t_splits(int m, int n) {
  const int tiles = (n + kWpassCols - 1) / kWpassCols;
  const int sp = (512 + tiles - 1) / tiles;
  return std::max(1, std::min(sp, std::min(4, m / 256)));
}

void sketch_split(int m, int n, int gran, int* nsplit, int* kps) {
  const int ntiles = (n + 63) / 64;
  int ns = 1;
  while (ntiles * ns < 512 && m / (ns * 2) >= 512) ns *= 2;
  int k = (m + ns - 1) / ns;
  k = (k + gran - 1) / gran * gran;
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

int launch_gaussian_t(hipStream_t s, int rows, int cols, uint64_t seed, uint64_t stream,
                      double* out, long long ld) {
  if (rows % 4 != 0 || ld < cols) return RQ_ERR_LIMIT;
  if (rows <= 0 || cols <= 0) return RQ_OK;
  long long grid = ((long long)rows / 4 * cols + GT - 1) / GT;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_gaussian_t, dim3((unsigned)grid), dim3(GT), 0, s, rows, cols, seed, stream,
                     out, ld);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

bool sketch_t_usable(int m, int l, const double* a, long long lda) {
  return m >= 2 && m % 2 == 0 && lda % 2 == 0 && l % 4 == 0 && l <= 128 &&
         reinterpret_cast<uintptr_t>(a) % 16 == 0;
}

int launch_sketch_t(hipStream_t s, int m, int n, int l, const double* omt, const double* a,
                    long long lda, double* b, long long ldb, double* partial) {
  if (!sketch_t_usable(m, l, a, lda) || reinterpret_cast<uintptr_t>(omt) % 16 != 0)
    return RQ_ERR_LIMIT;
  if (n <= 0) return RQ_OK;
  // part[z][j][q] = sum over the z-th row range of Omega(q, i) A(i, j)
  int got = 0;
  const int rc = wpass_partials<double>(s, m, l, n, n, omt, m, a, lda, a, lda, partial,
                                        sketch_t_splits(m, n), &got);
  if (rc) return rc;
  long long total = (long long)l * n;
  long long grid2 = (total + GT - 1) / GT;
  if (grid2 > 65536) grid2 = 65536;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)grid2), dim3(GT), 0, s, l, n, partial, total,
                     got, b, ldb);
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

size_t sketch_partial_doubles(int m, int n, int l) {
  int ns, kps, ns2, kps2;
  sketch_split(m, n, KT, &ns, &kps);
  sketch_split(m, n, LKT, &ns2, &kps2);
  if (ns2 > ns) ns = ns2;
  ns = std::max(ns, sketch_t_splits(m, n));
  return (size_t)ns * l * n;
}

size_t sketch_lp_bytes(int m, int n, int l, int stype) {
  if (stype != SK_BF16 && stype != SK_FP8) return 0;
  const size_t lpad = (size_t)(l + 15) / 16 * 16;
  const size_t mpad = (size_t)(m + LKT - 1) / LKT * LKT;
  const size_t es = stype == SK_BF16 ? 2 : 1;
  return (lpad * mpad * es + 255) / 256 * 256 + (size_t)n * sizeof(float);
}

template <typename TA>
struct SketchArgs {
  int m, n, l;
  const double* om;
  long long ldo;
  const TA* a;
  long long lda;
  double* out;
  long long ldout, stride;
  int kps;
  const void* oq;
  long long ldq;
  const float* scale;
};

template <int MB, typename TA>
static void launch_mb(hipStream_t s, dim3 grid, int stype, const SketchArgs<TA>& x) {
  if (stype == SK_F64)
    hipLaunchKernelGGL((k_sketch_f64<MB, TA>), grid, dim3(GT), 0, s, x.m, x.n, x.l, x.om, x.ldo,
                       x.a, x.lda, x.out, x.ldout, x.stride, x.kps);
  else if (stype == SK_BF16)
    hipLaunchKernelGGL((k_sketch_lp<MB, 0, TA>), grid, dim3(GT), 0, s, x.m, x.n, x.l, x.oq, x.ldq,
                       x.a, x.lda, x.scale, x.out, x.ldout, x.stride, x.kps);
  else
    hipLaunchKernelGGL((k_sketch_lp<MB, 1, TA>), grid, dim3(GT), 0, s, x.m, x.n, x.l, x.oq, x.ldq,
                       x.a, x.lda, x.scale, x.out, x.ldout, x.stride, x.kps);
}

template <typename TA>
int launch_sketch(hipStream_t s, int m, int n, int l, int stype, const double* om, long long ldo,
                  const TA* a, long long lda, double* b, long long ldb, double* partial,
                  void* lpbuf) {
  if (l > MAX_L) return RQ_ERR_LIMIT;
  if (stype != SK_F64 && stype != SK_BF16 && stype != SK_FP8) return RQ_ERR_UNSUPPORTED;
  const bool lp = stype != SK_F64;
  int ns, kps;
  sketch_split(m, n, lp ? LKT : KT, &ns, &kps);
  SketchArgs<TA> x;
  x.m = m;
  x.n = n;
  x.l = l;
  x.om = om;
  x.ldo = ldo;
  x.a = a;
  x.lda = lda;
  x.out = ns > 1 ? partial : b;
  x.ldout = ns > 1 ? l : ldb;
  x.stride = (long long)l * n;
  x.kps = kps;
  x.oq = nullptr;
  x.ldq = 0;
  x.scale = nullptr;
  if (lp) {
    const int lpad = (l + 15) / 16 * 16;
    const int mpad = (m + LKT - 1) / LKT * LKT;
    const size_t es = stype == SK_BF16 ? 2 : 1;
    float* scale = (float*)((char*)lpbuf + ((size_t)lpad * mpad * es + 255) / 256 * 256);
    const long long tot = (long long)lpad * mpad;
    const unsigned g = (unsigned)std::min<long long>((tot + GT - 1) / GT, 65536);
    if (stype == SK_BF16)
      hipLaunchKernelGGL(k_omega_lp<0>, dim3(g), dim3(GT), 0, s, l, m, om, ldo, lpbuf,
                         (long long)mpad, lpad, mpad);
    else {
      hipLaunchKernelGGL(k_omega_lp<1>, dim3(g), dim3(GT), 0, s, l, m, om, ldo, lpbuf,
                         (long long)mpad, lpad, mpad);
      hipLaunchKernelGGL(k_colscale<TA>, dim3((n + 3) / 4), dim3(GT), 0, s, m, n, a, lda, scale);
    }
    RQ_HIP_CHECK(hipGetLastError());
    x.oq = lpbuf;
    x.ldq = mpad;
    x.scale = scale;
  }
  dim3 grid((n + 63) / 64, ns);
  const int mb = (l + 15) / 16;
  switch (mb) {
    case 1: launch_mb<1>(s, grid, stype, x); break;
    case 2: launch_mb<2>(s, grid, stype, x); break;
    case 3: launch_mb<3>(s, grid, stype, x); break;
    case 4: launch_mb<4>(s, grid, stype, x); break;
    case 5: launch_mb<5>(s, grid, stype, x); break;
    case 6: launch_mb<6>(s, grid, stype, x); break;
    case 7: launch_mb<7>(s, grid, stype, x); break;
    case 8: launch_mb<8>(s, grid, stype, x); break;
    case 9: launch_mb<9>(s, grid, stype, x); break;
    case 10: launch_mb<10>(s, grid, stype, x); break;
    default: return RQ_ERR_LIMIT;
  }
  RQ_HIP_CHECK(hipGetLastError());
  if (ns > 1) {
    long long total = (long long)l * n;
    long long grid2 = (total + GT - 1) / GT;
    if (grid2 > 65536) grid2 = 65536;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)grid2), dim3(GT), 0, s, l, n, partial,
                       x.stride, ns, b, ldb);
    RQ_HIP_CHECK(hipGetLastError());
  }
  return RQ_OK;
}
template int launch_sketch<double>(hipStream_t, int, int, int, int, const double*, long long,
                                   const double*, long long, double*, long long, double*, void*);
template int launch_sketch<float>(hipStream_t, int, int, int, int, const double*, long long,
                                  const float*, long long, double*, long long, double*, void*);

}  // namespace rq
