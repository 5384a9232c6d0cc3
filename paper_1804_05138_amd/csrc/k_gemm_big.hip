// Large-tile GEMM on MFMA for the left-looking trailing update:
//     C = alpha op(A) B + beta C     (column-major, op(A) = A or A^T),
// or, for a split reduction, the raw partial sums of K ranges.
//
// Each wave owns a (16 XT) x (16 YT) block of C (XT x YT MFMA tiles of 16 x 16,
// FP64 v_mfma_f64_16x16x4f64 or FP32 v_mfma_f32_16x16x4f32); a workgroup of
// WM x WN waves covers a (16 XT WM) x (16 YT WN) tile.  K advances in steps of
// BK through two LDS buffers: the global loads of step t+1 are in registers
// while step t runs on the matrix cores, one barrier per step.  The large
// products use 128 x 128 tiles (twice the side of the generic GEMM's,
// k_gemm.hip), so each operand byte staged feeds twice the MFMA work.
//
// Loads move two consecutive elements of the contiguous index per lane
// (8- or 16-byte vector loads) when leading dimensions, bases and the
// contiguous extents allow it; otherwise one element.  Out-of-range elements
// are read from clamped (always valid) addresses and masked to zero.
//
// Tile order: consecutive workgroups go to different XCDs (the dispatcher
// deals them round-robin over the eight dies), so the linear index is
// remapped to give each die a contiguous range of tiles, walked in groups of
// eight tile rows, so the operand panels a die's workgroups share stay in its
// own L2.
#include <algorithm>

#include "internal.h"
#include "gemm.h"

namespace rq {
namespace {

template <typename T>
struct BigMfma;
template <>
struct BigMfma<double> {
  typedef v4d acc_t;
  static RQ_DEV acc_t run(double a, double b, acc_t c) { return mfma_f64(a, b, c); }
};
template <>
struct BigMfma<float> {
  typedef v4f acc_t;
  static RQ_DEV acc_t run(float a, float b, acc_t c) { return mfma_f32(a, b, c); }
};

constexpr int kPad = 1;  // LDS row padding (elements)

template <typename T, bool TA, int WM, int WN, int XT, int YT, int BK, int OCC, bool VEC>
__global__ __launch_bounds__(64 * WM * WN, OCC) void k_gemm_big(
    int M, int N, int K, T alpha, const T* __restrict__ A, long long lda, const T* __restrict__ B,
    long long ldb, T beta, T* __restrict__ C, long long ldc, int kchunk, T* __restrict__ part) {
  typedef typename BigMfma<T>::acc_t acc_t;
  typedef T T2 __attribute__((ext_vector_type(2)));
  constexpr int NT = 64 * WM * WN, BM = 16 * XT * WM, BN = 16 * YT * WN;
  constexpr int VW = VEC ? 2 : 1;
  constexpr int NLA = BM * BK / NT / VW, NLB = BN * BK / NT / VW;
  static_assert(NLA * NT * VW == BM * BK && NLB * NT * VW == BN * BK, "tiles split evenly");
  __shared__ T sA[2][BK][BM + kPad];
  __shared__ T sB[2][BK][BN + kPad];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;

  const int nbm = (M + BM - 1) / BM, nbn = (N + BN - 1) / BN, tiles = nbm * nbn;
  int tile = blockIdx.x;
  if ((tiles & 7) == 0) tile = (tile & 7) * (tiles >> 3) + (tile >> 3);
  constexpr int GM = 8;
  const int first = tile / (GM * nbn) * GM, gsz = min(nbm - first, GM);
  const int tm = first + (tile % (GM * nbn)) % gsz, tn = (tile % (GM * nbn)) / gsz;
  const int m0 = tm * BM, n0 = tn * BN;
  const int wm = (wave % WM) * 16 * XT, wn = (wave / WM) * 16 * YT;
  const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);

  acc_t acc[XT][YT];
#pragma unroll
  for (int x = 0; x < XT; ++x)
#pragma unroll
    for (int y = 0; y < YT; ++y) acc[x][y] = acc_t{0, 0, 0, 0};

  typedef T RegA[NLA * VW];
  typedef T RegB[NLB * VW];
  // Loads put raw values from clamped (always valid) addresses in registers;
  // the range masks are applied when the values go to LDS, after the MFMAs of
  // the current step, so nothing waits for the loads before then.
  auto ldraw = [&](const T* p, T* dst) {
    if constexpr (VEC) {
      const T2 v = *reinterpret_cast<const T2*>(p);
      dst[0] = v.x;
      dst[1] = v.y;
    } else {
      dst[0] = *p;
    }
  };
  // element (ci, oi) of a load: ci along the contiguous index (VW at a time)
  auto load = [&](int k0, RegA& ra, RegB& rb) {
#pragma unroll
    for (int j = 0; j < NLA; ++j) {
      const int u = tid + NT * j;
      if constexpr (!TA) {  // A(m, k) at A[k lda + m]: contiguous along m
        const int mi = (u % (BM / VW)) * VW, ki = u / (BM / VW);
        const int gm = m0 + mi, gk = k0 + ki;
        const int gmc = gm < M ? gm : ((M - 1) & ~(VW - 1)), gkc = gk < ke ? gk : ke - 1;
        ldraw(A + (long long)gkc * lda + gmc, ra + VW * j);
      } else {              // op(A)(m, k) = A[m lda + k]: contiguous along k
        const int ki = (u % (BK / VW)) * VW, mi = u / (BK / VW);
        const int gm = m0 + mi, gk = k0 + ki;
        const int gmc = gm < M ? gm : M - 1, gkc = gk < ke ? gk : ke - VW;
        ldraw(A + (long long)gmc * lda + gkc, ra + VW * j);
      }
    }
#pragma unroll
    for (int j = 0; j < NLB; ++j) {
      const int u = tid + NT * j;
      const int ki = (u % (BK / VW)) * VW, ni = u / (BK / VW);
      const int gn = n0 + ni, gk = k0 + ki;
      const int gnc = gn < N ? gn : N - 1, gkc = gk < ke ? gk : ke - VW;
      ldraw(B + (long long)gnc * ldb + gkc, rb + VW * j);
    }
  };
  auto stash = [&](int buf, int k0, const RegA& ra, const RegB& rb) {
#pragma unroll
    for (int j = 0; j < NLA; ++j) {
      const int u = tid + NT * j;
      if constexpr (!TA) {
        const int mi = (u % (BM / VW)) * VW, ki = u / (BM / VW);
        const int gm = m0 + mi;
        const bool kok = k0 + ki < ke;
#pragma unroll
        for (int v = 0; v < VW; ++v)
          sA[buf][ki][mi + v] = (kok && gm + v < M) ? ra[VW * j + v] : T(0);
      } else {
        const int ki = (u % (BK / VW)) * VW, mi = u / (BK / VW);
        const bool mok = m0 + mi < M;
#pragma unroll
        for (int v = 0; v < VW; ++v)
          sA[buf][ki + v][mi] = (mok && k0 + ki + v < ke) ? ra[VW * j + v] : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < NLB; ++j) {
      const int u = tid + NT * j;
      const int ki = (u % (BK / VW)) * VW, ni = u / (BK / VW);
      const bool nok = n0 + ni < N;
#pragma unroll
      for (int v = 0; v < VW; ++v)
        sB[buf][ki + v][ni] = (nok && k0 + ki + v < ke) ? rb[VW * j + v] : T(0);
    }
  };

  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      T av[XT], bv[YT];
#pragma unroll
      for (int x = 0; x < XT; ++x) av[x] = sA[buf][4 * ks + lg][wm + 16 * x + lr16];
#pragma unroll
      for (int y = 0; y < YT; ++y) bv[y] = sB[buf][4 * ks + lg][wn + 16 * y + lr16];
#pragma unroll
      for (int x = 0; x < XT; ++x)
#pragma unroll
        for (int y = 0; y < YT; ++y) acc[x][y] = BigMfma<T>::run(av[x], bv[y], acc[x][y]);
    }
  };

  {
    RegA ra;
    RegB rb;
    if (kb < ke) {
      load(kb, ra, rb);
      stash(0, kb, ra, rb);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) load(k0 + BK, ra, rb);
      compute(buf);
      if (more) stash(buf ^ 1, k0 + BK, ra, rb);
      __syncthreads();
      buf ^= 1;
    }
  }

  if (part) {
#pragma unroll
    for (int x = 0; x < XT; ++x)
#pragma unroll
      for (int y = 0; y < YT; ++y)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gm = m0 + wm + 16 * x + acc_row<T>(lg, e);
          const int gn = n0 + wn + 16 * y + lr16;
          if (gm < M && gn < N) part[((size_t)blockIdx.y * N + gn) * M + gm] = acc[x][y][e];
        }
    return;
  }
  // C = alpha acc + beta C, one MFMA row block (16 rows) at a time: its 4 YT
  // reads of C go out together from clamped addresses before any is used
#pragma unroll
  for (int x = 0; x < XT; ++x) {
    T cv[YT][4];
#pragma unroll
    for (int y = 0; y < YT; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = min(m0 + wm + 16 * x + acc_row<T>(lg, e), M - 1);
        const int gn = min(n0 + wn + 16 * y + lr16, N - 1);
        cv[y][e] = beta == T(0) ? T(0) : C[(long long)gn * ldc + gm];
      }
#pragma unroll
    for (int y = 0; y < YT; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wm + 16 * x + acc_row<T>(lg, e);
        const int gn = n0 + wn + 16 * y + lr16;
        const T v = alpha * acc[x][y][e];
        if (gm < M && gn < N) C[(long long)gn * ldc + gm] = (beta == T(0)) ? v : v + beta * cv[y][e];
      }
  }
}

template <typename T, bool TA, int WM, int WN, int BK, int OCC, int XT = 4, int YT = 4>
void launch_big(hipStream_t s, bool vec, int M, int N, int K, T alpha, const T* A, long long lda,
                const T* B, long long ldb, T beta, T* C, long long ldc, int kchunk, int nsplit,
                T* part) {
  constexpr int BM = 16 * XT * WM, BN = 16 * YT * WN;
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  const dim3 grid(tiles, nsplit), block(64 * WM * WN);
  if (vec)
    hipLaunchKernelGGL((k_gemm_big<T, TA, WM, WN, XT, YT, BK, OCC, true>), grid, block, 0, s,
                       M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
  else
    hipLaunchKernelGGL((k_gemm_big<T, TA, WM, WN, XT, YT, BK, OCC, false>), grid, block, 0, s,
                       M, N, K,
                       alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
}

// W pass of the left-looking schedule: for K rows in split z,
//     part[z][n][q] = sum_k V(k, q) B(k, n),   q < nq <= 16 QX,
// where the columns of B come from two segments (n < n1 from B1, the rest
// from B2), so the V^T V_prev Gram block can ride along with V^T A2.
// A wave owns 16 YN columns and all 16 QX rows q (QX YN MFMA tiles of 16 x 16);
// each lane streams its B fragments straight from memory into registers: in a
// chunk of KC rows, lane (g, c) loads the KC/4 consecutive rows g KC/4 ..
// of its columns, and MFMA step j takes row g KC/4 + j from every lane group,
// so no B data passes through LDS.  V (16 QX x KC per chunk, shared by the NW
// waves) goes through LDS.  Two chunks of B are in flight
// while one runs; loads past the range read clamped addresses and are never
// used (issued unconditionally so that waiting for one chunk never waits for
// the next).  Requires even leading dimensions, K and split ranges, and
// 16-byte aligned bases (two-element loads).
template <typename T, int QX, int KC, int YN, int NW, int OCC>
__global__ __launch_bounds__(64 * NW, OCC) void k_wpass(int K, int nq, int N, int n1,
                                                   const T* __restrict__ V, long long ldv,
                                                   const T* __restrict__ B1, long long ld1,
                                                   const T* __restrict__ B2, long long ld2,
                                                   int kchunk, T* __restrict__ part) {
  typedef T d2 __attribute__((ext_vector_type(2)));
  typedef typename BigMfma<T>::acc_t acc_t;
  constexpr int QR = 16 * QX;  // reflector rows q covered
  __shared__ T sV[2][KC][QR + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr16 = lane & 15, lg = lane >> 4;
  constexpr int NT = 64 * NW;
  const int n0 = (blockIdx.x * NW + wave) * 16 * YN;
  const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);
  const int nch = ke > kb ? (ke - kb + KC - 1) / KC : 0;  // uniform
  if (nch == 0) return;

  // this lane's YN columns
  const T* bcol[YN];
#pragma unroll
  for (int y = 0; y < YN; ++y) {
    int n = n0 + 16 * y + lr16;
    n = n < N ? n : N - 1;
    bcol[y] = n < n1 ? B1 + (long long)n * ld1 : B2 + (long long)(n - n1) * ld2;
  }
  constexpr int RL = KC / 4;  // rows per lane and chunk
  typedef T RegB[YN][RL];
  // B rows past the range read the range's last two rows again and are not
  // masked: V's rows there are zero in LDS, so they add nothing (for finite
  // data), and with no select on the loaded values the loads stay in flight
  // until the MFMAs that take them (a select right after each load made the
  // compiler wait for it there).
  auto load_b = [&](int k0, RegB& r) {
#pragma unroll
    for (int y = 0; y < YN; ++y)
#pragma unroll
      for (int p = 0; p < RL / 2; ++p) {
        const int k = k0 + RL * lg + 2 * p;
        const d2 v = *reinterpret_cast<const d2*>(bcol[y] + (k < ke ? k : ke - 2));
        r[y][2 * p] = v.x;
        r[y][2 * p + 1] = v.y;
      }
  };
  // V chunk: KC rows x QR columns, pairs along the rows
  constexpr int NVP = KC * QR / 2;                // pairs per chunk
  constexpr int NV = (NVP + NT - 1) / NT;         // pairs per thread
  // (raw values in registers; the mask is applied when they go to LDS, so
  // that nothing waits for these loads before the next chunk's compute)
  T rv[2 * NV];
  auto load_v = [&](int k0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int u = tid + NT * j;
      const int ki = (u % (KC / 2)) * 2, q = u / (KC / 2);
      const int k = k0 + ki;
      const d2 v = *reinterpret_cast<const d2*>(V + (long long)(q < nq ? q : nq - 1) * ldv +
                                                (k < ke ? k : ke - 2));
      rv[2 * j] = v.x;
      rv[2 * j + 1] = v.y;
    }
  };
  auto stash_v = [&](int buf, int k0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int u = tid + NT * j;
      const int ki = (u % (KC / 2)) * 2, q = u / (KC / 2);
      const bool ok = q < nq && k0 + ki < ke;   // k0 + ki even and ke even
      if (NV * NT == NVP || u < NVP) {          // (pairs past the chunk: none stored)
        sV[buf][ki][q] = ok ? rv[2 * j] : T(0);
        sV[buf][ki + 1][q] = ok ? rv[2 * j + 1] : T(0);
      }
    }
  };
  acc_t acc[QX][YN];
#pragma unroll
  for (int x = 0; x < QX; ++x)
#pragma unroll
    for (int y = 0; y < YN; ++y) acc[x][y] = acc_t{0, 0, 0, 0};
  auto compute = [&](int buf, const RegB& r) {
#pragma unroll
    for (int j = 0; j < RL; ++j) {
      T av[QX];
#pragma unroll
      for (int x = 0; x < QX; ++x) av[x] = sV[buf][RL * lg + j][16 * x + lr16];
#pragma unroll
      for (int x = 0; x < QX; ++x)
#pragma unroll
        for (int y = 0; y < YN; ++y) acc[x][y] = BigMfma<T>::run(av[x], r[y][j], acc[x][y]);
    }
  };

  // An even number of chunks (a trailing chunk past the range reads clamped
  // addresses, is masked to zero and adds nothing): a loop body without an
  // early exit keeps the accumulators in one register set (an exit between
  // the two halves made the compiler copy all of them every iteration).
  const int nch2 = (nch + 1) & ~1;
  // (each chunk's V load is issued before its B loads, here as in the loop,
  // so the wait for a V chunk never covers the B loads that follow it)
  RegB r0, r1;
  load_v(kb);
  load_b(kb, r0);
  stash_v(0, kb);
  load_v(kb + KC);
  load_b(kb + KC, r1);
  __syncthreads();
  for (int t = 0; t < nch2; t += 2) {
    compute(0, r0);
    stash_v(1, kb + (t + 1) * KC);
    load_v(kb + (t + 2) * KC);
    load_b(kb + (t + 2) * KC, r0);
    __syncthreads();
    compute(1, r1);
    stash_v(0, kb + (t + 2) * KC);
    load_v(kb + (t + 3) * KC);
    load_b(kb + (t + 3) * KC, r1);
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < QX; ++x)
#pragma unroll
    for (int y = 0; y < YN; ++y) {
      const int n = n0 + 16 * y + lr16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = 16 * x + acc_row<T>(lg, e);
        if (n < N && q < nq) part[((size_t)blockIdx.y * N + n) * nq + q] = acc[x][y][e];
      }
    }
}

// C = alpha sum_z part[z] + beta C (partials in split order)
template <typename T>
__global__ void k_big_sum(int M, int N, int S, const T* __restrict__ part, T alpha, T beta,
                          T* __restrict__ C, long long ldc) {
  const long long total = (long long)M * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    T acc = part[e];
    for (int z = 1; z < S; ++z) acc += part[(size_t)z * total + e];
    T* c = C + (e / M) * ldc + e % M;
    const T v = alpha * acc;
    *c = (beta == T(0)) ? v : v + beta * (*c);
  }
}

constexpr int kBK = 16;

unsigned grid_for(long long total) {
  const long long g = (total + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// Output tiles of the variant gemm_big picks for this shape.
int big_tiles(bool ta, int M, int N) {
  int bm = 128, bn = 128;
  if (ta && M <= 64) { bm = 64; bn = 256; }
  else if (!ta && M <= 64) { bm = 64; bn = 128; }
  else if (!ta && (N <= 64 || M <= 128)) { bm = 64; bn = 64; }
  return ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
}

template <typename T>
void big_launch(hipStream_t s, bool ta, int M, int N, int K, T alpha, const T* A, long long lda,
                const T* B, long long ldb, T beta, T* C, long long ldc, int kchunk, int nsplit,
                T* part) {
  // two-element loads: even leading dimensions and K, aligned bases, and an
  // even row count when A's rows are the contiguous index
  const uintptr_t al = 2 * sizeof(T);
  const bool vec = K > 0 && lda % 2 == 0 && ldb % 2 == 0 && K % 2 == 0 && kchunk % 2 == 0 &&
                   (reinterpret_cast<uintptr_t>(A) % al) == 0 &&
                   (reinterpret_cast<uintptr_t>(B) % al) == 0 && (ta || M % 2 == 0);
  if (ta) {
    if (M <= 64)
      launch_big<T, true, 1, 4, 8, 2>(s, vec, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                      kchunk, nsplit, part);
    else
      launch_big<T, true, 2, 2, kBK, 2>(s, vec, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                        kchunk, nsplit, part);
  } else {
    if (M <= 64)
      launch_big<T, false, 1, 2, kBK, 2>(s, vec, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                         kchunk, nsplit, part);
    else if (N <= 64 || M <= 128)   // 64 x 64 tiles as four waves of 32 x 32 (narrow or
                                    // short products: more tiles)
      launch_big<T, false, 2, 2, kBK, 2, 2, 2>(s, vec, M, N, K, alpha, A, lda, B, ldb, beta, C,
                                               ldc, kchunk, nsplit, part);
    else  // 128 x 128 tiles as eight waves of 64 x 32 (two workgroups per CU; 1.4%
          // faster than 32 x 64 on the 15360^2 x 1024 FP64 product)
      launch_big<T, false, 2, 4, kBK, 2, 4, 2>(s, vec, M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                  ldc, kchunk, nsplit, part);
  }
}

// K ranges of whole 16-steps for at most `want` splits: (kchunk, count)
void big_split(int K, int want, int* kchunk, int* nsplit) {
  if (want < 2 || K <= kBK) {
    *kchunk = K > 0 ? K : 1;
    *nsplit = 1;
    return;
  }
  *kchunk = ((K + want - 1) / want + kBK - 1) / kBK * kBK;
  *nsplit = (K + *kchunk - 1) / *kchunk;
}

}  // namespace

template <typename T>
int gemm_big(hipStream_t s, bool ta, int M, int N, int K, T alpha, const T* A, long long lda,
             const T* B, long long ldb, T beta, T* C, long long ldc, T* ws, size_t ws_elems) {
  if (M <= 0 || N <= 0) return RQ_OK;
  // few output tiles and a long reduction: split K so the grid covers the
  // chip (about 512 workgroups), raw partials in ws, summed in split order
  int want = 1;
  const int tiles = big_tiles(ta, M, N);
  if (ws && tiles < 512 && K >= 4 * kBK) {
    want = (512 + tiles - 1) / tiles;
    want = std::min(want, K / (2 * kBK));
    want = std::min<long long>(want, (long long)(ws_elems / ((size_t)M * N)));
    want = std::min(want, 64);
  }
  int kchunk = 1, nsplit = 1;
  big_split(K, want, &kchunk, &nsplit);
  if (nsplit > 1) {
    big_launch<T>(s, ta, M, N, K, T(1), A, lda, B, ldb, T(0), nullptr, 0, kchunk, nsplit, ws);
    hipLaunchKernelGGL(k_big_sum<T>, dim3(grid_for((long long)M * N)), dim3(256), 0, s, M, N,
                       nsplit, (const T*)ws, alpha, beta, C, ldc);
  } else {
    big_launch<T>(s, ta, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, 1, nullptr);
  }
  RQ_HIP_CHECK(hipGetLastError());
  return RQ_OK;
}

template <typename T>
int gemm_big_partials(hipStream_t s, bool ta, int M, int N, int K, const T* A, long long lda,
                      const T* B, long long ldb, T* part, int max_split, int* nsplit_out) {
  *nsplit_out = 0;
  if (M <= 0 || N <= 0) return RQ_OK;
  int kchunk = 1, nsplit = 1;
  big_split(K, max_split, &kchunk, &nsplit);
  big_launch<T>(s, ta, M, N, K, T(1), A, lda, B, ldb, T(0), nullptr, 0, kchunk, nsplit, part);
  RQ_HIP_CHECK(hipGetLastError());
  *nsplit_out = nsplit;
  return RQ_OK;
}

template <typename T>
int wpass_partials(hipStream_t s, int K, int nq, int N, int n1, const T* V, long long ldv,
                   const T* B1, long long ld1, const T* B2, long long ld2, T* part,
                   int max_split, int* nsplit_out) {
  *nsplit_out = 0;
  if (N <= 0 || nq <= 0) return RQ_OK;
  if (nq > (sizeof(T) == 8 ? 128 : 64)) return RQ_ERR_LIMIT;
  const uintptr_t al = 2 * sizeof(T);
  const bool fits = K >= 2 && K % 2 == 0 && ldv % 2 == 0 && ld1 % 2 == 0 && ld2 % 2 == 0 &&
                    reinterpret_cast<uintptr_t>(V) % al == 0 &&
                    reinterpret_cast<uintptr_t>(B1) % al == 0 &&
                    (n1 >= N || reinterpret_cast<uintptr_t>(B2) % al == 0);
  if (!fits) return RQ_ERR_LIMIT;
  constexpr int KC = 16, NW = 8;   // two workgroups of eight waves per CU
  static_assert(kWpassCols == 16 * NW, "one 16-column tile per wave");
  int want = std::max(1, max_split);
  int kchunk = ((K + want - 1) / want + KC - 1) / KC * KC;
  const int nsplit = (K + kchunk - 1) / kchunk;
  auto go = [&](auto kern, int cols) {
    hipLaunchKernelGGL(kern, dim3((N + cols - 1) / cols, nsplit), dim3(64 * NW), 0, s, K, nq, N,
                       n1, V, ldv, B1, ld1, B2, ld2, kchunk, part);
  };
  // 16 columns per wave, 128 per workgroup, two workgroups per CU (64
  // reflector rows: 82 registers; 128 rows, FP64 only: 128 registers; for FP32
  // storage with 128 rows the LDS-staged GEMM measured as fast).  At 64 rows,
  // 16384 x 16320 FP64, this measured 9% faster than 32 columns per wave.
  if (nq <= 64)
    go(&k_wpass<T, 4, KC, 1, NW, 4>, kWpassCols);
  else if constexpr (sizeof(T) == 8) {
    if (nq <= 80)   // e.g. the sketch's b + p = 72 rows
      go(&k_wpass<T, 5, KC, 1, NW, 4>, kWpassCols);
    else
      go(&k_wpass<T, 8, KC, 1, NW, 2>, kWpassCols);
  }
  RQ_HIP_CHECK(hipGetLastError());
  *nsplit_out = nsplit;
  return RQ_OK;
}
template int wpass_partials<double>(hipStream_t, int, int, int, int, const double*, long long,
                                    const double*, long long, const double*, long long, double*,
                                    int, int*);
template int wpass_partials<float>(hipStream_t, int, int, int, int, const float*, long long,
                                   const float*, long long, const float*, long long, float*, int,
                                   int*);

template int gemm_big<double>(hipStream_t, bool, int, int, int, double, const double*, long long,
                              const double*, long long, double, double*, long long, double*,
                              size_t);
template int gemm_big<float>(hipStream_t, bool, int, int, int, float, const float*, long long,
                             const float*, long long, float, float*, long long, float*, size_t);
template int gemm_big_partials<double>(hipStream_t, bool, int, int, int, const double*, long long,
                                       const double*, long long, double*, int, int*);
template int gemm_big_partials<float>(hipStream_t, bool, int, int, int, const float*, long long,
                                      const float*, long long, float*, int, int*);

}  // namespace rq
