// Shared device helpers for librqrcp (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RQ_DEV __device__ __forceinline__

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Status codes (mirrored in include/rqrcp.h)
// ---------------------------------------------------------------------------
enum {
  RQ_OK = 0,
  RQ_ERR_HIP = 1001,
  RQ_ERR_WORKSPACE = 1002,
  RQ_ERR_UNSUPPORTED = 1003,
  RQ_ERR_DEVICE = 1004,
  RQ_ERR_LIMIT = 1005,
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and Box-Muller normals.
// key = (seed, stream); normal number q uses counter (q/4 + 1, 0, 0, 0) and
// output word q%4; u = ((x >> 12) + 1/2) 2^-52.
// ---------------------------------------------------------------------------
namespace rq {

constexpr uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;
constexpr double TWO_PI = 6.283185307179586;

RQ_DEV void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(PHILOX_M0, c[0]);
    const uint64_t lo0 = PHILOX_M0 * c[0];
    const uint64_t hi1 = __umul64hi(PHILOX_M1, c[2]);
    const uint64_t lo1 = PHILOX_M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
}

RQ_DEV double philox_uniform(uint64_t x) {
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

// The four normals of counter block `blk` (= q/4) of stream (seed, stream).
RQ_DEV void philox_normals4(uint64_t blk, uint64_t seed, uint64_t stream, double z[4]) {
  uint64_t c[4] = {blk + 1, 0, 0, 0};
  philox4x64_10(c, seed, stream);
  const double u0 = philox_uniform(c[0]), u1 = philox_uniform(c[1]);
  const double u2 = philox_uniform(c[2]), u3 = philox_uniform(c[3]);
  const double r01 = sqrt(-2.0 * log(u0));
  const double r23 = sqrt(-2.0 * log(u2));
  const double t01 = TWO_PI * u1;
  const double t23 = TWO_PI * u3;
  z[0] = r01 * cos(t01);
  z[1] = r01 * sin(t01);
  z[2] = r23 * cos(t23);
  z[3] = r23 * sin(t23);
}

// ---------------------------------------------------------------------------
// MFMA wrappers.  Operand layouts of the 16x16x4 forms (64 lanes):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   C/D (16x16), FP64: lane l, element e holds D[l / 16 + 4 e][l % 16]
//   C/D (16x16), FP32: lane l, element e holds D[4 (l / 16) + e][l % 16]
// acc_row<T>(g, e) gives the row for g = l / 16.
// ---------------------------------------------------------------------------
RQ_DEV v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
RQ_DEV v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
RQ_DEV int acc_row(int g, int e);
template <>
RQ_DEV int acc_row<double>(int g, int e) { return g + 4 * e; }
template <>
RQ_DEV int acc_row<float>(int g, int e) { return 4 * g + e; }

// ---------------------------------------------------------------------------
// Grid-wide barrier for persistent (co-resident) grids.  Sense-reversing:
// the last arriving workgroup resets the counter and bumps the generation,
// so the state is reusable across barriers and launches.  Every wait is
// bounded: after `RQ_SPIN_LIMIT` polls the waiter raises *err and proceeds,
// so a grid that is not fully resident still terminates.
// ---------------------------------------------------------------------------
struct GridBarrier {
  unsigned count;
  unsigned gen;
  unsigned err;
  unsigned pad[61];  // keep the flag lines apart from other data
};

#ifndef RQ_SPIN_LIMIT
#define RQ_SPIN_LIMIT (1u << 24)
#endif

RQ_DEV unsigned atomic_load_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
RQ_DEV unsigned atomic_peek_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-workgroup barrier state kept in LDS: the generation this workgroup
// waits to see move, tracked locally so that arriving needs no extra read.
struct BarrierLocal {
  unsigned gen;
  unsigned last;
};

// Once per launch, by all threads, before the first barrier of the launch
// (safe: no barrier of this launch can complete before this workgroup arrives).
RQ_DEV void grid_sync_init(GridBarrier* bar, BarrierLocal* bl) {
  if (threadIdx.x == 0) bl->gen = atomic_peek_agent(&bar->gen);
  __syncthreads();
}

// Phase 1 (all threads): arrive with one acquire-release RMW.  Returns true in
// every thread of the last workgroup to arrive, which then sees every other
// workgroup's global writes made before their arrival.
RQ_DEV bool grid_arrive(GridBarrier* bar, unsigned nwg, BarrierLocal* bl) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned arrived =
        __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    bl->last = (arrived == nwg - 1) ? 1u : 0u;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(bl->last) != 0;  // uniform for the compiler too
}

// Two-level arrive: workgroups count themselves in groups of GRID_GROUP on
// separate counters (sub[grp * GRID_SUB_STRIDE]); the last of each group
// counts the group on bar->count.  Fewer atomics queue on any one address
// than with a single counter.  Same contract as grid_arrive: returns true in
// every thread of the workgroup that completed the barrier, which then sees
// every workgroup's writes made before its arrival (acquire-release chain).
constexpr int GRID_GROUP = 16;
constexpr int GRID_SUB_STRIDE = 32;  // one 128-byte line per group counter
RQ_DEV bool grid_arrive2(GridBarrier* bar, unsigned* sub, unsigned nwg, BarrierLocal* bl) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned grp = blockIdx.x / GRID_GROUP;
    const unsigned ngrp = (nwg + GRID_GROUP - 1) / GRID_GROUP;
    const unsigned gsize = min((unsigned)GRID_GROUP, nwg - grp * GRID_GROUP);
    unsigned* c = sub + grp * GRID_SUB_STRIDE;
    const unsigned a = __hip_atomic_fetch_add(c, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    unsigned last = 0u;
    if (a == gsize - 1) {
      __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned b =
          __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      last = (b == ngrp - 1) ? 1u : 0u;
    }
    bl->last = last;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(bl->last) != 0;  // uniform for the compiler too
}

// Phase 2a (all threads of the last workgroup): release the others.
RQ_DEV void grid_release(GridBarrier* bar, BarrierLocal* bl) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&bar->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    bl->gen += 1u;
  }
  __syncthreads();
}

// Phase 2b (all threads of the other workgroups): bounded wait.  Polls with
// relaxed loads; one acquire fence once the generation has moved.
RQ_DEV void grid_wait(GridBarrier* bar, BarrierLocal* bl) {
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    while (atomic_peek_agent(&bar->gen) == bl->gen) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > RQ_SPIN_LIMIT) {
        atomicOr(&bar->err, 1u);
        break;
      }
      if ((spins & 1023u) == 0 && atomic_peek_agent(&bar->err)) break;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    bl->gen += 1u;
  }
  __syncthreads();
}

// Publish-and-poll exchange: a workgroup publishes a record by writing it and
// then storing `seq` into the record's sequence word with release semantics
// (called by thread 0 after a workgroup barrier, so every thread's record
// writes are ordered before it).  Readers wait until the sequence words of
// all `n` records (stride `stride` 32-bit words) equal `seq`, then acquire.
// One workgroup-wide barrier; no shared counter, so no atomic contention.
RQ_DEV void publish_seq(unsigned* seqword, unsigned seq) {
  __hip_atomic_store(seqword, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
RQ_DEV void wait_all_seq(const unsigned* seq0, long long stride, int n, unsigned seq,
                         GridBarrier* bar) {
  if ((threadIdx.x >> 6) == 0) {
    const int lane = threadIdx.x & 63;
    for (int q = lane; q < n; q += 64) {
      const unsigned* w = seq0 + (long long)q * stride;
      // two polls in flight: each check waits only for the older one
      unsigned spins = 0;
      unsigned va = atomic_peek_agent(w);
      unsigned vb = atomic_peek_agent(w);
      for (;;) {
        if (va == seq) break;
        va = atomic_peek_agent(w);
        if (vb == seq) break;
        vb = atomic_peek_agent(w);
        spins += 2;
        if (spins > RQ_SPIN_LIMIT) {
          atomicOr(&bar->err, 1u);
          break;
        }
        if ((spins & 1022u) == 0 && atomic_peek_agent(&bar->err)) break;
      }
    }
    // one acquire for the workgroup (the invalidation is per cache, not per wave)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

RQ_DEV void grid_barrier(GridBarrier* bar, unsigned nwg, BarrierLocal* bl) {
  if (grid_arrive(bar, nwg, bl))
    grid_release(bar, bl);
  else
    grid_wait(bar, bl);
}

// ---------------------------------------------------------------------------
// Wave-wide reductions with DPP (data-parallel primitives of the VALU: row
// shifts within 16-lane rows, then row broadcasts).  The inclusive scan
// pattern row_shr 1,2,4,8 + row_bcast 15,31 leaves the total in lane 63,
// which readlane then broadcasts.  Much cheaper than LDS-routed shuffles.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
RQ_DEV double dpp_f64(double old, double v) {
  const long long ov = __double_as_longlong(old), vv = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)ov, (int)vv, CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO);
  const int hi = __builtin_amdgcn_update_dpp((int)(ov >> 32), (int)(vv >> 32), CTRL, ROW_MASK,
                                             BANK_MASK, BOUND_ZERO);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
RQ_DEV int dpp_i32(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO);
}
RQ_DEV double readlane_f64(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// DPP controls (GCN/CDNA encoding)
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114,
              DPP_ROW_SHR8 = 0x118, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143,
              DPP_QUAD_XOR1 = 0xB1,  // quad_perm [1,0,3,2]
              DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]

// Sum over the wave, returned in every lane.  The summation order is fixed.
RQ_DEV double wave_sum_dpp(double v) {
  v += dpp_f64<DPP_ROW_SHR1, 0xf, 0xf, true>(0.0, v);
  v += dpp_f64<DPP_ROW_SHR2, 0xf, 0xf, true>(0.0, v);
  v += dpp_f64<DPP_ROW_SHR4, 0xf, 0xe, true>(0.0, v);
  v += dpp_f64<DPP_ROW_SHR8, 0xf, 0xc, true>(0.0, v);
  v += dpp_f64<DPP_ROW_BCAST15, 0xa, 0xf, false>(0.0, v);
  v += dpp_f64<DPP_ROW_BCAST31, 0xc, 0xf, false>(0.0, v);
  return readlane_f64(v, 63);
}

// Sum of adjacent lane pairs (lane ^ 1), returned in both lanes.
RQ_DEV double pair_sum_dpp(double v) {
  return v + dpp_f64<DPP_QUAD_XOR1, 0xf, 0xf, false>(v, v);
}

// Sum over each quad of lanes (lane ^ 1, lane ^ 2), returned in all four.
RQ_DEV double quad_sum_dpp(double v) {
  v = pair_sum_dpp(v);
  return v + dpp_f64<DPP_QUAD_XOR2, 0xf, 0xf, false>(v, v);
}

// Arg-max over the wave of (n, then lowest p); s is carried along.  The
// result is returned in every lane.  Lanes with no candidate pass n < 0.
RQ_DEV bool argbetter(double n1, int p1, double n2, int p2) {
  return n1 > n2 || (n1 == n2 && p1 < p2);
}
template <int CTRL, int ROW_MASK, int BANK_MASK>
RQ_DEV void argmax_step(double& n, int& p, int& s) {
  // disabled / out-of-row lanes read their own value (old = own), a no-op
  const double n2 = dpp_f64<CTRL, ROW_MASK, BANK_MASK, false>(n, n);
  const int p2 = dpp_i32<CTRL, ROW_MASK, BANK_MASK, false>(p, p);
  const int s2 = dpp_i32<CTRL, ROW_MASK, BANK_MASK, false>(s, s);
  if (argbetter(n2, p2, n, p)) {
    n = n2;
    p = p2;
    s = s2;
  }
}
RQ_DEV void wave_argmax(double& n, int& p, int& s) {
  argmax_step<DPP_ROW_SHR1, 0xf, 0xf>(n, p, s);
  argmax_step<DPP_ROW_SHR2, 0xf, 0xf>(n, p, s);
  argmax_step<DPP_ROW_SHR4, 0xf, 0xe>(n, p, s);
  argmax_step<DPP_ROW_SHR8, 0xf, 0xc>(n, p, s);
  argmax_step<DPP_ROW_BCAST15, 0xa, 0xf>(n, p, s);
  argmax_step<DPP_ROW_BCAST31, 0xc, 0xf>(n, p, s);
  n = readlane_f64(n, 63);
  p = __builtin_amdgcn_readlane(p, 63);
  s = __builtin_amdgcn_readlane(s, 63);
}

// ---------------------------------------------------------------------------
// Misc.
// ---------------------------------------------------------------------------
RQ_DEV double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
RQ_DEV T ld_elem(const T* p) { return *p; }

}  // namespace rq

// Host-side helper
#define RQ_HIP_CHECK(expr)                                   \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return RQ_ERR_HIP;                 \
  } while (0)
