// Device building blocks of libmbdp: the sweep order, the grid barrier,
// wavefront reductions and order-preserving keys for atomic max/min.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mbdp_internal.h"

namespace mbdp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// ------------------------------------------------------------ sweep order
//
// Philox-4x32-10 (Salmon et al., SC'11): ten rounds of
//   (x0,x1,x2,x3) <- (hi(B*x2)^x1^k0, lo(B*x2), hi(A*x0)^x3^k1, lo(A*x0))
// with A = 0xD2511F53, B = 0xCD9E8D57 and the key advanced by the Weyl
// increments (0x9E3779B9, 0xBB67AE85) between rounds.  Only output word 0
// is needed by the order.
__device__ __forceinline__ uint32_t philox_word0(uint32_t x0, uint32_t x1, uint32_t x2,
                                                 uint32_t x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t a_hi = __umulhi(0xD2511F53u, x0), a_lo = 0xD2511F53u * x0;
    const uint32_t b_hi = __umulhi(0xCD9E8D57u, x2), b_lo = 0xCD9E8D57u * x2;
    const uint32_t y0 = b_hi ^ x1 ^ k0;
    const uint32_t y2 = a_hi ^ x3 ^ k1;
    x0 = y0;
    x1 = b_lo;
    x2 = y2;
    x3 = a_lo;
  }
  return x0;
}

// The order of sweep t: a 4-round Feistel network on [0, 4^h) with h the
// smallest h >= 1 such that 4^h >= n, round j mapping the right half R to
// word0(Philox(counter = (R, j, t_lo, t_hi), key = (seed_lo, seed_hi))) & mask,
// restricted to [0, n) by cycle walking.  Any round function gives a
// bijection; cycle walking keeps it one on [0, n).
struct OrderKey {
  uint32_t n, h, mask, s_lo, s_hi, t_lo, t_hi;
};

__device__ __forceinline__ OrderKey make_order_key(int64_t n, uint64_t seed, uint64_t t) {
  OrderKey k;
  k.n = (uint32_t)n;
  uint32_t h = 1;
  while ((1ull << (2 * h)) < (unsigned long long)n) ++h;
  k.h = h;
  k.mask = (1u << h) - 1u;
  k.s_lo = (uint32_t)seed;
  k.s_hi = (uint32_t)(seed >> 32);
  k.t_lo = (uint32_t)t;
  k.t_hi = (uint32_t)(t >> 32);
  return k;
}

__device__ __forceinline__ uint32_t feistel(uint32_t x, const OrderKey& k) {
  uint32_t left = x >> k.h, right = x & k.mask;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) {
    const uint32_t f = philox_word0(right, j, k.t_lo, k.t_hi, k.s_lo, k.s_hi) & k.mask;
    const uint32_t nr = left ^ f;
    left = right;
    right = nr;
  }
  return (left << k.h) | right;
}

__device__ __forceinline__ uint32_t sweep_order_at(uint32_t p, const OrderKey& k) {
  uint32_t y = feistel(p, k);
  while (y >= k.n) y = feistel(y, k);
  return y;
}

// The network run backwards: round j maps (L, R) to (R ^ f_j(L), L).
__device__ __forceinline__ uint32_t feistel_inverse(uint32_t y, const OrderKey& k) {
  uint32_t left = y >> k.h, right = y & k.mask;
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    const uint32_t f = philox_word0(left, (uint32_t)j, k.t_lo, k.t_hi, k.s_lo, k.s_hi) & k.mask;
    const uint32_t prev_left = right ^ f;
    right = left;
    left = prev_left;
  }
  return (left << k.h) | right;
}

// Position of state s in the order of sweep t, sigma_t^{-1}(s): cycle walking
// backwards through the values outside [0, n).
__device__ __forceinline__ uint32_t sweep_position_of(uint32_t s, const OrderKey& k) {
  uint32_t x = feistel_inverse(s, k);
  while (x >= k.n) x = feistel_inverse(x, k);
  return x;
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}

// (q, a) <- the smaller Q-value, the lower action index on ties, over lanes
// whose index differs in the bits of [first_off, 64).
__device__ __forceinline__ void wave_argmin(double& q, int& a, int first_off = 1) {
  for (int off = first_off; off < kWave; off <<= 1) {
    const double q2 = __shfl_xor(q, off);
    const int a2 = __shfl_xor(a, off);
    if (q2 < q || (q2 == q && a2 < a)) {
      q = q2;
      a = a2;
    }
  }
}

// The same over the lane bits [FIRST, 64) with constant offsets (unrolled).
template <int FIRST>
__device__ __forceinline__ void wave_argmin_from(double& q, int& a) {
#pragma unroll
  for (int off = FIRST; off < kWave; off <<= 1) {
    const double q2 = __shfl_xor(q, off);
    const int a2 = __shfl_xor(a, off);
    const bool take = q2 < q || (q2 == q && a2 < a);
    q = take ? q2 : q;
    a = take ? a2 : a;
  }
}

// Order-preserving 64-bit key of a double (monotone in the value).
__device__ __forceinline__ unsigned long long okey(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double okey_value(unsigned long long k) {
  const unsigned long long u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double((long long)u);
}

__device__ __forceinline__ unsigned long long atomic_load_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ grid barrier
//
// All workgroups of a cooperative launch meet here, once per batch.  The
// cost of a device-wide barrier on MI355X grows with the number of
// workgroups and with contention on one atomic counter, so arrival is
// contention-free: every wave first waits for its own memory operations
// (vmcnt(0)), then one thread per workgroup makes the workgroup's writes
// visible device-wide (agent-scope release: L2 write-back) and stores the
// barrier generation into the workgroup's own arrival slot.  Workgroup 0
// polls all slots in parallel (one per thread) and then publishes the
// generation in a single release word that the others poll, followed by an
// agent-scope acquire (L2 invalidate) before anyone reads shared data.
// Every wait gives up after `timeout` wall-clock ticks or when another
// workgroup raised the abort flag, so no wave can spin forever.  Returns
// false when aborted.
struct GridBarrier {
  Control* ctl;
  unsigned long long gen;      // barriers passed so far
  unsigned long long nblocks;
  unsigned long long timeout;
};

__device__ __forceinline__ void raise_abort(Control* ctl, unsigned int code) {
  atomicCAS(&ctl->error, 0u, code);
  __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spins until *word >= target; false on abort or timeout.
__device__ __forceinline__ bool wait_at_least(const unsigned long long* word,
                                              unsigned long long target, const GridBarrier& g) {
  const unsigned long long t0 = wall_clock64();
  while (atomic_load_agent(word) < target) {
    if (__hip_atomic_load(&g.ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (wall_clock64() - t0 > g.timeout) {
      raise_abort(g.ctl, kDevBarrierTimeout);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

__device__ __forceinline__ bool grid_sync(GridBarrier& g) {
  __shared__ int s_abort;
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads and stores are done
  __syncthreads();
  g.gen += 1;
  unsigned long long* slots = g.ctl->bar_slots;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomic_store_agent(&slots[blockIdx.x], g.gen);
  }
  int ok = 1;
  if (blockIdx.x == 0) {
    for (unsigned i = threadIdx.x; i < g.nblocks && ok; i += blockDim.x)
      ok = wait_at_least(&slots[i], g.gen, g);
    // Workgroup 0 relays the arrivals: an acquire after observing them and a
    // release before publishing make every arrival happen before the release
    // word's store, so each workgroup's acquire below synchronises with all
    // arrivals through workgroup 0 (release -> acquire at agent scope, then
    // the workgroup barrier, then release -> acquire again).
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomic_store_agent(&g.ctl->bar_release, g.gen);
    }
  }
  if (threadIdx.x == 0) {
    if (ok) ok = wait_at_least(&g.ctl->bar_release, g.gen, g);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok) ok = __hip_atomic_load(&g.ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    s_abort = !ok;
  }
  __syncthreads();
  return s_abort == 0;
}

}  // namespace mbdp
