// HIP kernels of libmbdp for gfx950 (MI355X).
//
// One persistent, cooperatively launched kernel runs a whole call: one sweep
// (mb_sweep), MB-VI (vi_solve) or MB-MPI (mpi_solve).  A sweep of the
// mini-batch operator (Sec. III-A, eqs. (10)-(12)) processes the states in
// the order sigma_t, cut into batches of b consecutive positions; the
// states of one batch are computed in parallel from the values before the
// batch and committed together, so later batches see them.  Between batches
// every workgroup meets at a device-wide barrier (one per batch), instead
// of one kernel launch per batch.
//
// Visibility of V across batches uses two buffers.  In the phase of batch k
// the kernel reads buffer R (complete up to batch k-1) and writes into the
// other buffer W the new values of batch k and a copy of batch k-1 (still
// missing there).  After the barrier the roles swap.  No state of a batch
// can therefore read a value of its own batch (Jacobi inside a batch, as
// eq. (11) requires: M_b(i) holds only earlier batches).  Batches of one
// sweep are disjoint, but the first batch of sweep t+1 may share states with
// the last batch of sweep t (all of them when b = n); such states are
// stamped when the first batch's order is drawn and not copied forward, so
// the copy can never overwrite their new value.  Stamps live in two arrays
// by sweep parity: with b = n the next sweep's stamps are written in the
// same phase that reads the current sweep's.
//
// The hot loop is the row gather + dot product Q(s,a) = c(s,a) +
// gamma * sum_s' P(s,a,s') V(s'):
//  * dense: a workgroup per (state, column block), all m rows of the state
//    streamed with non-temporal 16-byte loads, V reused from registers for
//    the m rows, partial sums reduced through LDS (and, for small b, across
//    workgroups with per-state arrival counters);
//  * constant row length k (ELL): a wavefront per state, k/4 lanes per row,
//    one 16-byte load of columns and one of weights per lane, V gathered;
//  * general CSR: a wavefront per state, lanes striding over each row.
// Dot products accumulate in FP32; cost, discount and the action minimum
// are done in FP64 and the result rounded to FP32.
//
// The order of the next batch is computed during the current one and
// stored, so its ALU work overlaps the memory stream.

#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>

#include "mbdp_device.h"
#include "mbdp_internal.h"

namespace mbdp {

// ------------------------------------------------------------ accumulators

// Accumulators of the current epoch: max |dW|, max error against V_ref,
// max |TW - W|, the range of W and the policy changes.  Two forms with one
// interface.  RegAcc keeps them per thread in registers (committing lanes
// only) and reduces them at the flush; LdsAcc keeps one copy per workgroup
// in LDS, updated with LDS atomics, and holds no registers, for the dense
// engine whose row tiles need every register (it commits few states).
struct RegAcc {
  double v[3];  // kAccDv, kAccErr, kAccResid slots below
  double wmax, wmin;
  unsigned long long changes;

  __device__ __forceinline__ static int idx(int i) { return i == kAccDv ? 0 : (i == kAccErr ? 1 : 2); }
  __device__ __forceinline__ void init() {
    v[0] = v[1] = v[2] = 0.0;
    wmax = -INFINITY;
    wmin = INFINITY;
    changes = 0;
  }
  __device__ __forceinline__ void max_abs(int i, double x) { v[idx(i)] = fmax(v[idx(i)], x); }
  __device__ __forceinline__ void range(double w) {
    wmax = fmax(wmax, w);
    wmin = fmin(wmin, w);
  }
  __device__ __forceinline__ void count_change() { changes += 1; }

  // Merges the workgroup's values into epoch slot `slot` and clears them.
  // Every thread of the workgroup must call it.
  __device__ __forceinline__ void flush(Control* ctl, int slot) {
    __shared__ double sh[16][5];
    __shared__ unsigned long long shc[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const double dv = wave_max_d(v[0]), err = wave_max_d(v[1]), res = wave_max_d(v[2]);
    const double hi = wave_max_d(wmax), lo = wave_min_d(wmin);
    unsigned long long ch = changes;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ch += __shfl_xor(ch, off);
    if (lane == 0) {
      sh[w][0] = dv;
      sh[w][1] = err;
      sh[w][2] = res;
      sh[w][3] = hi;
      sh[w][4] = lo;
      shc[w] = ch;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = sh[0][0], b = sh[0][1], c = sh[0][2], d = sh[0][3], e = sh[0][4];
      unsigned long long f = shc[0];
      for (int i = 1; i < nw; ++i) {
        a = fmax(a, sh[i][0]);
        b = fmax(b, sh[i][1]);
        c = fmax(c, sh[i][2]);
        d = fmax(d, sh[i][3]);
        e = fmin(e, sh[i][4]);
        f += shc[i];
      }
      unsigned long long* acc = ctl->acc[slot];
      if (a > 0.0) atomicMax(&acc[kAccDv], (unsigned long long)__double_as_longlong(a));
      if (b > 0.0) atomicMax(&acc[kAccErr], (unsigned long long)__double_as_longlong(b));
      if (c > 0.0) atomicMax(&acc[kAccResid], (unsigned long long)__double_as_longlong(c));
      if (d > -INFINITY) atomicMax(&acc[kAccWmax], okey(d));
      if (e < INFINITY) atomicMin(&acc[kAccWmin], okey(e));
      if (f) atomicAdd(&acc[kAccChanges], f);
    }
    __syncthreads();
    init();
  }
};

struct LdsAcc {
  unsigned long long* a;  // [kNumAcc]: doubles >= 0 as bits, the W range as ordered keys

  __device__ __forceinline__ void init() {
    __shared__ unsigned long long acc[kNumAcc];
    a = acc;
    if (threadIdx.x == 0)  // visible after the next barrier, before any commit
      for (int i = 0; i < kNumAcc; ++i) a[i] = (i == kAccWmin) ? ~0ull : 0ull;
  }
  __device__ __forceinline__ void max_abs(int i, double x) {  // NaN is ignored, as by fmax
    if (x == x) atomicMax(&a[i], (unsigned long long)__double_as_longlong(x));
  }
  __device__ __forceinline__ void range(double w) {
    atomicMax(&a[kAccWmax], okey(w));
    atomicMin(&a[kAccWmin], okey(w));
  }
  __device__ __forceinline__ void count_change() { atomicAdd(&a[kAccChanges], 1ull); }

  __device__ __forceinline__ void flush(Control* ctl, int slot) {
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long* acc = ctl->acc[slot];
      if (a[kAccDv]) atomicMax(&acc[kAccDv], a[kAccDv]);
      if (a[kAccErr]) atomicMax(&acc[kAccErr], a[kAccErr]);
      if (a[kAccResid]) atomicMax(&acc[kAccResid], a[kAccResid]);
      if (a[kAccWmax]) atomicMax(&acc[kAccWmax], a[kAccWmax]);
      if (a[kAccWmin] != ~0ull) atomicMin(&acc[kAccWmin], a[kAccWmin]);
      if (a[kAccChanges]) atomicAdd(&acc[kAccChanges], a[kAccChanges]);
      for (int i = 0; i < kNumAcc; ++i) a[i] = (i == kAccWmin) ? ~0ull : 0ull;
    }
    __syncthreads();
  }
};

__device__ __forceinline__ void reset_slot(Control* ctl, int slot) {
  for (int i = 0; i < kNumAcc; ++i) {
    unsigned long long v = 0ull;
    if (i == kAccWmin) v = ~0ull;
    atomic_store_agent(&ctl->acc[slot][i], v);
  }
}

__device__ __forceinline__ double slot_double(Control* ctl, int slot, int i) {
  return __longlong_as_double((long long)atomic_load_agent(&ctl->acc[slot][i]));
}

// ------------------------------------------------------------ per-state commit

template <class VT>
struct CtxT {
  VT* rd;   // read buffer: W before the current batch (complete)
  VT* wr;   // write buffer
};
using Ctx = CtxT<float>;

// Costs of a row: the solvers always read the FP64 shifted costs (equal to
// c until the first re-centring), a single sweep reads c itself.  The
// choice is made at compile time so the hot loops carry no branch for it.
template <bool CE>
__device__ __forceinline__ double cost_of(const KParams& p, int64_t row) {
  if constexpr (CE)
    return p.ceff[row];
  else
    return (double)p.c32[row];
}

// What a state's commit needs besides its new value is loaded with the
// state's row data, so that the commit waits for no further memory round
// trip: in the sweeps of a solve, aux = V_ref(s) - R(s) (kept in the
// workspace array tgt), the target of the error check W + R - V_ref =
// W - aux; in improvement passes, the old policy entry.  The loads are
// unconditional, so no wait is placed before the row loads.
template <bool CE, bool IDENT>
__device__ __forceinline__ double commit_aux(const KParams& p, int32_t s) {
  if constexpr (IDENT)
    return (double)p.policy[s];
  else if constexpr (CE)
    return p.tgt[s];
  else
    return 0.0;
}

// Marks aux as used by every lane here.  Only one lane per state commits;
// without a use on the other lanes' path the load of aux would still count
// as pending at the loop's back edge, and the compiler would wait for all
// memory operations (the commit's stores included) before the next
// iteration's loads.  aux was loaded with the row data, so it has arrived.
__device__ __forceinline__ void consume(double aux) { __asm__ volatile("" ::"v"(aux)); }

// New value of state s from the FP64 bracket minimum q with action a.  The
// solvers iterate W = V - R for an FP64 anchor R (see Driver::recentre).
template <class Acc>
__device__ __forceinline__ void commit_sweep(const KParams& p, const Ctx& c, int32_t s, double q,
                                             int a, float old, double aux, Acc& L) {
  const float w = (float)q;
  c.wr[s] = w;
  if (p.argmin_out) p.argmin_out[s] = a;
  L.max_abs(kAccDv, fabs((double)w - (double)old));
  if (p.vref) L.max_abs(kAccErr, fabs((double)w - aux));
  L.range((double)w);
}

// Policy improvement of state s (Algorithm 1): V is not written.
template <class Acc>
__device__ __forceinline__ void commit_improve(const KParams& p, int32_t s, double q, int a,
                                               float old, bool count, double aux, Acc& L) {
  if (count && (int)aux != a) L.count_change();
  p.policy[s] = a;
  L.max_abs(kAccResid, fabs(q - (double)old));
}

enum Mode : int { kModeMin = 0, kModePolicy = 1, kModeImprove = 2, kModeImproveCount = 3 };


// ------------------------------------------------------------ storage of P
//
// Transition values are FP32, or BF16 / FP8 E4M3 (OCP E4M3FN) with one FP32
// scale per row: P(r, j) = scale_r * decode(q_rj).  Decoding is exact (BF16 is
// the upper half of an FP32; FP8 goes through the hardware converter), the
// dot products accumulate the decoded values in FP32 and the row scale is
// applied once per row, in FP64 with the cost.

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ f4 fp8x4(unsigned w) {
  const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);  // bytes 0, 1
  const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);   // bytes 2, 3
  return f4{lo[0], lo[1], hi[0], hi[1]};
}

struct ValF32 {
  static constexpr int kType = kF32;
  static constexpr int kBytes = 4;
  // ELL entries e .. e+3 (e a multiple of 4)
  __device__ __forceinline__ static f4 ell4(const KParams& p, size_t e) {
    return __builtin_nontemporal_load(reinterpret_cast<const f4*>(p.val + e));
  }
  __device__ __forceinline__ static float scale(const KParams&, int64_t) { return 1.f; }
  __device__ __forceinline__ static float dense_at(const KParams& p, size_t i) {
    return __builtin_nontemporal_load(p.P + i);
  }
};

struct ValBF16 {
  static constexpr int kType = kBF16;
  static constexpr int kBytes = 2;
  __device__ __forceinline__ static f4 ell4(const KParams& p, size_t e) {
    const u2 w = __builtin_nontemporal_load(
        reinterpret_cast<const u2*>(static_cast<const uint16_t*>(p.pq) + e));
    return f4{bf16_lo(w.x), bf16_hi(w.x), bf16_lo(w.y), bf16_hi(w.y)};
  }
  __device__ __forceinline__ static float scale(const KParams& p, int64_t row) {
    return p.rscale[row];
  }
  __device__ __forceinline__ static float dense_at(const KParams& p, size_t i) {
    return __uint_as_float((unsigned)static_cast<const uint16_t*>(p.pq)[i] << 16);
  }
  // word w (values 2w, 2w+1) of a 16-byte load of 8 values, times V
  __device__ __forceinline__ static void fma_word(unsigned x, int w, const f4* v, float& acc) {
    const f4& vv = v[w >> 1];
    acc = fmaf(bf16_lo(x), (w & 1) ? vv.z : vv.x, acc);
    acc = fmaf(bf16_hi(x), (w & 1) ? vv.w : vv.y, acc);
  }
};

struct ValFP8 {
  static constexpr int kType = kFP8;
  static constexpr int kBytes = 1;
  __device__ __forceinline__ static f4 ell4(const KParams& p, size_t e) {
    return fp8x4(__builtin_nontemporal_load(
        reinterpret_cast<const unsigned*>(static_cast<const uint8_t*>(p.pq) + e)));
  }
  __device__ __forceinline__ static float scale(const KParams& p, int64_t row) {
    return p.rscale[row];
  }
  __device__ __forceinline__ static float dense_at(const KParams& p, size_t i) {
    return fp8x4((unsigned)static_cast<const uint8_t*>(p.pq)[i]).x;
  }
  // word w (values 4w .. 4w+3) of a 16-byte load of 16 values, times V
  __device__ __forceinline__ static void fma_word(unsigned x, int w, const f4* v, float& acc) {
    const f4 d = fp8x4(x);
    acc = fmaf(d.x, v[w].x, acc);
    acc = fmaf(d.y, v[w].y, acc);
    acc = fmaf(d.z, v[w].z, acc);
    acc = fmaf(d.w, v[w].w, acc);
  }
};

// ------------------------------------------------------------ dense engine

// acc[r] += sum_{j in [j0, j1), this thread's columns} rows[r][j] * V[j],
// for thread tid of nthr threads sharing the rows.  Row bases are uniform
// across the workgroup and column offsets are 32-bit, so every load is a
// scalar base plus one vector offset.
template <int R, int VEC, int U>
__device__ __forceinline__ void dense_dot(const float* __restrict__ rows, uint32_t n, int nrows,
                                          const float* __restrict__ V, uint32_t j0, uint32_t j1,
                                          uint32_t tid, uint32_t nthr, float (&acc)[R]) {
  const uint32_t step = nthr * VEC;
  for (uint32_t j = j0 + tid * VEC; j < j1; j += step * U) {
    if constexpr (VEC == 4) {
      f4 v[U];
      f4 x[U][R];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t jj = j + u * step;
        const bool ok = jj < j1;
        v[u] = ok ? *reinterpret_cast<const f4*>(V + jj) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < R; ++r)
          x[u][r] = (ok && r < nrows)
                        ? __builtin_nontemporal_load(
                              reinterpret_cast<const f4*>(rows + (size_t)r * n + jj))
                        : f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          acc[r] = fmaf(x[u][r].x, v[u].x, acc[r]);
          acc[r] = fmaf(x[u][r].y, v[u].y, acc[r]);
          acc[r] = fmaf(x[u][r].z, v[u].z, acc[r]);
          acc[r] = fmaf(x[u][r].w, v[u].w, acc[r]);
        }
    } else {
      float v[U];
      float x[U][R];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t jj = j + u * step;
        const bool ok = jj < j1;
        v[u] = ok ? V[jj] : 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r)
          x[u][r] = (ok && r < nrows) ? __builtin_nontemporal_load(rows + (size_t)r * n + jj) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fmaf(x[u][r], v[u], acc[r]);
    }
  }
}

// The same for BF16 / FP8 rows: each 16-byte load holds EPL = 16 / kBytes
// consecutive values of a row, decoded and multiplied by EPL values of V.
// rows is the byte address of the first row; n % EPL == 0.
template <int R, class T, int U>
__device__ __forceinline__ void dense_dot_q(const uint8_t* __restrict__ rows, uint32_t n,
                                            int nrows, const float* __restrict__ V, uint32_t j0,
                                            uint32_t j1, uint32_t tid, uint32_t nthr,
                                            float (&acc)[R]) {
  constexpr int EPL = 16 / T::kBytes;
  const uint32_t step = nthr * EPL;
  const size_t rbytes = (size_t)n * T::kBytes;
  for (uint32_t j = j0 + tid * EPL; j < j1; j += step * U) {
    f4 v[U][EPL / 4];
    u4 x[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t jj = j + u * step;
      const bool ok = jj < j1;
#pragma unroll
      for (int q = 0; q < EPL / 4; ++q)
        v[u][q] = ok ? *reinterpret_cast<const f4*>(V + jj + 4 * q) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < R; ++r)
        x[u][r] = (ok && r < nrows)
                      ? __builtin_nontemporal_load(reinterpret_cast<const u4*>(
                            rows + (size_t)r * rbytes + (size_t)jj * T::kBytes))
                      : u4{0u, 0u, 0u, 0u};
    }
    // word by word across the rows, so each decoded word dies at once
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int r = 0; r < R; ++r) T::fma_word(x[u][r][w], w, v[u], acc[r]);
  }
}

// out[g * R + r] (LDS) = sum of acc[r] over the wpg waves of group g (the
// workgroup's waves split into consecutive groups of wpg), r < R, in a fixed
// order.  Every thread of the workgroup must call it.
template <int R>
__device__ __forceinline__ void group_sum(float (&acc)[R], float* out, int wpg) {
  __shared__ float red[16][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, groups = (blockDim.x >> 6) / wpg;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float v = wave_sum(acc[r]);
    if (lane == 0) red[w][r] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < R * groups) {
    const int g = threadIdx.x / R, r = threadIdx.x % R;
    float s = 0.f;
    for (int i = 0; i < wpg; ++i) s += red[g * wpg + i][r];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// out[r] (LDS) = block-wide FP64 sum of acc[r], r < R.
template <int R>
__device__ __forceinline__ void block_sum_d(double (&acc)[R], double* out) {
  __shared__ double red_d[16][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double v = wave_sum_d(acc[r]);
    if (lane == 0) red_d[w][r] = v;
  }
  __syncthreads();
  if (threadIdx.x < R) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red_d[i][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

constexpr int kMaxActions = 1024;

template <int R, int VEC, class T = ValF32>
struct DenseEngine {
  static constexpr bool kBand = false;
  using Acc = LdsAcc;
  // 16-byte row loads in flight per thread and step: 16 for FP32 and BF16;
  // 8 for FP8, whose tiles also hold 16 values of V per load
  static constexpr int kLoads = T::kType == kFP8 ? 8 : 16;
  // (at most 4 steps at once: each step also holds VEC values of V)
  static constexpr int kRowUnroll = VEC == 1 ? 4 : (R >= kLoads ? 1 : (kLoads / R < 4 ? kLoads / R : 4));
  // one row per state in policy sweeps: a BF16 / FP8 row of n values is
  // n * 2 or n bytes, at most a few loads per thread
  static constexpr int kPolicyUnroll = VEC == 1 ? 16 : (T::kType == kF32 ? 8 : 2);

  // Partial dot products of the rows row0 .. row0+nrows-1 (VEC: FP32 values
  // per load, or the values of one 16-byte load for BF16 / FP8).
  template <int RR, int U>
  __device__ __forceinline__ static void dot(const KParams& p, size_t row0, uint32_t n,
                                             int nrows, const float* V, uint32_t j0, uint32_t j1,
                                             uint32_t tid, uint32_t nthr, float (&acc)[RR]) {
    if constexpr (T::kType == kF32)
      dense_dot<RR, VEC, U>(p.P + row0 * n, n, nrows, V, j0, j1, tid, nthr, acc);
    else
      dense_dot_q<RR, T, U>(static_cast<const uint8_t*>(p.pq) + row0 * n * T::kBytes, n, nrows,
                            V, j0, j1, tid, nthr, acc);
  }

  // Column range of split q of S, rounded to whole block-wide vector steps.
  __device__ __forceinline__ static void split_range(uint32_t n, int S, int q, uint32_t& j0,
                                                     uint32_t& j1) {
    if (S == 1) {
      j0 = 0;
      j1 = n;
      return;
    }
    const uint32_t quantum = blockDim.x * VEC;
    uint32_t cs = (n + S - 1) / S;
    cs = (cs + quantum - 1) / quantum * quantum;
    j0 = min((uint32_t)q * cs, n);
    j1 = min(j0 + cs, n);
  }

  // Processes this workgroup's units of one batch (IDENT: the states are
  // the positions themselves).  Without column splits a workgroup with
  // several states of the batch streams up to four of them at once, each
  // with its own group of waves, so that the start-up latency of a state's
  // row stream is paid once per group of states rather than per state.
  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch(const KParams& p, const int32_t* ord, int64_t bk,
                                               const Ctx& c, int mode, Acc& L) {
    __shared__ float s_sum[64];
    __shared__ double s_q[kMaxActions];
    __shared__ int s_last;
    const int64_t n = p.n;
    const int m = p.m;
    const bool improve = mode >= kModeImprove;
    const int S = improve ? 1 : p.splits;
    const int64_t units = bk * S;
    const int mr = (mode == kModePolicy) ? 1 : m;  // rows of a state that are read
    // states streamed at once by one workgroup
    const int nw = blockDim.x >> 6;
    int G = 1;
    if (S == 1) {
      const int64_t per_wg = (units + gridDim.x - 1) / gridDim.x;
      G = per_wg >= 4 ? 4 : (per_wg >= 2 ? 2 : 1);
      while (G > 1 && (nw % G != 0 || G * m > kMaxActions)) G >>= 1;
    }
    const int wpg = nw / G;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int grp = wave / wpg;
    const uint32_t gtid = threadIdx.x - (uint32_t)(grp * wpg * kWave);
    const uint32_t gthr = (uint32_t)(wpg * kWave);
    const bool lead_wave = (wave % wpg) == 0;
    double* sq = s_q + grp * m;
    for (int64_t ub = blockIdx.x; ub * G < units; ub += gridDim.x) {
      const int64_t u = ub * G + grp;
      const bool active = u < units;
      const int64_t uc = active ? u : ub * G;
      const int64_t i = uc / S;
      const int q = (int)(uc % S);
      int32_t s;
      if constexpr (IDENT)
        s = (int32_t)i;
      else
        s = ord[i];
      // the state is uniform over each wave: keep it (and the row bases) scalar
      s = __builtin_amdgcn_readfirstlane(s);
      uint32_t j0, j1;
      split_range((uint32_t)n, S, q, j0, j1);
      int apol = (mode == kModePolicy) ? __builtin_amdgcn_readfirstlane(p.policy[s]) : 0;
      if (apol < 0 || apol >= m) {
        if (active && gtid == 0) raise_abort(p.ctl, kDevBadPolicy);
        apol = 0;
      }
      // 1. partial dot products of the m (or 1) rows over [j0, j1)
      if (mode == kModePolicy) {
        float acc[1] = {0.f};
        if (active)
          dot<1, kPolicyUnroll>(p, (size_t)s * m + apol, (uint32_t)n, 1, c.rd, j0, j1, gtid, gthr,
                                acc);
        group_sum<1>(acc, s_sum, wpg);
        if (active && gtid == 0) {
          const int64_t row = (int64_t)s * m + apol;
          if (S == 1)
            sq[0] = cost_of<CE>(p, row) + p.gamma * ((double)s_sum[grp] * (double)T::scale(p, row));
          else
            p.partial[(size_t)(i * S + q)] = s_sum[0];
        }
      } else {
        for (int a0 = 0; a0 < m; a0 += R) {
          const int nrows = min(R, m - a0);
          float acc[R];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = 0.f;
          if (active)
            dot<R, kRowUnroll>(p, (size_t)s * m + a0, (uint32_t)n, nrows, c.rd, j0, j1, gtid,
                               gthr, acc);
          group_sum<R>(acc, s_sum, wpg);
          if (active && (int)gtid < nrows) {
            const int a = a0 + gtid;
            const int64_t row = (int64_t)s * m + a;
            const float sum = s_sum[grp * R + gtid];
            if (S == 1)
              sq[a] = cost_of<CE>(p, row) + p.gamma * ((double)sum * (double)T::scale(p, row));
            else
              p.partial[(size_t)(i * S + q) * m + a] = sum;
          }
        }
      }
      // the commit's inputs (issued before the reductions that precede the commit)
      const float old = c.rd[s];
      const double aux = commit_aux<CE, IDENT>(p, s);
      // 2. combine the splits (G == 1): the last workgroup to arrive finishes the state
      if (S > 1) {
        __syncthreads();
        if (threadIdx.x == 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          const unsigned prev = atomicAdd(&p.unit_count[i], 1u);
          int last = prev == (unsigned)(S - 1);
          if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            p.unit_count[i] = 0u;  // ready for the next batch using slot i
          }
          s_last = last;
        }
        __syncthreads();
        if (!s_last) continue;
        for (int a = threadIdx.x; a < mr; a += blockDim.x) {
          double sum = 0.0;
          for (int qq = 0; qq < S; ++qq) sum += (double)p.partial[(size_t)(i * S + qq) * mr + a];
          const int64_t row = (int64_t)s * m + ((mode == kModePolicy) ? apol : a);
          s_q[a] = cost_of<CE>(p, row) + p.gamma * (sum * (double)T::scale(p, row));
        }
      }
      __syncthreads();
      consume(aux);
      // 3. action minimum (lowest index on ties) and commit, in the group's first wave
      if (active && lead_wave) {
        const int lane = threadIdx.x & 63;
        double qv = INFINITY;
        int av = 0x7fffffff;
        if (mode == kModePolicy) {
          qv = sq[0];
          av = apol;
        } else {
          for (int a = lane; a < m; a += kWave) {
            const double x = sq[a];
            if (x < qv) {  // strictly smaller keeps the lowest index per lane
              qv = x;
              av = a;
            }
          }
          wave_argmin(qv, av);
          if (av == 0x7fffffff) av = 0;
        }
        consume(aux);
        if (lane == 0) {
          if (improve)
            commit_improve(p, s, qv, av, old, mode == kModeImproveCount, aux, L);
          else
            commit_sweep(p, c, s, qv, av, old, aux, L);
        }
      }
      __syncthreads();
    }
  }

  // c'(s,a) = c(s,a) - R(s) + gamma * (P R)(s,a) in FP64, a workgroup per state.
  __device__ __forceinline__ static void shift_costs(const KParams& p) {
    __shared__ double s_sumd[16];
    const int m = p.m;
    const uint32_t n = (uint32_t)p.n;
    for (int64_t s = blockIdx.x; s < p.n; s += gridDim.x) {
      const double rs = p.shift[s];
      for (int a0 = 0; a0 < m; a0 += R) {
        const int nrows = min(R, m - a0);
        const size_t base = ((size_t)s * m + a0) * (size_t)n;
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
          const double rj = p.shift[j];
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (r < nrows)
              acc[r] = fma((double)T::dense_at(p, base + (size_t)r * n + j), rj, acc[r]);
        }
        block_sum_d<R>(acc, s_sumd);
        if (threadIdx.x < nrows) {
          const int64_t row = (int64_t)s * m + a0 + threadIdx.x;
          p.ceff[row] = (double)p.c32[row] - rs +
                        p.gamma * (s_sumd[threadIdx.x] * (double)T::scale(p, row));
        }
      }
    }
  }
};

// ------------------------------------------------------------ ELL engine
//
// Constant row length k, k % 4 == 0, k <= 256.  A row is served by LPR =
// (k/4 rounded up to a power of two) lanes; a wavefront covers RPP = 64/LPR
// rows per pass.  In the minimum modes a wavefront serves UNR states at a
// time; in the policy mode each lane group serves its own state.  LPR is a
// template parameter so that the lane reductions unroll with constant
// shuffle offsets.
template <int UNR, int LPR, class T = ValF32>
struct EllEngine {
  static constexpr bool kBand = false;
  using Acc = RegAcc;


  // One wavefront iteration serves UNR states (min modes) or UNR lane
  // groups of states (policy mode).  The states of the next iteration are
  // fetched one iteration ahead, and the costs and old values are loaded
  // together with the columns and weights, so an iteration waits for two
  // round trips (the row stream, then the V gathers).  Every load uses a
  // valid address (positions past the batch end read state 0, lanes beyond a
  // row read the row's first entries, rows past m read row m-1) and unused
  // results are discarded by selects, so the loads issue back to back
  // without branches.
  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch(const KParams& p, const int32_t* ord, int64_t bk,
                                               const Ctx& c, int mode, Acc& L) {
    const int m = p.m, k = p.ell_k;
    constexpr int lpr = LPR, rpp = kWave / LPR;
    const int lane = threadIdx.x & 63, g = lane / lpr, l = lane % lpr;
    const bool lane_has_data = l * 4 < k;
    const int lcol = lane_has_data ? l * 4 : 0;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const bool improve = mode >= kModeImprove;
    const bool pol = mode == kModePolicy;
    // positions of a unit: min modes UNR states, policy mode UNR groups of rpp
    const int64_t per_unit = pol ? (int64_t)rpp * UNR : (int64_t)UNR;
    const int64_t units = (bk + per_unit - 1) / per_unit;
    // state at slot x of unit u, or -1 past the batch end
    auto state_at = [&](int64_t u, int x) -> int32_t {
      const int64_t pos = pol ? u * per_unit + (int64_t)x * rpp + g : u * per_unit + x;
      const bool valid = u < units && pos < bk;
      const int64_t pc = valid ? pos : 0;
      int32_t v;
      if constexpr (IDENT)
        v = (int32_t)pc;
      else
        v = ord[pc];
      return valid ? v : -1;
    };
    const float* __restrict__ rd = c.rd;
    int32_t s_next[UNR];
#pragma unroll
    for (int x = 0; x < UNR; ++x) s_next[x] = state_at(gw, x);
    for (int64_t u = gw; u < units; u += nw) {
      int32_t s[UNR], sc[UNR];
      float old[UNR];
      double aux[UNR];
#pragma unroll
      for (int x = 0; x < UNR; ++x) {
        s[x] = s_next[x];
        sc[x] = s[x] >= 0 ? s[x] : 0;
        old[x] = rd[sc[x]];
        aux[x] = commit_aux<CE, IDENT>(p, sc[x]);
      }
      if (pol) {
        int a[UNR];
        i4 cc[UNR];
        f4 vv[UNR];
        double cost[UNR];
        float scl[UNR];
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          int av = p.policy[sc[x]];
          if (av < 0 || av >= m) {
            if (s[x] >= 0) raise_abort(p.ctl, kDevBadPolicy);
            av = 0;
          }
          a[x] = av;
          const size_t e = ((size_t)sc[x] * m + av) * (size_t)k + (size_t)lcol;
          cc[x] = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p.col + e));
          vv[x] = T::ell4(p, e);
          cost[x] = cost_of<CE>(p, (int64_t)sc[x] * m + av);
          scl[x] = T::scale(p, (int64_t)sc[x] * m + av);
        }
#pragma unroll
        for (int x = 0; x < UNR; ++x) s_next[x] = state_at(u + nw, x);
        f4 gv[UNR];  // all V gathers of the iteration are issued before any use
#pragma unroll
        for (int x = 0; x < UNR; ++x)
          gv[x] = f4{rd[cc[x].x], rd[cc[x].y], rd[cc[x].z], rd[cc[x].w]};
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          float part = vv[x].x * gv[x].x;
          part = fmaf(vv[x].y, gv[x].y, part);
          part = fmaf(vv[x].z, gv[x].z, part);
          part = fmaf(vv[x].w, gv[x].w, part);
          part = lane_has_data ? part : 0.f;
          #pragma unroll
          for (int off = LPR >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off);
          consume(aux[x]);
          if (l == 0 && s[x] >= 0)
            commit_sweep(p, c, s[x], cost[x] + p.gamma * ((double)part * (double)scl[x]), a[x],
                         old[x], aux[x], L);
        }
        continue;
      }
      double qb[UNR];
      int ab[UNR];
#pragma unroll
      for (int x = 0; x < UNR; ++x) {
        qb[x] = INFINITY;
        ab[x] = 0x7fffffff;
      }
      for (int a0 = 0; a0 < m; a0 += rpp) {
        const int a = a0 + g;
        const bool row_ok = a < m;
        const int ac = row_ok ? a : m - 1;
        i4 cc[UNR];
        f4 vv[UNR];
        double cost[UNR];
        float scl[UNR];
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          const size_t e = ((size_t)sc[x] * m + ac) * (size_t)k + (size_t)lcol;
          cc[x] = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p.col + e));
          vv[x] = T::ell4(p, e);
          cost[x] = cost_of<CE>(p, (int64_t)sc[x] * m + ac);
          scl[x] = T::scale(p, (int64_t)sc[x] * m + ac);
        }
        if (a0 == 0) {
#pragma unroll
          for (int x = 0; x < UNR; ++x) s_next[x] = state_at(u + nw, x);
        }
        f4 gv[UNR];  // all V gathers of the iteration are issued before any use
#pragma unroll
        for (int x = 0; x < UNR; ++x)
          gv[x] = f4{rd[cc[x].x], rd[cc[x].y], rd[cc[x].z], rd[cc[x].w]};
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          float part = vv[x].x * gv[x].x;
          part = fmaf(vv[x].y, gv[x].y, part);
          part = fmaf(vv[x].z, gv[x].z, part);
          part = fmaf(vv[x].w, gv[x].w, part);
          part = lane_has_data ? part : 0.f;
          #pragma unroll
          for (int off = LPR >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off);
          const bool use = row_ok && s[x] >= 0;
          // computed on every lane, then selected: keeps the cost load unconditional
          const double qa = cost[x] + p.gamma * ((double)part * (double)scl[x]);
          double q = use ? qa : INFINITY;
          int aq = use ? a : 0x7fffffff;
          wave_argmin_from<LPR>(q, aq);
          const bool better = q < qb[x] || (q == qb[x] && aq < ab[x]);
          qb[x] = better ? q : qb[x];
          ab[x] = better ? aq : ab[x];
        }
      }
#pragma unroll
      for (int x = 0; x < UNR; ++x) consume(aux[x]);
      if (lane == 0) {
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          if (s[x] < 0) continue;
          const int av = ab[x] == 0x7fffffff ? 0 : ab[x];
          if (improve)
            commit_improve(p, s[x], qb[x], av, old[x], mode == kModeImproveCount, aux[x], L);
          else
            commit_sweep(p, c, s[x], qb[x], av, old[x], aux[x], L);
        }
      }
    }
  }

  // c'(s,a) = c(s,a) - R(s) + gamma * (P R)(s,a) in FP64, a wavefront per state.
  __device__ __forceinline__ static void shift_costs(const KParams& p) {
    const int m = p.m, k = p.ell_k;
    constexpr int lpr = LPR, rpp = kWave / LPR;
    const int lane = threadIdx.x & 63, g = lane / lpr, l = lane % lpr;
    const bool lane_has_data = l * 4 < k;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t s = gw; s < p.n; s += nw) {
      const double rs = p.shift[s];
      for (int a0 = 0; a0 < m; a0 += rpp) {
        const int a = a0 + g;
        double part = 0.0;
        if (a < m && lane_has_data) {
          const size_t e = ((size_t)s * m + a) * (size_t)k + (size_t)l * 4;
          const i4 cc = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p.col + e));
          const f4 vv = T::ell4(p, e);
          part = (double)vv.x * p.shift[cc.x] + (double)vv.y * p.shift[cc.y] +
                 (double)vv.z * p.shift[cc.z] + (double)vv.w * p.shift[cc.w];
        }
        #pragma unroll
          for (int off = LPR >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off);
        if (l == 0 && a < m) {
          const int64_t row = s * m + a;
          p.ceff[row] = (double)p.c32[row] - rs + p.gamma * (part * (double)T::scale(p, row));
        }
      }
    }
  }
};

// ------------------------------------------------------------ band-local ELL engine
//
// When every column of the rows of state s lies within a band |s' - s| <=
// beta, workgroup w owns one contiguous chunk of D states and computes, in
// each batch, exactly the states of the batch that fall in its chunk.  Their
// reads stay inside the window [w D - beta, (w+1) D + beta) of V, which the
// workgroup copies into LDS with coalesced loads at the start of the batch,
// so the k reads per row are LDS reads instead of scattered memory reads.
// A batch is a set of states that all read the values from before the batch
// (eq. (11)), so the order inside it is free: at the start of a sweep the
// workgroup sorts its chunk by batch index sigma_t^{-1}(s) / b (the Feistel
// network run backwards) with a counting sort in LDS, and batch k is then
// one contiguous run of that list.
constexpr int kWinCap = 16384;   // V entries staged in LDS (64 KB)
constexpr int kChunkCap = 8192;  // states of one workgroup's chunk
constexpr int kBatchCap = 4096;  // batches per sweep

struct BandShared {
  float win[kWinCap];               // V[wlo, wlo + wn) of the current batch; sort scratch
  uint16_t lst[2][kChunkCap];       // chunk offsets ordered by batch, by sweep parity
  int32_t off[kBatchCap + 1];       // batch k is lst[.][off[k], off[k+1])
  uint32_t first0[kChunkCap / 32];  // bit i: state c0 + i is in batch 0 of the newest sweep
  int32_t wsum[16];                 // per-wave partial sums of the scan
};

__device__ __forceinline__ BandShared& band_shared() {
  __shared__ BandShared sh;
  return sh;
}

struct BandGeom {
  int64_t c0;   // first state of the chunk
  int dw;       // states in the chunk
  int64_t wlo;  // first V entry of the window
  int wn;       // entries in the window
};

__device__ __forceinline__ BandGeom band_geom(const KParams& p) {
  const int64_t D = (p.n + gridDim.x - 1) / gridDim.x;
  BandGeom g;
  g.c0 = min(p.n, (int64_t)blockIdx.x * D);
  const int64_t c1 = min(p.n, g.c0 + D);
  g.dw = (int)(c1 - g.c0);
  g.wlo = max((int64_t)0, g.c0 - (int64_t)p.band);
  g.wn = g.dw > 0 ? (int)(min(p.n, c1 + (int64_t)p.band) - g.wlo) : 0;
  return g;
}

// a[0, cnt) <- its exclusive prefix sums, in place, over the workgroup.
__device__ __forceinline__ void block_exclusive_scan(int32_t* a, int cnt, int32_t* wsum) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, w = tid >> 6;
  const int per = (cnt + nt - 1) / nt;
  const int i0 = min(cnt, tid * per), i1 = min(cnt, i0 + per);
  int sum = 0;
  for (int i = i0; i < i1; ++i) sum += a[i];
  int x = sum;  // inclusive scan over the wavefront
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  int run = x - sum;
  for (int j = 0; j < w; ++j) run += wsum[j];
  for (int i = i0; i < i1; ++i) {
    const int v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
}

// lst[buf] <- the chunk's offsets ordered by batch of sweep t; off, first0.
__device__ __forceinline__ void band_sort(const KParams& p, BandShared& sh, const BandGeom& bg,
                                          uint64_t t, int buf, int nb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i <= nb; i += nt) sh.off[i] = 0;
  for (int i = tid; i < (bg.dw + 31) / 32; i += nt) sh.first0[i] = 0u;
  __syncthreads();
  uint32_t* kr = reinterpret_cast<uint32_t*>(sh.win);  // (batch << 16) | rank in batch
  const OrderKey key = make_order_key(p.n, p.seed, t);
  const uint32_t b = (uint32_t)p.b;
  for (int i = tid; i < bg.dw; i += nt) {
    const uint32_t kb = sweep_position_of((uint32_t)(bg.c0 + i), key) / b;
    const uint32_t r = (uint32_t)atomicAdd(&sh.off[kb], 1);
    kr[i] = (kb << 16) | r;
  }
  __syncthreads();
  block_exclusive_scan(sh.off, nb, sh.wsum);
  if (tid == 0) sh.off[nb] = bg.dw;
  __syncthreads();
  for (int i = tid; i < bg.dw; i += nt) {
    const uint32_t v = kr[i];
    const uint32_t kb = v >> 16;
    sh.lst[buf][sh.off[kb] + (int)(v & 0xFFFFu)] = (uint16_t)i;
    if (kb == 0) atomicOr(&sh.first0[i >> 5], 1u << (i & 31));
  }
  __syncthreads();
}

// The ELL loop of EllEngine with state ids from the workgroup's list and V
// read from the window in LDS.  Row streams, costs and policies still come
// from memory; the recentring pass (shift_costs) is EllEngine's.
template <int UNR, int LPR, class T = ValF32>
struct BandEngine : EllEngine<UNR, LPR, T> {
  static constexpr bool kBand = true;

  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch_band(const KParams& p, const BandShared& sh,
                                                    const uint16_t* lst, int cnt,
                                                    const BandGeom& bg, const Ctx& c, int mode,
                                                    Acc& L) {
    const int m = p.m, k = p.ell_k;
    constexpr int rpp = kWave / LPR;
    const int lane = threadIdx.x & 63, g = lane / LPR, l = lane % LPR;
    const bool lane_has_data = l * 4 < k;
    const int lcol = lane_has_data ? l * 4 : 0;
    const int wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    const bool improve = mode >= kModeImprove;
    const bool pol = mode == kModePolicy;
    const int per_unit = pol ? rpp * UNR : UNR;
    const int units = (cnt + per_unit - 1) / per_unit;
    const float* win = sh.win;
    const int32_t wlo = (int32_t)bg.wlo;
    const uint32_t wlast = (uint32_t)(bg.wn > 0 ? bg.wn - 1 : 0);
    // V(j) from the window; the clamp only keeps an index inside the array
    auto at = [&](int32_t j) -> float { return win[min((uint32_t)(j - wlo), wlast)]; };
    for (int u = wv; u < units; u += nwv) {
      int32_t s[UNR], sc[UNR];
      float old[UNR];
      double aux[UNR];
#pragma unroll
      for (int x = 0; x < UNR; ++x) {
        const int pos = pol ? u * per_unit + x * rpp + g : u * per_unit + x;
        const bool valid = pos < cnt;
        const int pc = valid ? pos : 0;
        int o;
        if constexpr (IDENT)
          o = pc;
        else
          o = (int)lst[pc];
        sc[x] = (int32_t)bg.c0 + o;
        s[x] = valid ? sc[x] : -1;
        old[x] = at(sc[x]);
        aux[x] = commit_aux<CE, IDENT>(p, sc[x]);
      }
      if (pol) {
        int a[UNR];
        i4 cc[UNR];
        f4 vv[UNR];
        double cost[UNR];
        float scl[UNR];
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          int av = p.policy[sc[x]];
          if (av < 0 || av >= m) {
            if (s[x] >= 0) raise_abort(p.ctl, kDevBadPolicy);
            av = 0;
          }
          a[x] = av;
          const size_t e = ((size_t)sc[x] * m + av) * (size_t)k + (size_t)lcol;
          cc[x] = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p.col + e));
          vv[x] = T::ell4(p, e);
          cost[x] = cost_of<CE>(p, (int64_t)sc[x] * m + av);
          scl[x] = T::scale(p, (int64_t)sc[x] * m + av);
        }
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          float part = vv[x].x * at(cc[x].x);
          part = fmaf(vv[x].y, at(cc[x].y), part);
          part = fmaf(vv[x].z, at(cc[x].z), part);
          part = fmaf(vv[x].w, at(cc[x].w), part);
          part = lane_has_data ? part : 0.f;
#pragma unroll
          for (int off = LPR >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off);
          consume(aux[x]);
          if (l == 0 && s[x] >= 0)
            commit_sweep(p, c, s[x], cost[x] + p.gamma * ((double)part * (double)scl[x]), a[x],
                         old[x], aux[x], L);
        }
        continue;
      }
      double qb[UNR];
      int ab[UNR];
#pragma unroll
      for (int x = 0; x < UNR; ++x) {
        qb[x] = INFINITY;
        ab[x] = 0x7fffffff;
      }
      for (int a0 = 0; a0 < m; a0 += rpp) {
        const int a = a0 + g;
        const bool row_ok = a < m;
        const int ac = row_ok ? a : m - 1;
        i4 cc[UNR];
        f4 vv[UNR];
        double cost[UNR];
        float scl[UNR];
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          const size_t e = ((size_t)sc[x] * m + ac) * (size_t)k + (size_t)lcol;
          cc[x] = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p.col + e));
          vv[x] = T::ell4(p, e);
          cost[x] = cost_of<CE>(p, (int64_t)sc[x] * m + ac);
          scl[x] = T::scale(p, (int64_t)sc[x] * m + ac);
        }
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          float part = vv[x].x * at(cc[x].x);
          part = fmaf(vv[x].y, at(cc[x].y), part);
          part = fmaf(vv[x].z, at(cc[x].z), part);
          part = fmaf(vv[x].w, at(cc[x].w), part);
          part = lane_has_data ? part : 0.f;
#pragma unroll
          for (int off = LPR >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off);
          const bool use = row_ok && s[x] >= 0;
          // computed on every lane, then selected: keeps the cost load unconditional
          const double qa = cost[x] + p.gamma * ((double)part * (double)scl[x]);
          double q = use ? qa : INFINITY;
          int aq = use ? a : 0x7fffffff;
          wave_argmin_from<LPR>(q, aq);
          const bool better = q < qb[x] || (q == qb[x] && aq < ab[x]);
          qb[x] = better ? q : qb[x];
          ab[x] = better ? aq : ab[x];
        }
      }
#pragma unroll
      for (int x = 0; x < UNR; ++x) consume(aux[x]);
      if (lane == 0) {
#pragma unroll
        for (int x = 0; x < UNR; ++x) {
          if (s[x] < 0) continue;
          const int av = ab[x] == 0x7fffffff ? 0 : ab[x];
          if (improve)
            commit_improve(p, s[x], qb[x], av, old[x], mode == kModeImproveCount, aux[x], L);
          else
            commit_sweep(p, c, s[x], qb[x], av, old[x], aux[x], L);
        }
      }
    }
  }
};

// ------------------------------------------------------------ column-block engine
//
// For b = n (the whole state set is one batch, which reads only the values
// before it: eq. (11) with M_n(i) empty, i.e. T of eq. (7)) the order in
// which a batch's products are summed is free.  A constant-row-length MDP
// may then carry a second copy of its entries in column-sorted blocks
// (mdp_column_blocks_prepare / _attach): block B holds the entries of the
// rows of states [B * bs, (B + 1) * bs) (bs * m <= 4096 rows), sorted by
// column and packed into groups of 64 entries whose rows are distinct, each
// entry a 32-bit key (column << 12 | row within the block) and an FP32 value
// (padding entries have value 0).  A wavefront takes a block and its groups
// in order, gathers V for a group's 64 columns -- sorted, so they fall on a
// few cache lines instead of 64 -- and adds value * V into the block's row
// sums in its own part of the LDS (the rows of a group are distinct, so a
// wave's 64 lanes never collide, and no other wave writes there: no
// atomics).  Then the cost is added in FP64, the minimum taken and
// committed as by the other engines.  Policy sweeps (one row per state) and
// b < n use the row-major engine, whose re-centring pass is also used.
constexpr int kColWaves = 8;     // wavefronts per workgroup, one block's row sums each

struct ColShared {
  float acc[kColWaves][kColRows] __attribute__((aligned(16)));
};

__device__ __forceinline__ ColShared& col_shared() {
  __shared__ ColShared sh;
  return sh;
}

template <int UNR, int LPR>
struct ColEngine : EllEngine<UNR, LPR, ValF32> {
  static constexpr bool kBand = false;
  using Base = EllEngine<UNR, LPR, ValF32>;
  using Acc = typename Base::Acc;
  static constexpr int U = 16;      // groups of 64 entries in flight per wavefront
  static constexpr int kAlign = 1;  // rounds of U groups between workgroup barriers

  // Each wavefront owns one block of a set of W consecutive blocks (its own
  // LDS row sums, no copies to add), and the workgroup's wavefronts walk V
  // in column order side by side: a workgroup barrier every kAlign rounds
  // keeps them within a few groups of each other, so a V line that one
  // wavefront brings into the compute unit's L1 is still there when the
  // others gather from it.  (Without the barriers the wavefronts drift
  // apart and every gather line goes to L2.)
  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch(const KParams& p, const int32_t* ord, int64_t bk,
                                               const Ctx& c, int mode, Acc& L) {
    if (mode == kModePolicy || bk != p.n || !p.cb_keys || (blockDim.x >> 6) > kColWaves) {
      Base::template batch<CE, IDENT>(p, ord, bk, c, mode, L);
      return;
    }
    const int m = p.m;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = (int)(blockDim.x >> 6);  // <= kColWaves (the launch uses 512 threads)
    const int64_t bs = p.cb_states, n = p.n;
    const int64_t nblk = (n + bs - 1) / bs;
    const float* __restrict__ rd = c.rd;
    float* a = col_shared().acc[wv];
    for (int64_t set = blockIdx.x; set * W < nblk; set += gridDim.x) {
      const int64_t blk = set * W + wv;
      const bool have = blk < nblk;
      for (int i = lane; i < kColRows / 4; i += kWave)
        reinterpret_cast<f4*>(a)[i] = f4{0.f, 0.f, 0.f, 0.f};
      const int64_t g0 = have ? p.cb_gptr[blk] : 0, g1 = have ? p.cb_gptr[blk + 1] : 0;
      // every wavefront runs as many rounds (and barriers) as the set's
      // longest block needs
      int64_t gmax = 0;
      for (int w = 0; w < W; ++w) {
        const int64_t b2 = set * W + w;
        if (b2 < nblk) gmax = max(gmax, (int64_t)(p.cb_gptr[b2 + 1] - p.cb_gptr[b2]));
      }
      int round = 0;
      for (int64_t it = 0; it < gmax; it += U, ++round) {
        if (g0 + it < g1) {
          uint32_t kk[U];
          float vv[U], gv[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t gr = g0 + it + u;
            const bool ok = gr < g1;
            const size_t e = (size_t)(ok ? gr : g0) * kWave + lane;  // a valid group either way
            kk[u] = __builtin_nontemporal_load(p.cb_keys + e);
            vv[u] = ok ? __builtin_nontemporal_load(p.cb_vals + e) : 0.f;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) gv[u] = rd[kk[u] >> 12];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const uint32_t r = kk[u] & (kColRows - 1);
            a[r] = fmaf(vv[u], gv[u], a[r]);
          }
        }
        if (round % kAlign == kAlign - 1) __builtin_amdgcn_s_barrier();
      }
      // the block's states: cost in FP64, minimum, commit (a lane per state)
      if (have) {
        const int64_t s0 = blk * bs;
        const int ns = (int)min(bs, n - s0);
        for (int i = lane; i < ns; i += kWave) {
          const int32_t s = (int32_t)(s0 + i);
          const float old = rd[s];
          const double aux = commit_aux<CE, IDENT>(p, s);
          double qb = INFINITY;
          int ab = 0;
          for (int act = 0; act < m; ++act) {
            const double q = cost_of<CE>(p, (int64_t)s * m + act) + p.gamma * (double)a[i * m + act];
            if (q < qb) {  // ascending actions: strictly smaller keeps the lowest
              qb = q;
              ab = act;
            }
          }
          if (mode >= kModeImprove)
            commit_improve(p, s, qb, ab, old, mode == kModeImproveCount, aux, L);
          else
            commit_sweep(p, c, s, qb, ab, old, aux, L);
        }
      }
    }
  }
};

// ------------------------------------------------------------ general CSR engine

struct CsrEngine {
  static constexpr bool kBand = false;
  using Acc = RegAcc;

  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch(const KParams& p, const int32_t* ord, int64_t bk,
                                               const Ctx& c, int mode, Acc& L) {
    const int m = p.m;
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const bool improve = mode >= kModeImprove;
    for (int64_t u = gw; u < bk; u += nw) {
      int32_t s;
      if constexpr (IDENT)
        s = (int32_t)u;
      else
        s = ord[u];
      const float old = c.rd[s];
      const double aux = commit_aux<CE, IDENT>(p, s);
      double qb = INFINITY;
      int ab = 0x7fffffff;
      int a_lo = mode == kModePolicy ? p.policy[s] : 0;
      if (a_lo < 0 || a_lo >= m) {
        if (lane == 0) raise_abort(p.ctl, kDevBadPolicy);
        a_lo = 0;
      }
      const int a_hi = mode == kModePolicy ? a_lo + 1 : m;
      for (int a = a_lo; a < a_hi; ++a) {
        const int64_t row = (int64_t)s * m + a;
        const int64_t e0 = p.row_ptr[row], e1 = p.row_ptr[row + 1];
        float part = 0.f;
        for (int64_t e = e0 + lane; e < e1; e += kWave)
          part = fmaf(__builtin_nontemporal_load(p.val + e), c.rd[p.col[e]], part);
        part = wave_sum(part);
        const double q = cost_of<CE>(p, row) + p.gamma * (double)part;
        if (q < qb) {
          qb = q;
          ab = a;
        }
      }
      if (ab == 0x7fffffff) ab = a_lo;
      consume(aux);
      if (lane == 0) {
        if (improve)
          commit_improve(p, s, qb, ab, old, mode == kModeImproveCount, aux, L);
        else
          commit_sweep(p, c, s, qb, ab, old, aux, L);
      }
    }
  }

  // c'(s,a) = c(s,a) - R(s) + gamma * (P R)(s,a) in FP64, a wavefront per state.
  __device__ __forceinline__ static void shift_costs(const KParams& p) {
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t s = gw; s < p.n; s += nw) {
      const double rs = p.shift[s];
      for (int a = 0; a < p.m; ++a) {
        const int64_t row = s * p.m + a;
        double part = 0.0;
        for (int64_t e = p.row_ptr[row] + lane; e < p.row_ptr[row + 1]; e += kWave)
          part = fma((double)p.val[e], p.shift[p.col[e]], part);
        part = wave_sum_d(part);
        if (lane == 0) p.ceff[row] = (double)p.c32[row] - rs + p.gamma * part;
      }
    }
  }
};

// ------------------------------------------------------------ the persistent kernel

// VT is the type of the value buffers: float for the solvers (W = V - R),
// double for the FP64 correction (V itself).
template <class Acc, class VT = float>
struct Driver {
  const KParams& p;
  GridBarrier g;
  Acc L;
  VT* buf0;
  VT* buf1;
  int64_t phase;          // batches processed (parity selects the read buffer)
  const int32_t* prev_order;
  int64_t prev_count;     // states of the previous batch still to copy forward
  unsigned epoch;         // sweeps + improvement passes, selects accumulator slot
  int64_t gtid, gthreads;
  // band-local engine: this workgroup's part of the previous batch, a run of
  // list buffer band_prev_buf (-1: none yet)
  int band_prev_buf, band_prev_lo, band_prev_hi;

  __device__ __forceinline__ explicit Driver(const KParams& kp) : p(kp) {
    g.ctl = p.ctl;
    g.gen = 0;
    g.nblocks = gridDim.x;
    g.timeout = p.timeout_ticks;
    L.init();
    if constexpr (sizeof(VT) == sizeof(double)) {
      buf0 = p.vd0;
      buf1 = p.vd1;
    } else {
      buf0 = p.vbuf0;
      buf1 = p.vbuf1;
    }
    phase = 0;
    prev_order = nullptr;
    prev_count = 0;
    epoch = 0;
    gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    gthreads = (int64_t)gridDim.x * blockDim.x;
    band_prev_buf = -1;
    band_prev_lo = band_prev_hi = 0;
  }

  // Stamp of sweep t in first_mark (never 0, the cleared value).
  __device__ __forceinline__ static uint32_t stamp(uint64_t t) {
    const uint32_t v = (uint32_t)(t + 1);
    return v ? v : 1u;
  }

  // order[t % 3][pos] for pos in [begin, begin + count): sigma_t or perm.
  // The states of a sweep's first batch (begin == 0) are stamped.
  __device__ __forceinline__ void fill_order(uint64_t t, int64_t begin, int64_t count) {
    int32_t* dst = p.order + (size_t)(t % 3) * (size_t)p.n;
    const bool first = begin == 0;
    const uint32_t st = stamp(t);
    uint32_t* mark = p.first_mark + (size_t)(t & 1) * (size_t)p.n;
    if (p.perm) {
      for (int64_t i = gtid; i < count; i += gthreads) {
        int32_t v = p.perm[begin + i];
        if (v < 0 || (int64_t)v >= p.n) {
          raise_abort(p.ctl, kDevBadPerm);
          v = 0;
        }
        dst[begin + i] = v;
        if (first) mark[v] = st;
      }
      return;
    }
    const OrderKey key = make_order_key(p.n, p.seed, t);
    for (int64_t i = gtid; i < count; i += gthreads) {
      const int32_t v = (int32_t)sweep_order_at((uint32_t)(begin + i), key);
      dst[begin + i] = v;
      if (first) mark[v] = st;
    }
  }

  // buffer holding V before the current batch (complete) / the other one
  __device__ __forceinline__ VT* rd_buf() const { return (phase & 1) ? buf1 : buf0; }
  __device__ __forceinline__ VT* wr_buf() const { return (phase & 1) ? buf0 : buf1; }

  __device__ __forceinline__ int slot() const { return (int)(epoch % 3); }

  template <class Eng, bool CE>
  __device__ __forceinline__ bool sweep(uint64_t t, int mode) {
    if constexpr (Eng::kBand) return sweep_band<Eng, CE>(t, mode);
    const int64_t n = p.n, b = p.b, nb = (n + b - 1) / b;
    if (blockIdx.x == 0 && threadIdx.x == 0) reset_slot(p.ctl, (int)((epoch + 1) % 3));
    const int32_t* ord = p.order + (size_t)(t % 3) * (size_t)n;
    for (int64_t k = 0; k < nb; ++k) {
      const int64_t kb = k * b, bk = min(b, n - kb);
      CtxT<VT> c{rd_buf(), wr_buf()};
      // copy the previous batch forward, except states this batch rewrites
      // (only possible for the first batch, whose states are stamped)
      const uint32_t st = stamp(t);
      const uint32_t* mark = p.first_mark + (size_t)(t & 1) * (size_t)n;
      for (int64_t i = gtid; i < prev_count; i += gthreads) {
        const int32_t s = prev_order[i];
        if (k != 0 || mark[s] != st) c.wr[s] = c.rd[s];
      }
      if (k + 1 < nb)
        fill_order(t, kb + b, min(b, n - kb - b));
      else
        fill_order(t + 1, 0, min(b, n));
      Eng::template batch<CE, false>(p, ord + kb, bk, c, mode, L);
      prev_order = ord + kb;
      prev_count = bk;
      if (k == nb - 1) L.flush(p.ctl, slot());
      if (!grid_sync(g)) return false;
      ++phase;
    }
    ++epoch;
    return true;
  }

  // Band-local sweep: the workgroup computes the states of each batch that
  // lie in its chunk, reading V from the batch's window in LDS.  It copies
  // forward its own states of the previous batch (from the window, which
  // holds them), except, in the first batch, those the batch rewrites.
  template <class Eng, bool CE>
  __device__ __forceinline__ bool sweep_band(uint64_t t, int mode) {
    BandShared& sh = band_shared();
    const BandGeom bg = band_geom(p);
    const int nb = (int)((p.n + p.b - 1) / p.b);
    const int buf = (int)(t & 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) reset_slot(p.ctl, (int)((epoch + 1) % 3));
    band_sort(p, sh, bg, t, buf, nb);
    for (int k = 0; k < nb; ++k) {
      Ctx c{rd_buf(), wr_buf()};
      for (int i = threadIdx.x; i < bg.wn; i += blockDim.x) sh.win[i] = c.rd[bg.wlo + i];
      __syncthreads();
      if (band_prev_buf >= 0) {
        const uint16_t* prev = sh.lst[band_prev_buf];
        for (int i = band_prev_lo + (int)threadIdx.x; i < band_prev_hi; i += blockDim.x) {
          const int o = prev[i];
          if (k == 0 && ((sh.first0[o >> 5] >> (o & 31)) & 1u)) continue;
          c.wr[bg.c0 + o] = sh.win[bg.c0 + o - bg.wlo];
        }
      }
      const int lo = sh.off[k], hi = sh.off[k + 1];
      Eng::template batch_band<CE, false>(p, sh, sh.lst[buf] + lo, hi - lo, bg, c, mode, L);
      band_prev_buf = buf;
      band_prev_lo = lo;
      band_prev_hi = hi;
      if (k == nb - 1) L.flush(p.ctl, slot());
      if (!grid_sync(g)) return false;
      ++phase;
    }
    ++epoch;
    return true;
  }

  template <class Eng, bool CE>
  __device__ __forceinline__ bool improve_band(bool count) {
    BandShared& sh = band_shared();
    const BandGeom bg = band_geom(p);
    if (blockIdx.x == 0 && threadIdx.x == 0) reset_slot(p.ctl, (int)((epoch + 1) % 3));
    Ctx c{rd_buf(), wr_buf()};
    for (int i = threadIdx.x; i < bg.wn; i += blockDim.x) sh.win[i] = c.rd[bg.wlo + i];
    __syncthreads();
    Eng::template batch_band<CE, true>(p, sh, nullptr, bg.dw, bg, c,
                                       count ? kModeImproveCount : kModeImprove, L);
    L.flush(p.ctl, slot());
    if (!grid_sync(g)) return false;
    ++epoch;
    return true;
  }

  template <class Eng, bool CE>
  __device__ __forceinline__ bool improve(bool count) {
    if constexpr (Eng::kBand) return improve_band<Eng, CE>(count);
    if (blockIdx.x == 0 && threadIdx.x == 0) reset_slot(p.ctl, (int)((epoch + 1) % 3));
    CtxT<VT> c{rd_buf(), wr_buf()};
    Eng::template batch<CE, true>(p, nullptr, p.n, c, count ? kModeImproveCount : kModeImprove, L);
    L.flush(p.ctl, slot());
    if (!grid_sync(g)) return false;
    ++epoch;
    return true;
  }

  // Re-centring (exact in real arithmetic): fold the iterate into the FP64
  // anchor, R <- R + W, set W = 0 in both buffers, and rebuild the shifted
  // costs c'(s,a) = c(s,a) - R(s) + gamma (P R)(s,a).  Every value a state
  // reads is V(j) = W(j) + R(j), old or new alike, so the sweep on W with c'
  // is the sweep on V minus R for any order and batch size.  Afterwards W
  // carries only the change since the fold, so FP32 resolves it relative to
  // the remaining error rather than to |V|.
  template <class Eng>
  __device__ __forceinline__ bool recentre(long long& count) {
    const float* cur = rd_buf();
    for (int64_t s = gtid; s < p.n; s += gthreads) {
      const double r = p.shift[s] + (double)cur[s];
      p.shift[s] = r;
      if (p.vref) p.tgt[s] = p.vref[s] - r;
      buf0[s] = 0.f;
      buf1[s] = 0.f;
    }
    if (!grid_sync(g)) return false;
    Eng::shift_costs(p);
    ++count;
    return grid_sync(g);
  }

  // True when FP32 resolution of W is about to limit the iteration: the
  // last sweep changed W by less than 2^-14 of its magnitude.
  __device__ __forceinline__ bool want_recentre(int slot_, double last_dv, long long since) const {
    if (p.recentre_every <= 0 || since < p.recentre_every) return false;
    const double wmax = okey_value(atomic_load_agent(&p.ctl->acc[slot_][kAccWmax]));
    const double wmin = okey_value(atomic_load_agent(&p.ctl->acc[slot_][kAccWmin]));
    const double wabs = fmax(fabs(wmax), fabs(wmin));
    if (!isfinite(wabs) || wabs <= 0.0) return false;
    return p.recentre_force || wabs > 16384.0 * last_dv;
  }

  // Final V into the caller's buffer (V = W + R) and the statistics.
  __device__ __forceinline__ void finish(long long sweeps, long long outer, long long changes_last,
                                         long long recentrings, double last_dv, double last_err,
                                         int converged) {
    const float* cur = rd_buf();
    if (p.shift) {
      for (int64_t s = gtid; s < p.n; s += gthreads) {
        const double v = (double)cur[s] + p.shift[s];
        p.vbuf0[s] = (float)v;
        if (p.v64_out) p.v64_out[s] = v;
      }
    } else {
      if (cur != p.vbuf0)
        for (int64_t s = gtid; s < p.n; s += gthreads) p.vbuf0[s] = cur[s];
      if (p.v64_out)
        for (int64_t s = gtid; s < p.n; s += gthreads) p.v64_out[s] = (double)cur[s];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Control* ctl = p.ctl;
      ctl->sweeps = sweeps;
      ctl->outer_iters = outer;
      ctl->policy_changes_last = changes_last;
      ctl->recentrings = recentrings;
      ctl->final_dv_inf = last_dv;
      ctl->final_err_ref = last_err;
      ctl->converged = converged;
      ctl->dv_last = (float)last_dv;
    }
  }
};

// Threads per workgroup and waves per SIMD of an engine's launch: one
// 1024-thread workgroup per CU is 4 waves per SIMD, so the compiler may use
// the 128 VGPRs that allows rather than serialise loads for occupancy; the
// column-block engine runs 512-thread workgroups (its LDS holds one per CU),
// 2 waves per SIMD and up to 256 VGPRs.
template <class Eng>
struct LaunchOf {
  static constexpr int kThreads = 1024, kWavesPerEU = 4;
};
template <int UNR, int LPR>
struct LaunchOf<ColEngine<UNR, LPR>> {
  static constexpr int kThreads = kColThreads, kWavesPerEU = 2;
};

template <class Eng, int TASK>
__global__ void __launch_bounds__(LaunchOf<Eng>::kThreads)
    __attribute__((amdgpu_waves_per_eu(LaunchOf<Eng>::kWavesPerEU, LaunchOf<Eng>::kWavesPerEU)))
solve_kernel(KParams p) {
  Driver<typename Eng::Acc> d(p);
  const int64_t n = p.n;
  uint64_t t = p.first_sweep;
  // prologue: second buffer, row sums and shifted costs, first order
  for (int64_t s = d.gtid; s < n; s += d.gthreads) p.vbuf1[s] = p.vbuf0[s];
  if (TASK != kTaskSweep) {
    if (p.shift)
      for (int64_t s = d.gtid; s < n; s += d.gthreads) p.shift[s] = 0.0;
    for (int64_t s = d.gtid; s < n; s += d.gthreads) p.tgt[s] = p.vref ? p.vref[s] : 0.0;
    for (int64_t i = d.gtid; i < n * p.m; i += d.gthreads) p.ceff[i] = (double)p.c32[i];
  }
  long long since_recentre = 0;
  if constexpr (!Eng::kBand) d.fill_order(t, 0, min(p.b, n));
  if (blockIdx.x == 0 && threadIdx.x == 0) reset_slot(p.ctl, 0);
  if (!grid_sync(d.g)) return;

  long long sweeps = 0, outer = 0, changes_last = -1, recentrings = 0;
  double last_dv = NAN, last_err = NAN;
  int converged = 0;

  if constexpr (TASK == kTaskSweep) {
    if (!d.template sweep<Eng, false>(t, p.policy_sweep ? kModePolicy : kModeMin)) return;
    sweeps = 1;
    last_dv = slot_double(p.ctl, (int)((d.epoch - 1) % 3), kAccDv);
    converged = 1;
  } else if constexpr (TASK == kTaskVI) {
    while (true) {
      if (!d.template sweep<Eng, true>(t, kModeMin)) return;
      ++t;
      ++sweeps;
      const int sl = (int)((d.epoch - 1) % 3);
      last_dv = slot_double(p.ctl, sl, kAccDv);
      bool stop = p.tol_dv >= 0.0 && last_dv <= p.tol_dv;
      if (p.vref) {
        last_err = slot_double(p.ctl, sl, kAccErr);
        stop = stop || last_err <= p.eps;
      }
      if (stop) {
        converged = 1;
        break;
      }
      if (sweeps >= p.max_sweeps) break;
      if (d.want_recentre(sl, last_dv, ++since_recentre)) {
        if (!d.template recentre<Eng>(recentrings)) return;
        since_recentre = 0;
      }
    }
    if (p.want_policy_out)
      if (!d.template improve<Eng, true>(false)) return;
  } else {  // MPI, Algorithm 1
    if (!p.policy_is_init)
      if (!d.template improve<Eng, true>(false)) return;
    bool done = false;
    while (!done) {
      for (int k = 0; k < p.K; ++k) {
        if (!d.template sweep<Eng, true>(t, kModePolicy)) return;
        ++t;
        ++sweeps;
        const int sl = (int)((d.epoch - 1) % 3);
        if (p.vref) {
          last_err = slot_double(p.ctl, sl, kAccErr);
          if (last_err <= p.eps) {
            converged = 1;
            done = true;
            break;
          }
        }
        if (d.want_recentre(sl, slot_double(p.ctl, sl, kAccDv), ++since_recentre)) {
          if (!d.template recentre<Eng>(recentrings)) return;
          since_recentre = 0;
        }
      }
      if (done) break;
      if (!d.template improve<Eng, true>(true)) return;
      ++outer;
      const int sl = (int)((d.epoch - 1) % 3);
      changes_last = (long long)atomic_load_agent(&p.ctl->acc[sl][kAccChanges]);
      last_dv = slot_double(p.ctl, sl, kAccResid);
      if (changes_last == 0 && p.tol_dv >= 0.0 && last_dv <= p.tol_dv) {
        converged = 1;
        break;
      }
      if (outer >= p.max_outer) break;
    }
  }
  d.finish(sweeps, outer, changes_last, recentrings, last_dv, last_err, converged);
}

// The instantiation of the solve kernel for an engine and task.

template <class Eng>
inline SolveFn solve_fn(int task) {
  if (task == kTaskSweep) return &solve_kernel<Eng, kTaskSweep>;
  if (task == kTaskVI) return &solve_kernel<Eng, kTaskVI>;
  return &solve_kernel<Eng, kTaskMPI>;
}

}  // namespace mbdp
