// Many independent dense MDPs of uneven size in one launch.
//
// A workgroup takes the next MDP from a queue and runs MB-VI on it alone:
// the sweep order sigma_t of its own n and seed, batches of its own b, and
// between batches only a workgroup barrier, since no other workgroup
// touches the MDP.  V (FP64, up to 8192 states) lives in LDS for the whole
// solve; the rows stream from HBM, FP32 / BF16 / FP8 values decoded exactly
// and accumulated in FP64, so no re-centring is needed.  The launch is an
// ordinary one (no cooperative launch) and can be captured in a hipGraph.
//
// The heaviest MDPs (bytes per sweep times the sweeps gamma asks for) are
// served by a team of workgroups instead, so that one long solve does not
// hold the whole launch on one compute unit: the members split each batch's
// states, publish the new values in a global buffer, meet at a team barrier
// (an arrival counter), and each copies the batch into its own LDS V.  The
// queue hands out the teams' tickets first and the host keeps the members of
// all teams within the compute units of the device, so every member of every
// team is resident from the start and no member waits for a workgroup that
// is busy with another MDP.
//
// A lane group of LANES lanes serves one state at a time: lanes split the
// row's columns, 16 bytes of the row per lane and step, and the rows of the
// state are taken 8 (FP8: 4) at a time so the V values a lane loads from
// LDS serve all of them.

#include <hip/hip_runtime.h>

#include <math.h>

#include "mbdp_engines.h"

namespace mbdp {

// rows of a state taken together: FP8 holds 16 values of V per step, so 4
template <int VT>
constexpr int batch_rows() {
  return VT == kFP8 ? 4 : 8;
}

template <int VT>
struct BatchVals;

template <>
struct BatchVals<kF32> {
  static constexpr int kEpl = 4;  // values per 16-byte load
  static constexpr int kBytes = 4;
  __device__ __forceinline__ static void decode(const u4& x, double (&out)[kEpl]) {
    out[0] = (double)__uint_as_float(x.x);
    out[1] = (double)__uint_as_float(x.y);
    out[2] = (double)__uint_as_float(x.z);
    out[3] = (double)__uint_as_float(x.w);
  }
};

template <>
struct BatchVals<kBF16> {
  static constexpr int kEpl = 8;
  static constexpr int kBytes = 2;
  __device__ __forceinline__ static void decode(const u4& x, double (&out)[kEpl]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      out[2 * w] = (double)bf16_lo(x[w]);
      out[2 * w + 1] = (double)bf16_hi(x[w]);
    }
  }
};

template <>
struct BatchVals<kFP8> {
  static constexpr int kEpl = 16;
  static constexpr int kBytes = 1;
  __device__ __forceinline__ static void decode(const u4& x, double (&out)[kEpl]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const f4 d = fp8x4(x[w]);
      out[4 * w] = (double)d.x;
      out[4 * w + 1] = (double)d.y;
      out[4 * w + 2] = (double)d.z;
      out[4 * w + 3] = (double)d.w;
    }
  }
};

// The item table holds generic pointers; these views make the compiler use
// global (not flat) memory instructions for them.
#define MBDP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const MBDP_GLOBAL T* gview(const void* p) {
  return (const MBDP_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ MBDP_GLOBAL T* gview_mut(void* p) {
  return (MBDP_GLOBAL T*)p;
}

struct BatchShared {
  double V[kBatchMaxN];
  double newv[kBatchMaxB];
  int32_t sidx[kBatchMaxB];
  double red[16];
  int item, rank, ok;
};

// min_a Q(s, a) (FP64) and its action, lowest index on ties, for the lane
// group of `sl` (lane within the group) serving state s.  Every lane of the
// group returns the same result.
template <int VT, int LANES>
__device__ __forceinline__ void batch_state(const BatchItem& I, const double* V, int32_t s,
                                            int sl, double& qbest, int& abest) {
  using B = BatchVals<VT>;
  constexpr int EPL = B::kEpl;
  constexpr int kBatchRows = batch_rows<VT>();
  const int64_t m = I.m, ld = I.ld;
  const MBDP_GLOBAL uint8_t* P = gview<uint8_t>(I.P);
  const MBDP_GLOBAL float* C = gview<float>(I.c);
  const MBDP_GLOBAL float* RS = gview<float>(I.rscale);
  qbest = INFINITY;
  abest = 0;
  for (int a0 = 0; a0 < m; a0 += kBatchRows) {
    double acc[kBatchRows];
#pragma unroll
    for (int r = 0; r < kBatchRows; ++r) acc[r] = 0.0;
    const size_t row0 = (size_t)s * m + a0;
    for (int64_t j = (int64_t)sl * EPL; j < ld; j += (int64_t)LANES * EPL) {
      double v[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) v[e] = V[j + e];
      u4 x[kBatchRows];
#pragma unroll
      for (int r = 0; r < kBatchRows; ++r)
        x[r] = (a0 + r < m) ? __builtin_nontemporal_load((const MBDP_GLOBAL u4*)(
                                  P + ((row0 + r) * (size_t)ld + (size_t)j) * B::kBytes))
                            : u4{0u, 0u, 0u, 0u};
#pragma unroll
      for (int r = 0; r < kBatchRows; ++r) {
        double d[EPL];
        B::decode(x[r], d);
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[r] = fma(d[e], v[e], acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < kBatchRows; ++r) {
#pragma unroll
      for (int off = LANES >> 1; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
      const int a = a0 + r;
      if (a < m) {
        const size_t row = row0 + r;
        const double scale = VT == kF32 ? 1.0 : (double)RS[row];
        const double q = (double)C[row] + I.gamma * (scale * acc[r]);
        if (q < qbest) {  // strictly smaller keeps the lowest action on ties
          qbest = q;
          abest = a;
        }
      }
    }
  }
}

template <int VT, int LANES>
__device__ void batch_solve_item(const BatchItem& I, BatchShared& sh, BatchStat* stats,
                                 double tol, long long max_sweeps) {
  constexpr int GPW = kWave / LANES;  // lane groups per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sl = lane % LANES;
  const int group = wave * GPW + lane / LANES;
  const int groups = (blockDim.x >> 6) * GPW;
  const int64_t n = I.n, b = I.b, nb = (n + b - 1) / b;
  const MBDP_GLOBAL double* V0 = gview<double>(I.V);
  for (int64_t j = threadIdx.x; j < I.ld; j += blockDim.x) sh.V[j] = j < n ? V0[j] : 0.0;
  __syncthreads();
  const unsigned long long t_start = wall_clock64();
  long long sweeps = 0;
  double dv = INFINITY;
  int converged = 0;
  for (uint64_t t = 0; (long long)t < max_sweeps; ++t) {
    const OrderKey key = make_order_key(n, I.seed, t);
    double dvl = 0.0;
    for (int64_t k = 0; k < nb; ++k) {
      const int64_t kb = k * b, bk = min(b, n - kb);
      for (int64_t i = group; i < bk; i += groups) {
        const int32_t s = (int32_t)sweep_order_at((uint32_t)(kb + i), key);
        double q;
        int a;
        batch_state<VT, LANES>(I, sh.V, s, sl, q, a);
        if (sl == 0) {
          sh.newv[i] = q;
          sh.sidx[i] = s;
          dvl = fmax(dvl, fabs(q - sh.V[s]));
        }
      }
      __syncthreads();  // every state of the batch read the values before it
      for (int64_t i = threadIdx.x; i < bk; i += blockDim.x) sh.V[sh.sidx[i]] = sh.newv[i];
      __syncthreads();  // committed before the next batch reads
    }
    ++sweeps;
    dvl = wave_max_d(dvl);
    if (lane == 0) sh.red[wave] = dvl;
    __syncthreads();
    dv = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) dv = fmax(dv, sh.red[w]);
    __syncthreads();
    if (dv <= tol) {
      converged = 1;
      break;
    }
  }
  // results: V, and the greedy policy at the final V
  MBDP_GLOBAL double* Vout = gview_mut<double>(I.V);
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) Vout[j] = sh.V[j];
  if (I.policy) {
    MBDP_GLOBAL int32_t* pol = gview_mut<int32_t>(I.policy);
    for (int64_t s = group; s < n; s += groups) {
      double q;
      int a;
      batch_state<VT, LANES>(I, sh.V, (int32_t)s, sl, q, a);
      if (sl == 0) pol[s] = a;
    }
  }
  if (threadIdx.x == 0) {
    BatchStat st;
    st.sweeps = sweeps;
    st.dv = dv;
    st.converged = converged;
    st.pad = 0;
    st.t_start = t_start;
    st.t_end = wall_clock64();
    stats[I.index] = st;
  }
  __syncthreads();
}

// Team of K workgroups on one MDP (see the file comment).  The arrival
// counter only grows: the p-th barrier of the solve (p = 0, 1, ...) ends when
// it reaches (p + 1) K.  Release by one thread after every wave's memory
// operations are done makes the workgroup's writes visible device-wide;
// acquire after the wait makes the others' writes visible to it.  Gives up
// (false, and raises the launch's abort flag) after `timeout` ticks or when
// another team gave up.
__device__ __forceinline__ bool team_sync(unsigned long long* arrive, unsigned* abort,
                                          unsigned long long target,
                                          unsigned long long timeout, BatchShared& sh) {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads and stores are done
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(arrive, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const unsigned long long t0 = wall_clock64();
    while (atomic_load_agent(arrive) < target) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (wall_clock64() - t0 > timeout) {
        __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sh.ok = ok;
  }
  __syncthreads();
  return sh.ok != 0;
}

// Member `rank` of a team of I.team workgroups.  Every member runs the same
// sequence of barriers (the stop decision is taken on the same values by
// all), so no member waits for a barrier that another skips.
template <int VT, int LANES>
__device__ void batch_solve_team(const BatchItem& I, int rank, BatchShared& sh,
                                 const BatchArgs& A) {
  constexpr int GPW = kWave / LANES;
  const int K = I.team;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sl = lane % LANES;
  const int groups = (blockDim.x >> 6) * GPW;
  const int gid = rank * groups + wave * GPW + lane / LANES;  // lane group within the team
  const int gstride = K * groups;
  const int64_t n = I.n, b = I.b, nb = (n + b - 1) / b;
  unsigned long long* arrive = &A.ctl->arrive[I.slot];
  double* dvm = A.team_dv + (size_t)I.slot * 2 * kBatchMaxTeam;  // [2][kBatchMaxTeam]
  MBDP_GLOBAL double* gnew = gview_mut<double>(A.team_new + (size_t)I.slot * 2 * kBatchMaxB);
  const MBDP_GLOBAL double* V0 = gview<double>(I.V);
  for (int64_t j = threadIdx.x; j < I.ld; j += blockDim.x) sh.V[j] = j < n ? V0[j] : 0.0;
  __syncthreads();
  const unsigned long long t_start = wall_clock64();
  long long sweeps = 0;
  double dv = INFINITY;
  int converged = 0;
  unsigned long long phase = 0;
  bool ok = true;
  for (uint64_t t = 0; ok && (long long)t < A.max_sweeps; ++t) {
    const OrderKey key = make_order_key(n, I.seed, t);
    double dvl = 0.0;
    for (int64_t k = 0; k < nb; ++k) {
      const int64_t kb = k * b, bk = min(b, n - kb);
      MBDP_GLOBAL double* buf = gnew + (phase & 1) * kBatchMaxB;
      for (int64_t i = gid; i < bk; i += gstride) {
        const int32_t s = (int32_t)sweep_order_at((uint32_t)(kb + i), key);
        double q;
        int a;
        batch_state<VT, LANES>(I, sh.V, s, sl, q, a);
        if (sl == 0) {
          buf[i] = q;
          dvl = fmax(dvl, fabs(q - sh.V[s]));
        }
      }
      if (k == nb - 1) {  // this member's max |dV| of the sweep, by sweep parity
        dvl = wave_max_d(dvl);
        if (lane == 0) sh.red[wave] = dvl;
        __syncthreads();
        if (threadIdx.x == 0) {
          double d = 0.0;
          for (int w = 0; w < (int)(blockDim.x >> 6); ++w) d = fmax(d, sh.red[w]);
          gview_mut<double>(dvm)[(t & 1) * kBatchMaxTeam + rank] = d;
        }
      }
      // buffers of parity p are rewritten at phase p + 2, after barrier p + 1,
      // which every member reaches only once it has read them
      ok = team_sync(arrive, &A.ctl->abort, (phase + 1) * (unsigned long long)K,
                     A.timeout_ticks, sh);
      if (!ok) break;
      for (int64_t i = threadIdx.x; i < bk; i += blockDim.x)
        sh.V[sweep_order_at((uint32_t)(kb + i), key)] = buf[i];
      ++phase;
      __syncthreads();  // committed before the next batch reads
    }
    if (!ok) break;
    ++sweeps;
    dv = 0.0;
    for (int r = 0; r < K; ++r) dv = fmax(dv, gview<double>(dvm)[(t & 1) * kBatchMaxTeam + r]);
    if (dv <= A.tol) {
      converged = 1;
      break;
    }
  }
  if (ok) {
    if (rank == 0) {
      MBDP_GLOBAL double* Vout = gview_mut<double>(I.V);
      for (int64_t j = threadIdx.x; j < n; j += blockDim.x) Vout[j] = sh.V[j];
    }
    if (I.policy) {
      MBDP_GLOBAL int32_t* pol = gview_mut<int32_t>(I.policy);
      for (int64_t s = gid; s < n; s += gstride) {
        double q;
        int a;
        batch_state<VT, LANES>(I, sh.V, (int32_t)s, sl, q, a);
        if (sl == 0) pol[s] = a;
      }
    }
  }
  if (rank == 0 && threadIdx.x == 0) {
    BatchStat st;
    st.sweeps = sweeps;
    st.dv = dv;
    st.converged = ok ? converged : 0;
    st.pad = ok ? 0 : 1;
    st.t_start = t_start;  // member 0's: the team starts together
    st.t_end = wall_clock64();
    A.stats[I.index] = st;
  }
  __syncthreads();
}

template <int VT>
__device__ __forceinline__ void batch_dispatch_lanes(const BatchItem& I, int rank,
                                                     BatchShared& sh, const BatchArgs& A) {
  if (I.team > 1) {
    if (I.lanes == 16)
      batch_solve_team<VT, 16>(I, rank, sh, A);
    else if (I.lanes == 32)
      batch_solve_team<VT, 32>(I, rank, sh, A);
    else
      batch_solve_team<VT, 64>(I, rank, sh, A);
  } else if (I.lanes == 16) {
    batch_solve_item<VT, 16>(I, sh, A.stats, A.tol, A.max_sweeps);
  } else if (I.lanes == 32) {
    batch_solve_item<VT, 32>(I, sh, A.stats, A.tol, A.max_sweeps);
  } else {
    batch_solve_item<VT, 64>(I, sh, A.stats, A.tol, A.max_sweeps);
  }
}

// Tickets 0, 1, ... are handed out in order; item i owns the tickets
// [ticket0, ticket0 + team), the items ordered by ticket0.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4)))
batch_kernel(BatchArgs A) {
  __shared__ BatchShared sh;
  const BatchItem& last = A.items[A.count - 1];
  const long long tickets = last.ticket0 + last.team;
  while (true) {
    if (threadIdx.x == 0) {
      const long long u = (long long)atomicAdd(&A.ctl->queue, 1u);
      int it = A.count;
      if (u < tickets) {  // the last item whose first ticket is <= u
        int lo = 0, hi = A.count - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (A.items[mid].ticket0 <= u) lo = mid; else hi = mid - 1;
        }
        it = lo;
        sh.rank = (int)(u - A.items[lo].ticket0);
      }
      sh.item = it;
    }
    __syncthreads();
    const int it = sh.item, rank = sh.rank;
    __syncthreads();
    if (it >= A.count) break;
    const BatchItem I = A.items[it];
    if (I.dtype == kBF16)
      batch_dispatch_lanes<kBF16>(I, rank, sh, A);
    else if (I.dtype == kFP8)
      batch_dispatch_lanes<kFP8>(I, rank, sh, A);
    else
      batch_dispatch_lanes<kF32>(I, rank, sh, A);
    if (__hip_atomic_load(&A.ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
  }
}

int launch_batch(const BatchArgs& a, int blocks, void* stream) {
  hipLaunchKernelGGL(batch_kernel, dim3(blocks), dim3(1024), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mbdp
