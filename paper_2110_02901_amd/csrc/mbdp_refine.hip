// The FP64 correction of libmbdp (mdp_refine): the iterate V, the
// accumulation of every dot product, the costs, the minimum and the
// stopping tests are FP64; the transition rows are the handle's FP32 values,
// widened exactly.  It closes the gap between the solution of a reduced-
// precision copy of an MDP and the MDP itself.
//
// Certificate (Sec. III-B): every B_{sigma,b} (eq. (11)) is a gamma-
// contraction in the max norm with fixed point J*, for any order and batch
// size, and so is T (eq. (7)).  Hence max|V - J*| <= max|TV - V| / (1 - gamma)
// for any V, and after a sweep V' = B V,
//   max|V' - J*| <= min(gamma max|V' - V| / (1 - gamma), gamma max|V - J*|).
// The kernel evaluates max|TV - V| of its input in one pass over all states
// (V fixed), then either applies sweeps of B_{sigma_t,b} until the second
// bound certifies eps (K = 0), or runs Algorithm 1 -- the improvement step,
// which yields the residual, then K sweeps of B_{mu,sigma_t,b} -- until an
// improvement step's residual certifies eps (K >= 1).
//
// One persistent cooperative launch runs the whole correction with the
// solvers' driver (orders, batches, ping-pong buffers, grid barriers) over
// FP64 buffers.  The engines:
//  * dense: a workgroup per state streams the state's m rows (8 rows at a
//    time, two 16-byte loads per row and thread, V reused from registers
//    across the rows) against V staged in LDS (n <= 8192) or read from
//    memory; in policy sweeps a wavefront per state;
//  * constant row length k: a wavefront per state, k/4 lanes per row, V
//    gathered in FP64; in policy sweeps a lane group per state;
//  * general CSR: a wavefront per state, lanes striding each row.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>

#include "mbdp_engines.h"

namespace mbdp {

namespace {

// New value q (action a) of state s in a sweep.
template <class Acc>
__device__ __forceinline__ void commit64(const KParams& p, const CtxT<double>& c, int32_t s,
                                         double q, int a, double old, Acc& L) {
  c.wr[s] = q;
  if (p.argmin_out) p.argmin_out[s] = a;
  L.max_abs(kAccDv, fabs(q - old));
  if (p.vref) L.max_abs(kAccErr, fabs(q - p.vref[s]));
}

// Improvement step at state s (V fixed): the residual |(TV)(s) - V(s)|, the
// greedy action, and the error of V(s) itself against V_ref.
template <class Acc>
__device__ __forceinline__ void improve64(const KParams& p, int32_t s, double q, int a,
                                          double old, bool count, Acc& L) {
  if (p.policy) {
    if (count && p.policy[s] != a) L.count_change();
    p.policy[s] = a;
  }
  L.max_abs(kAccResid, fabs(q - old));
  if (p.vref) L.max_abs(kAccErr, fabs(old - p.vref[s]));
}

// Lowest-index minimum of s_q[0, m) in wavefront 0 of the workgroup; every
// lane of that wavefront gets the result.
__device__ __forceinline__ void lds_argmin(const double* s_q, int m, double& qv, int& av) {
  const int lane = threadIdx.x & 63;
  qv = INFINITY;
  av = 0x7fffffff;
  for (int a = lane; a < m; a += kWave) {
    const double x = s_q[a];
    if (x < qv) {
      qv = x;
      av = a;
    }
  }
  wave_argmin(qv, av);
  if (av == 0x7fffffff) av = 0;
}

constexpr int kStage64 = 8192;  // FP64 values of V staged in LDS (64 KB)

// LDS of the dense engine, one instance per kernel whatever the template
// instantiations that use it (a __shared__ variable inside a template
// exists once per instantiation).
struct Dense64Shared {
  double v[kStage64];        // V staged for the batch
  double q[kMaxActions];     // Q of the state's actions
  double red[16][8];         // per-wavefront row sums
};

__device__ __forceinline__ Dense64Shared& dense64_shared() {
  __shared__ Dense64Shared sh;
  return sh;
}

}  // namespace

// ------------------------------------------------------------ dense, FP64

template <int VEC>
struct Dense64Engine {
  static constexpr bool kBand = false;
  using Acc = LdsAcc;
  static constexpr int R = 8;   // rows of a state per pass
  static constexpr int U = 1;   // column steps in flight (R * U 16-byte loads per thread)

  // acc[r] += row r . V over this thread's columns (all n), rows r < nrows.
  template <bool STAGED>
  __device__ __forceinline__ static void dot_rows(const float* __restrict__ rows, uint32_t n,
                                                  int nrows, const double* __restrict__ V,
                                                  double (&acc)[R]) {
    const uint32_t step = blockDim.x * VEC;
    for (uint32_t j0 = threadIdx.x * VEC; j0 < n; j0 += step * U) {
      if constexpr (VEC == 4) {
        f4 x[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const uint32_t j = j0 + u * step;
            x[u][r] = (r < nrows && j < n)
                          ? __builtin_nontemporal_load(
                                reinterpret_cast<const f4*>(rows + (size_t)r * n + j))
                          : f4{0.f, 0.f, 0.f, 0.f};
          }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t j = j0 + u * step;
          if (j >= n) break;
          const double v0 = V[j], v1 = V[j + 1], v2 = V[j + 2], v3 = V[j + 3];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            acc[r] = fma((double)x[u][r].x, v0, acc[r]);
            acc[r] = fma((double)x[u][r].y, v1, acc[r]);
            acc[r] = fma((double)x[u][r].z, v2, acc[r]);
            acc[r] = fma((double)x[u][r].w, v3, acc[r]);
          }
        }
      } else {
        float x[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const uint32_t j = j0 + u * step;
            x[u][r] = (r < nrows && j < n) ? __builtin_nontemporal_load(rows + (size_t)r * n + j)
                                           : 0.f;
          }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t j = j0 + u * step;
          if (j >= n) break;
          const double v = V[j];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = fma((double)x[u][r], v, acc[r]);
        }
      }
    }
  }

  template <bool STAGED, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch_min(const KParams& p, const int32_t* ord,
                                                   int64_t bk, const CtxT<double>& c,
                                                   const double* V, int mode, Acc& L) {
    Dense64Shared& sh = dense64_shared();
    double (&red)[16][8] = sh.red;
    double* s_q = sh.q;
    const uint32_t n = (uint32_t)p.n;
    const int m = p.m;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t i = blockIdx.x; i < bk; i += gridDim.x) {
      int32_t s;
      if constexpr (IDENT)
        s = (int32_t)i;
      else
        s = ord[i];
      s = __builtin_amdgcn_readfirstlane(s);
      for (int a0 = 0; a0 < m; a0 += R) {
        const int nrows = min(R, m - a0);
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        dot_rows<STAGED>(p.P + ((size_t)s * m + a0) * n, n, nrows, V, acc);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double x = wave_sum_d(acc[r]);
          if (lane == 0) red[w][r] = x;
        }
        __syncthreads();
        if ((int)threadIdx.x < nrows) {
          double sum = 0.0;
          for (int i2 = 0; i2 < nw; ++i2) sum += red[i2][threadIdx.x];
          const int64_t row = (int64_t)s * m + a0 + threadIdx.x;
          s_q[a0 + threadIdx.x] = (double)p.c32[row] + p.gamma * sum;
        }
        __syncthreads();
      }
      if (w == 0) {
        double qv;
        int av;
        lds_argmin(s_q, m, qv, av);
        if (lane == 0) {
          const double old = c.rd[s];
          if (mode >= kModeImprove)
            improve64(p, s, qv, av, old, mode == kModeImproveCount, L);
          else
            commit64(p, c, s, qv, av, old, L);
        }
      }
      __syncthreads();
    }
  }

  // Policy sweeps: a wavefront per state, the state's one row.
  template <bool STAGED, class Acc>
  __device__ __forceinline__ static void batch_policy(const KParams& p, const int32_t* ord,
                                                      int64_t bk, const CtxT<double>& c,
                                                      const double* V, Acc& L) {
    constexpr int U = 4;
    const uint32_t n = (uint32_t)p.n;
    const int m = p.m;
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t i = gw; i < bk; i += nwv) {
      const int32_t s = __builtin_amdgcn_readfirstlane(ord[i]);
      int a = __builtin_amdgcn_readfirstlane(p.policy[s]);
      if (a < 0 || a >= m) {
        if (lane == 0) raise_abort(p.ctl, kDevBadPolicy);
        a = 0;
      }
      const int64_t row = (int64_t)s * m + a;
      const float* rp = p.P + (size_t)row * n;
      double acc = 0.0;
      const uint32_t step = kWave * VEC;
      for (uint32_t j0 = lane * VEC; j0 < n; j0 += step * U) {
        if constexpr (VEC == 4) {
          f4 x[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + u * step;
            x[u] = j < n ? __builtin_nontemporal_load(reinterpret_cast<const f4*>(rp + j))
                         : f4{0.f, 0.f, 0.f, 0.f};
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + u * step;
            if (j < n) {
              acc = fma((double)x[u].x, V[j], acc);
              acc = fma((double)x[u].y, V[j + 1], acc);
              acc = fma((double)x[u].z, V[j + 2], acc);
              acc = fma((double)x[u].w, V[j + 3], acc);
            }
          }
        } else {
          float x[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + u * step;
            x[u] = j < n ? __builtin_nontemporal_load(rp + j) : 0.f;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + u * step;
            if (j < n) acc = fma((double)x[u], V[j], acc);
          }
        }
      }
      acc = wave_sum_d(acc);
      if (lane == 0) commit64(p, c, s, (double)p.c32[row] + p.gamma * acc, a, c.rd[s], L);
    }
  }

  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch(const KParams& p, const int32_t* ord, int64_t bk,
                                               const CtxT<double>& c, int mode, Acc& L) {
    double* s_v = dense64_shared().v;
    const int64_t units_per_wg = mode == kModePolicy ? (int64_t)(blockDim.x >> 6) : 1;
    if ((int64_t)blockIdx.x * units_per_wg >= bk) return;  // uniform over the workgroup
    if (p.n <= kStage64) {
      for (int64_t j = threadIdx.x; j < p.n; j += blockDim.x) s_v[j] = c.rd[j];
      __syncthreads();
      if (mode == kModePolicy)
        batch_policy<true>(p, ord, bk, c, s_v, L);
      else
        batch_min<true, IDENT>(p, ord, bk, c, s_v, mode, L);
      __syncthreads();  // s_v is rewritten by the next batch
    } else {
      if (mode == kModePolicy)
        batch_policy<false>(p, ord, bk, c, c.rd, L);
      else
        batch_min<false, IDENT>(p, ord, bk, c, c.rd, mode, L);
    }
  }
};

// ------------------------------------------------------------ constant row length, FP64

template <int LPR>
struct Ell64Engine {
  static constexpr bool kBand = false;
  using Acc = RegAcc;
  static constexpr int kRpp = kWave / LPR;  // rows per wavefront pass

  // FP64 dot product of this lane's (up to) 4 entries at entry e with V,
  // summed over the LPR lanes of the row (every lane of the group gets it).
  __device__ __forceinline__ static double row_part(const KParams& p, size_t e, bool has,
                                                    const double* __restrict__ V) {
    const i4 cc = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p.col + e));
    const f4 vv = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p.val + e));
    const double g0 = V[cc.x], g1 = V[cc.y], g2 = V[cc.z], g3 = V[cc.w];
    double part = (double)vv.x * g0;
    part = fma((double)vv.y, g1, part);
    part = fma((double)vv.z, g2, part);
    part = fma((double)vv.w, g3, part);
    part = has ? part : 0.0;
#pragma unroll
    for (int off = LPR >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off);
    return part;
  }

  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch(const KParams& p, const int32_t* ord, int64_t bk,
                                               const CtxT<double>& c, int mode, Acc& L) {
    const int m = p.m, k = p.ell_k;
    const int lane = threadIdx.x & 63, g = lane / LPR, l = lane % LPR;
    const bool has = l * 4 < k;
    const int lcol = has ? l * 4 : 0;  // lanes beyond the row read its first entries
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x >> 6);
    const double* __restrict__ V = c.rd;
    if (mode == kModePolicy) {  // a lane group per state
      for (int64_t u = gw; u * kRpp < bk; u += nwv) {
        const int64_t pos = u * kRpp + g;
        const bool valid = pos < bk;
        const int32_t s = ord[valid ? pos : 0];
        int a = p.policy[s];
        if (a < 0 || a >= m) {
          if (valid) raise_abort(p.ctl, kDevBadPolicy);
          a = 0;
        }
        const int64_t row = (int64_t)s * m + a;
        const double part = row_part(p, (size_t)row * k + lcol, has, V);
        if (l == 0 && valid) commit64(p, c, s, (double)p.c32[row] + p.gamma * part, a, V[s], L);
      }
      return;
    }
    for (int64_t u = gw; u < bk; u += nwv) {  // a wavefront per state
      int32_t s;
      if constexpr (IDENT)
        s = (int32_t)u;
      else
        s = ord[u];
      double qb = INFINITY;
      int ab = 0x7fffffff;
      for (int a0 = 0; a0 < m; a0 += kRpp) {
        const int a = a0 + g;
        const bool row_ok = a < m;
        const int64_t row = (int64_t)s * m + (row_ok ? a : m - 1);
        const double part = row_part(p, (size_t)row * k + lcol, has, V);
        double q = row_ok ? (double)p.c32[row] + p.gamma * part : INFINITY;
        int aq = row_ok ? a : 0x7fffffff;
        wave_argmin_from<LPR>(q, aq);
        const bool better = q < qb || (q == qb && aq < ab);
        qb = better ? q : qb;
        ab = better ? aq : ab;
      }
      if (lane == 0) {
        const int av = ab == 0x7fffffff ? 0 : ab;
        if (mode >= kModeImprove)
          improve64(p, s, qb, av, V[s], mode == kModeImproveCount, L);
        else
          commit64(p, c, s, qb, av, V[s], L);
      }
    }
  }
};

// ------------------------------------------------------------ general CSR, FP64

struct Csr64Engine {
  static constexpr bool kBand = false;
  using Acc = RegAcc;

  __device__ __forceinline__ static double row_dot(const KParams& p, int64_t row,
                                                   const double* __restrict__ V) {
    const int lane = threadIdx.x & 63;
    const int64_t e0 = p.row_ptr[row], e1 = p.row_ptr[row + 1];
    double part = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += kWave) part = fma((double)p.val[e], V[p.col[e]], part);
    return wave_sum_d(part);
  }

  template <bool CE, bool IDENT, class Acc>
  __device__ __forceinline__ static void batch(const KParams& p, const int32_t* ord, int64_t bk,
                                               const CtxT<double>& c, int mode, Acc& L) {
    const int m = p.m;
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x >> 6);
    const double* __restrict__ V = c.rd;
    for (int64_t u = gw; u < bk; u += nwv) {
      int32_t s;
      if constexpr (IDENT)
        s = (int32_t)u;
      else
        s = ord[u];
      s = __builtin_amdgcn_readfirstlane(s);
      if (mode == kModePolicy) {
        int a = __builtin_amdgcn_readfirstlane(p.policy[s]);
        if (a < 0 || a >= m) {
          if (lane == 0) raise_abort(p.ctl, kDevBadPolicy);
          a = 0;
        }
        const int64_t row = (int64_t)s * m + a;
        const double part = row_dot(p, row, V);
        if (lane == 0) commit64(p, c, s, (double)p.c32[row] + p.gamma * part, a, V[s], L);
        continue;
      }
      double qb = INFINITY;
      int ab = 0;
      for (int a = 0; a < m; ++a) {
        const int64_t row = (int64_t)s * m + a;
        const double q = (double)p.c32[row] + p.gamma * row_dot(p, row, V);
        if (q < qb) {  // strictly smaller keeps the lowest index
          qb = q;
          ab = a;
        }
      }
      if (lane == 0) {
        if (mode >= kModeImprove)
          improve64(p, s, qb, ab, V[s], mode == kModeImproveCount, L);
        else
          commit64(p, c, s, qb, ab, V[s], L);
      }
    }
  }
};

// ------------------------------------------------------------ the correction kernel

template <class Eng>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4)))
refine_kernel(KParams p) {
  Driver<typename Eng::Acc, double> d(p);
  const int64_t n = p.n;
  const double gamma = p.gamma, inv = 1.0 / (1.0 - gamma);
  uint64_t t = p.first_sweep;
  for (int64_t s = d.gtid; s < n; s += d.gthreads) p.vd1[s] = p.vd0[s];
  d.fill_order(t, 0, min(p.b, n));
  if (blockIdx.x == 0 && threadIdx.x == 0) reset_slot(p.ctl, 0);
  if (!grid_sync(d.g)) return;

  // the input: residual max|TV - V| (its certificate) and the greedy policy
  if (!d.template improve<Eng, false>(false)) return;
  int sl = (int)((d.epoch - 1) % 3);
  const double residual_in = slot_double(p.ctl, sl, kAccResid);
  double residual = residual_in;
  double bound = residual_in * inv;
  double err = p.vref ? slot_double(p.ctl, sl, kAccErr) : (double)NAN;
  double last_dv = NAN;
  bool fresh = true;  // the last improvement step was at the current V
  bool done = p.vref ? err <= p.eps : bound <= p.eps;
  long long sweeps = 0, outer = 0;

  if (p.K == 0) {  // sweeps of B_{sigma_t,b}, the contraction bound
    while (!done && sweeps < p.max_sweeps) {
      if (!d.template sweep<Eng, false>(t, kModeMin)) return;
      ++t;
      ++sweeps;
      fresh = false;
      sl = (int)((d.epoch - 1) % 3);
      last_dv = slot_double(p.ctl, sl, kAccDv);
      bound = fmin(gamma * last_dv * inv, gamma * bound);
      if (p.vref) err = slot_double(p.ctl, sl, kAccErr);
      done = p.vref ? err <= p.eps : bound <= p.eps;
    }
  } else {  // Algorithm 1, certified at its improvement steps
    while (!done && outer < p.max_outer) {
      for (int k = 0; k < p.K; ++k) {
        if (!d.template sweep<Eng, false>(t, kModePolicy)) return;
        ++t;
        ++sweeps;
        fresh = false;
        sl = (int)((d.epoch - 1) % 3);
        last_dv = slot_double(p.ctl, sl, kAccDv);
        if (p.vref) {
          err = slot_double(p.ctl, sl, kAccErr);
          if (err <= p.eps) {
            done = true;
            break;
          }
        }
      }
      if (done) break;
      if (!d.template improve<Eng, false>(true)) return;
      ++outer;
      fresh = true;
      sl = (int)((d.epoch - 1) % 3);
      residual = slot_double(p.ctl, sl, kAccResid);
      bound = residual * inv;
      if (!p.vref) done = bound <= p.eps;
    }
  }
  // the output's residual and greedy policy, when wanted and not current
  double residual_out = fresh ? residual : (double)NAN;
  if (!fresh && (p.policy || p.K > 0)) {
    if (!d.template improve<Eng, false>(false)) return;
    sl = (int)((d.epoch - 1) % 3);
    residual_out = slot_double(p.ctl, sl, kAccResid);
  }
  if (p.K > 0) bound = residual_out * inv;
  // the result into the caller's buffer
  const double* cur = d.rd_buf();
  if (cur != p.vd0)
    for (int64_t s = d.gtid; s < n; s += d.gthreads) p.vd0[s] = cur[s];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Control* ctl = p.ctl;
    ctl->sweeps = sweeps;
    ctl->outer_iters = outer;
    ctl->final_dv_inf = last_dv;
    ctl->final_err_ref = err;
    ctl->converged = done ? 1 : 0;
    ctl->residual_in = residual_in;
    ctl->residual_out = residual_out;
    ctl->bound_out = bound;
  }
}

// ------------------------------------------------------------ launch

static SolveFn pick_refine(const KParams& p) {
  if (p.vdtype != kF32) return nullptr;
  if (p.storage == kDense)
    return (p.n % 4 == 0) ? &refine_kernel<Dense64Engine<4>> : &refine_kernel<Dense64Engine<1>>;
  if (p.storage == kEll) {
    const int lanes = (p.ell_k + 3) / 4;
    if (lanes <= 1) return &refine_kernel<Ell64Engine<1>>;
    if (lanes <= 2) return &refine_kernel<Ell64Engine<2>>;
    if (lanes <= 4) return &refine_kernel<Ell64Engine<4>>;
    if (lanes <= 8) return &refine_kernel<Ell64Engine<8>>;
    if (lanes <= 16) return &refine_kernel<Ell64Engine<16>>;
    if (lanes <= 32) return &refine_kernel<Ell64Engine<32>>;
    if (lanes <= 64) return &refine_kernel<Ell64Engine<64>>;
    return &refine_kernel<Csr64Engine>;
  }
  return &refine_kernel<Csr64Engine>;
}

int launch_refine(KParams p, LaunchShape shape, void* stream, char* err, size_t errlen) {
  SolveFn f = pick_refine(p);
  if (!f) {
    snprintf(err, errlen, "the FP64 correction needs FP32 transition values");
    return -1;
  }
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &occ, reinterpret_cast<const void*>(f), shape.threads, 0);
  if (e != hipSuccess || occ < 1) {
    snprintf(err, errlen, "occupancy query failed (%d blocks/CU): %s", occ, hipGetErrorString(e));
    return -1;
  }
  const int bpc = shape.blocks_per_cu < occ ? shape.blocks_per_cu : occ;
  int blocks = shape.cus * bpc;
  if (blocks > kMaxBlocks) blocks = kMaxBlocks;
  p.splits = 1;
  void* args[] = {&p};
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(f), dim3(blocks),
                                 dim3(shape.threads), args, 0,
                                 reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    snprintf(err, errlen, "cooperative launch (%d x %d) failed: %s", blocks, shape.threads,
             hipGetErrorString(e));
    return -1;
  }
  return 0;
}

}  // namespace mbdp
