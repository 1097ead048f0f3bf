// Several value vectors against one dense P on the matrix cores.
//
// r value vectors V[:, j], one per cost vector C[:, :, j], share P (BF16
// codes with one FP32 scale per row), gamma, the batch size b and the sweep
// order sigma_t; each follows MB-VI (Sec. III-B) of its own MDP.  For one
// batch the expected values of all vectors are a matrix product: the batch's
// rows (s, a) of P against V [n x r], which these kernels run on MFMA
// (v_mfma_f32_16x16x32_bf16).
//
// Precision.  MFMA multiplies BF16 operands and accumulates in FP32.  The
// codes of P are BF16 already; V is held as V = R + W with an FP64 anchor R
// and a small difference W, and only W goes through the matrix cores, split
// into two BF16 terms (hi + lo carry 16 significant bits): the anchor's share
// P R is computed once per re-centring in FP64.  The error of a backup is
// then a small multiple of 2^-16 max|W|, which the host keeps below a
// fraction of the current change per sweep by folding W into R (the same
// idea as the single-vector anchor).
//
// A sweep starts with `multi_order_kernel`, which writes sigma_t into a table
// of the workspace.  One batch is two launches: `multi_gemm_kernel` writes the partial products
// of a K-range of P per (row, vector) (split over K so that a batch of a few
// thousand rows still fills the device), `multi_commit_kernel` adds the
// partials in FP64 with the cost, the anchor share and the row scale, takes
// the minimum over actions and commits the batch.  `multi_end_kernel` closes
// a sweep (its max |dV| from the commits' per-position maxima, the stop flag).  Every kernel returns at once when
// the stop flag is set, so the host can enqueue several sweeps and read the
// control block once.

#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "mbdp_device.h"
#include "mbdp_internal.h"

namespace mbdp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

#define MBDP_GLOBAL __attribute__((address_space(1)))

// round-to-nearest-even FP32 -> BF16 bits (NaN is not produced here: W is finite)
__device__ __forceinline__ unsigned multi_bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return ((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16) & 0xFFFFu;
}

__device__ __forceinline__ bool multi_done(const MultiControl* ctl) {
  return __hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Row `row` of a launch over positions kb, kb + 1, ... : its state and
// action.  Positions are those of sweep order sigma_t (the table the sweep's
// order kernel wrote), or (full) the states themselves, for the greedy policy.
__device__ __forceinline__ void multi_row_state(int64_t row, int32_t m, int full, int64_t kb,
                                                const int32_t* order, int64_t& s, int32_t& a) {
  const int64_t p = row / m;
  a = (int32_t)(row - p * m);
  s = full ? kb + p : (int64_t)order[kb + p];
}

// sigma_t of a whole sweep, once per sweep: every product and commit launch
// of the sweep reads its states from this table instead of evaluating the
// Feistel network per row (40 Philox rounds of 32-bit multiplies each).
// A wavefront runs its cycle walk until its slowest lane is done, so only
// kMultiOrderLanes lanes of each take a position (the expected longest of 16
// walks is about 5 Feistel passes, of 64 about 7) and the positions spread
// over four times as many wavefronts.
constexpr int kMultiOrderLanes = 16;
__global__ void __launch_bounds__(256) multi_order_kernel(MultiArgs A, uint64_t t) {
  if (multi_done(A.ctl)) return;  // uniform over the launch
  if ((threadIdx.x & 63) >= kMultiOrderLanes) return;
  const OrderKey key = make_order_key(A.n, A.seed, t);
  const int64_t lane_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64 * kMultiOrderLanes +
                          (threadIdx.x & 63);
  const int64_t lanes = (int64_t)gridDim.x * (blockDim.x / 64) * kMultiOrderLanes;
  for (int64_t p = lane_id; p < A.n; p += lanes)
    A.order[p] = (int32_t)sweep_order_at((uint32_t)p, key);
}

// Partial products of one K-range: part[split][row][j] = sum over k in the
// range of code(row, k) * (hi + lo)(k, j).  A wavefront owns 16 RT rows and
// all NCT * 16 vectors; lane l feeds rows l % 16 of each row tile and vectors
// l % 16 of each column tile, 8 consecutive k from 8 (l / 16) (the same k map
// for both operands).  K runs in rounds: the rows come straight from
// HBM (every load of a round issued before its products), while the W terms
// of the round, shared by the workgroup's four wavefronts, are staged in LDS
// once per workgroup with whole-line loads (double buffered: the next
// round's W is fetched during this round's products).  Reading W per
// wavefront from L2 in 64-byte pieces cost more than the row stream itself.
// Rounds are 256 wide for 32 vectors, 128 for 16 and 64 above (measured:
// wider rounds were slower for 16 and 48 vectors; 64 needs the registers).
// A row load brings 64 bytes of each of 16 rows (the MFMA operand layout),
// so each 128-byte line is asked for by two loads of the same wavefront;
// plain loads, which L1 keeps, serve the second half from the first
// (non-temporal ones were 1-7% slower).
template <int RT, int NCT, int ROUND>  // ROUND: K per round (64, 128 or 256)
__global__ void __launch_bounds__(256) multi_gemm_kernel(MultiArgs A, uint64_t t, int64_t k,
                                                         int full) {
  constexpr int U = ROUND / 32;
  constexpr int PITCH = ROUND + 8;                     // staged W row, 16-byte pad
  constexpr int PPR = ROUND / 8;                       // 16-byte pieces per staged row
  constexpr int WROWS = 2 * NCT * 16;                  // staged W rows: 2 terms x r vectors
  constexpr int WPIECES = WROWS * PPR;                 // pieces per round
  constexpr int WPER = (WPIECES + 255) / 256;          // per thread
  __shared__ __attribute__((aligned(16))) uint16_t Wl[2][WROWS][PITCH];
  if (!full && multi_done(A.ctl)) return;  // uniform over the launch
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t kb = k * A.b;
  const int64_t rows = min(A.b, A.n - kb) * A.m;
  const int64_t wg0 = (int64_t)blockIdx.x * 4 * (16 * RT);
  if (wg0 >= rows) return;  // whole workgroup: no barrier is skipped by part of it
  const int64_t tile0 = wg0 + wave * (16 * RT);
  const int i = lane & 15, g = lane >> 4;
  const int64_t n = A.n;
  const MBDP_GLOBAL uint16_t* P = (const MBDP_GLOBAL uint16_t*)A.P;
  const MBDP_GLOBAL uint16_t* Ws = (const MBDP_GLOBAL uint16_t*)A.Ws;
  const MBDP_GLOBAL uint16_t* arow[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    int64_t row = tile0 + rt * 16 + i;
    row = row < rows ? row : rows - 1;  // ragged tile: a valid row, result dropped
    int64_t s;
    int32_t a;
    multi_row_state(row, A.m, full, kb, A.order, s, a);
    arow[rt] = P + ((size_t)s * A.m + a) * (size_t)n + 8 * g;
  }
  f32x4 acc[RT][NCT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[rt][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t k0 = (int64_t)blockIdx.y * A.kchunk;
  const int64_t k1 = min(n, k0 + A.kchunk);
  // staged W row w = h * r + j holds W term h of vector j; piece q of a round
  // is row q / PPR, values 8 (q % PPR) .. +7
  auto fetch_w = [&](int64_t kk, u32x4 (&wr)[WPER]) {
#pragma unroll
    for (int e = 0; e < WPER; ++e) {
      const int q = threadIdx.x + 256 * e;
      const int w = q / PPR, c8 = (q % PPR) * 8;
      if (q < WPIECES && kk + c8 < k1) {
        const int h = w / (NCT * 16), j = w - h * (NCT * 16);
        wr[e] = *(const MBDP_GLOBAL u32x4*)(Ws + ((size_t)h * A.r + j) * (size_t)n + kk + c8);
      } else {
        wr[e] = u32x4{0u, 0u, 0u, 0u};
      }
    }
  };
  auto store_w = [&](int buf, const u32x4 (&wr)[WPER]) {
#pragma unroll
    for (int e = 0; e < WPER; ++e) {
      const int q = threadIdx.x + 256 * e;
      if (q < WPIECES) *(u32x4*)&Wl[buf][q / PPR][(q % PPR) * 8] = wr[e];
    }
  };
  {
    u32x4 wr[WPER];
    fetch_w(k0, wr);
    store_w(0, wr);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t kk = k0; kk < k1; kk += ROUND, buf ^= 1) {
    const int steps = (int)min((int64_t)U, (k1 - kk) / 32);  // last round may be short
    u32x4 av[U][RT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        av[u][rt] = u < steps ? *(const MBDP_GLOBAL u32x4*)(arow[rt] + kk + 32 * u)
                              : u32x4{0u, 0u, 0u, 0u};
    const bool next = kk + ROUND < k1;
    u32x4 wr[WPER];
    if (next) fetch_w(kk + ROUND, wr);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u >= steps) break;
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const u32x4 bv = *(const u32x4*)&Wl[buf][h * NCT * 16 + c * 16 + i][32 * u + 8 * g];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, av[u][rt]), __builtin_bit_cast(bf16x8, bv), acc[rt][c],
                0, 0, 0);
        }
    }
    // the other buffer was last read in the previous round, before its barrier
    if (next) store_w(buf ^ 1, wr);
    __syncthreads();
  }
  if (tile0 >= rows) return;  // after the last barrier
  // lane l holds rows 4 (l / 16) + v of each 16-row tile, vector l % 16 of each column tile
  MBDP_GLOBAL float* part = (MBDP_GLOBAL float*)A.part + (size_t)blockIdx.y * A.part_rows * A.r;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = tile0 + rt * 16 + 4 * g + v;
      if (row < rows) {
#pragma unroll
        for (int c = 0; c < NCT; ++c) part[(size_t)row * A.r + c * 16 + i] = acc[rt][c][v];
      }
    }
}

// Commit of batch k (mode 0), or the greedy action of states kb .. kb + b - 1
// (mode 1): a workgroup per state.  Thread (al, j) serves vector j and the
// actions a = al, al + AL, ... (AL = 256 / r action lanes); the lanes' minima
// meet in LDS, lowest action on ties.
__global__ void __launch_bounds__(256) multi_commit_kernel(MultiArgs A, uint64_t t, int64_t k,
                                                           int mode) {
  __shared__ double qs[256];
  __shared__ int32_t as[256];
  const int64_t kb = k * A.b;
  const int64_t p = blockIdx.x;                // position in the launch (< min(b, n - kb))
  const int AL = 256 / A.r;
  const int al = threadIdx.x / A.r, j = threadIdx.x - al * A.r;
  // The stop flag is requested with the state (the table is read in either
  // mode, so neither load waits behind a branch) and tested only before the
  // first store; the state's old W and R are requested with its costs.
  const unsigned done = __hip_atomic_load(&A.ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t o = A.order[kb + p];
  const bool stop = mode == 0 && done != 0u;
  const int64_t s = mode ? kb + p : o;
  const size_t e = (size_t)s * A.r + j;
  const bool commit = mode == 0 && al == 0;
  const double w_old = commit ? A.W[e] : 0.0, r_old = commit ? A.R[e] : 0.0;
  double best = INFINITY;
  int32_t besta = 0;
  if (al < AL) {
    for (int32_t a = al; a < A.m; a += AL) {
      const int64_t lrow = p * A.m + a;      // row of the launch
      const int64_t grow = s * A.m + a;      // row of P
      double acc = 0.0;
#pragma unroll 4
      for (int sp = 0; sp < A.splits; ++sp)
        acc += (double)A.part[((size_t)sp * A.part_rows + lrow) * A.r + j];
      const double q = (double)A.C[(size_t)grow * A.r + j] +
                       A.gamma * ((double)A.rscale[grow] * acc + A.PR[(size_t)grow * A.r + j]);
      if (q < best) {  // ascending actions: strictly smaller keeps the lowest
        best = q;
        besta = a;
      }
    }
  }
  qs[threadIdx.x] = best;
  as[threadIdx.x] = besta;
  __syncthreads();
  if (stop) return;  // uniform over the launch; nothing was stored
  double dv = 0.0;
  if (al == 0) {
    for (int l = 1; l < AL; ++l) {
      const double q2 = qs[l * A.r + j];
      const int32_t a2 = as[l * A.r + j];
      if (q2 < best || (q2 == best && a2 < besta)) {
        best = q2;
        besta = a2;
      }
    }
    if (mode == 1) {
      A.policy[e] = besta;
    } else {
      const double wnew = best - r_old;
      dv = fabs(wnew - w_old);
      A.W[e] = wnew;
      const unsigned hi = multi_bf16_rne((float)wnew);
      const unsigned lo = multi_bf16_rne((float)(wnew - (double)__uint_as_float(hi << 16)));
      A.Ws[(size_t)j * A.n + s] = (uint16_t)hi;
      A.Ws[((size_t)A.r + j) * A.n + s] = (uint16_t)lo;
    }
  }
  if (mode == 0 && threadIdx.x < 64) {  // the r <= 64 threads with al == 0 are in wavefront 0
    dv = wave_max_d(dv);
    // one slot per position of the sweep (every sweep writes all n), reduced
    // by the end-of-sweep kernel: no contended atomic per workgroup
    if (threadIdx.x == 0) A.dvs[kb + p] = dv;
  }
}

// End of sweep t: its max |dV| (over the per-position maxima the commits
// wrote), the bound on max |W|, the stop flag.  One workgroup.
__global__ void __launch_bounds__(256) multi_end_kernel(MultiArgs A) {
  __shared__ double red[4];
  if (multi_done(A.ctl)) return;  // uniform over the workgroup
  double dv = 0.0;
#pragma unroll 8  // independent loads, so several are in flight
  for (int64_t e = threadIdx.x; e < A.n; e += blockDim.x) dv = fmax(dv, A.dvs[e]);
  dv = wave_max_d(dv);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dv;
  __syncthreads();
  if (threadIdx.x != 0) return;
  dv = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  MultiControl* c = A.ctl;
  c->dv_last = dv;
  c->w_bound += dv;
  c->sweeps += 1;
  if (A.tol >= 0.0 && dv <= A.tol)
    __hip_atomic_store(&c->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// mode 0: R = V, W = 0 (start); mode 1: R += W, W = 0 (re-centring);
// mode 2: V = R + W (result).  Clears the split copy of W in modes 0 and 1.
__global__ void __launch_bounds__(256) multi_anchor_kernel(MultiArgs A, double* V, int mode) {
  const int64_t total = A.n * A.r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (mode == 2) {
      V[e] = A.R[e] + A.W[e];
      continue;
    }
    A.R[e] = mode == 0 ? V[e] : A.R[e] + A.W[e];
    A.W[e] = 0.0;
    const int64_t s = e / A.r, j = e - s * A.r;
    A.Ws[(size_t)j * A.n + s] = 0;
    A.Ws[((size_t)A.r + j) * A.n + s] = 0;
  }
  if (mode != 2 && blockIdx.x == 0 && threadIdx.x == 0) A.ctl->w_bound = 0.0;
}

// PR[row][j] = scale(row) * sum_k code(row, k) R[k][j] in FP64: a workgroup
// per 64 rows x 64 vectors, K in chunks of 32 through LDS, a 4 x 4 block of
// outputs per thread.
__global__ void __launch_bounds__(256) multi_pr_kernel(MultiArgs A) {
  __shared__ double Pt[64][33];
  __shared__ double Rt[32][64];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const int64_t rows = A.n * A.m;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
  for (int64_t k0 = 0; k0 < A.n; k0 += 32) {
    {  // 64 rows x 32 codes: 8 per thread
      const int lr = tid >> 2, lk = (tid & 3) * 8;
      const int64_t row = min(row0 + lr, rows - 1);
      const u32x4 x = *(const u32x4*)(A.P + (size_t)row * A.n + k0 + lk);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        Pt[lr][lk + 2 * w] = (double)__uint_as_float(x[w] << 16);
        Pt[lr][lk + 2 * w + 1] = (double)__uint_as_float(x[w] & 0xFFFF0000u);
      }
    }
    for (int e = tid; e < 32 * 64; e += 256) {
      const int kk = e >> 6, j = e & 63;
      Rt[kk][j] = j < A.r ? A.R[(size_t)(k0 + kk) * A.r + j] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 32; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) a[x] = Pt[ty * 4 + x][kk];
#pragma unroll
      for (int x = 0; x < 4; ++x) b[x] = Rt[kk][tx * 4 + x];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int64_t row = row0 + ty * 4 + x;
    if (row >= rows) continue;
    const double sc = (double)A.rscale[row];
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int j = tx * 4 + y;
      if (j < A.r) A.PR[(size_t)row * A.r + j] = sc * acc[x][y];
    }
  }
}

// ------------------------------------------------------------------ launches

typedef void (*MultiGemmFn)(MultiArgs, uint64_t, int64_t, int);

static MultiGemmFn multi_gemm_fn(int32_t r) {
  switch (r) {
    case 16: return multi_gemm_kernel<1, 1, 128>;
    case 32: return multi_gemm_kernel<2, 2, 256>;
    case 48: return multi_gemm_kernel<3, 3, 64>;
    case 64: return multi_gemm_kernel<4, 4, 64>;
    default: return nullptr;
  }
}


int launch_multi_gemm(const MultiArgs& a, uint64_t t, int64_t k, int full, void* stream) {
  MultiGemmFn f = multi_gemm_fn(a.r);
  if (!f) return -1;
  const int64_t rows = std::min<int64_t>(a.b, a.n - k * a.b) * a.m;
  const int64_t per_block = 4 * (int64_t)multi_rows_per_wave(a.r);  // 4 wavefronts
  const int64_t bx = (rows + per_block - 1) / per_block;
  const int64_t by = (a.n + a.kchunk - 1) / a.kchunk;
  hipLaunchKernelGGL(f, dim3((unsigned)bx, (unsigned)by), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a, t, k, full);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_multi_commit(const MultiArgs& a, uint64_t t, int64_t k, int mode, void* stream) {
  const int64_t blocks = std::min<int64_t>(a.b, a.n - k * a.b);  // a workgroup per state
  hipLaunchKernelGGL(multi_commit_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a, t, k, mode);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_multi_end(const MultiArgs& a, void* stream) {
  hipLaunchKernelGGL(multi_end_kernel, dim3(1), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_multi_order(const MultiArgs& a, uint64_t t, void* stream) {
  const int64_t per_block = 4 * kMultiOrderLanes;  // positions per 256-thread workgroup and pass
  int64_t blocks = (a.n + per_block - 1) / per_block;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(multi_order_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a, t);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_multi_anchor(const MultiArgs& a, double* V, int mode, void* stream) {
  int64_t blocks = (a.n * a.r + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(multi_anchor_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a, V, mode);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_multi_pr(const MultiArgs& a, void* stream) {
  const int64_t blocks = (a.n * a.m + 63) / 64;
  hipLaunchKernelGGL(multi_pr_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mbdp
