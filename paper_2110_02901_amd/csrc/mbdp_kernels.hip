// Launchers and small kernels of libmbdp (FP32 transition data); the
// engines and the persistent solve kernel are in mbdp_engines.h.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>

#include "mbdp_engines.h"

namespace mbdp {

// ------------------------------------------------------------ small kernels

__global__ void zero_kernel(unsigned int* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void permutation_kernel(int64_t n, uint64_t seed, uint64_t t, int32_t* out) {
  const OrderKey key = make_order_key(n, seed, t);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)sweep_order_at((uint32_t)i, key);
}

// flags[0]: rows whose length differs from k; flags[1]: decreasing row_ptr
// entries or entries outside [0, nnz]; flags[2]: row_ptr[0] != 0 or
// row_ptr[rows] != nnz; flags[3]: columns outside [0, n); flags[4]: with k
// rows of length k, max |s' - s| over the entries s' of the rows of state s.
__global__ void csr_inspect_kernel(const int64_t* row_ptr, const int32_t* col, int64_t rows,
                                   int64_t n, int64_t nnz, int64_t k, unsigned long long* flags) {
  unsigned long long not_k = 0, bad_ptr = 0, bad_col = 0, band = 0;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = tid; r < rows; r += nth) {
    const int64_t a = row_ptr[r], b = row_ptr[r + 1];
    not_k += (b - a) != k;
    bad_ptr += (b < a) || a < 0 || b > nnz;
  }
  const int64_t per_state = k > 0 ? k * (rows / n) : 0;  // entries of one state's rows
  for (int64_t e = tid; e < nnz; e += nth) {
    const int32_t c = col[e];
    bad_col += c < 0 || (int64_t)c >= n;
    if (per_state > 0) {
      const int64_t d = (int64_t)c - e / per_state;
      const unsigned long long ad = (unsigned long long)(d < 0 ? -d : d);
      band = ad > band ? ad : band;
    }
  }
  if (not_k) atomicAdd(&flags[0], not_k);
  if (bad_ptr) atomicAdd(&flags[1], bad_ptr);
  if (bad_col) atomicAdd(&flags[3], bad_col);
  if (band) atomicMax(&flags[4], band);
  if (tid == 0)
    if (row_ptr[0] != 0 || row_ptr[rows] != nnz) atomicAdd(&flags[2], 1ull);
}

// Transition value i (dense index or CSR entry) as stored, decoded, before the
// row scale.
__device__ __forceinline__ float stored_value(const KParams& p, size_t i) {
  if (p.vdtype == kBF16) return ValBF16::dense_at(p, i);
  if (p.vdtype == kFP8) return ValFP8::dense_at(p, i);
  return p.storage == kDense ? p.P[i] : p.val[i];
}

__device__ __forceinline__ double stored_scale(const KParams& p, int64_t row) {
  return p.vdtype == kF32 ? 1.0 : (double)p.rscale[row];
}

// out: [0] bad probability, [1] bad row sum, [2] empty rows, [3] bad column,
// [4] bad row_ptr, [5] bad cost, [6] no admissible action, [7] max |rowsum-1|
// (double bits).
__global__ void validate_kernel(KParams p, double tol, unsigned long long* out) {
  const int64_t rows = p.n * p.m;
  unsigned long long bad_p = 0, bad_sum = 0, empty = 0, bad_col = 0, bad_ptr = 0;
  double dev = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    if (p.storage == kDense) {
      const size_t base = (size_t)r * (size_t)p.n;
      for (int64_t j = 0; j < p.n; ++j) {
        const float x = stored_value(p, base + (size_t)j);
        if (!(x >= 0.f) || isinf(x)) ++bad_p;
        s += (double)x;
      }
    } else {
      const int64_t e0 = p.row_ptr[r], e1 = p.row_ptr[r + 1];
      if (e1 < e0) ++bad_ptr;
      if (e1 <= e0) ++empty;
      for (int64_t e = e0; e < e1; ++e) {
        const float x = stored_value(p, (size_t)e);
        if (!(x >= 0.f) || isinf(x)) ++bad_p;
        const int32_t cidx = p.col[e];
        if (cidx < 0 || (int64_t)cidx >= p.n) ++bad_col;
        s += (double)x;
      }
    }
    s *= stored_scale(p, r);
    const double d = fabs(s - 1.0);
    if (!(d <= tol)) ++bad_sum;
    if (d > dev || isnan(d)) dev = isnan(d) ? INFINITY : d;
  }
  unsigned long long bad_cost = 0, no_adm = 0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < p.n;
       s += (int64_t)gridDim.x * blockDim.x) {
    int finite = 0;
    for (int a = 0; a < p.m; ++a) {
      const float x = p.c32[s * p.m + a];
      if (isnan(x) || (isinf(x) && x < 0.f)) ++bad_cost;
      if (isfinite(x)) finite = 1;
    }
    if (!finite) ++no_adm;
  }
  if (bad_p) atomicAdd(&out[0], bad_p);
  if (bad_sum) atomicAdd(&out[1], bad_sum);
  if (empty) atomicAdd(&out[2], empty);
  if (bad_col) atomicAdd(&out[3], bad_col);
  if (bad_ptr) atomicAdd(&out[4], bad_ptr);
  if (bad_cost) atomicAdd(&out[5], bad_cost);
  if (no_adm) atomicAdd(&out[6], no_adm);
  if (dev > 0.0) atomicMax(&out[7], (unsigned long long)__double_as_longlong(dev));
}

// ------------------------------------------------------------ row quantiser
//
// BF16: round to nearest even of the FP32 bits.  FP8 E4M3 (OCP E4M3FN: bias
// 7, subnormals m * 2^-9, largest finite 448, NaN S.1111.111, no infinity):
// nearest value, ties to the even code, saturating at 448.  Each FP8 row is
// first multiplied by the power of two 2^(7 - E), E the binary exponent of
// its largest magnitude (clamped to [-100, 127]), so the scaling is exact and
// the largest entry lands in [128, 256).  The row scale makes the stored row
// sum to 1: scale = 1 / sum_j decode(q_j), summed in FP64.

__device__ __forceinline__ unsigned encode_bf16(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return ((u >> 16) | 0x40u) & 0xFFFFu;
  return ((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16) & 0xFFFFu;
}

__device__ __forceinline__ unsigned encode_e4m3(float x) {
  const unsigned u = __float_as_uint(x);
  const unsigned sign = (u >> 24) & 0x80u;
  const unsigned a = u & 0x7FFFFFFFu;
  if (a > 0x7F800000u) return 0x7Fu | sign;
  const int e = (int)(a >> 23) - 127;
  unsigned code;
  if (e >= -6) {
    const unsigned keep = ((unsigned)(e + 7) << 3) | ((a >> 20) & 7u);
    const unsigned rest = a & 0xFFFFFu;
    const bool up = rest > 0x80000u || (rest == 0x80000u && (keep & 1u));
    code = keep + (up ? 1u : 0u);
  } else {
    code = (unsigned)__builtin_rintf(__builtin_fabsf(x) * 512.0f);  // multiples of 2^-9
  }
  return (code < 0x7Eu ? code : 0x7Eu) | sign;
}

__global__ void quantize_kernel(const float* src, int64_t rows, int64_t len, int32_t dtype,
                                void* dst, float* scale) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t r = gw; r < rows; r += nw) {
    const float* row = src + r * len;
    float alpha = 1.f;
    if (dtype == kFP8) {
      float amax = 0.f;
      for (int64_t j = lane; j < len; j += kWave) amax = fmaxf(amax, fabsf(row[j]));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
      int e = (int)((__float_as_uint(amax) >> 23) & 0xFFu) - 127;
      e = e < -100 ? -100 : (e > 127 ? 127 : e);
      if (amax > 0.f) alpha = __uint_as_float((unsigned)(127 + 7 - e) << 23);
    }
    double sum = 0.0;
    for (int64_t j = lane; j < len; j += kWave) {
      const float x = row[j] * alpha;
      if (dtype == kBF16) {
        const unsigned q = encode_bf16(x);
        static_cast<uint16_t*>(dst)[r * len + j] = (uint16_t)q;
        sum += (double)__uint_as_float(q << 16);
      } else {
        const unsigned q = encode_e4m3(x);
        static_cast<uint8_t*>(dst)[r * len + j] = (uint8_t)q;
        sum += (double)fp8x4(q).x;
      }
    }
    sum = wave_sum_d(sum);
    if (lane == 0) scale[r] = sum > 0.0 ? (float)(1.0 / sum) : 0.f;
  }
}

// ------------------------------------------------------------ adjoint
//
// The adjoint equation (I - gamma P_mu)^T lambda = g of L = g^T J* is a
// policy evaluation on the transposed policy rows: lambda = g + gamma
// P_mu^T lambda.  These kernels build P_mu^T in CSR form from the ELL rows
// (s, mu(s)): in-degree counts, an exclusive scan, a scatter, and a sort of
// each transposed row by source state so the result does not depend on the
// order of the scatter's atomics.  flags[0] counts policy entries outside
// [0, m).

__device__ __forceinline__ int policy_action(const KParams& p, const int32_t* policy, int64_t s,
                                             unsigned* flags) {
  int a = policy[s];
  if (a < 0 || a >= p.m) {
    atomicAdd(&flags[0], 1u);
    a = 0;
  }
  return a;
}

__global__ void adj_count_kernel(KParams p, const int32_t* policy, unsigned* cnt,
                                 unsigned* flags) {
  const int64_t k = p.ell_k;
  const int64_t total = p.n * k;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / k;
    const int a = policy_action(p, policy, s, flags);
    atomicAdd(&cnt[p.col[(s * p.m + a) * k + i % k]], 1u);
  }
}

// row_ptr[0..n] <- exclusive prefix sums of cnt[0..n) (one workgroup).
__global__ void adj_scan_kernel(const unsigned* cnt, int64_t n, int64_t* row_ptr) {
  __shared__ int64_t part[1024];
  const int64_t nt = blockDim.x, per = (n + nt - 1) / nt;
  const int64_t i0 = min(n, (int64_t)threadIdx.x * per), i1 = min(n, i0 + per);
  int64_t sum = 0;
  for (int64_t i = i0; i < i1; ++i) sum += cnt[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t v = part[t];
      part[t] = run;
      run += v;
    }
    row_ptr[n] = run;
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int64_t i = i0; i < i1; ++i) {
    row_ptr[i] = run;
    run += cnt[i];
  }
}

__global__ void adj_fill_kernel(KParams p, const int32_t* policy, const int64_t* row_ptr,
                                unsigned* cursor, int32_t* col_t, float* val_t, unsigned* flags) {
  const int64_t k = p.ell_k;
  const int64_t total = p.n * k;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / k;
    const int a = policy_action(p, policy, s, flags);
    const int64_t e = (s * p.m + a) * k + i % k;
    const int32_t j = p.col[e];
    const int64_t pos = row_ptr[j] + atomicAdd(&cursor[j], 1u);
    col_t[pos] = (int32_t)s;
    val_t[pos] = p.val[e];
  }
}

// Each transposed row in increasing source state (insertion sort; rows hold
// a few dozen entries).
__global__ void adj_sort_kernel(const int64_t* row_ptr, int64_t n, int32_t* col_t, float* val_t) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e0 = row_ptr[j], e1 = row_ptr[j + 1];
    for (int64_t e = e0 + 1; e < e1; ++e) {
      const int32_t c = col_t[e];
      const float v = val_t[e];
      int64_t f = e - 1;
      while (f >= e0 && col_t[f] > c) {
        col_t[f + 1] = col_t[f];
        val_t[f + 1] = val_t[f];
        --f;
      }
      col_t[f + 1] = c;
      val_t[f + 1] = v;
    }
  }
}

// grad_c[s*m+a] = lambda(s) [a == mu(s)]; grad_val[e] = gamma lambda(s) V(col[e])
// on the entries of row (s, mu(s)), 0 on the other rows.
__global__ void adj_grad_kernel(KParams p, const int32_t* policy, const double* lambda,
                                const double* V, double* grad_c, double* grad_val,
                                unsigned* flags) {
  const int64_t k = p.ell_k, m = p.m;
  const int64_t rows = p.n * m;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = r / m;
    const bool on = (r % m) == policy_action(p, policy, s, flags);
    const double ls = lambda[s];
    if (grad_c) grad_c[r] = on ? ls : 0.0;
    if (grad_val)
      for (int64_t e = r * k; e < (r + 1) * k; ++e)
        grad_val[e] = on ? p.gamma * ls * V[p.col[e]] : 0.0;
  }
}

// ------------------------------------------------------------ launchers

// Result words of the CSR structure inspection done by mdp_create_csr (the
// only device memory the library owns; callers serialise its use).
__device__ unsigned long long g_inspect_flags[8];

int inspect_flags_ptr(void** out) {
  return (int)hipGetSymbolAddress(out, HIP_SYMBOL(g_inspect_flags));
}


// Picks the kernel instantiation for the launch.
static SolveFn pick(const KParams& p, int units_per_wave_hint) {
  if (p.storage == kDense) {
    const bool vec = p.n % 4 == 0;
    const int m = p.m;
    if (vec) {
      if (m >= 16) return solve_fn<DenseEngine<16, 4>>(p.task);
      if (m >= 8) return solve_fn<DenseEngine<8, 4>>(p.task);
      if (m >= 4) return solve_fn<DenseEngine<4, 4>>(p.task);
      if (m >= 2) return solve_fn<DenseEngine<2, 4>>(p.task);
      return solve_fn<DenseEngine<1, 4>>(p.task);
    }
    if (m >= 16) return solve_fn<DenseEngine<16, 1>>(p.task);
    if (m >= 8) return solve_fn<DenseEngine<8, 1>>(p.task);
    if (m >= 4) return solve_fn<DenseEngine<4, 1>>(p.task);
    if (m >= 2) return solve_fn<DenseEngine<2, 1>>(p.task);
    return solve_fn<DenseEngine<1, 1>>(p.task);
  }
  if (p.storage == kEll) {
    // two states per wavefront iteration keep the pipelined loop within 128 VGPRs
    int lpr = 1;
    while (lpr * 4 < p.ell_k) lpr <<= 1;
    const bool two = units_per_wave_hint >= 2;
    switch (lpr) {
      case 1: return two ? solve_fn<EllEngine<2, 1>>(p.task) : solve_fn<EllEngine<1, 1>>(p.task);
      case 2: return two ? solve_fn<EllEngine<2, 2>>(p.task) : solve_fn<EllEngine<1, 2>>(p.task);
      case 4: return two ? solve_fn<EllEngine<2, 4>>(p.task) : solve_fn<EllEngine<1, 4>>(p.task);
      case 8: return two ? solve_fn<EllEngine<2, 8>>(p.task) : solve_fn<EllEngine<1, 8>>(p.task);
      case 16: return two ? solve_fn<EllEngine<2, 16>>(p.task) : solve_fn<EllEngine<1, 16>>(p.task);
      case 32: return two ? solve_fn<EllEngine<2, 32>>(p.task) : solve_fn<EllEngine<1, 32>>(p.task);
      default: return two ? solve_fn<EllEngine<2, 64>>(p.task) : solve_fn<EllEngine<1, 64>>(p.task);
    }
  }
  return solve_fn<CsrEngine>(p.task);
}

// The band-local instantiation for ELL rows of LPR <= 16 lanes, or null.
static SolveFn pick_band(const KParams& p, int units_per_wave_hint) {
  int lpr = 1;
  while (lpr * 4 < p.ell_k) lpr <<= 1;
  const bool two = units_per_wave_hint >= 2;
  switch (lpr) {
    case 1: return two ? solve_fn<BandEngine<2, 1>>(p.task) : solve_fn<BandEngine<1, 1>>(p.task);
    case 2: return two ? solve_fn<BandEngine<2, 2>>(p.task) : solve_fn<BandEngine<1, 2>>(p.task);
    case 4: return two ? solve_fn<BandEngine<2, 4>>(p.task) : solve_fn<BandEngine<1, 4>>(p.task);
    case 8: return two ? solve_fn<BandEngine<2, 8>>(p.task) : solve_fn<BandEngine<1, 8>>(p.task);
    case 16: return two ? solve_fn<BandEngine<2, 16>>(p.task) : solve_fn<BandEngine<1, 16>>(p.task);
    default: return nullptr;
  }
}

// The column-block instantiation (b = n with an attached layout), or null.
static SolveFn pick_col(const KParams& p, int units_per_wave_hint) {
  int lpr = 1;
  while (lpr * 4 < p.ell_k) lpr <<= 1;
  const bool two = units_per_wave_hint >= 2;
  switch (lpr) {
    case 1: return two ? solve_fn<ColEngine<2, 1>>(p.task) : solve_fn<ColEngine<1, 1>>(p.task);
    case 2: return two ? solve_fn<ColEngine<2, 2>>(p.task) : solve_fn<ColEngine<1, 2>>(p.task);
    case 4: return two ? solve_fn<ColEngine<2, 4>>(p.task) : solve_fn<ColEngine<1, 4>>(p.task);
    case 8: return two ? solve_fn<ColEngine<2, 8>>(p.task) : solve_fn<ColEngine<1, 8>>(p.task);
    case 16: return two ? solve_fn<ColEngine<2, 16>>(p.task) : solve_fn<ColEngine<1, 16>>(p.task);
    default: return nullptr;
  }
}

// Whether the band-local engine's LDS holds a chunk, its window and the
// batch offsets for a grid of `blocks` workgroups.
static bool band_fits(const KParams& p, int blocks) {
  if (p.storage != kEll || p.band < 0 || p.perm || blocks < 1) return false;
  const int64_t D = (p.n + blocks - 1) / blocks;
  const int64_t nb = (p.n + p.b - 1) / p.b;
  return D <= kChunkCap && D + 2 * (int64_t)p.band <= kWinCap && nb <= kBatchCap;
}

static int grid_blocks(SolveFn f, const LaunchShape& shape, int* blocks, char* err,
                       size_t errlen) {
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &occ, reinterpret_cast<const void*>(f), shape.threads, 0);
  if (e != hipSuccess || occ < 1) {
    snprintf(err, errlen, "occupancy query failed (%d blocks/CU): %s", occ, hipGetErrorString(e));
    return -1;
  }
  const int bpc = shape.blocks_per_cu < occ ? shape.blocks_per_cu : occ;
  *blocks = shape.cus * bpc;
  if (*blocks > kMaxBlocks) *blocks = kMaxBlocks;
  return 0;
}

// The instantiation a launch runs and its grid.
static int choose(const KParams& p, LaunchShape& shape, SolveFn* fn, int* blocks,
                  int* engine, char* err, size_t errlen) {
  // a banded MDP keeps the band-local engine (its V window in LDS beats the
  // column blocks); otherwise, at b = n with column blocks attached, those
  bool band_ok = false;
  if (p.storage == kEll && p.band >= 0 && !p.perm && p.vdtype == kF32) {
    SolveFn fb = pick_band(p, 1);
    int bb = 0;
    if (fb && grid_blocks(fb, shape, &bb, err, errlen) == 0) band_ok = band_fits(p, bb);
  }
  if (!band_ok && p.storage == kEll && p.cb_keys && p.b == p.n && p.vdtype == kF32) {
    LaunchShape cs = shape;
    cs.threads = kColThreads;
    const int64_t waves = (int64_t)cs.cus * cs.blocks_per_cu * (kColThreads / kWave);
    const int64_t per_wave = waves > 0 ? p.b / waves : 1;
    SolveFn fc = pick_col(p, (int)(per_wave > 4 ? 4 : per_wave));
    if (fc) {
      shape = cs;
      *fn = fc;
      *engine = kEngineCol;
      return grid_blocks(fc, shape, blocks, err, errlen);
    }
  }
  const int waves_per_block = shape.threads / kWave;
  // ELL: states per wavefront iteration from the batch size and a full grid
  const int64_t waves_guess = (int64_t)shape.cus * shape.blocks_per_cu * waves_per_block;
  const int64_t per_wave = waves_guess > 0 ? p.b / waves_guess : 1;
  const int hint = (int)(per_wave > 4 ? 4 : per_wave);
  const bool lp = p.vdtype != kF32;
  if (p.storage == kEll && p.band >= 0 && !p.perm) {
    SolveFn fb = lp ? pick_band_lp(p, hint) : pick_band(p, hint);
    if (fb) {
      if (grid_blocks(fb, shape, blocks, err, errlen) != 0) return -1;
      if (band_fits(p, *blocks)) {
        *fn = fb;
        *engine = kEngineBand;
        return 0;
      }
    }
  }
  if (lp)
    *fn = p.storage == kDense ? pick_dense_lp(p)
                              : (p.storage == kEll ? pick_ell_lp(p, hint) : nullptr);
  else
    *fn = pick(p, hint);
  if (!*fn) {
    snprintf(err, errlen, "no kernel for this storage and value type");
    return -1;
  }
  *engine = p.storage == kDense ? kEngineDense : p.storage == kEll ? kEngineEll : kEngineCsr;
  return grid_blocks(*fn, shape, blocks, err, errlen);
}

int query_engine(const KParams& p, LaunchShape shape, int* engine, char* err, size_t errlen) {
  SolveFn f = nullptr;
  int blocks = 0;
  return choose(p, shape, &f, &blocks, engine, err, errlen);
}

int launch_solve(KParams p, LaunchShape shape, void* stream, char* err, size_t errlen) {
  SolveFn f = nullptr;
  int blocks = 0, engine = 0;
  if (choose(p, shape, &f, &blocks, &engine, err, errlen) != 0) return -1;
  // dense: split the columns of a state over several workgroups when the
  // batch has fewer states than there are workgroups
  p.splits = 1;
  if (p.storage == kDense && p.b < blocks) p.splits = (int)((blocks + p.b - 1) / p.b);
  void* args[] = {&p};
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(f), dim3(blocks),
                                 dim3(shape.threads), args, 0,
                                 reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    snprintf(err, errlen, "cooperative launch (%d x %d) failed: %s", blocks, shape.threads,
             hipGetErrorString(e));
    return -1;
  }
  return 0;
}

int launch_zero(void* ptr, size_t bytes, void* stream) {
  const size_t words = bytes / 4;
  int blocks = (int)((words + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), static_cast<unsigned int*>(ptr), words);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_permutation(int64_t n, uint64_t seed, uint64_t t, int32_t* out, void* stream) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(permutation_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), n, seed, t, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_csr_inspect(const int64_t* row_ptr, const int32_t* col, int64_t rows, int64_t n,
                       int64_t nnz, int64_t k, unsigned long long* flags, void* stream) {
  int64_t work = rows > nnz ? rows : nnz;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(csr_inspect_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), row_ptr, col, rows, n, nnz, k, flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_quantize(const float* src, int64_t rows, int64_t row_len, int32_t dtype, void* dst,
                    float* row_scale, void* stream) {
  int64_t blocks = (rows + 3) / 4;  // four rows (waves) per 256-thread block
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), src, rows, row_len, dtype, dst,
                     row_scale);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

static unsigned grid_for(int64_t work) {
  int64_t blocks = (work + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

int launch_policy_transpose(const KParams& p, const int32_t* policy, int64_t* row_ptr_t,
                            int32_t* col_t, float* val_t, unsigned* scratch, void* stream) {
  // scratch: flags[1] (padded to 64 words), counts[n], cursors[n]; zeroed by the caller
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned* flags = scratch;
  unsigned* cnt = scratch + 64;
  unsigned* cursor = cnt + p.n;
  const int64_t total = p.n * p.ell_k;
  hipLaunchKernelGGL(adj_count_kernel, dim3(grid_for(total)), dim3(256), 0, st, p, policy, cnt,
                     flags);
  hipLaunchKernelGGL(adj_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, p.n, row_ptr_t);
  hipLaunchKernelGGL(adj_fill_kernel, dim3(grid_for(total)), dim3(256), 0, st, p, policy,
                     row_ptr_t, cursor, col_t, val_t, flags);
  hipLaunchKernelGGL(adj_sort_kernel, dim3(grid_for(p.n)), dim3(256), 0, st, row_ptr_t, p.n,
                     col_t, val_t);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_value_gradients(const KParams& p, const int32_t* policy, const double* lambda,
                           const double* V, double* grad_c, double* grad_val, unsigned* flags,
                           void* stream) {
  hipLaunchKernelGGL(adj_grad_kernel, dim3(grid_for(p.n * p.m)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), p, policy, lambda, V, grad_c,
                     grad_val, flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_validate(const KParams& p, double tol, unsigned long long* out, void* stream) {
  int64_t rows = p.n * p.m;
  int64_t blocks = (rows + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), p, tol, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mbdp
