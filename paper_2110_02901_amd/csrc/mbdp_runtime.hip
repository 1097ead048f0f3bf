// Host runtime of libmbdp: the C-ABI declared in include/mbdp.h.
//
// Every entry point checks its arguments before any device work, maps HIP
// failures to MBDP_ERR_HIP with a message, and never throws.  The library
// allocates no device memory: scratch space is the caller's workspace, and
// the one tiny result buffer of mdp_create_csr is a file-scope device array.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "mbdp.h"
#include "mbdp_internal.h"

using namespace mbdp;

struct mbdp_mdp {
  int32_t storage;
  int32_t m;
  int64_t n;
  double gamma;
  const float* P;
  const int64_t* row_ptr;
  const int32_t* col;
  const float* val;
  int64_t nnz;
  int32_t ell_k;
  int32_t band;  // kEll: max |s' - s| over the entries of the rows of state s
  int32_t vdtype;        // kF32, kBF16, kFP8
  const void* pq;        // BF16 / FP8 values (P or val)
  const float* rscale;   // BF16 / FP8 per-row scales
  const float* c;
  int device;
  int cus;
  unsigned long long wall_khz;
  mbdp_tuning tuning;
  // column-sorted blocks (constant row length, FP32, b = n): the host layout
  // of mdp_column_blocks_prepare until mdp_column_blocks_attach copies it
  // into the caller's buffer
  std::vector<uint32_t> cb_keys_h;
  std::vector<float> cb_vals_h;
  std::vector<int32_t> cb_gptr_h;
  int64_t cb_states = 0;
  const uint32_t* cb_keys = nullptr;
  const float* cb_vals = nullptr;
  const int32_t* cb_gptr = nullptr;
};

namespace {

thread_local std::string g_err;

mbdp_status fail(mbdp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define MBDP_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(MBDP_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int64_t kMaxStates = (int64_t)1 << 31;  // state indices are int32
constexpr int32_t kMaxDenseActions = 1024;        // LDS holds one Q per action
constexpr double kBarrierTimeoutSeconds = 30.0;
// A team member waits for the others' batch: seconds at most for these sizes.
constexpr double kBatchTeamTimeoutSeconds = 60.0;

bool gamma_ok(double g) { return isfinite(g) && g > 0.0 && g < 1.0; }

mbdp_status query_device(mbdp_mdp* h) {
  MBDP_HIP(hipGetDevice(&h->device));
  int cus = 0, khz = 0, coop = 0;
  MBDP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
  MBDP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device));
  MBDP_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, h->device));
  if (!coop) return fail(MBDP_ERR_UNSUPPORTED, "device %d has no cooperative launch", h->device);
  if (cus < 1) return fail(MBDP_ERR_HIP, "device reports %d compute units", cus);
  h->cus = cus;
  h->wall_khz = khz > 0 ? (unsigned long long)khz : 100000ull;
  return MBDP_OK;
}

int64_t max_units(const mbdp_mdp* h) { return h->n + (int64_t)h->cus * kMaxBlocksPerCu; }

WsLayout layout(const mbdp_mdp* h) { return ws_layout(h->storage, h->n, h->m, max_units(h)); }

mbdp_status check_ws(const mbdp_mdp* h, void* ws, size_t bytes) {
  const WsLayout w = layout(h);
  if (!ws) return fail(MBDP_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", w.total);
  if (((uintptr_t)ws) % 256) return fail(MBDP_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (bytes < w.total)
    return fail(MBDP_ERR_WORKSPACE, "workspace has %zu bytes, need %zu", bytes, w.total);
  return MBDP_OK;
}

LaunchShape shape_of(const mbdp_mdp* h) {
  LaunchShape s;
  s.cus = h->cus;
  // One 1024-thread workgroup per CU: the grid barrier's cost grows with
  // the number of workgroups, and 16 waves per CU keep enough loads in flight.
  s.threads = 1024;
  s.blocks_per_cu = 1;
  if (h->tuning.threads_per_block == 256 || h->tuning.threads_per_block == 512 ||
      h->tuning.threads_per_block == 1024)
    s.threads = h->tuning.threads_per_block;
  if (h->tuning.blocks_per_cu > 0)
    s.blocks_per_cu =
        h->tuning.blocks_per_cu < kMaxBlocksPerCu ? h->tuning.blocks_per_cu : kMaxBlocksPerCu;
  return s;
}

// Minimum sweeps between re-centrings (0: no FP64 anchor).
int recentre_interval(const mbdp_mdp* h) {
  if (h->tuning.recentre_every < 0) return 0;
  return h->tuning.recentre_every > 0 ? h->tuning.recentre_every : 8;
}

KParams base_params(const mbdp_mdp* h, void* ws, float* V, int64_t b) {
  const WsLayout w = layout(h);
  char* base = static_cast<char*>(ws);
  KParams p{};
  p.storage = h->storage;
  p.m = h->m;
  p.n = h->n;
  p.gamma = h->gamma;
  p.P = h->P;
  p.row_ptr = h->row_ptr;
  p.col = h->col;
  p.val = h->val;
  p.ell_k = h->ell_k;
  p.band = (h->storage == kEll && h->tuning.band_window >= 0) ? h->band : -1;
  p.vdtype = h->vdtype;
  p.pq = h->pq;
  p.rscale = h->rscale;
  p.c32 = h->c;
  p.vbuf0 = V;
  p.vbuf1 = reinterpret_cast<float*>(base + w.vbuf1);
  p.b = b;
  p.ctl = reinterpret_cast<Control*>(base + w.ctl);
  p.order = reinterpret_cast<int32_t*>(base + w.order);
  p.first_mark = reinterpret_cast<uint32_t*>(base + w.first_mark);
  p.partial = reinterpret_cast<float*>(base + w.partial);
  p.unit_count = reinterpret_cast<unsigned int*>(base + w.unit_count);
  p.timeout_ticks = (unsigned long long)(kBarrierTimeoutSeconds * 1000.0 * (double)h->wall_khz);
  p.tol_dv = -1.0;
  p.splits = 1;
  p.cb_keys = h->cb_keys;
  p.cb_vals = h->cb_vals;
  p.cb_gptr = h->cb_gptr;
  p.cb_states = h->cb_states;
  return p;
}

mbdp_status launch(const mbdp_mdp* h, const KParams& p, void* ws, hipStream_t stream) {
  const WsLayout w = layout(h);
  if (launch_zero(ws, w.zero_bytes, stream) != 0)
    return fail(MBDP_ERR_HIP, "workspace clear failed: %s", hipGetErrorString(hipGetLastError()));
  char err[256] = {0};
  if (launch_solve(p, shape_of(h), stream, err, sizeof err) != 0)
    return fail(MBDP_ERR_HIP, "%s", err);
  return MBDP_OK;
}

const char* device_error_text(unsigned code) {
  switch (code) {
    case kDevBadPerm: return "explicit order has an entry outside [0, n)";
    case kDevBarrierTimeout: return "grid barrier timed out";
    case kDevBadPolicy: return "policy has an entry outside [0, m)";
    default: return "unknown device error";
  }
}

// Synchronises and copies the control block back; maps device errors.
mbdp_status finish(void* ws, hipStream_t stream, Control* out) {
  MBDP_HIP(hipMemcpyAsync(out, ws, sizeof(Control), hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  if (out->error)
    return fail(MBDP_ERR_DEVICE, "device error %u: %s", out->error, device_error_text(out->error));
  return MBDP_OK;
}

void fill_stats(const Control& c, bool with_ref, mbdp_stats* st) {
  if (!st) return;
  st->sweeps = c.sweeps;
  st->outer_iters = c.outer_iters;
  st->policy_changes_last = c.policy_changes_last;
  st->recentrings = c.recentrings;
  st->final_dv_inf = c.final_dv_inf;
  st->final_err_ref = with_ref ? c.final_err_ref : NAN;
  st->converged = c.converged;
  st->reserved = 0;
}

std::mutex g_inspect_mutex;

}  // namespace

namespace mbdp {
int inspect_flags_ptr(void** out);  // mbdp_kernels.hip
}

extern "C" {

const char* mbdp_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

int values_per_load(int32_t dtype) { return dtype == kBF16 ? 8 : 16; }

bool dtype_ok(int32_t dtype) { return dtype == MBDP_BF16 || dtype == MBDP_FP8_E4M3; }

mbdp_status create_dense(int64_t n, int32_t m, const float* P, const void* Pq, int32_t dtype,
                         const float* row_scale, const float* c, double gamma, mbdp_mdp_t* out) {
  if (!out) return fail(MBDP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || n >= kMaxStates) return fail(MBDP_ERR_INVALID_ARG, "n = %lld not in [1, 2^31)", (long long)n);
  if (m < 1) return fail(MBDP_ERR_INVALID_ARG, "m = %d < 1", m);
  if (m > kMaxDenseActions)
    return fail(MBDP_ERR_UNSUPPORTED, "dense storage supports m <= %d (got %d)", kMaxDenseActions, m);
  if (dtype == kF32 ? !P : (!Pq || !row_scale)) return fail(MBDP_ERR_INVALID_ARG, "P or row_scale is NULL");
  if (!c) return fail(MBDP_ERR_INVALID_ARG, "c is NULL");
  if (!gamma_ok(gamma)) return fail(MBDP_ERR_INVALID_ARG, "gamma = %g not in (0, 1)", gamma);
  if (dtype != kF32 && n % values_per_load(dtype) != 0)
    return fail(MBDP_ERR_UNSUPPORTED, "%s dense rows need n %% %d == 0 (got n = %lld)",
                dtype == kBF16 ? "BF16" : "FP8", values_per_load(dtype), (long long)n);
  mbdp_mdp* h = new (std::nothrow) mbdp_mdp();
  if (!h) return fail(MBDP_ERR_HIP, "out of host memory");
  h->storage = kDense;
  h->n = n;
  h->m = m;
  h->gamma = gamma;
  h->P = P;
  h->vdtype = dtype;
  h->pq = Pq;
  h->rscale = row_scale;
  h->c = c;
  const mbdp_status st = query_device(h);
  if (st != MBDP_OK) {
    delete h;
    return st;
  }
  *out = h;
  return MBDP_OK;
}

mbdp_status create_csr(int64_t n, int32_t m, const int64_t* row_ptr, const int32_t* col,
                       const float* val, const void* valq, int32_t dtype, const float* row_scale,
                       int64_t nnz, const float* c, double gamma, hipStream_t stream,
                       mbdp_mdp_t* out);

}  // namespace

extern "C" {

mbdp_status mdp_create_dense(int64_t n, int32_t m, const float* P, const float* c, double gamma,
                             mbdp_mdp_t* out) {
  return create_dense(n, m, P, nullptr, kF32, nullptr, c, gamma, out);
}

mbdp_status mdp_create_dense_q(int64_t n, int32_t m, const void* P, int32_t dtype,
                               const float* row_scale, const float* c, double gamma,
                               mbdp_mdp_t* out) {
  if (out) *out = nullptr;
  if (!dtype_ok(dtype)) return fail(MBDP_ERR_INVALID_ARG, "dtype %d is not BF16 or FP8 E4M3", dtype);
  return create_dense(n, m, nullptr, P, dtype, row_scale, c, gamma, out);
}

mbdp_status mdp_create_csr(int64_t n, int32_t m, const int64_t* row_ptr, const int32_t* col,
                           const float* val, int64_t nnz, const float* c, double gamma,
                           hipStream_t stream, mbdp_mdp_t* out) {
  return create_csr(n, m, row_ptr, col, val, nullptr, kF32, nullptr, nnz, c, gamma, stream, out);
}

mbdp_status mdp_create_csr_q(int64_t n, int32_t m, const int64_t* row_ptr, const int32_t* col,
                             const void* val, int32_t dtype, const float* row_scale, int64_t nnz,
                             const float* c, double gamma, hipStream_t stream, mbdp_mdp_t* out) {
  if (out) *out = nullptr;
  if (!dtype_ok(dtype)) return fail(MBDP_ERR_INVALID_ARG, "dtype %d is not BF16 or FP8 E4M3", dtype);
  return create_csr(n, m, row_ptr, col, nullptr, val, dtype, row_scale, nnz, c, gamma, stream, out);
}

mbdp_status mdp_quantize_rows(const float* src, int64_t rows, int64_t row_len, int32_t dtype,
                              void* dst, float* row_scale, hipStream_t stream) {
  if (!dtype_ok(dtype)) return fail(MBDP_ERR_INVALID_ARG, "dtype %d is not BF16 or FP8 E4M3", dtype);
  if (rows < 1 || row_len < 1) return fail(MBDP_ERR_INVALID_ARG, "rows and row_len must be >= 1");
  if (!src || !dst || !row_scale) return fail(MBDP_ERR_INVALID_ARG, "src, dst or row_scale is NULL");
  if (launch_quantize(src, rows, row_len, dtype, dst, row_scale, stream) != 0)
    return fail(MBDP_ERR_HIP, "quantize launch failed: %s", hipGetErrorString(hipGetLastError()));
  return MBDP_OK;
}

}  // extern "C"

namespace {

mbdp_status create_csr(int64_t n, int32_t m, const int64_t* row_ptr, const int32_t* col,
                       const float* val, const void* valq, int32_t dtype, const float* row_scale,
                       int64_t nnz, const float* c, double gamma, hipStream_t stream,
                       mbdp_mdp_t* out) {
  if (!out) return fail(MBDP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || n >= kMaxStates) return fail(MBDP_ERR_INVALID_ARG, "n = %lld not in [1, 2^31)", (long long)n);
  if (m < 1) return fail(MBDP_ERR_INVALID_ARG, "m = %d < 1", m);
  if (nnz < 0) return fail(MBDP_ERR_INVALID_ARG, "nnz = %lld < 0", (long long)nnz);
  const bool have_vals = dtype == kF32 ? val != nullptr : (valq != nullptr && row_scale != nullptr);
  if (!row_ptr || !c || (nnz > 0 && (!col || !have_vals)))
    return fail(MBDP_ERR_INVALID_ARG, "row_ptr, col, val, row_scale or c is NULL");
  if (!gamma_ok(gamma)) return fail(MBDP_ERR_INVALID_ARG, "gamma = %g not in (0, 1)", gamma);
  mbdp_mdp* h = new (std::nothrow) mbdp_mdp();
  if (!h) return fail(MBDP_ERR_HIP, "out of host memory");
  h->storage = kCsr;
  h->n = n;
  h->m = m;
  h->gamma = gamma;
  h->row_ptr = row_ptr;
  h->col = col;
  h->val = val;
  h->vdtype = dtype;
  h->pq = valq;
  h->rscale = row_scale;
  h->nnz = nnz;
  h->c = c;
  mbdp_status st = query_device(h);
  if (st != MBDP_OK) {
    delete h;
    return st;
  }
  // Inspect the structure on the device: constant row length, monotone
  // row_ptr consistent with nnz, columns in range.
  const int64_t rows = n * (int64_t)m;
  const int64_t k = (nnz % rows == 0) ? nnz / rows : -1;
  unsigned long long flags[8] = {0};
  {
    std::lock_guard<std::mutex> lock(g_inspect_mutex);
    void* dflags = nullptr;
    hipError_t e = (hipError_t)inspect_flags_ptr(&dflags);
    if (e == hipSuccess && launch_zero(dflags, sizeof flags, stream) != 0) e = hipGetLastError();
    if (e == hipSuccess &&
        launch_csr_inspect(row_ptr, col, rows, n, nnz, k,
                           static_cast<unsigned long long*>(dflags), stream) != 0)
      e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(flags, dflags, sizeof flags, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      delete h;
      return fail(MBDP_ERR_HIP, "CSR inspection failed: %s", hipGetErrorString(e));
    }
  }
  if (flags[1] || flags[2]) {
    delete h;
    return fail(MBDP_ERR_INVALID_ARG, "row_ptr is not non-decreasing from 0 to nnz");
  }
  if (flags[3]) {
    delete h;
    return fail(MBDP_ERR_INVALID_ARG, "%llu column indices outside [0, n)", flags[3]);
  }
  if (flags[0] == 0 && k >= 4 && k <= 256 && k % 4 == 0) {
    h->storage = kEll;
    h->ell_k = (int32_t)k;
    h->band = (int32_t)flags[4];
  }
  if (dtype != kF32 && !(h->storage == kEll && k <= 64)) {
    delete h;
    return fail(MBDP_ERR_UNSUPPORTED,
                "BF16 / FP8 values need a constant row length k with k %% 4 == 0, 4 <= k <= 64");
  }
  *out = h;
  return MBDP_OK;
}

}  // namespace

extern "C" {

mbdp_status mdp_destroy(mbdp_mdp_t h) {
  delete h;
  return MBDP_OK;
}

mbdp_status mdp_set_tuning(mbdp_mdp_t h, const mbdp_tuning* t) {
  if (!h || !t) return fail(MBDP_ERR_INVALID_ARG, "handle or tuning is NULL");
  if (t->threads_per_block != 0 && t->threads_per_block != 256 && t->threads_per_block != 512 &&
      t->threads_per_block != 1024)
    return fail(MBDP_ERR_INVALID_ARG, "threads_per_block must be 0, 256, 512 or 1024");
  if (t->band_window != 0 && t->band_window != -1)
    return fail(MBDP_ERR_INVALID_ARG, "band_window must be 0 or -1");
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > kMaxBlocksPerCu)
    return fail(MBDP_ERR_INVALID_ARG, "blocks_per_cu must be in [0, %d]", kMaxBlocksPerCu);
  h->tuning = *t;
  return MBDP_OK;
}

size_t mdp_workspace_bytes(mbdp_mdp_t h, int64_t b) {
  if (!h || b < 1 || b > h->n) return 0;
  return layout(h).total;
}

mbdp_status mdp_engine(mbdp_mdp_t h, int64_t b, const char** name) {
  if (!h || !name) return fail(MBDP_ERR_INVALID_ARG, "handle or name is NULL");
  *name = nullptr;
  if (b < 1 || b > h->n) return fail(MBDP_ERR_INVALID_ARG, "b = %lld not in [1, n]", (long long)b);
  KParams p = base_params(h, nullptr, nullptr, b);
  p.task = kTaskVI;
  int engine = 0;
  char err[256] = {0};
  if (query_engine(p, shape_of(h), &engine, err, sizeof err) != 0) return fail(MBDP_ERR_HIP, "%s", err);
  static const char* const names[] = {"dense", "ell", "ell-band", "csr", "ell-colblock"};
  *name = names[engine];
  return MBDP_OK;
}

}  // extern "C"

namespace {

constexpr int64_t kColMaxStates = (int64_t)1 << 20;  // 20-bit column field of a key

struct ColLayoutSizes {
  size_t gptr, keys, vals, total;
};

ColLayoutSizes col_sizes(const mbdp_mdp* h) {
  ColLayoutSizes z{};
  z.gptr = 0;
  z.keys = align_up(h->cb_gptr_h.size() * sizeof(int32_t), 256);
  z.vals = align_up(z.keys + h->cb_keys_h.size() * sizeof(uint32_t), 256);
  z.total = align_up(z.vals + h->cb_vals_h.size() * sizeof(float), 256);
  return z;
}

// Entries of block b (states [b bs, (b + 1) bs)) sorted by column, then
// packed greedily into groups of 64 with distinct rows (an entry whose row
// is already in the current group waits for the next one, ahead of the
// rest); the last group is padded with zero values on unused rows.
void build_col_block(const int32_t* col, const float* val, int64_t n, int32_t m, int32_t k,
                     int64_t bs, int64_t b, std::vector<uint32_t>& keys, std::vector<float>& vals) {
  const int64_t r0 = b * bs * m, r1 = std::min(n, (b + 1) * bs) * m;
  std::vector<std::pair<uint32_t, float>> e;
  e.reserve((size_t)(r1 - r0) * k);
  for (int64_t r = r0; r < r1; ++r)
    for (int32_t i = 0; i < k; ++i) {
      const size_t x = (size_t)r * k + i;
      e.push_back({((uint32_t)col[x] << 12) | (uint32_t)(r - r0), val[x]});
    }
  std::stable_sort(e.begin(), e.end(),
                   [](const std::pair<uint32_t, float>& a, const std::pair<uint32_t, float>& c) {
                     return a.first < c.first;
                   });
  std::vector<int> mark(kColRows, -1);
  std::vector<std::pair<uint32_t, float>> pend, next;
  size_t i = 0;
  int group = 0;
  while (i < e.size() || !pend.empty()) {
    int cnt = 0;
    uint32_t last = 0;
    next.clear();
    auto take = [&](const std::pair<uint32_t, float>& x) {
      const uint32_t r = x.first & (kColRows - 1);
      if (mark[r] == group) return false;
      mark[r] = group;
      keys.push_back(x.first);
      vals.push_back(x.second);
      last = x.first;
      ++cnt;
      return true;
    };
    for (size_t q = 0; q < pend.size(); ++q)
      if (cnt == kColGroup || !take(pend[q])) next.push_back(pend[q]);
    pend.swap(next);
    while (i < e.size() && cnt < kColGroup)
      if (!take(e[i++])) pend.push_back(e[i - 1]);
    for (uint32_t r = 0; cnt < kColGroup; ++r)
      if (mark[r] != group) {
        mark[r] = group;
        keys.push_back((last & ~(uint32_t)(kColRows - 1)) | r);
        vals.push_back(0.f);
        ++cnt;
      }
    ++group;
  }
}

}  // namespace

extern "C" {

mbdp_status mdp_column_blocks_prepare(mbdp_mdp_t h, hipStream_t stream, size_t* bytes) {
  if (!h || !bytes) return fail(MBDP_ERR_INVALID_ARG, "handle or bytes is NULL");
  *bytes = 0;
  if (h->storage != kEll || h->vdtype != kF32)
    return fail(MBDP_ERR_UNSUPPORTED, "column blocks need constant-row-length FP32 rows");
  if (h->n > kColMaxStates)
    return fail(MBDP_ERR_UNSUPPORTED, "column blocks need n <= 2^20 (n = %lld)", (long long)h->n);
  if (h->m > kColRows) return fail(MBDP_ERR_UNSUPPORTED, "column blocks need m <= %d", kColRows);
  // Blocks hold at most 4096 / m states (4096 rows of LDS sums); the block
  // size is then shrunk so that the blocks fill whole passes of the grid
  // (one 8-wavefront workgroup per CU, a wavefront per block), but not
  // below half of that (fewer rows per block leave more padding in the
  // groups): at 10^6 states and m = 8, 2045 blocks of 489 states give every
  // CU one set of 8 instead of 1954 blocks of 512 on 245 of them.
  const int64_t n = h->n, bmax = kColRows / h->m;
  const int64_t slots = (int64_t)std::max(h->cus, 1) * (kColThreads / 64);
  const int64_t passes = ((n + bmax - 1) / bmax + slots - 1) / slots;
  const int64_t bs = std::max((n + passes * slots - 1) / (passes * slots), (bmax + 1) / 2);
  const int64_t nblk = (n + bs - 1) / bs;
  const size_t nnz = (size_t)h->nnz;
  std::vector<int32_t> col(nnz);
  std::vector<float> val(nnz);
  MBDP_HIP(hipMemcpyAsync(col.data(), h->col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipMemcpyAsync(val.data(), h->val, nnz * sizeof(float), hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  // blocks are built on host threads, each over a contiguous range of
  // blocks, then concatenated in block order (the result does not depend
  // on the thread count)
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 32u));
  std::vector<std::vector<uint32_t>> tk(nt);
  std::vector<std::vector<float>> tv(nt);
  std::vector<std::vector<int64_t>> tg(nt);  // groups per block
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      const int64_t b0 = nblk * t / nt, b1 = nblk * (t + 1) / nt;
      for (int64_t b = b0; b < b1; ++b) {
        const size_t before = tk[t].size();
        build_col_block(col.data(), val.data(), n, h->m, h->ell_k, bs, b, tk[t], tv[t]);
        tg[t].push_back((int64_t)((tk[t].size() - before) / kColGroup));
      }
    });
  for (auto& x : th) x.join();
  h->cb_keys_h.clear();
  h->cb_vals_h.clear();
  h->cb_gptr_h.assign(1, 0);
  int64_t groups = 0;
  for (unsigned t = 0; t < nt; ++t) {
    h->cb_keys_h.insert(h->cb_keys_h.end(), tk[t].begin(), tk[t].end());
    h->cb_vals_h.insert(h->cb_vals_h.end(), tv[t].begin(), tv[t].end());
    for (int64_t g : tg[t]) {
      groups += g;
      if (groups > INT32_MAX) return fail(MBDP_ERR_UNSUPPORTED, "too many column-block groups");
      h->cb_gptr_h.push_back((int32_t)groups);
    }
  }
  h->cb_states = bs;
  *bytes = col_sizes(h).total;
  return MBDP_OK;
}

mbdp_status mdp_column_blocks_attach(mbdp_mdp_t h, void* buffer, size_t bytes,
                                     hipStream_t stream) {
  if (!h || !buffer) return fail(MBDP_ERR_INVALID_ARG, "handle or buffer is NULL");
  if (h->cb_gptr_h.empty())
    return fail(MBDP_ERR_INVALID_ARG, "no column blocks prepared (mdp_column_blocks_prepare)");
  if (((uintptr_t)buffer) % 256) return fail(MBDP_ERR_INVALID_ARG, "buffer is not 256-byte aligned");
  const ColLayoutSizes z = col_sizes(h);
  if (bytes < z.total)
    return fail(MBDP_ERR_INVALID_ARG, "buffer has %zu bytes, need %zu", bytes, z.total);
  char* base = static_cast<char*>(buffer);
  MBDP_HIP(hipMemcpyAsync(base + z.gptr, h->cb_gptr_h.data(),
                          h->cb_gptr_h.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  MBDP_HIP(hipMemcpyAsync(base + z.keys, h->cb_keys_h.data(),
                          h->cb_keys_h.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
  MBDP_HIP(hipMemcpyAsync(base + z.vals, h->cb_vals_h.data(),
                          h->cb_vals_h.size() * sizeof(float), hipMemcpyHostToDevice, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  h->cb_gptr = reinterpret_cast<const int32_t*>(base + z.gptr);
  h->cb_keys = reinterpret_cast<const uint32_t*>(base + z.keys);
  h->cb_vals = reinterpret_cast<const float*>(base + z.vals);
  std::vector<uint32_t>().swap(h->cb_keys_h);
  std::vector<float>().swap(h->cb_vals_h);
  std::vector<int32_t>().swap(h->cb_gptr_h);
  return MBDP_OK;
}

mbdp_status mdp_policy_transpose(mbdp_mdp_t h, const int32_t* policy, int64_t* row_ptr_t,
                                 int32_t* col_t, float* val_t, void* workspace, size_t ws_bytes,
                                 hipStream_t stream) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (!policy || !row_ptr_t || !col_t || !val_t)
    return fail(MBDP_ERR_INVALID_ARG, "policy, row_ptr_t, col_t or val_t is NULL");
  if (h->storage != kEll || h->vdtype != kF32)
    return fail(MBDP_ERR_UNSUPPORTED,
                "the policy transpose needs FP32 rows of constant length (ELL storage)");
  mbdp_status st = check_ws(h, workspace, ws_bytes);
  if (st != MBDP_OK) return st;
  const size_t scratch = (64 + 2 * (size_t)h->n) * sizeof(unsigned);
  if (launch_zero(workspace, scratch, stream) != 0)
    return fail(MBDP_ERR_HIP, "clear failed: %s", hipGetErrorString(hipGetLastError()));
  KParams p = base_params(h, workspace, nullptr, 1);
  if (launch_policy_transpose(p, policy, row_ptr_t, col_t, val_t,
                              static_cast<unsigned*>(workspace), stream) != 0)
    return fail(MBDP_ERR_HIP, "transpose launch failed: %s", hipGetErrorString(hipGetLastError()));
  unsigned bad = 0;
  MBDP_HIP(hipMemcpyAsync(&bad, workspace, sizeof bad, hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  if (bad) return fail(MBDP_ERR_INVALID_ARG, "%u policy entries outside [0, m)", bad);
  return MBDP_OK;
}

mbdp_status mdp_value_gradients(mbdp_mdp_t h, const int32_t* policy, const double* lambda,
                                const double* V, double* grad_c, double* grad_val,
                                void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (!policy || !lambda || !V) return fail(MBDP_ERR_INVALID_ARG, "policy, lambda or V is NULL");
  if (!grad_c && !grad_val) return fail(MBDP_ERR_INVALID_ARG, "grad_c and grad_val are NULL");
  if (h->storage != kEll || h->vdtype != kF32)
    return fail(MBDP_ERR_UNSUPPORTED,
                "value gradients need FP32 rows of constant length (ELL storage)");
  mbdp_status st = check_ws(h, workspace, ws_bytes);
  if (st != MBDP_OK) return st;
  if (launch_zero(workspace, 256, stream) != 0)
    return fail(MBDP_ERR_HIP, "clear failed: %s", hipGetErrorString(hipGetLastError()));
  KParams p = base_params(h, workspace, nullptr, 1);
  if (launch_value_gradients(p, policy, lambda, V, grad_c, grad_val,
                             static_cast<unsigned*>(workspace), stream) != 0)
    return fail(MBDP_ERR_HIP, "gradient launch failed: %s", hipGetErrorString(hipGetLastError()));
  unsigned bad = 0;
  MBDP_HIP(hipMemcpyAsync(&bad, workspace, sizeof bad, hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  if (bad) return fail(MBDP_ERR_INVALID_ARG, "%u policy entries outside [0, m)", bad);
  return MBDP_OK;
}

size_t mdp_batch_workspace_bytes(int32_t count) {
  if (count < 1) return 0;
  return batch_layout(count).total;
}

mbdp_status mdp_batch_upload(const mbdp_batch_item* items, int32_t count, void* workspace,
                             size_t ws_bytes, hipStream_t stream) {
  if (count < 1 || !items) return fail(MBDP_ERR_INVALID_ARG, "need count >= 1 items");
  const BatchLayout L = batch_layout(count);
  if (!workspace || ((uintptr_t)workspace) % 256 || ws_bytes < L.total)
    return fail(MBDP_ERR_WORKSPACE, "batch workspace must be 256-byte aligned with %zu bytes",
                L.total);
  std::vector<BatchItem> table((size_t)count);
  std::vector<double> work((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    const mbdp_batch_item& it = items[i];
    if (it.n < 1 || it.n > kBatchMaxN)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: n = %lld not in [1, %lld]", i,
                  (long long)it.n, (long long)kBatchMaxN);
    if (it.m < 1 || it.m > kBatchMaxM)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: m = %d not in [1, %d]", i, it.m, kBatchMaxM);
    if (it.ld < it.n || it.ld % 16 != 0 || it.ld > kBatchMaxN)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: ld = %lld must be >= n, <= %lld and a multiple of 16",
                  i, (long long)it.ld, (long long)kBatchMaxN);
    if (it.b < 1 || it.b > it.n || it.b > kBatchMaxB)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: b = %lld not in [1, min(n, %lld)]", i,
                  (long long)it.b, (long long)kBatchMaxB);
    if (!gamma_ok(it.gamma)) return fail(MBDP_ERR_INVALID_ARG, "item %d: gamma not in (0, 1)", i);
    if (it.dtype != MBDP_F32 && it.dtype != MBDP_BF16 && it.dtype != MBDP_FP8_E4M3)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: unknown dtype %d", i, it.dtype);
    if (!it.P || !it.c || !it.V || (it.dtype != MBDP_F32 && !it.row_scale))
      return fail(MBDP_ERR_INVALID_ARG, "item %d: P, c, V or row_scale is NULL", i);
    if (((uintptr_t)it.P) % 16)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: P must be 16-byte aligned", i);
    if (it.lanes != 0 && it.lanes != 16 && it.lanes != 32 && it.lanes != 64)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: lanes must be 0, 16, 32 or 64", i);
    if (it.team < 0 || it.team > kBatchMaxTeam)
      return fail(MBDP_ERR_INVALID_ARG, "item %d: team = %d not in [0, %d]", i, it.team,
                  kBatchMaxTeam);
    BatchItem& b = table[(size_t)i];
    b.n = it.n;
    b.ld = it.ld;
    b.b = it.b;
    b.m = it.m;
    b.dtype = it.dtype;
    b.P = it.P;
    b.rscale = it.row_scale;
    b.c = it.c;
    b.gamma = it.gamma;
    b.seed = it.seed;
    b.V = it.V;
    b.policy = it.policy;
    // default lane group: a step of the group should cover about a row
    const int epl = it.dtype == MBDP_F32 ? 4 : (it.dtype == MBDP_BF16 ? 8 : 16);
    b.lanes = it.lanes ? it.lanes : (it.ld >= 64 * epl ? 64 : (it.ld >= 32 * epl ? 32 : 16));
    b.index = i;
    b.team = it.team;
    b.slot = -1;
    b.ticket0 = 0;
    // work estimate: bytes per sweep times sweeps to shrink the error 1e6-fold
    const double bytes = (double)it.n * it.m * it.ld * (it.dtype == MBDP_F32 ? 4 : it.dtype == MBDP_BF16 ? 2 : 1);
    work[(size_t)i] = bytes * (13.8 / -log(it.gamma));
  }
  // Team sizes.  An MDP whose work exceeds the device's fair share (total
  // work / compute units) gets that many workgroups, at most kBatchMaxTeam
  // and at most 2 b / (lane groups per workgroup); all members of all teams
  // must fit on the device at once (one workgroup per compute unit).
  int device = 0, cus = 0;
  MBDP_HIP(hipGetDevice(&device));
  MBDP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  double total = 0.0;
  for (double w : work) total += w;
  const double share = total / (double)(cus > 0 ? cus : 1);
  std::vector<int32_t> by_work((size_t)count);
  for (int32_t i = 0; i < count; ++i) by_work[(size_t)i] = i;
  std::stable_sort(by_work.begin(), by_work.end(),
                   [&](int32_t x, int32_t y) { return work[(size_t)x] > work[(size_t)y]; });
  const int32_t slots = batch_team_slots(count);
  int64_t members = 0;
  int32_t teams = 0;
  for (int32_t i = 0; i < count; ++i) {
    BatchItem& b = table[(size_t)i];
    if (b.team != 0 || cus < 2 * kBatchMaxTeam) continue;
    const int64_t groups = 1024 / b.lanes;
    // a team runs below one workgroup's rate per member (team barriers), so
    // it gets half again its share, to end with the rest of the launch
    int64_t k = (int64_t)ceil(1.5 * work[(size_t)i] / share);
    // at least half a state per lane group of each member per batch
    const int64_t kcap = std::min<int64_t>(kBatchMaxTeam, std::max<int64_t>(1, 2 * b.b / groups));
    b.team = (int32_t)std::max<int64_t>(1, std::min(k, kcap));
  }
  for (int32_t i = 0; i < count; ++i) {
    BatchItem& b = table[(size_t)i];
    if (b.team == 0) b.team = 1;
    if (b.team > 1) {
      members += b.team;
      ++teams;
    }
  }
  // too many: the lightest automatic teams fall back to one workgroup
  for (int32_t j = count - 1; j >= 0 && (members > cus || teams > slots); --j) {
    const int32_t i = by_work[(size_t)j];
    BatchItem& b = table[(size_t)i];
    if (b.team > 1 && items[i].team == 0) {
      members -= b.team;
      --teams;
      b.team = 1;
    }
  }
  if (members > cus || teams > slots)
    return fail(MBDP_ERR_UNSUPPORTED,
                "teams need %lld workgroups in %d teams; the device runs %d at once and a "
                "launch serves %d teams", (long long)members, teams, cus, slots);
  // queue order: the teams first (all their members start at once), then the
  // single workgroups, each part heaviest per workgroup first
  std::vector<int32_t> order((size_t)count);
  for (int32_t i = 0; i < count; ++i) order[(size_t)i] = i;
  auto per_member = [&](int32_t i) { return work[(size_t)i] / table[(size_t)i].team; };
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const bool tx = table[(size_t)x].team > 1, ty = table[(size_t)y].team > 1;
    if (tx != ty) return tx;
    return per_member(x) > per_member(y);
  });
  std::vector<BatchItem> sorted((size_t)count);
  int64_t ticket = 0;
  int32_t slot = 0;
  for (int32_t i = 0; i < count; ++i) {
    BatchItem b = table[(size_t)order[(size_t)i]];
    b.ticket0 = ticket;
    ticket += b.team;
    if (b.team > 1) b.slot = slot++;
    sorted[(size_t)i] = b;
  }
  char* base = static_cast<char*>(workspace);
  MBDP_HIP(hipMemcpyAsync(base + L.items, sorted.data(), sorted.size() * sizeof(BatchItem),
                          hipMemcpyHostToDevice, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  return MBDP_OK;
}

mbdp_status mdp_batch_launch(int32_t count, double tol_dv, int64_t max_sweeps, void* workspace,
                             size_t ws_bytes, hipStream_t stream) {
  if (count < 1) return fail(MBDP_ERR_INVALID_ARG, "count must be >= 1");
  if (max_sweeps < 1) return fail(MBDP_ERR_INVALID_ARG, "max_sweeps must be >= 1");
  const BatchLayout L = batch_layout(count);
  if (!workspace || ((uintptr_t)workspace) % 256 || ws_bytes < L.total)
    return fail(MBDP_ERR_WORKSPACE, "batch workspace must be 256-byte aligned with %zu bytes",
                L.total);
  int device = 0, cus = 0, khz = 0;
  MBDP_HIP(hipGetDevice(&device));
  MBDP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  MBDP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
  char* base = static_cast<char*>(workspace);
  // kernels only (a fill kernel clears the control words), so the call can be captured
  if (launch_zero(base + L.control, sizeof(BatchControl), stream) != 0)
    return fail(MBDP_ERR_HIP, "clear failed: %s", hipGetErrorString(hipGetLastError()));
  BatchArgs a{};
  a.items = reinterpret_cast<const BatchItem*>(base + L.items);
  a.count = count;
  a.ctl = reinterpret_cast<BatchControl*>(base + L.control);
  a.stats = reinterpret_cast<BatchStat*>(base + L.stats);
  a.team_dv = reinterpret_cast<double*>(base + L.team_dv);
  a.team_new = reinterpret_cast<double*>(base + L.team_new);
  a.tol = tol_dv;
  a.max_sweeps = (long long)max_sweeps;
  a.timeout_ticks = (unsigned long long)(kBatchTeamTimeoutSeconds * 1000.0 *
                                         (double)(khz > 0 ? khz : 100000));
  // one workgroup per compute unit at most (the LDS holds one), and at least
  // every member of every team, which the upload kept within the device
  const int64_t want = (int64_t)count * kBatchMaxTeam;
  const int blocks = (int)std::min<int64_t>(cus, want);
  if (launch_batch(a, blocks, stream) != 0)
    return fail(MBDP_ERR_HIP, "batch launch failed: %s", hipGetErrorString(hipGetLastError()));
  return MBDP_OK;
}

mbdp_status mdp_batch_read_stats(void* workspace, int32_t count, mbdp_batch_stats* out,
                                 hipStream_t stream) {
  if (count < 1 || !workspace || !out) return fail(MBDP_ERR_INVALID_ARG, "bad arguments");
  const BatchLayout L = batch_layout(count);
  std::vector<BatchStat> st((size_t)count);
  BatchControl ctl{};
  MBDP_HIP(hipMemcpyAsync(st.data(), static_cast<char*>(workspace) + L.stats,
                          st.size() * sizeof(BatchStat), hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipMemcpyAsync(&ctl, static_cast<char*>(workspace) + L.control, sizeof ctl,
                          hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  if (ctl.abort)
    return fail(MBDP_ERR_DEVICE, "a team barrier of the batched launch timed out");
  std::vector<BatchItem> table((size_t)count);
  MBDP_HIP(hipMemcpyAsync(table.data(), static_cast<char*>(workspace) + L.items,
                          table.size() * sizeof(BatchItem), hipMemcpyDeviceToHost, stream));
  int device = 0, khz = 0;
  MBDP_HIP(hipGetDevice(&device));
  MBDP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
  MBDP_HIP(hipStreamSynchronize(stream));
  const double us_per_tick = 1000.0 / (double)(khz > 0 ? khz : 100000);
  unsigned long long t0 = ~0ull;
  for (const BatchStat& s : st) t0 = std::min(t0, s.t_start);
  for (int32_t i = 0; i < count; ++i) {
    out[i].sweeps = st[(size_t)i].sweeps;
    out[i].final_dv_inf = st[(size_t)i].dv;
    out[i].converged = st[(size_t)i].converged;
    out[i].team = 0;
    out[i].start_us = (double)(st[(size_t)i].t_start - t0) * us_per_tick;
    out[i].end_us = (double)(st[(size_t)i].t_end - t0) * us_per_tick;
  }
  for (const BatchItem& b : table)
    if (b.index >= 0 && b.index < count) out[b.index].team = b.team;
  return MBDP_OK;
}

namespace {

mbdp_status multi_check(const mbdp_mdp* h, int32_t r, int64_t b) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (h->storage != kDense || h->vdtype != kBF16)
    return fail(MBDP_ERR_UNSUPPORTED, "multi-vector backups need a dense BF16 handle (mdp_create_dense_q)");
  if (h->n % 32 != 0)
    return fail(MBDP_ERR_UNSUPPORTED, "multi-vector backups need n %% 32 == 0 (got n = %lld)",
                (long long)h->n);
  if (r != 16 && r != 32 && r != 48 && r != 64)
    return fail(MBDP_ERR_INVALID_ARG, "r = %d is not 16, 32, 48 or 64", r);
  if (b < 1 || b > h->n) return fail(MBDP_ERR_INVALID_ARG, "b = %lld not in [1, n]", (long long)b);
  return MBDP_OK;
}

// Fold W into the anchor when the products' error bound (2^-16 max|W|)
// would reach a twentieth of the last sweep's change.
constexpr double kMultiSplitError = 1.0 / 65536.0;
constexpr double kMultiErrorShare = 0.05;
constexpr int kMultiChunk = 8;  // sweeps enqueued between reads of the control block

}  // namespace

size_t mdp_multi_workspace_bytes(mbdp_mdp_t h, int32_t r, int64_t b) {
  if (multi_check(h, r, b) != MBDP_OK) return 0;
  return multi_layout(h->n, h->m, r, b).total;
}

mbdp_status mdp_multi_solve(mbdp_mdp_t h, int32_t r, const float* C, double* V, int32_t* policy,
                            int64_t b, uint64_t seed, uint64_t first_sweep, double tol_dv,
                            int64_t max_sweeps, void* workspace, size_t ws_bytes,
                            hipStream_t stream, mbdp_multi_stats* stats) {
  mbdp_status st = multi_check(h, r, b);
  if (st != MBDP_OK) return st;
  if (!C || !V) return fail(MBDP_ERR_INVALID_ARG, "C or V is NULL");
  if (max_sweeps < 1) return fail(MBDP_ERR_INVALID_ARG, "max_sweeps must be >= 1");
  const MultiLayout L = multi_layout(h->n, h->m, r, b);
  if (!workspace || ((uintptr_t)workspace) % 256 || ws_bytes < L.total)
    return fail(MBDP_ERR_WORKSPACE, "multi-vector workspace must be 256-byte aligned with %zu bytes",
                L.total);
  MBDP_HIP(hipSetDevice(h->device));
  char* base = static_cast<char*>(workspace);
  MultiArgs a{};
  a.n = h->n;
  a.m = h->m;
  a.r = r;
  a.gamma = h->gamma;
  a.b = b;
  a.seed = seed;
  a.tol = tol_dv;
  a.P = static_cast<const uint16_t*>(h->pq);
  a.rscale = h->rscale;
  a.C = C;
  a.R = reinterpret_cast<double*>(base + L.R);
  a.W = reinterpret_cast<double*>(base + L.W);
  a.Ws = reinterpret_cast<uint16_t*>(base + L.Ws);
  a.PR = reinterpret_cast<double*>(base + L.PR);
  a.part = reinterpret_cast<float*>(base + L.part);
  a.part_rows = b * h->m;
  a.kchunk = L.kchunk;
  a.splits = L.splits;
  a.policy = policy;
  a.dvs = reinterpret_cast<double*>(base + L.dvs);
  a.order = reinterpret_cast<int32_t*>(base + L.order);
  a.ctl = reinterpret_cast<MultiControl*>(base + L.ctl);
  const char* what = nullptr;
  auto ok = [&](int rc, const char* name) {
    if (rc != 0 && !what) what = name;
    return rc == 0;
  };
  // anchor at V0: R = V0, W = 0, PR = P R
  ok(launch_zero(base + L.ctl, sizeof(MultiControl), stream), "clear");
  ok(launch_multi_anchor(a, V, 0, stream), "anchor");
  ok(launch_multi_pr(a, stream), "anchor products");
  if (what) return fail(MBDP_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(hipGetLastError()));
  const int64_t nb = (h->n + b - 1) / b;
  int64_t launched = 0, recentrings = 0;
  MultiControl ctl{};
  uint64_t t = first_sweep;
  while (launched < max_sweeps) {
    const int64_t chunk = std::min<int64_t>(kMultiChunk, max_sweeps - launched);
    for (int64_t c = 0; c < chunk && !what; ++c, ++t) {
      ok(launch_multi_order(a, t, stream), "sweep order");
      for (int64_t k = 0; k < nb && !what; ++k) {
        ok(launch_multi_gemm(a, t, k, 0, stream), "product");
        ok(launch_multi_commit(a, t, k, 0, stream), "commit");
      }
      ok(launch_multi_end(a, stream), "end of sweep");
    }
    if (what) return fail(MBDP_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(hipGetLastError()));
    launched += chunk;
    MBDP_HIP(hipMemcpyAsync(&ctl, base + L.ctl, sizeof ctl, hipMemcpyDeviceToHost, stream));
    MBDP_HIP(hipStreamSynchronize(stream));
    if (ctl.done || launched >= max_sweeps) break;
    if (ctl.w_bound * kMultiSplitError > kMultiErrorShare * ctl.dv_last) {
      ok(launch_multi_anchor(a, V, 1, stream), "re-centring");
      ok(launch_multi_pr(a, stream), "anchor products");
      ++recentrings;
      if (what) return fail(MBDP_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(hipGetLastError()));
    }
  }
  ok(launch_multi_anchor(a, V, 2, stream), "result");
  if (policy) {
    for (int64_t k = 0; k < nb && !what; ++k) {
      ok(launch_multi_gemm(a, 0, k, 1, stream), "policy product");
      ok(launch_multi_commit(a, 0, k, 1, stream), "policy");
    }
  }
  if (what) return fail(MBDP_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(hipGetLastError()));
  MBDP_HIP(hipStreamSynchronize(stream));
  if (stats) {
    stats->sweeps = ctl.sweeps;
    stats->final_dv_inf = ctl.dv_last;
    stats->recentrings = recentrings;
    stats->converged = ctl.done ? 1 : 0;
    stats->reserved = 0;
  }
  return ctl.done || tol_dv < 0 ? MBDP_OK : MBDP_ERR_NOT_CONVERGED;
}

mbdp_status mdp_validate(mbdp_mdp_t h, double row_sum_tol, void* workspace, size_t ws_bytes,
                         hipStream_t stream, mbdp_validation* report) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (!(row_sum_tol >= 0.0)) return fail(MBDP_ERR_INVALID_ARG, "row_sum_tol must be >= 0");
  mbdp_status st = check_ws(h, workspace, ws_bytes);
  if (st != MBDP_OK) return st;
  KParams p = base_params(h, workspace, nullptr, 1);
  unsigned long long* out = static_cast<unsigned long long*>(workspace);
  unsigned long long res[8] = {0};
  if (launch_zero(out, sizeof res, stream) != 0)
    return fail(MBDP_ERR_HIP, "clear failed: %s", hipGetErrorString(hipGetLastError()));
  if (launch_validate(p, row_sum_tol, out, stream) != 0)
    return fail(MBDP_ERR_HIP, "validate launch failed: %s", hipGetErrorString(hipGetLastError()));
  MBDP_HIP(hipMemcpyAsync(res, out, sizeof res, hipMemcpyDeviceToHost, stream));
  MBDP_HIP(hipStreamSynchronize(stream));
  mbdp_validation v;
  v.bad_probability = (int64_t)res[0];
  v.bad_row_sum = (int64_t)res[1];
  v.empty_rows = (int64_t)res[2];
  v.bad_column = (int64_t)res[3];
  v.bad_row_ptr = (int64_t)res[4];
  v.bad_cost = (int64_t)res[5];
  v.no_admissible_action = (int64_t)res[6];
  double dev;
  memcpy(&dev, &res[7], sizeof dev);
  v.max_row_sum_dev = dev;
  if (report) *report = v;
  if (v.bad_probability || v.bad_row_sum || v.empty_rows || v.bad_column || v.bad_row_ptr ||
      v.bad_cost || v.no_admissible_action)
    return fail(MBDP_ERR_VALIDATION,
                "invalid MDP: %lld bad probabilities, %lld bad row sums (max dev %g), %lld empty "
                "rows, %lld bad columns, %lld bad costs, %lld states without admissible action",
                (long long)v.bad_probability, (long long)v.bad_row_sum, v.max_row_sum_dev,
                (long long)v.empty_rows, (long long)v.bad_column, (long long)v.bad_cost,
                (long long)v.no_admissible_action);
  return MBDP_OK;
}

mbdp_status mbdp_permutation(int64_t n, uint64_t seed, uint64_t sweep_index, int32_t* out,
                             hipStream_t stream) {
  if (n < 1 || n >= kMaxStates) return fail(MBDP_ERR_INVALID_ARG, "n = %lld not in [1, 2^31)", (long long)n);
  if (!out) return fail(MBDP_ERR_INVALID_ARG, "out is NULL");
  if (launch_permutation(n, seed, sweep_index, out, stream) != 0)
    return fail(MBDP_ERR_HIP, "permutation launch failed: %s", hipGetErrorString(hipGetLastError()));
  return MBDP_OK;
}

mbdp_status mb_sweep(mbdp_mdp_t h, float* V, const int32_t* policy, int64_t b, uint64_t seed,
                     uint64_t sweep_index, const int32_t* perm, int32_t* argmin_out,
                     float* dv_out, void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (!V) return fail(MBDP_ERR_INVALID_ARG, "V is NULL");
  if (b < 1 || b > h->n)
    return fail(MBDP_ERR_INVALID_ARG, "batch size b = %lld not in [1, n = %lld]", (long long)b,
                (long long)h->n);
  mbdp_status st = check_ws(h, workspace, ws_bytes);
  if (st != MBDP_OK) return st;
  KParams p = base_params(h, workspace, V, b);
  p.task = kTaskSweep;
  p.policy = const_cast<int32_t*>(policy);
  p.policy_sweep = policy != nullptr;
  p.perm = perm;
  p.argmin_out = argmin_out;
  p.seed = seed;
  p.first_sweep = sweep_index;
  st = launch(h, p, workspace, stream);
  if (st != MBDP_OK) return st;
  if (dv_out)
    MBDP_HIP(hipMemcpyAsync(dv_out, &p.ctl->dv_last, sizeof(float), hipMemcpyDeviceToDevice, stream));
  return MBDP_OK;
}

mbdp_status mbdp_sync_status(void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!workspace || ws_bytes < sizeof(Control))
    return fail(MBDP_ERR_WORKSPACE, "workspace missing or too small");
  Control c;
  return finish(workspace, stream, &c);
}

}  // extern "C"

namespace {

mbdp_status vi_solve_impl(mbdp_mdp_t h, float* V, double* V64_out, int32_t* policy_out,
                          int64_t b, uint64_t seed, uint64_t first_sweep, double tol_dv,
                          double eps, const double* V_ref, int64_t max_sweeps, void* workspace,
                          size_t ws_bytes, hipStream_t stream, mbdp_stats* stats) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (!V) return fail(MBDP_ERR_INVALID_ARG, "V is NULL");
  if (b < 1 || b > h->n)
    return fail(MBDP_ERR_INVALID_ARG, "batch size b = %lld not in [1, n = %lld]", (long long)b,
                (long long)h->n);
  if (max_sweeps < 1) return fail(MBDP_ERR_INVALID_ARG, "max_sweeps must be >= 1");
  if (isnan(tol_dv)) return fail(MBDP_ERR_INVALID_ARG, "tol_dv is NaN");
  if (V_ref && !(eps >= 0.0)) return fail(MBDP_ERR_INVALID_ARG, "eps must be >= 0 with V_ref");
  mbdp_status st = check_ws(h, workspace, ws_bytes);
  if (st != MBDP_OK) return st;
  const WsLayout w = layout(h);
  KParams p = base_params(h, workspace, V, b);
  p.task = kTaskVI;
  p.v64_out = V64_out;
  p.policy = policy_out;
  p.want_policy_out = policy_out != nullptr;
  p.seed = seed;
  p.first_sweep = first_sweep;
  p.tol_dv = tol_dv;
  p.eps = eps;
  p.vref = V_ref;
  p.max_sweeps = max_sweeps;
  p.recentre_every = recentre_interval(h);
  p.recentre_force = h->tuning.recentre_force != 0;
  p.ceff = reinterpret_cast<double*>(static_cast<char*>(workspace) + w.ceff);
  p.tgt = reinterpret_cast<double*>(static_cast<char*>(workspace) + w.tgt);
  if (p.recentre_every > 0)
    p.shift = reinterpret_cast<double*>(static_cast<char*>(workspace) + w.shift);
  st = launch(h, p, workspace, stream);
  if (st != MBDP_OK) return st;
  Control c;
  st = finish(workspace, stream, &c);
  if (st != MBDP_OK) return st;
  fill_stats(c, V_ref != nullptr, stats);
  if (!c.converged)
    return fail(MBDP_ERR_NOT_CONVERGED, "no stopping rule fired within %lld sweeps",
                (long long)max_sweeps);
  return MBDP_OK;
}

// The no-allocation variant's scratch memory: a file-scope device array
// (one copy per device, held until the process ends).  In host code its
// name is only a host-side stand-in; the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// The current device's address of `scratch` (looked up on first use).
mbdp_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(MBDP_ERR_UNSUPPORTED, "device %d is beyond the %d devices served", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MBDP_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return MBDP_OK;
}

}  // namespace

extern "C" {

mbdp_status vi_solve(mbdp_mdp_t h, float* V, double* V64_out, int32_t* policy_out, int64_t b,
                     uint64_t seed, uint64_t first_sweep, double tol_dv, double eps,
                     const double* V_ref, int64_t max_sweeps, void* workspace, size_t ws_bytes,
                     hipStream_t stream, mbdp_stats* stats) {
  return vi_solve_impl(h, V, V64_out, policy_out, b, seed, first_sweep, tol_dv, eps, V_ref,
                       max_sweeps, workspace, ws_bytes, stream, stats);
}

mbdp_status vi_solve_noalloc(mbdp_mdp_t h, float* V, double* V64_out, int32_t* policy_out,
                             int64_t b, uint64_t seed, uint64_t first_sweep, double tol_dv,
                             double eps, const double* V_ref, int64_t max_sweeps,
                             hipStream_t stream, mbdp_stats* stats) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  const size_t need = layout(h).total;
  if (need > kScratchBytes)
    return fail(MBDP_ERR_INVALID_ARG,
                "vi_solve_noalloc: this MDP needs %zu bytes of scratch memory, more than the "
                "%zu bytes the library holds (use vi_solve with a workspace)",
                need, kScratchBytes);
  int device = -1;
  MBDP_HIP(hipGetDevice(&device));
  if (device != h->device)
    return fail(MBDP_ERR_INVALID_ARG,
                "vi_solve_noalloc: the current device (%d) is not the handle's (%d)", device,
                h->device);
  void* ws = nullptr;
  const mbdp_status st = scratch_address(device, &ws);
  if (st != MBDP_OK) return st;
  return vi_solve_impl(h, V, V64_out, policy_out, b, seed, first_sweep, tol_dv, eps, V_ref,
                       max_sweeps, ws, kScratchBytes, stream, stats);
}

mbdp_status mpi_solve(mbdp_mdp_t h, float* V, double* V64_out, int32_t* policy,
                      int32_t policy_is_init, int32_t K, int64_t b, uint64_t seed,
                      uint64_t first_sweep, double tol_dv, double eps, const double* V_ref,
                      int64_t max_outer, void* workspace, size_t ws_bytes, hipStream_t stream,
                      mbdp_stats* stats) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (!V || !policy) return fail(MBDP_ERR_INVALID_ARG, "V or policy is NULL");
  if (K < 1) return fail(MBDP_ERR_INVALID_ARG, "K = %d < 1", K);
  if (b < 1 || b > h->n)
    return fail(MBDP_ERR_INVALID_ARG, "batch size b = %lld not in [1, n = %lld]", (long long)b,
                (long long)h->n);
  if (max_outer < 1) return fail(MBDP_ERR_INVALID_ARG, "max_outer must be >= 1");
  if (isnan(tol_dv)) return fail(MBDP_ERR_INVALID_ARG, "tol_dv is NaN");
  if (V_ref && !(eps >= 0.0)) return fail(MBDP_ERR_INVALID_ARG, "eps must be >= 0 with V_ref");
  mbdp_status st = check_ws(h, workspace, ws_bytes);
  if (st != MBDP_OK) return st;
  const WsLayout w = layout(h);
  KParams p = base_params(h, workspace, V, b);
  p.task = kTaskMPI;
  p.v64_out = V64_out;
  p.policy = policy;
  p.policy_is_init = policy_is_init != 0;
  p.K = K;
  p.seed = seed;
  p.first_sweep = first_sweep;
  p.tol_dv = tol_dv;
  p.eps = eps;
  p.vref = V_ref;
  p.max_outer = max_outer;
  p.recentre_every = recentre_interval(h);
  p.recentre_force = h->tuning.recentre_force != 0;
  p.ceff = reinterpret_cast<double*>(static_cast<char*>(workspace) + w.ceff);
  p.tgt = reinterpret_cast<double*>(static_cast<char*>(workspace) + w.tgt);
  if (p.recentre_every > 0)
    p.shift = reinterpret_cast<double*>(static_cast<char*>(workspace) + w.shift);
  st = launch(h, p, workspace, stream);
  if (st != MBDP_OK) return st;
  Control c;
  st = finish(workspace, stream, &c);
  if (st != MBDP_OK) return st;
  fill_stats(c, V_ref != nullptr, stats);
  if (!c.converged)
    return fail(MBDP_ERR_NOT_CONVERGED, "no stopping rule fired within %lld outer iterations",
                (long long)max_outer);
  return MBDP_OK;
}

mbdp_status mdp_refine(mbdp_mdp_t h, double* V, int32_t* policy_out, int32_t K, int64_t b,
                       uint64_t seed, uint64_t first_sweep, double eps, const double* V_ref,
                       int64_t max_iters, void* workspace, size_t ws_bytes, hipStream_t stream,
                       mbdp_refine_stats* stats) {
  if (!h) return fail(MBDP_ERR_INVALID_ARG, "handle is NULL");
  if (!V) return fail(MBDP_ERR_INVALID_ARG, "V is NULL");
  if (h->vdtype != kF32)
    return fail(MBDP_ERR_UNSUPPORTED, "the FP64 correction needs a handle with FP32 values");
  if (K < 0) return fail(MBDP_ERR_INVALID_ARG, "K = %d < 0", K);
  if (b < 1 || b > h->n)
    return fail(MBDP_ERR_INVALID_ARG, "batch size b = %lld not in [1, n = %lld]", (long long)b,
                (long long)h->n);
  if (max_iters < 0) return fail(MBDP_ERR_INVALID_ARG, "max_iters must be >= 0");
  if (!(eps >= 0.0)) return fail(MBDP_ERR_INVALID_ARG, "eps must be >= 0");
  mbdp_status st = check_ws(h, workspace, ws_bytes);
  if (st != MBDP_OK) return st;
  const WsLayout w = layout(h);
  char* base = static_cast<char*>(workspace);
  KParams p = base_params(h, workspace, nullptr, b);
  p.task = kTaskRefine;
  p.vd0 = V;
  p.vd1 = reinterpret_cast<double*>(base + w.shift);  // n doubles
  // Algorithm 1 needs a policy: the caller's, or n words of the workspace
  p.policy = policy_out ? policy_out
                        : (K > 0 ? reinterpret_cast<int32_t*>(base + w.vbuf1) : nullptr);
  p.K = K;
  p.seed = seed;
  p.first_sweep = first_sweep;
  p.eps = eps;
  p.vref = V_ref;
  p.max_sweeps = max_iters;
  p.max_outer = max_iters;
  if (launch_zero(workspace, w.zero_bytes, stream) != 0)
    return fail(MBDP_ERR_HIP, "workspace clear failed: %s", hipGetErrorString(hipGetLastError()));
  char err[256] = {0};
  if (launch_refine(p, shape_of(h), stream, err, sizeof err) != 0)
    return fail(MBDP_ERR_HIP, "%s", err);
  Control c;
  st = finish(workspace, stream, &c);
  if (st != MBDP_OK) return st;
  if (stats) {
    stats->residual_in = c.residual_in;
    stats->residual_out = c.residual_out;
    stats->bound_out = c.bound_out;
    stats->final_dv_inf = c.final_dv_inf;
    stats->final_err_ref = V_ref ? c.final_err_ref : NAN;
    stats->sweeps = c.sweeps;
    stats->outer_iters = c.outer_iters;
    stats->converged = c.converged;
    stats->reserved = 0;
  }
  if (!c.converged)
    return fail(MBDP_ERR_NOT_CONVERGED, "eps not reached within %lld %s", (long long)max_iters,
                K > 0 ? "outer iterations" : "sweeps");
  return MBDP_OK;
}

}  // extern "C"
