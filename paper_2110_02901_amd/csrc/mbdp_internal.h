// Internal definitions shared by the HIP kernels and the host runtime of
// libmbdp.so.  Not part of the public C-ABI (include/mbdp.h).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace mbdp {

enum Storage : int32_t { kDense = 0, kEll = 1, kCsr = 2 };
// Storage of transition probabilities (values of mbdp_dtype in include/mbdp.h).
enum ValueType : int32_t { kF32 = 0, kBF16 = 1, kFP8 = 2 };
enum Task : int32_t { kTaskSweep = 0, kTaskVI = 1, kTaskMPI = 2, kTaskRefine = 3 };

// Device-side error codes recorded in Control::error.
enum DeviceError : uint32_t {
  kDevOk = 0,
  kDevBadPerm = 1,        // explicit order entry outside [0, n)
  kDevBarrierTimeout = 2, // a grid barrier waited longer than the limit
  kDevBadPolicy = 3,      // policy entry outside [0, m)
};

// Accumulators of one epoch (a sweep or an improvement pass).  Doubles are
// kept as order-preserving 64-bit keys so that atomic max/min on unsigned
// integers give the max/min of the values.
enum Acc : int {
  kAccDv = 0,      // max |W_new - W_old| (non-negative double bits)
  kAccErr = 1,     // max |W_new + r - V_ref|
  kAccWmax = 2,    // max W_new (ordered key)
  kAccWmin = 3,    // min W_new (ordered key)
  kAccChanges = 4, // policy changes (count)
  kAccResid = 5,   // max |TW - W| (non-negative double bits)
  kNumAcc = 6
};

constexpr int kMaxBlocks = 4096;  // persistent workgroups per launch (arrival slots)

struct alignas(256) Control {
  unsigned long long bar_release;  // last barrier generation released by workgroup 0
  unsigned long long pad0[31];
  unsigned int abort;            // nonzero: every workgroup leaves
  unsigned int error;            // DeviceError
  unsigned long long pad1[31];
  unsigned long long acc[3][16]; // rotating epoch accumulators, kNumAcc used
  // results written by workgroup 0 at the end of a launch
  long long sweeps;
  long long outer_iters;
  long long policy_changes_last;
  long long recentrings;
  double final_dv_inf;
  double final_err_ref;
  int converged;
  int pad2;
  float dv_last;                 // last sweep's max |dV| as FP32 (mb_sweep)
  float pad3;
  double residual_in;            // FP64 correction: max |TV - V| of the input
  double residual_out;           // FP64 correction: max |TV - V| of the output (NaN: not evaluated)
  double bound_out;              // FP64 correction: certified bound on max |V - J*|
  unsigned long long bar_slots[kMaxBlocks] __attribute__((aligned(256)));  // arrival generations
};

struct KParams {
  // the MDP
  int32_t storage;
  int32_t m;
  int64_t n;
  double gamma;
  const float* P;          // dense [n][m][n] (FP32 storage)
  const int64_t* row_ptr;  // CSR
  const int32_t* col;
  const float* val;
  int32_t ell_k;           // constant row length (kEll), else 0
  int32_t band;            // kEll: max |s' - s| over the entries of state s's rows; -1 unknown or off
  int32_t vdtype;          // storage of the transition values: kF32, kBF16, kFP8
  int32_t pad3;
  const void* pq;          // BF16 / FP8 values: dense [n][m][n], or ELL [nnz]
  const float* rscale;     // BF16 / FP8: per-row scale, P(r, j) = rscale[r] * decode(q_rj)
  const float* c32;        // plain costs [n*m]
  double* ceff;            // shifted costs [n*m] (solvers), workspace
  double* shift;           // FP64 anchor R[n] with V = W + R (solvers), workspace
  double* tgt;             // V_ref - R [n] (solvers; zeros without a reference), workspace
  double* v64_out;         // optional FP64 copy of the final V
  // vectors
  float* vbuf0;            // caller's V
  float* vbuf1;            // ping-pong partner, workspace
  double* vd0;             // FP64 correction: caller's V
  double* vd1;             // FP64 correction: ping-pong partner, workspace
  int32_t* policy;         // B_{mu,b} policy in; improvement out
  int32_t* argmin_out;
  const int32_t* perm;     // explicit order or null
  const double* vref;       // FP64 reference values (measurement mode)
  // schedule
  int32_t task;
  int32_t policy_sweep;    // mb_sweep with a policy
  int64_t b;
  uint64_t seed;
  uint64_t first_sweep;
  int64_t max_sweeps;      // VI
  int64_t max_outer;       // MPI
  int32_t K;               // MPI evaluation sweeps
  int32_t policy_is_init;  // MPI
  int32_t recentre_every;  // 0: plain costs, no anchor; else min sweeps between re-centrings
  int32_t want_policy_out; // VI: greedy policy at the end into `policy`
  int32_t recentre_force;  // re-centre after every sweep (respecting recentre_every)
  int32_t pad2;
  double tol_dv;
  double eps;
  // decomposition
  int32_t splits;          // dense: workgroups per state when b is small
  int32_t pad1;
  // workspace
  Control* ctl;
  int32_t* order;          // [3][n] sweep orders, by sweep index mod 3
  uint32_t* first_mark;    // [2][n] stamp (t + 1) of the states in batch 0 of sweep t, by t % 2 (cleared per launch)
  float* partial;          // dense split partial sums
  unsigned int* unit_count;// dense split arrival counters
  unsigned long long timeout_ticks;
  // column-sorted blocks of a constant-row-length FP32 MDP (b = n), or null
  const uint32_t* cb_keys;  // [groups * 64]: column << 12 | row within the block
  const float* cb_vals;     // [groups * 64]
  const int32_t* cb_gptr;   // [blocks + 1]: first group of each block
  int64_t cb_states;        // states per block
};

// Workspace layout, shared by the size query and the launches.
struct WsLayout {
  size_t ctl, unit_count, partial, order, first_mark, vbuf1, ceff, shift, tgt, total;
  size_t zero_bytes;  // prefix cleared before every launch (control + counters)
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// max_units bounds the (state, split) units of one dense batch: b * splits
// < b + blocks <= n + max_blocks.
inline WsLayout ws_layout(int32_t storage, int64_t n, int32_t m, int64_t max_units) {
  WsLayout w{};
  size_t off = 0;
  // cleared before every launch: control block, split counters, first-batch stamps
  w.ctl = off;        off = align_up(off + sizeof(Control), 256);
  w.unit_count = off;
  if (storage == kDense) off = align_up(off + (size_t)max_units * sizeof(unsigned int), 256);
  w.first_mark = off; off = align_up(off + 2 * (size_t)n * sizeof(uint32_t), 256);
  w.zero_bytes = off;
  w.partial = off;
  if (storage == kDense) off = align_up(off + (size_t)max_units * (size_t)m * sizeof(float), 256);
  w.order = off;      off = align_up(off + 3 * (size_t)n * sizeof(int32_t), 256);
  w.vbuf1 = off;      off = align_up(off + (size_t)n * sizeof(float), 256);
  w.ceff = off;       off = align_up(off + (size_t)n * (size_t)m * sizeof(double), 256);
  w.shift = off;      off = align_up(off + (size_t)n * sizeof(double), 256);
  w.tgt = off;        off = align_up(off + (size_t)n * sizeof(double), 256);
  w.total = off;
  return w;
}

// Launch entry points implemented in mbdp_kernels.hip.
struct LaunchShape {
  int cus;            // compute units of the device
  int blocks_per_cu;  // requested persistent workgroups per CU (clamped to occupancy)
  int threads;        // threads per workgroup
};

constexpr int kMaxBlocksPerCu = 16;

// Kernel families a launch can run.
enum Engine : int { kEngineDense = 0, kEngineEll = 1, kEngineBand = 2, kEngineCsr = 3,
                     kEngineCol = 4 };
constexpr int kColThreads = 512;  // threads of a column-block launch (8 wavefronts)
constexpr int kColRows = 4096;    // rows per column block (the 12-bit row field of a key)
constexpr int kColGroup = 64;     // entries per group (one per lane of a wavefront)

// Fills p.splits from the grid actually used and launches the persistent
// kernel cooperatively.  Returns 0 or -1 with a message in err.
int launch_solve(KParams p, LaunchShape shape, void* stream, char* err, size_t errlen);
// The FP64 correction kernel (mbdp_refine.hip) for an FP32 handle; the same
// contract as launch_solve.
int launch_refine(KParams p, LaunchShape shape, void* stream, char* err, size_t errlen);
// The kernel family launch_solve would run for p (no device work).
int query_engine(const KParams& p, LaunchShape shape, int* engine, char* err, size_t errlen);
int launch_zero(void* ptr, size_t bytes, void* stream);
int launch_permutation(int64_t n, uint64_t seed, uint64_t t, int32_t* out, void* stream);
int launch_csr_inspect(const int64_t* row_ptr, const int32_t* col, int64_t rows, int64_t n,
                       int64_t nnz, int64_t k, unsigned long long* flags, void* stream);
int launch_validate(const KParams& p, double tol, unsigned long long* out, void* stream);
int launch_quantize(const float* src, int64_t rows, int64_t row_len, int32_t dtype, void* dst,
                    float* row_scale, void* stream);
// scratch: (64 + 2 n) words, zeroed; scratch[0] counts bad policy entries
int launch_policy_transpose(const KParams& p, const int32_t* policy, int64_t* row_ptr_t,
                            int32_t* col_t, float* val_t, unsigned* scratch, void* stream);
int launch_value_gradients(const KParams& p, const int32_t* policy, const double* lambda,
                           const double* V, double* grad_c, double* grad_val, unsigned* flags,
                           void* stream);

// Many small dense MDPs solved in one launch (mbdp_batch.hip): a workgroup
// (or a team of up to kBatchMaxTeam workgroups) per MDP, V in LDS, FP64
// arithmetic.
constexpr int64_t kBatchMaxN = 8192;  // states (and row stride) per MDP
constexpr int64_t kBatchMaxB = 4096;  // batch size per MDP
constexpr int32_t kBatchMaxM = 64;    // actions per MDP
constexpr int32_t kBatchMaxTeam = 16; // workgroups per MDP
constexpr int32_t kBatchTeamSlots = 256;  // MDPs served by a team at once

struct BatchItem {
  int64_t n, ld, b;
  int32_t m, dtype;
  const void* P;
  const float* rscale;
  const float* c;
  double gamma;
  uint64_t seed;
  double* V;
  int32_t* policy;
  int32_t lanes;   // lanes per state: 16, 32 or 64
  int32_t index;   // position in the caller's list (results go there)
  int32_t team;    // workgroups serving the MDP
  int32_t slot;    // team slot (teams only)
  int64_t ticket0; // first queue ticket of the MDP; tickets [ticket0, ticket0 + team)
};

struct BatchStat {
  long long sweeps;
  double dv;
  int converged;
  int pad;
  unsigned long long t_start, t_end;  // device wall clock when the solve started / ended
};

// Control words of a batched launch (cleared per launch): the ticket
// counter, the abort flag raised by a team barrier that timed out, and one
// barrier arrival counter per team slot.
struct BatchControl {
  unsigned queue;
  unsigned abort;
  unsigned pad[14];
  unsigned long long arrive[kBatchTeamSlots];
};

inline int32_t batch_team_slots(int32_t count) {
  return count < kBatchTeamSlots ? count : kBatchTeamSlots;
}

// Workspace of a batched solve: control words, the item table, the
// statistics, and per team slot the members' sweep maxima [2][kBatchMaxTeam]
// and the new values of a batch [2][kBatchMaxB] (both by parity).
struct BatchLayout {
  size_t control, items, stats, team_dv, team_new, total;
};
inline BatchLayout batch_layout(int32_t count) {
  BatchLayout l{};
  const size_t slots = (size_t)batch_team_slots(count);
  size_t off = 0;
  l.control = off;  off = align_up(off + sizeof(BatchControl), 256);
  l.items = off;    off = align_up(off + (size_t)count * sizeof(BatchItem), 256);
  l.stats = off;    off = align_up(off + (size_t)count * sizeof(BatchStat), 256);
  l.team_dv = off;  off = align_up(off + slots * 2 * kBatchMaxTeam * sizeof(double), 256);
  l.team_new = off; off = align_up(off + slots * 2 * (size_t)kBatchMaxB * sizeof(double), 256);
  l.total = off;
  return l;
}

struct BatchArgs {
  const BatchItem* items;
  int count;
  BatchControl* ctl;
  BatchStat* stats;
  double* team_dv;
  double* team_new;
  double tol;
  long long max_sweeps;
  unsigned long long timeout_ticks;  // a team barrier gives up after this many wall-clock ticks
};

int launch_batch(const BatchArgs& a, int blocks, void* stream);

// Several value vectors against one dense BF16 P (mbdp_multi.hip).
constexpr int32_t kMultiMaxR = 64;

struct MultiControl {
  double dv_last;              // max |dV| of the last completed sweep
  double w_bound;              // sum of the sweeps' max |dV| since the last re-centring (>= max |W|)
  long long sweeps;            // sweeps completed
  unsigned done;               // a sweep met the stop rule: the sweep kernels return at once
  unsigned pad[7];
};

struct MultiArgs {
  int64_t n;
  int32_t m, r;
  double gamma;
  int64_t b;
  uint64_t seed;
  double tol;
  const uint16_t* P;     // BF16 codes [n][m][n]
  const float* rscale;   // [n * m]
  const float* C;        // [n][m][r]
  double* R;             // anchor [n][r]
  double* W;             // V - R [n][r]
  uint16_t* Ws;          // W as two BF16 terms [2][r][n]
  double* PR;            // scale * codes . R per row [n * m][r]
  float* part;           // partial products [splits][part_rows][r]
  int64_t part_rows;     // b * m
  int64_t kchunk;        // K per split, a multiple of 32
  int32_t splits;
  int32_t* policy;       // [n][r] or null
  double* dvs;           // [n] max |dV| over the vectors per position of the sweep
  int32_t* order;        // [n] sigma_t of the sweep being run, written at its start
  MultiControl* ctl;
};

// rows of P per wavefront of the product kernel: 16 per 16 vectors
inline int64_t multi_rows_per_wave(int32_t r) { return r; }

struct MultiLayout {
  size_t ctl, R, W, Ws, PR, part, dvs, order, total;
  int64_t kchunk;
  int32_t splits;
};
// Split K so that a batch's product runs on about 2048 wavefronts (measured
// against 1024 and 4096 on the dense 8192 x 16 workload).
inline MultiLayout multi_layout(int64_t n, int32_t m, int32_t r, int64_t b) {
  MultiLayout l{};
  const int64_t tiles = (b * m + multi_rows_per_wave(r) - 1) / multi_rows_per_wave(r);
  int64_t splits = (2048 + tiles - 1) / tiles;
  const int64_t max_splits = n / 256 > 0 ? n / 256 : 1;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  l.kchunk = ((n + splits - 1) / splits + 31) / 32 * 32;
  l.splits = (int32_t)((n + l.kchunk - 1) / l.kchunk);
  size_t off = 0;
  l.ctl = off;  off = align_up(off + sizeof(MultiControl), 256);
  l.R = off;    off = align_up(off + (size_t)n * r * sizeof(double), 256);
  l.W = off;    off = align_up(off + (size_t)n * r * sizeof(double), 256);
  l.Ws = off;   off = align_up(off + 2 * (size_t)r * n * sizeof(uint16_t), 256);
  l.PR = off;   off = align_up(off + (size_t)n * m * r * sizeof(double), 256);
  l.part = off; off = align_up(off + (size_t)l.splits * b * m * r * sizeof(float), 256);
  l.dvs = off;  off = align_up(off + (size_t)n * sizeof(double), 256);
  l.order = off; off = align_up(off + (size_t)n * sizeof(int32_t), 256);
  l.total = off;
  return l;
}

int launch_multi_gemm(const MultiArgs& a, uint64_t t, int64_t k, int full, void* stream);
int launch_multi_commit(const MultiArgs& a, uint64_t t, int64_t k, int mode, void* stream);
int launch_multi_end(const MultiArgs& a, void* stream);
int launch_multi_order(const MultiArgs& a, uint64_t t, void* stream);
int launch_multi_anchor(const MultiArgs& a, double* V, int mode, void* stream);
int launch_multi_pr(const MultiArgs& a, void* stream);

// BF16 / FP8 instantiations (mbdp_kernels_lp_*.hip): null when the shape has
// none (ELL rows of more than 64 entries).
typedef void (*SolveFn)(KParams);
SolveFn pick_dense_lp(const KParams& p);
SolveFn pick_ell_lp(const KParams& p, int units_per_wave_hint);
SolveFn pick_band_lp(const KParams& p, int units_per_wave_hint);

}  // namespace mbdp
