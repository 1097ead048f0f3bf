/*
 * mbdp.h -- C-ABI of the MI355X (gfx950) randomized mini-batch Bellman
 * operator library, libmbdp.so.
 *
 * Paper: M. Gargiani, A. Martinelli, M. Ruts Martinez, J. Lygeros, "Parallel
 * and Flexible Dynamic Programming via the Randomized Mini-Batch Operator",
 * arXiv 2110.02901.  Section and equation numbers below are the paper's.
 *
 * Problem (Sec. II-A): a finite MDP with n states, m actions per state,
 * transition probabilities P(s, a, s'), stage costs c(s, a) and a discount
 * gamma in (0, 1); the goal is the minimal discounted cost J* (eq. (2)).
 * A cost of +inf marks an action that is not admissible in its state (the
 * paper's U(i)); every state needs at least one finite-cost action.  The
 * paper's batch size "m" is called b here; its "alpha" is gamma and its cost
 * vector J is V.
 *
 * Conventions for every entry point:
 *  - All arrays named as device arrays live in HBM of the current HIP device
 *    and are BORROWED: the caller allocates them, keeps them alive and does
 *    not modify them while a call that uses them may run.  The library
 *    allocates no device memory; scratch space comes from a caller-provided
 *    workspace of mdp_workspace_bytes() bytes (256-byte aligned).
 *  - Transition row r = s*m + a.  Dense P is [n][m][n] FP32, row-major, so
 *    the m rows of a state are contiguous.  Costs c are [n][m] FP32.  V is
 *    FP32[n].  Policies are int32[n] with entries in [0, m).
 *  - Arguments are checked before any device work; a bad argument returns
 *    MBDP_ERR_INVALID_ARG and touches nothing.  No entry point throws or
 *    exits.  mbdp_last_error() gives a message for the last failure on the
 *    calling thread.
 *  - A handle and a workspace are used by one stream at a time; calls that
 *    share a workspace must not overlap.
 *  - Device work runs on the given stream.  mb_sweep and mbdp_permutation
 *    are asynchronous; mdp_create_csr, mdp_validate, vi_solve and mpi_solve
 *    synchronise the stream before returning.
 */
#ifndef MBDP_H
#define MBDP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbdp_mdp* mbdp_mdp_t; /* opaque handle */

typedef enum {
  MBDP_OK = 0,
  MBDP_ERR_INVALID_ARG = 1,   /* bad size, pointer, batch size, gamma, K ... */
  MBDP_ERR_UNSUPPORTED = 2,   /* valid request the library cannot serve */
  MBDP_ERR_WORKSPACE = 3,     /* workspace missing, too small or misaligned */
  MBDP_ERR_HIP = 4,           /* a HIP runtime call failed */
  MBDP_ERR_NOT_CONVERGED = 5, /* soft: iteration limit reached, V and stats valid */
  MBDP_ERR_VALIDATION = 6,    /* mdp_validate found an invalid MDP */
  MBDP_ERR_DEVICE = 7         /* device-side error (bad explicit order, barrier timeout) */
} mbdp_status;

/* Statistics of a solve (vi_solve, mpi_solve). */
typedef struct {
  int64_t sweeps;              /* sweeps of B_b or B_{mu,b} applied */
  int64_t outer_iters;         /* MPI policy-improvement steps (0 for VI) */
  int64_t policy_changes_last; /* states whose action changed in the last improvement (-1: none) */
  int64_t recentrings;         /* number of re-centring steps */
  double final_dv_inf;         /* VI: max|V_{t+1} - V_t| of the last sweep;
                                  MPI: Bellman residual max|TV - V| of the last improvement */
  double final_err_ref;        /* max|V - V_ref| after the last sweep (NaN without V_ref) */
  int32_t converged;           /* 1 if a stopping rule fired before the limit */
  int32_t reserved;
} mbdp_stats;

/* Result of mdp_validate. */
typedef struct {
  int64_t bad_probability;     /* entries < 0, NaN or inf in P */
  int64_t bad_row_sum;         /* rows whose FP64 sum differs from 1 by more than the tolerance */
  int64_t empty_rows;          /* CSR rows without entries */
  int64_t bad_column;          /* CSR column outside [0, n) */
  int64_t bad_row_ptr;         /* CSR row_ptr not non-decreasing / inconsistent with nnz */
  int64_t bad_cost;            /* costs NaN or -inf */
  int64_t no_admissible_action;/* states whose costs are all +inf */
  double max_row_sum_dev;      /* max |sum_s' P(s,a,s') - 1| over rows */
} mbdp_validation;

/* Tuning knobs of a handle (all fields 0 = library default). */
typedef struct {
  int32_t blocks_per_cu;       /* persistent workgroups per compute unit */
  int32_t threads_per_block;   /* 256, 512 or 1024 */
  int32_t recentre_every;      /* solvers: minimum sweeps between re-centrings; -1 disables */
  int32_t recentre_force;      /* nonzero: re-centre after every recentre_every sweeps
                                  whatever the size of the change (testing) */
  int32_t band_window;         /* constant-row-length sparse MDPs whose columns stay in a
                                  band around their state: 0 stages the band of V in LDS
                                  when it fits, -1 never does (V is gathered from memory) */
} mbdp_tuning;

/* Storage types of the transition probabilities. */
typedef enum {
  MBDP_F32 = 0,      /* IEEE binary32 */
  MBDP_BF16 = 1,     /* bfloat16 codes (uint16) with one FP32 scale per row */
  MBDP_FP8_E4M3 = 2  /* OCP FP8 E4M3FN codes (uint8) with one FP32 scale per row */
} mbdp_dtype;

/* Dense MDP (P as in Sec. II-A, stored [n][m][n]).  Records the pointers;
 * does no device work.  P and c are device arrays. */
mbdp_status mdp_create_dense(int64_t n, int32_t m, const float* P, const float* c,
                             double gamma, mbdp_mdp_t* out);

/* Sparse MDP: CSR over the n*m transition rows.  row_ptr int64[n*m + 1]
 * (row_ptr[0] = 0, row_ptr[n*m] = nnz), col int32[nnz] in [0, n), val
 * FP32[nnz]; a repeated column contributes once per entry.  All are device
 * arrays.  Inspects row_ptr on the device (synchronising `stream`) to detect
 * a constant row length k, which selects a faster kernel. */
mbdp_status mdp_create_csr(int64_t n, int32_t m, const int64_t* row_ptr, const int32_t* col,
                           const float* val, int64_t nnz, const float* c, double gamma,
                           hipStream_t stream, mbdp_mdp_t* out);

/* Releases the handle (not the borrowed arrays).  NULL is a no-op. */
mbdp_status mdp_destroy(mbdp_mdp_t h);

/* Reduced-precision storage (the paper fixes no precision; this variant
 * trades accuracy for bytes per backup).  Row r of `rows` FP32 rows of
 * `row_len` entries (device, row-major, `src`) is stored as codes q_r in
 * `dst` (device; uint16 per entry for MBDP_BF16, uint8 for MBDP_FP8_E4M3)
 * and one FP32 scale in `row_scale[r]` (device) such that the stored row
 * P'(r, j) = row_scale[r] * decode(q_rj) sums to 1 (row_scale = 1 / sum_j
 * decode(q_rj), summed in FP64; 0 for a row that encodes to zeros).
 * Encoding rounds to nearest, ties to even.  FP8 rows are first multiplied
 * by the power of two 2^(7 - E), E the binary exponent of the row's largest
 * magnitude (clamped to [-100, 127]), an exact scaling that places the
 * largest entry in [128, 256); values beyond 448 saturate.  The MDP that the
 * BF16 / FP8 handles below solve is P', not the FP32 input: its solution
 * differs from the FP32 one by up to ~ gamma / (1 - gamma) times the
 * relative storage error (2^-9 BF16, 2^-4 FP8).  Asynchronous on `stream`. */
mbdp_status mdp_quantize_rows(const float* src, int64_t rows, int64_t row_len, int32_t dtype,
                              void* dst, float* row_scale, hipStream_t stream);

/* Dense MDP with P stored as BF16 / FP8 codes [n][m][n] and row scales
 * [n*m] (as written by mdp_quantize_rows).  n must be a multiple of 8
 * (BF16) or 16 (FP8), else MBDP_ERR_UNSUPPORTED.  Borrowed pointers. */
mbdp_status mdp_create_dense_q(int64_t n, int32_t m, const void* P, int32_t dtype,
                               const float* row_scale, const float* c, double gamma,
                               mbdp_mdp_t* out);

/* Sparse MDP with BF16 / FP8 values and row scales [n*m].  Needs a constant
 * row length k with k % 4 == 0 and 4 <= k <= 64 (else
 * MBDP_ERR_UNSUPPORTED); otherwise as mdp_create_csr. */
mbdp_status mdp_create_csr_q(int64_t n, int32_t m, const int64_t* row_ptr, const int32_t* col,
                             const void* val, int32_t dtype, const float* row_scale, int64_t nnz,
                             const float* c, double gamma, hipStream_t stream, mbdp_mdp_t* out);

/* Differentiation (an extension: the paper stops at J*).  For L = g^T J*
 * with a unique optimal policy mu, J* = (I - gamma P_mu)^-1 c_mu near the
 * data (eq. (4)), so with the adjoint lambda = (I - gamma P_mu)^-T g:
 *   dL/dc(s, a) = lambda(s) [a == mu(s)],
 *   dL/dP(s, a, s') = gamma lambda(s) J*(s') [a == mu(s)]
 * (partial derivatives with respect to the stored entries).  The adjoint
 * equation lambda = g + gamma P_mu^T lambda is a policy evaluation on the
 * transposed policy rows: mdp_policy_transpose writes P_mu^T as CSR arrays
 * (row_ptr_t int64[n+1], col_t int32[n*k], val_t FP32[n*k], each row in
 * increasing source state; all device, caller-allocated) and a handle made
 * from them with mdp_create_csr (m = 1, costs g, the same gamma) solves it
 * with vi_solve: the same mini-batch sweep, on the transpose.  Both calls
 * need an FP32 handle with constant row length k (else
 * MBDP_ERR_UNSUPPORTED), use the workspace of mdp_workspace_bytes(h, 1),
 * reject policy entries outside [0, m) (MBDP_ERR_INVALID_ARG) and
 * synchronise `stream`. */
mbdp_status mdp_policy_transpose(mbdp_mdp_t h, const int32_t* policy, int64_t* row_ptr_t,
                                 int32_t* col_t, float* val_t, void* workspace, size_t ws_bytes,
                                 hipStream_t stream);

/* grad_c FP64[n*m] and grad_val FP64[n*m*k] (either may be NULL) from the
 * policy, the adjoint lambda FP64[n] and J* FP64[n] by the formulas above;
 * entries of rows that mu does not select get 0. */
mbdp_status mdp_value_gradients(mbdp_mdp_t h, const int32_t* policy, const double* lambda,
                                const double* V, double* grad_c, double* grad_val,
                                void* workspace, size_t ws_bytes, hipStream_t stream);

/* Batching (an extension: many independent dense MDPs of uneven size in
 * one launch).  Each MDP is solved by MB-VI (Sec. III-B) on one workgroup:
 * its own sweep orders (seed), batch size b and stop rule, V in LDS, FP64
 * arithmetic on FP32 / BF16 / FP8 rows (decoded exactly), so its iterates
 * are the FP64 MB-VI iterates of the stored MDP.  Workgroups take MDPs from
 * a queue, heaviest first.  An MDP much heavier than the rest (bytes per
 * sweep times the sweeps its gamma needs, against the total over the
 * device's compute units) is served by a team of workgroups that split each
 * batch and exchange its new values through device memory; the iterates are
 * the same.  The members of all teams together must fit on the device at
 * once (one workgroup per compute unit). */
typedef struct {
  int64_t n;              /* states, 1 <= n <= 8192 */
  int32_t m;              /* actions, 1 <= m <= 64 */
  int32_t dtype;          /* MBDP_F32, MBDP_BF16 or MBDP_FP8_E4M3 */
  int64_t ld;             /* row stride of P in values: >= n, <= 8192, a multiple of 16 */
  const void* P;          /* device, [n][m][ld], 16-byte aligned, padding columns zero */
  const float* row_scale; /* device [n*m] (BF16 / FP8; see mdp_quantize_rows), else NULL */
  const float* c;         /* device [n][m] */
  double gamma;           /* in (0, 1) */
  int64_t b;              /* batch size, 1 <= b <= min(n, 4096) */
  uint64_t seed;          /* sweep orders sigma_t of this MDP */
  double* V;              /* device [n]: V0 in, the last iterate out */
  int32_t* policy;        /* device [n]: greedy policy at the last iterate, or NULL */
  int32_t lanes;          /* lanes per state: 16, 32 or 64; 0 picks by row length */
  int32_t team;           /* workgroups serving the MDP, 1..16; 0 picks by work */
} mbdp_batch_item;

typedef struct {
  int64_t sweeps;
  double final_dv_inf;    /* max |dV| of the last sweep */
  int32_t converged;      /* final_dv_inf <= tol_dv */
  int32_t team;           /* workgroups that served the MDP */
  double start_us;        /* when its solve started and ended, in microseconds */
  double end_us;          /* after the earliest start of the launch (device clock) */
} mbdp_batch_stats;

/* Workspace bytes of a batch of `count` MDPs (0 if count < 1). */
size_t mdp_batch_workspace_bytes(int32_t count);

/* Checks the items, sizes the teams for the current device and writes the
 * item table (teams first, then by work per workgroup, heaviest first) into
 * the workspace; synchronises `stream`.  Explicit team sizes that do not fit
 * on the device give MBDP_ERR_UNSUPPORTED; automatic ones are reduced.
 * Pointers are borrowed until the last launch using them has finished. */
mbdp_status mdp_batch_upload(const mbdp_batch_item* items, int32_t count, void* workspace,
                             size_t ws_bytes, hipStream_t stream);

/* Runs every uploaded MDP to max |dV| <= tol_dv or max_sweeps sweeps.
 * Enqueues kernels only (no copies, no synchronisation, no allocation), so
 * it can be captured in a hipGraph and replayed; V is read at the start of
 * each launch. */
mbdp_status mdp_batch_launch(int32_t count, double tol_dv, int64_t max_sweeps, void* workspace,
                             size_t ws_bytes, hipStream_t stream);

/* Statistics of the last launch, in the order of the uploaded items;
 * synchronises `stream`.  MBDP_ERR_DEVICE if a team barrier gave up (a team
 * member did not arrive within 60 s; the launch then stops early and the
 * statistics are incomplete). */
mbdp_status mdp_batch_read_stats(void* workspace, int32_t count, mbdp_batch_stats* out,
                                 hipStream_t stream);

/* Several value vectors against one P (an extension): r cost vectors
 * C[:, :, j] share the handle's transition probabilities, gamma, the batch
 * size b and the sweep orders sigma_t; V[:, j] follows MB-VI (Sec. III-B,
 * eqs. (10)-(12)) of the MDP with costs C[:, :, j] (the handle's own costs
 * are not used).  For one batch the expected values of all r vectors are
 * one matrix product (the batch's rows of P against V), run on the matrix
 * cores.  V is held as an FP64 anchor plus a small difference that goes
 * through the products as two BF16 terms; the anchor is refreshed (an FP64
 * pass over P) whenever the products' error bound would reach a twentieth
 * of the last sweep's change, so the iterates follow the FP64 ones. */
typedef struct {
  int64_t sweeps;        /* sweeps applied */
  double final_dv_inf;   /* max over vectors and states of |dV| in the last sweep */
  int64_t recentrings;   /* anchor refreshes after the start */
  int32_t converged;     /* final_dv_inf <= tol_dv */
  int32_t reserved;
} mbdp_multi_stats;

/* Workspace bytes of mdp_multi_solve for this handle, r and b (0 if the
 * handle is not dense BF16 with n % 32 == 0, r is not 16, 32, 48 or 64, or b
 * is not in [1, n]). */
size_t mdp_multi_workspace_bytes(mbdp_mdp_t h, int32_t r, int64_t b);

/* MB-VI on r vectors at once.  C: device FP32 [n][m][r]; V: device FP64
 * [n][r], V0 in, the last iterate out; policy: device int32 [n][r], the
 * greedy actions at the last iterate (lowest index on ties), or NULL.  Sweep
 * t (t = first_sweep, first_sweep + 1, ...) uses sigma_t of `seed`.  Stops
 * after the first sweep with max |dV| <= tol_dv (over all vectors; tol_dv < 0
 * disables the rule) or after max_sweeps; MBDP_ERR_NOT_CONVERGED (soft) when
 * the limit was reached with tol_dv >= 0.  Needs a dense BF16 handle
 * (mdp_create_dense_q) with n % 32 == 0 and r in {16, 32, 48, 64};
 * synchronises `stream`. */
mbdp_status mdp_multi_solve(mbdp_mdp_t h, int32_t r, const float* C, double* V, int32_t* policy,
                            int64_t b, uint64_t seed, uint64_t first_sweep, double tol_dv,
                            int64_t max_sweeps, void* workspace, size_t ws_bytes,
                            hipStream_t stream, mbdp_multi_stats* stats);

/* Column-sorted blocks for b = n (an MI355X layout; the method is unchanged).
 * With b = n the whole state set is one batch that reads only the values
 * from before it (eq. (11) with an empty updated set: the Bellman operator T,
 * eq. (7)), so a backup's products may be summed in any order.  For a
 * constant-row-length FP32 MDP with n <= 2^20 states (and m <= 4096) the
 * library can keep a second copy of the entries, grouped by blocks of at
 * most 4096 / m states (fewer, down to half that, so that the blocks fill
 * whole passes of the device's compute units, 8 blocks to a compute unit)
 * and sorted by column inside each block, packed into groups
 * of 64 entries with distinct rows (padding entries have value 0): the V
 * gathers of a wavefront then fall on a few cache lines instead of 64, and
 * the products are summed in LDS without atomics.  Solves and sweeps with
 * b = n (min and improvement passes) then run the "ell-colblock" kernel;
 * policy sweeps and b < n keep the row-major kernels.  The sums are
 * grouped differently from the row-major kernels (FP32 rounding differs;
 * results are deterministic).
 * mdp_column_blocks_prepare copies col / val to the host, builds the layout
 * on host threads and returns in *bytes the device buffer it needs (about
 * 8 bytes per entry); synchronises `stream`.  mdp_column_blocks_attach
 * copies it into `buffer` (device, 256-byte aligned, at least *bytes,
 * borrowed like the other arrays) and releases the host copy; synchronises
 * `stream`.  MBDP_ERR_UNSUPPORTED for other MDPs. */
mbdp_status mdp_column_blocks_prepare(mbdp_mdp_t h, hipStream_t stream, size_t* bytes);
mbdp_status mdp_column_blocks_attach(mbdp_mdp_t h, void* buffer, size_t bytes,
                                     hipStream_t stream);

/* Replaces the handle's tuning knobs. */
mbdp_status mdp_set_tuning(mbdp_mdp_t h, const mbdp_tuning* t);

/* Workspace bytes that mb_sweep, vi_solve, mpi_solve and mdp_validate need
 * for this handle with batch size b (0 on a bad handle or batch size). */
size_t mdp_workspace_bytes(mbdp_mdp_t h, int64_t b);

/* Name of the kernel family that mb_sweep (without an explicit order),
 * vi_solve and mpi_solve run for this handle and batch size b: "dense",
 * "ell" (constant row length, V gathered from memory), "ell-band" (constant
 * row length with every column within a band around its state: each
 * workgroup owns a chunk of states and stages the band of V it reads in
 * LDS), "ell-colblock" (b = n with column blocks attached) or "csr".  The choice follows the handle's tuning.  *name points to
 * a static string.  No device work. */
mbdp_status mdp_engine(mbdp_mdp_t h, int64_t b, const char** name);

/* Optional input checks: P entries in [0, inf), FP64 row sums within
 * row_sum_tol of 1, CSR structure, costs not NaN/-inf and at least one
 * finite cost per state.  Fills *report (may be NULL) and returns MBDP_OK
 * or MBDP_ERR_VALIDATION.  Synchronises `stream`. */
mbdp_status mdp_validate(mbdp_mdp_t h, double row_sum_tol, void* workspace, size_t ws_bytes,
                         hipStream_t stream, mbdp_validation* report);

/* The sweep order sigma_t of the states (Sec. III-A processes states in a
 * random order, re-drawn every sweep; Sec. IV-A shuffles before every
 * operator evaluation): out[p] = state processed at position p of sweep
 * `sweep_index` under `seed`, for p in [0, n).  out is a device int32[n].
 * The order is a 4-round Feistel network on [0, 4^h) (h the smallest h >= 1
 * with 4^h >= n) whose round function j maps R to word 0 of
 * Philox-4x32-10(counter = (R, j, t_lo, t_hi), key = (seed_lo, seed_hi))
 * masked to h bits, restricted to [0, n) by cycle walking. */
mbdp_status mbdp_permutation(int64_t n, uint64_t seed, uint64_t sweep_index, int32_t* out,
                             hipStream_t stream);

/* One sweep of the mini-batch operator, eqs. (10)-(12).  The states are
 * processed in the order sigma_t (t = sweep_index), or in the explicit order
 * perm (device int32[n], a permutation of [0, n)) when perm != NULL, cut into
 * consecutive batches of b (the last batch may be shorter).  Each state of a
 * batch reads the new values of earlier batches and the old values of its
 * own and later batches; the batch is committed after all its reads.
 *   policy == NULL: B_b,      V(s) <- min_a [c(s,a) + gamma sum_s' P(s,a,s') V(s')]
 *   policy != NULL: B_{mu,b}, V(s) <- c(s,mu(s)) + gamma sum_s' P(s,mu(s),s') V(s')
 * 1 <= b <= n; b = n is the Bellman operator T (eq. (7)) and b = 1 the
 * Gauss-Seidel operator F (Sec. II-D).  V (device FP32[n]) is updated in
 * place.  argmin_out (device int32[n], may be NULL) receives the lowest
 * minimising action (or mu(s)).  dv_out (device float[1], may be NULL)
 * receives max_s |V_new(s) - V_old(s)|.  Dot products accumulate in FP32;
 * the cost is added and the minimum taken in FP64, then rounded to FP32.
 * Asynchronous; device-side errors (an out-of-range perm entry) are
 * reported by mbdp_sync_status. */
mbdp_status mb_sweep(mbdp_mdp_t h, float* V, const int32_t* policy, int64_t b, uint64_t seed,
                     uint64_t sweep_index, const int32_t* perm, int32_t* argmin_out,
                     float* dv_out, void* workspace, size_t ws_bytes, hipStream_t stream);

/* Synchronises `stream` and returns the device-side status recorded in
 * `workspace` by the last mb_sweep/vi_solve/mpi_solve that used it. */
mbdp_status mbdp_sync_status(void* workspace, size_t ws_bytes, hipStream_t stream);

/* MB-VI (Sec. III-B): from the caller's V (the paper starts at 0, Sec.
 * IV-A), apply sweeps t = first_sweep, first_sweep + 1, ... of B_b with
 * order sigma_t until max|V_{t+1} - V_t| <= tol_dv (tol_dv < 0 disables),
 * or -- when V_ref (device FP64[n]) is given -- max|V_{t+1} - V_ref| <= eps,
 * or max_sweeps sweeps.  All sweeps run in one persistent kernel launch
 * with a device-wide barrier between batches.
 * Precision: the iterate is kept as V = W + R with W in FP32 and an FP64
 * anchor R, iterating W with the costs c(s,a) - R(s) + gamma (P R)(s,a);
 * this is exact in real arithmetic for any order and batch size.  Whenever
 * a sweep changes W by less than 2^-14 of its magnitude, W is folded into R
 * (one extra pass over P), so FP32 resolves the remaining error rather than
 * |V|.  By the contraction property (Sec. III-B), max|V_{t+1} - V_t| <= tol
 * implies max|V_{t+1} - J*| <= tol * gamma / (1 - gamma).
 * On return V holds the last iterate in FP32, V64_out (device FP64[n], may
 * be NULL) the same iterate W + R in FP64, and policy_out (device int32[n],
 * may be NULL) the greedy policy at V (lowest index on ties).  stats may be
 * NULL.  Returns MBDP_ERR_NOT_CONVERGED when the limit was reached. */
mbdp_status vi_solve(mbdp_mdp_t h, float* V, double* V64_out, int32_t* policy_out, int64_t b,
                     uint64_t seed, uint64_t first_sweep, double tol_dv, double eps,
                     const double* V_ref, int64_t max_sweeps, void* workspace, size_t ws_bytes,
                     hipStream_t stream, mbdp_stats* stats);

/* vi_solve for callers that cannot allocate memory or pass a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same solve, the same arguments except the workspace,
 * and the same results, bit for bit.  Its scratch memory is a file-scope
 * device array of the library, 32 MiB on each device it runs on, held until
 * the process ends; its address is looked up once per device (with that
 * device current).  The call allocates nothing.  MDPs whose workspace
 * (mdp_workspace_bytes) exceeds 32 MiB are rejected with
 * MBDP_ERR_INVALID_ARG (dense n = 8192, m = 16 needs about 2.3 MB; sparse
 * MDPs with k = 32, m = 8 up to about 300 000 states fit).  The handle's
 * device must be current.  Every call on a device shares that device's
 * array, which keeps the last call's contents (the control words are
 * cleared at the start of each call): calls that overlap on one device --
 * on different streams or from different threads -- race and must not be
 * made.  Synchronises `stream`. */
mbdp_status vi_solve_noalloc(mbdp_mdp_t h, float* V, double* V64_out, int32_t* policy_out,
                             int64_t b, uint64_t seed, uint64_t first_sweep, double tol_dv,
                             double eps, const double* V_ref, int64_t max_sweeps,
                             hipStream_t stream, mbdp_stats* stats);

/* MB-MPI: Algorithm 1 with its K policy-evaluation steps done by B_{mu,b}
 * (warm start from the current V).  policy (device int32[n]) is the initial
 * policy when policy_is_init != 0; otherwise the initial policy is the
 * greedy policy at the caller's V.  Each outer iteration runs K sweeps of
 * B_{mu,b} (orders sigma_t, t counting evaluation sweeps from first_sweep)
 * and then the improvement step over all states (V fixed).  Stops when an
 * improvement changes no action and the Bellman residual max|TV - V| is
 * <= tol_dv, or -- with V_ref -- after the first evaluation sweep with
 * max|V - V_ref| <= eps, or after max_outer outer iterations.  Precision
 * and V64_out as for vi_solve.  On return V and policy hold the last
 * iterate. */
mbdp_status mpi_solve(mbdp_mdp_t h, float* V, double* V64_out, int32_t* policy,
                      int32_t policy_is_init, int32_t K, int64_t b, uint64_t seed,
                      uint64_t first_sweep, double tol_dv, double eps, const double* V_ref,
                      int64_t max_outer, void* workspace, size_t ws_bytes, hipStream_t stream,
                      mbdp_stats* stats);

/* Certified FP64 correction (an extension: the paper fixes no precision).
 * Typical use: V is the solution of a reduced-precision copy of this MDP
 * (mdp_create_dense_q / mdp_create_csr_q), which differs from this MDP's J*
 * by the storage error; the correction brings it to within eps of this
 * MDP's J*, with a certificate.  Everything is FP64 on the GPU: V, the
 * accumulation of every dot product with the handle's FP32 transition
 * values (widened exactly), costs, minima and tests.
 * The certificate is the contraction property (Sec. III-B): every B_{sigma,b}
 * of eq. (11), like T of eq. (7), is a gamma-contraction in the max norm
 * with fixed point J*, so max|V - J*| <= max|TV - V| / (1 - gamma), and a
 * sweep V' = B V gives max|V' - J*| <= min(gamma max|V' - V| / (1 - gamma),
 * gamma max|V - J*|) (bounds of exact arithmetic).
 * Steps: one pass of eq. (7) over all states at the input gives its residual
 * max|TV - V|.  Then
 *   K = 0:  sweeps t = first_sweep, first_sweep + 1, ... of B_{sigma_t,b}
 *           until the chained bound above is <= eps (max_iters sweeps at
 *           most);
 *   K >= 1: Algorithm 1: K sweeps of B_{mu,sigma_t,b} with mu the greedy
 *           policy of the last improvement step, then the improvement step
 *           (a pass of eq. (7), V fixed), until an improvement step's
 *           residual / (1 - gamma) is <= eps (max_iters improvement steps
 *           at most).
 * The input itself is returned unchanged when its residual certifies eps.
 * With V_ref (device FP64[n]) the stop is instead the first V (the input or
 * a sweep's result) with max|V - V_ref| <= eps (measurement mode).
 * V: device FP64[n], in and out.  policy_out: device int32[n], the greedy
 * policy at the output (lowest index on ties), or NULL.  The handle must
 * hold FP32 values (MBDP_ERR_UNSUPPORTED otherwise); the workspace is that
 * of mdp_workspace_bytes(h, b).  Synchronises `stream`.  Returns
 * MBDP_ERR_NOT_CONVERGED (soft) when the limit was reached. */
typedef struct {
  double residual_in;   /* max|TV - V| at the input */
  double residual_out;  /* max|TV - V| at the output; NaN when not evaluated
                           (K = 0 without policy_out after at least one sweep) */
  double bound_out;     /* certified bound on max|V - J*| at the output:
                           K = 0 the chained sweep bound, K >= 1 residual_out / (1 - gamma) */
  double final_dv_inf;  /* max|V_t - V_{t-1}| of the last sweep (NaN if none) */
  double final_err_ref; /* max|V - V_ref| at the output (NaN without V_ref) */
  int64_t sweeps;       /* sweeps applied */
  int64_t outer_iters;  /* K >= 1: improvement steps after the input's */
  int32_t converged;    /* 1 if the stopping rule fired */
  int32_t reserved;
} mbdp_refine_stats;

mbdp_status mdp_refine(mbdp_mdp_t h, double* V, int32_t* policy_out, int32_t K, int64_t b,
                       uint64_t seed, uint64_t first_sweep, double eps, const double* V_ref,
                       int64_t max_iters, void* workspace, size_t ws_bytes, hipStream_t stream,
                       mbdp_refine_stats* stats);

/* Message of the last failed call on this thread ("" if none). */
const char* mbdp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MBDP_H */
