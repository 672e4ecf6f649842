/*
 * rlgl.h - C ABI of the MI355X (gfx950) Red-Light-Green-Light solver.
 *
 * The method is the one of Avrachenkov, Brown and Litvak, "Red Light Green
 * Light Method for Solving Large Markov Chains" (J. Sci. Comput. 93:18, 2022):
 * every state i holds cash C_i; at step t a green-light set G_t moves its
 * cash along the transition matrix P, the moved cash accumulates in the
 * history H, and pi_hat_t = H_t / (H_t 1) estimates the stationary
 * distribution pi* = pi* P (Sec. 2.1, eqs. (1)-(6), Algorithm 1).
 *
 * Conventions for every call
 *   - Graph arrays, the workspace and the output vector are DEVICE pointers
 *     owned by the caller; they must stay alive until rlgl_destroy.  The
 *     library allocates no device memory and frees nothing it did not create.
 *     It allocates a small host-side context only.
 *   - All device work is enqueued on the caller's hipStream_t given to
 *     rlgl_create.  rlgl_step/rlgl_solve/rlgl_get_state return after the work
 *     they enqueued has finished and the host-visible results are final.
 *   - Calls on one context must not overlap (one host thread at a time).
 *     Distinct contexts are independent.
 *   - Errors are reported through the return code; rlgl_last_error() gives a
 *     human-readable message for the calling thread.  No C++ exception
 *     crosses this interface.
 */
#ifndef RLGL_H
#define RLGL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlgl_ctx rlgl_ctx;

typedef enum {
  RLGL_OK = 0,
  RLGL_EINVAL = -1,          /* bad argument; nothing was enqueued */
  RLGL_ENOMEM = -2,          /* workspace smaller than rlgl_workspace_bytes() or host allocation failed */
  RLGL_EHIP = -3,            /* a HIP runtime call failed */
  RLGL_EZERO_HISTORY = -4,   /* |H_t 1| <= 1e-300 or <= 1e-12 ||H_t||_1: the "restart" case of Sec. 2.1 / Example 1 */
  RLGL_ENOT_CONVERGED = -5,  /* max_steps reached before the stop test; pi is still written */
  RLGL_ENONFINITE = -6,      /* ||C_t||_1 or H_t 1 is not finite */
  RLGL_EBUSY = -7            /* pool: no free slot or arena block right now, or the chain has not finished */
} rlgl_status;

/* Green-light rules (Sec. 6, "cash-dependent heuristics"; G_t is chosen from
 * the cash snapshot C_t and all green nodes move at once, eq. (4)). */
typedef enum {
  RLGL_SCHED_ALL = 0,        /* G_t = [N]: power iteration (Sec. 2.3.1) */
  RLGL_SCHED_THRESHOLD = 1,  /* |C_t,i| >= theta_t, theta_t = (sum_j |C_t,j|^r / N)^(1/r) (RLGL_Theta, all nodes at once) */
  RLGL_SCHED_TOPK = 2,       /* the k largest |C_t,i|, ties broken by smaller node id (Gauss-Southwell style) */
  RLGL_SCHED_MAXC = 3,       /* every node with |C_t,i| = max_j |C_t,j| (RLGL_MaxC) */
  RLGL_SCHED_PC = 4          /* RLGL_PC drawn for every node at once: node i is green with probability
                                |C_t,i| / max_j |C_t,j|, green iff u < |C_t,i| / max_j |C_t,j| with
                                u = (splitmix64(seed) output number t 2^32 + i) >> 11, times 2^-53 */
} rlgl_sched;

/* Arithmetic.  Cash routing runs in the cash type; H_t 1, ||C_t||_1, theta
 * and all other reductions run in FP64. */
typedef enum {
  RLGL_FP64 = 0,             /* C, P values and H in double */
  RLGL_FP32C_FP64H = 1,      /* C and P values in float, H in double */
  RLGL_FP32C_KAHANH = 2      /* C and P values in float, H as a compensated (Neumaier) float pair */
} rlgl_precision;

/* How the moved cash M_t reaches the destinations (the product M_t P of eq. (6)). */
typedef enum {
  RLGL_ROUTE_PUSH = 0,       /* scatter along the CSR rows of the green nodes (atomic adds) */
  RLGL_ROUTE_PULL = 1,       /* gather along the CSC columns of every node (needs the CSC arrays) */
  RLGL_ROUTE_AUTO = 2        /* per step: pull when the previous step's green links >= pull_alpha * nnz */
} rlgl_route;

/* The chain.  W is given in CSR (out-links) and optionally in CSC (in-links,
 * the transpose of the same matrix).  The transition matrix is
 *   P_ij = c * W_ij + (1 - c) / N   for a row i with at least one stored link,
 *   P_ij = 1 / N                    for a row with none (dangling),
 * i.e. the Google matrix of Sec. 3.2 with uniform restart; duplicate (i,j)
 * entries add up.  Rows of W must sum to 1 (the caller's contract).
 * Value arrays hold double for RLGL_FP64 and float otherwise; a NULL value
 * array means 1/outdeg(i) for every stored link of row i. */
typedef struct {
  int32_t n;                  /* number of states N >= 1 */
  int64_t nnz;                /* stored links, must equal csr_rowptr[n] and be < 2^31 */
  const int32_t *csr_rowptr;  /* [n+1], non-decreasing, csr_rowptr[0] = 0 */
  const int32_t *csr_col;     /* [nnz], each in [0, n) */
  const void *csr_val;        /* [nnz] or NULL */
  const int32_t *csc_colptr;  /* [n+1] or NULL: then only push routing is possible */
  const int32_t *csc_row;     /* [nnz] source of each in-link */
  const void *csc_val;        /* [nnz] or NULL (1/outdeg of the source) */
  double damping;             /* c in (0, 1] */
} rlgl_graph;

typedef struct {
  int32_t sched;              /* rlgl_sched */
  double r;                   /* power-mean order of the threshold, r >= 1 (default 1) */
  int64_t k;                  /* top-k size, >= 1 */
  int32_t theta_period;       /* recompute theta every theta_period steps (>= 1, default 1) */
  int32_t precision;          /* rlgl_precision */
  int32_t route;              /* rlgl_route */
  double pull_alpha;          /* AUTO switch point as a fraction of nnz (default 0.05) */
  int32_t check_period;       /* rlgl_solve: steps enqueued between host reads of the stop flag; 0 = adaptive */
  int32_t record_green;       /* non-zero: keep the green mask of the last step for rlgl_get_green */
  int32_t refresh;            /* rebuild C_t = H_t P - H_t in FP64 (needs the CSC; see rlgl_refresh):
                                 0 never; 1 in rlgl_solve before a stop is accepted and whenever |C_t 1| exceeds
                                 ||C_t||_1 / 2 (rounding drift); k > 1 also every k steps of rlgl_solve */
  int32_t relabel;            /* non-zero: rlgl_create renumbers the states internally by decreasing out-degree
                                 (ties by id) and keeps relabelled copies of the CSR/CSC in the workspace, so
                                 the cash of the states gathered most often shares cache lines; every value
                                 that crosses this interface (C, H, the green mask, pi_hat) stays in the
                                 caller's numbering.  Not with RLGL_SCHED_TOPK or _PC (they use the ids) */
  uint64_t seed;              /* RLGL_SCHED_PC: the splitmix64 seed of the draws */
} rlgl_options;

/* Snapshot of the solver after the last enqueued step. */
typedef struct {
  int64_t t;                  /* index of the current state C_t, H_t (t = 1 after rlgl_create) */
  int64_t green;              /* |G| of the last step */
  int64_t green_total;        /* sum of |G_t| over the steps t >= 1 */
  int64_t edges_pushed;       /* stored links of green nodes that moved non-zero cash, step 0 included */
  double l1_cash;             /* ||C_t||_1 */
  double h_sum;               /* H_t 1 */
  double resid;               /* ||C_t||_1 / |H_t 1| = ||pi_hat_t - pi_hat_t P||_1 (Algorithm 1, step (7)) */
  double theta;               /* threshold used by the last step (THRESHOLD), else 0 */
  double cash_sum;            /* C_t 1 (zero in exact arithmetic) */
  int32_t status;             /* rlgl_status of the last call */
  int32_t last_route;         /* rlgl_route used by the last step (PUSH or PULL) */
} rlgl_step_info;

/* Debug check of a graph against the contract above (Sec. 2: P must be
 * stochastic, so every row of W with a stored link sums to one), run on
 * `stream` over the device arrays; waits for the stream.  Checks:
 *   - csr_rowptr runs from 0 to nnz without decreasing; every csr_col is in
 *     [0, n);
 *   - with csr_val: no value is negative or non-finite, and every row with a
 *     stored link sums to 1 within 1e-12 (precision RLGL_FP64, double values)
 *     or 1e-6 (float values);
 *   - with the CSC: csc_colptr runs from 0 to nnz without decreasing, every
 *     csc_row is in [0, n), and the CSC holds exactly the CSR's links (i, j),
 *     with bit-identical values when both value arrays are given.  The links
 *     are compared as multisets, through every column's length against the
 *     CSR in-degree and a 64-bit sum of link hashes (a difference goes
 *     unnoticed with probability about 2^-64).
 * dev_scratch: caller-owned device memory of at least
 * rlgl_validate_scratch_bytes(g) bytes (about 4n), overwritten.
 * *max_row_dev (host, may be NULL): max |row sum - 1| over the rows with a
 * link (0 without csr_val).  Every array read is bounds-checked against n
 * and nnz.  Returns RLGL_OK, or RLGL_EINVAL with the first failed check in
 * rlgl_last_error(). */
size_t rlgl_validate_scratch_bytes(const rlgl_graph *g);
rlgl_status rlgl_validate(const rlgl_graph *g, int32_t precision, void *dev_scratch, size_t scratch_bytes,
                          void *stream, double *max_row_dev);

/* Fills *opt with the defaults: THRESHOLD, r = 1, k = 1, theta_period = 1,
 * FP32C_FP64H, AUTO, pull_alpha = 0.05, check_period = 0, record_green = 0,
 * refresh = 1, relabel = 0, seed = 0. */
void rlgl_default_options(rlgl_options *opt);

/* Device workspace the context needs, in bytes (0 on a bad argument).  Depends
 * on n, nnz, the precision, whether the CSC and the link values are given and
 * on relabel. */
size_t rlgl_workspace_bytes(const rlgl_graph *g, const rlgl_options *opt);

/* Checks the arguments, lays out the workspace, builds the static pull plan
 * from the CSC column pointers (setup: one device-to-host copy of csc_colptr)
 * and performs step 0 of Algorithm 1 (eq. (3) with uniform M_0 = (1/N) 1), so
 * the context holds C_1, H_1 and t = 1.  `stream` is a hipStream_t (NULL =
 * the default stream).  *out is set only on RLGL_OK. */
rlgl_status rlgl_create(const rlgl_graph *g, const rlgl_options *opt, void *dev_workspace, size_t ws_bytes,
                        void *stream, rlgl_ctx **out);

/* Performs nsteps >= 0 green-light steps (eqs. (4)-(6)) without any stop test
 * on the residual; stops early only on RLGL_EZERO_HISTORY or RLGL_ENONFINITE.
 * info (host pointer, may be NULL) receives the state after the last step. */
rlgl_status rlgl_step(rlgl_ctx *ctx, int32_t nsteps, rlgl_step_info *info);

/* Runs Algorithm 1 from the current state until ||C_t||_1 / |H_t 1| < eps for
 * some t >= 2 (step (7)), or until max_steps more steps were taken
 * (RLGL_ENOT_CONVERGED).  Then writes pi_hat_t = H_t / (H_t 1) as n doubles
 * into dev_pi (device pointer, may be NULL).  For c < 1 the L1 distance of
 * pi_hat to pi* is at most resid / (1 - c). */
rlgl_status rlgl_solve(rlgl_ctx *ctx, double eps, int64_t max_steps, double *dev_pi, rlgl_step_info *info);

/* One green-light step (Algorithm 1, steps (4)-(6); eqs. (4)-(6)) whose green
 * set G_t is given by the caller instead of the schedule: node i is green
 * when dev_mask[i] != 0 (device memory, n bytes, caller's numbering; a green
 * node with zero cash moves nothing).  This runs any rule for G_t, e.g. the
 * block schedules of the mean-field SBM (Sec. 5).  No stop test; the route
 * follows opt.route.  RLGL_EINVAL when the context was created with relabel.
 * *info (may be NULL) as for rlgl_step. */
rlgl_status rlgl_step_mask(rlgl_ctx *ctx, const uint8_t *dev_mask, rlgl_step_info *info);

/* ---- one-workgroup solves --------------------------------------------
 *
 * Algorithm 1 from step 0 to its stop test (step (7)) and pi_hat = H / (H 1)
 * (eq. (2)), for a chain small enough that one workgroup's LDS holds its cash
 * vector, in ONE kernel launch on `stream`.  Meant for latency-bound chains
 * (one green node per step in RLGL_MaxC, Sec. 6, takes N-scale step counts).
 * Rules: RLGL_SCHED_ALL, _THRESHOLD (r, theta_period), _MAXC and _PC; TOPK is
 * RLGL_EINVAL.  Precision: RLGL_FP64, or FP32 cash (either FP32 option) with
 * an FP64 history.  With FP64 cash and RLGL_MaxC the cash moves in the order
 * of the plain serial method (C -= M for the green nodes, their links in
 * increasing node order, then the uniform restart share), so every green set
 * and every cash value equal the serial method's.  With FP32 cash and
 * opt->refresh > 0 a stop is accepted only on C_t = H_t P - H_t rebuilt in
 * FP64 (eq. (7)).  opt->route, pull_alpha, check_period, record_green and
 * relabel are ignored.
 *
 * g: both the CSR and the CSC are required (device arrays, as for
 * rlgl_create); n <= rlgl_small_max_n(precision).
 * dev_workspace: caller-owned device memory of at least
 * rlgl_small_workspace_bytes(n) bytes (history, moved cash, result record),
 * overwritten.  dev_pi: n doubles (device, may be NULL), written when the
 * solve stops on eps (RLGL_OK) or at max_steps (RLGL_ENOT_CONVERGED).
 * Synchronises `stream` before returning; *info (host, may be NULL) as for
 * rlgl_solve, with last_route PUSH for a step routed from the green list and
 * PULL for a column step.  Errors: RLGL_EINVAL (arguments, n above the
 * capacity, csr_rowptr[n] or csc_colptr[n] != nnz; nothing launched),
 * RLGL_ENOMEM (workspace too small), RLGL_EHIP, and the solve outcomes
 * RLGL_ENOT_CONVERGED, RLGL_EZERO_HISTORY, RLGL_ENONFINITE. */
int32_t rlgl_small_max_n(int32_t precision);
size_t rlgl_small_workspace_bytes(int32_t n);
rlgl_status rlgl_solve_small(const rlgl_graph *g, const rlgl_options *opt, double eps, int64_t max_steps,
                             double *dev_pi, void *dev_workspace, size_t ws_bytes, void *stream,
                             rlgl_step_info *info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * rlgl_solve_small with its workspace taken from a static device array of
 * RLGL_SMALL_STATIC_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends.  Same arguments, behaviour and errors as
 * rlgl_solve_small without dev_workspace and ws_bytes; RLGL_EINVAL when
 * rlgl_small_workspace_bytes(g->n) exceeds RLGL_SMALL_STATIC_BYTES (n above
 * about 32,700).  Calls no hipMalloc, hipFree or other allocating routine.
 * Every call on one GPU uses that GPU's array, which keeps the last call's
 * contents (every solve writes its history and moved cash before reading
 * them): calls whose work overlaps on one GPU (from several host threads,
 * or on streams that run concurrently) race and must not be made. */
#define RLGL_SMALL_STATIC_BYTES (512u * 1024u)
rlgl_status rlgl_solve_small_static(const rlgl_graph *g, const rlgl_options *opt, double eps, int64_t max_steps,
                                    double *dev_pi, void *stream, rlgl_step_info *info);

/* ---- pull plans (host only; no GPU is used) ---------------------------
 *
 * The static work partition of the column sums of eq. (6) (the pull route,
 * C_{t+1,k} = (C_t - M_t)_k + sum over the in-links j -> k of c P'_jk M_j +
 * the restart share), built from CSC column pointers held in HOST memory.
 * rlgl_create builds the same plan for a single chain and rlgl_batch_create /
 * rlgl_pool_admit the batched one for each chain; these calls return it so it
 * can be inspected.
 *
 * Item i is items[4i .. 4i+3] = {x, y, p0, p1}, links [p0, p1) of the CSC:
 *   x >= 0: a run of the whole columns [x, y);
 *   x <  0: a piece of column y, whose in-links exceed one run; its partial sum
 *           goes to long-column slot -1 - x, and long_cols[slot] = y.
 * Single chain (rlgl_pull_plan): runs hold at most 512 links and 64 columns,
 * pieces 512 links, and the pieces are spread over the first three quarters
 * of the runs.  Batched (rlgl_batch_chain_plan): all pieces first (*n_pieces
 * of them, at most 4096 links each, for columns of more than 2048 in-links),
 * then runs of at most 2048 links and 1024 columns.  Every column lies in
 * exactly one run or is a long column; every link lies in exactly one item.
 *
 * host_colptr: n + 1 non-decreasing ints from 0 to nnz (caller-owned host
 * memory, read only).  items / long_cols: caller-owned host arrays of
 * 4 * max_items and max_long ints (may be NULL when the max is 0).  Returns
 * the number of items (>= 0), RLGL_EINVAL for bad pointers or column
 * pointers, RLGL_ENOMEM when max_items or max_long is too small (the counts
 * are still returned through n_long and n_pieces).  *item_bound (may be NULL)
 * receives the item count the device workspace is sized for. */
int64_t rlgl_pull_plan(const int32_t *host_colptr, int32_t n, int64_t nnz, int32_t *items, int64_t max_items,
                       int32_t *long_cols, int64_t max_long, int64_t *n_long, int64_t *item_bound);
int64_t rlgl_batch_chain_plan(const int32_t *host_colptr, int32_t n, int64_t nnz, int32_t *items, int64_t max_items,
                              int32_t *long_cols, int64_t max_long, int64_t *n_long, int64_t *n_pieces,
                              int64_t *item_bound);

/* Releases the host context.  Does not touch the caller's device memory. */
void rlgl_destroy(rlgl_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *rlgl_last_error(void);

/* ---- extensions ------------------------------------------------------- */

/* Re-runs step 0: the context is back at t = 1 (same as right after create). */
rlgl_status rlgl_reset(rlgl_ctx *ctx);

/* Copies C_t and H_t out as n doubles each (device pointers, either may be
 * NULL).  A compensated history is returned as hi + lo. */
rlgl_status rlgl_get_state(rlgl_ctx *ctx, double *dev_C, double *dev_H, rlgl_step_info *info);

/* Replaces the state by (C, H, H 1 = h_sum) at index t >= 1.  C is rounded to
 * the cash type; h_sum NaN means "sum of H".  The checkpoint of eq. (7): any
 * (C, H) with H + C = H P continues the method exactly. */
rlgl_status rlgl_set_state(rlgl_ctx *ctx, const double *dev_C, const double *dev_H, double h_sum, int64_t t);

/* Rebuilds the cash of the current state from its history with the balance
 * identity of Sec. 2.2 (eq. (7), C_0 = 0): C_t = H_t P - H_t, evaluated in FP64
 * along the CSC columns and rounded once to the cash type.  Needs the CSC
 * arrays (RLGL_EINVAL otherwise).  The method's state is unchanged in exact
 * arithmetic; the rounding accumulated by FP32 routing is removed. */
rlgl_status rlgl_refresh(rlgl_ctx *ctx, rlgl_step_info *info);

/* Green mask of the last step as n bytes (1 = green), device pointer.  Needs
 * record_green in the options; RLGL_EINVAL otherwise. */
rlgl_status rlgl_get_green(rlgl_ctx *ctx, uint8_t *dev_mask);

/* Per-kernel timing of the steps enqueued since the last call (HIP events on
 * the context's stream around every launch while enabled).  Fills up to 8
 * entries; the return value is the number of entries (or a negative
 * rlgl_status).  `bytes` counts what the method itself must move (the cost
 * of the links used, Sec. 6): a pull launch 4 B of source index, the link
 * value when stored and the gathered moved cash per link of a green node
 * that moved cash, plus 4 B of column pointer, the cash read and written and
 * the moved cash per node; a push launch the link index, value and
 * destination read-modify-write per such link plus the frontier entry per
 * green row; a select launch the cash per node and the row pointers and
 * history read-modify-write per green node (plus the frontier or the send
 * values it writes).  `bytes_touched` counts what the launch's access
 * pattern reads and writes: a pull reads every stored link, red or green,
 * and a push adds into FP64 sums. */
typedef struct {
  char name[24];
  int64_t launches;
  double ms;
  double bytes;               /* algorithmic bytes */
  double bytes_touched;       /* bytes of the access pattern */
  int64_t green_links;        /* links of green nodes that moved cash, over the launches */
} rlgl_kernel_stat;
rlgl_status rlgl_profile_enable(rlgl_ctx *ctx, int32_t on);
int32_t rlgl_profile_read(rlgl_ctx *ctx, rlgl_kernel_stat *out, int32_t max_entries);

/* ---- batched solves ----------------------------------------------------
 *
 * Many independent chains of uneven size solved together.  Each chain is the
 * chain of rlgl_graph with its own damping; the method, readings and stop
 * test are those of rlgl_solve (Algorithm 1 from uniform M_0, stop at
 * ||C_t||_1 / |H_t 1| < eps_k, t >= 2, confirmed on C_t = H_t P - H_t when
 * refresh is set).  The arrays of all chains are concatenated; node ids
 * inside a chain are local (0-based).  The CSC is required (the batched route
 * is the CSC gather).  Same conventions as above: device arrays and workspace
 * belong to the caller and must outlive the batch; the library allocates no
 * device memory.
 *
 * The engine (RLGL_BATCH_LOCKSTEP): every unfinished chain advances one step
 * per iteration of three launches (select, route, control) that span all of
 * them, so a large chain is spread over the whole GPU; link weights are
 * implicit (1/outdeg in FP64) and csr_val/csc_val are not read.  (Value 0,
 * an engine that ran each chain's whole solve in one workgroup, is no
 * longer offered: one CU per chain made the large chains of a batch slower
 * than solving the chains one after another.) */
typedef enum { RLGL_BATCH_LOCKSTEP = 1 } rlgl_batch_engine;
typedef struct rlgl_batch rlgl_batch;

typedef struct {
  int32_t n_chains;           /* >= 1 */
  const int64_t *node_off;    /* host [n_chains+1], non-decreasing, node_off[0] = 0: chain k owns entries
                                 node_off[k] .. node_off[k+1]-1 of every per-node vector (n_k >= 1) */
  const int64_t *edge_off;    /* host [n_chains+1]: chain k owns links edge_off[k] .. edge_off[k+1]-1 */
  const double *damping;      /* host [n_chains], each in (0, 1] */
  const int32_t *csr_rowptr;  /* device: chain k's n_k+1 local row pointers start at node_off[k] + k */
  const int32_t *csr_col;     /* device [total links]: local target ids */
  const void *csr_val;        /* device [total links] or NULL (1/outdeg); float, or double for RLGL_FP64 */
  const int32_t *csc_colptr;  /* device, laid out like csr_rowptr */
  const int32_t *csc_row;     /* device [total links]: local source ids */
  const void *csc_val;        /* device or NULL, as csr_val */
  const double *tol_l1;       /* host [n_chains] or NULL: chain k stops at ||C_t||_1 / |H_t 1| < tol_l1[k] (1 - c_k),
                                 which bounds the L1 error of pi_hat by tol_l1[k] (Lemma 1 with
                                 ||sum_k (P^k - 1 pi)||_1 <= 1 / (1 - c)); NULL: options.eps for every chain.
                                 With tol_l1 given, every damping must be below 1 (at c = 1 there is no such
                                 bound and the target would be 0): RLGL_EINVAL otherwise */
} rlgl_batch_graphs;

typedef struct {
  int32_t sched;              /* RLGL_SCHED_ALL, _THRESHOLD or _MAXC */
  double r;                   /* threshold power-mean order, >= 1 */
  int32_t precision;          /* rlgl_precision */
  double eps;                 /* stop test on ||C_t||_1 / |H_t 1| */
  int64_t max_steps;          /* per chain */
  int32_t refresh;            /* confirm the stop on the cash rebuilt from the history (0/1) */
  int32_t wg_size;            /* threads per route workgroup, 256 or 512 */
  int32_t wg_per_cu;          /* route workgroups per CU the plan items are strided over, 1..16, or 0 for one
                                 workgroup per item */
  int32_t engine;             /* rlgl_batch_engine: RLGL_BATCH_LOCKSTEP (anything else is RLGL_EINVAL) */
  int32_t check_period;       /* iterations between host checks of the finished count (>= 1) */
  int32_t relabel;            /* non-zero: every chain is solved in a relabelled copy of its graph (states
                                 renumbered by decreasing out-degree, ties by id) kept in the workspace, so
                                 the sources that send on most links share cache lines; pi_hat comes back in
                                 the caller's numbering.  Costs 4 (2 n + 2 + nnz) + 4 n bytes of workspace
                                 per chain */
} rlgl_batch_options;

/* Outcome of one chain. */
typedef struct {
  int64_t t;                  /* final state index */
  int64_t edges_pushed;       /* as in rlgl_step_info */
  double resid;               /* ||C_t||_1 / |H_t 1| at the stop */
  double h_sum;               /* H_t 1 */
  int32_t status;             /* rlgl_status of the chain */
  int32_t green_steps;        /* green-light steps taken after step 0 */
  double start_us, end_us;    /* device wall clock, microseconds since the launch began */
} rlgl_chain_result;

/* Defaults: THRESHOLD, r = 1, FP32C_KAHANH, eps = 1e-7, max_steps = 100000,
 * refresh = 1, wg_size = 256, wg_per_cu = 0, engine = LOCKSTEP,
 * check_period = 8, relabel = 1. */
void rlgl_batch_default_options(rlgl_batch_options *opt);

size_t rlgl_batch_workspace_bytes(const rlgl_batch_graphs *g, const rlgl_batch_options *opt);

/* Checks the arguments, copies the column pointers to the host once to build
 * each chain's static plan, and orders the chains by decreasing link count.
 * With opt->relabel it also copies the row pointers, renumbers every chain
 * and writes the relabelled row pointers and CSC into the workspace (the
 * caller's arrays are only read); RLGL_EINVAL when a chain's row or column
 * pointers decrease or its column pointers do not run from 0 to its link
 * count. */
rlgl_status rlgl_batch_create(const rlgl_batch_graphs *g, const rlgl_batch_options *opt, void *dev_workspace,
                              size_t ws_bytes, void *stream, rlgl_batch **out);

/* Solves every chain with the configured engine.  dev_pi (device, total
 * nodes doubles) receives pi_hat of every chain in the concatenated layout;
 * results (host, n_chains entries, may be NULL) the per-chain outcome;
 * *elapsed_ms (may be NULL) the time from the first launch to the last
 * chain's stop.  Returns RLGL_OK when every chain stopped on its test, else
 * the first failing chain's status. */
rlgl_status rlgl_batch_solve(rlgl_batch *b, double *dev_pi, rlgl_chain_result *results, double *elapsed_ms);

/* Autotuner: times one batch solve for every candidate launch shape (route
 * wg_size in {256, 512} x wg_per_cu in {0, 4, 8}) with HIP events and keeps
 * the fastest in the batch; *best (may be NULL) receives the chosen options. */
rlgl_status rlgl_batch_autotune(rlgl_batch *b, double *dev_pi, rlgl_batch_options *best);

void rlgl_batch_destroy(rlgl_batch *b);

/* ---- serving pool -------------------------------------------------------
 *
 * Continuous batching of independent solves.  A pool owns a device arena (a
 * part of the caller's workspace) in which admitted chains stay resident:
 * their CSC, row pointers, plan, cash, history and pi_hat.  rlgl_pool_admit
 * takes a chain held in host memory, reserves its footprint in the arena
 * (first fit) and enqueues its upload on a copy stream of the pool's own; a
 * chain joins the step-synchronous iteration of the other resident chains
 * at the first rlgl_pool_advance after its upload has landed, so requests
 * that arrive while others run are admitted as slots and memory free up,
 * and their steps share launches with the others'.  The method, the readings
 * and the stop test are those of the lockstep batch engine; link weights are
 * implicit (1/outdeg, FP64).  Calls on one pool must not overlap. */
typedef struct rlgl_pool rlgl_pool;

typedef struct {
  int32_t sched;              /* RLGL_SCHED_ALL, _THRESHOLD or _MAXC */
  double r;                   /* threshold power-mean order, >= 1 */
  int32_t precision;          /* rlgl_precision */
  int32_t refresh;            /* confirm the stop on the cash rebuilt from the history (0/1) */
  int32_t wg_size;            /* threads per route workgroup: 256 or 512 */
  int32_t max_chains;         /* slots: chains resident at once, >= 1 */
  int64_t max_steps;          /* per chain */
  int32_t route_per_cu;       /* route workgroups per CU the plan items are strided over, 1..16; 0: one per item */
} rlgl_pool_options;

/* One request: a chain of the form of rlgl_graph (damping c, uniform restart,
 * dangling rows uniform, weights 1/outdeg) held in HOST memory.  Page-locked
 * memory makes the upload asynchronous.  The arrays must stay valid until
 * the chain's result has been reported by rlgl_pool_poll or the slot has been
 * released. */
typedef struct {
  int32_t n;                  /* >= 1 */
  int64_t nnz;                /* < 2^31 */
  const int32_t *csr_rowptr;  /* host [n+1], 0 .. nnz, non-decreasing: the out-degrees */
  const int32_t *csc_colptr;  /* host [n+1], 0 .. nnz, non-decreasing */
  const int32_t *csc_row;     /* host [nnz], local source ids (NULL allowed when nnz = 0) */
  double damping;             /* c in (0, 1): a request stops on an L1 certificate, which c = 1 does not
                                 have (RLGL_EINVAL) */
  double tol_l1;              /* stop at ||C_t||_1 / |H_t 1| < tol_l1 (1 - c), which bounds the L1 error of
                                 pi_hat by tol_l1 (Lemma 1); >= 0 */
} rlgl_request;

/* Defaults: THRESHOLD, r = 1, FP32C_KAHANH, refresh = 1, wg_size = 256,
 * max_chains = 256, max_steps = 100000, route_per_cu = 8. */
void rlgl_pool_default_options(rlgl_pool_options *opt);

/* Workspace for a pool whose arena holds arena_bytes (control records of
 * max_chains slots added); 0 on bad options. */
size_t rlgl_pool_workspace_bytes(const rlgl_pool_options *opt, size_t arena_bytes);

/* Arena bytes one resident chain of n states and nnz links takes (upper
 * bound; the plan's exact size is known at admission). */
size_t rlgl_pool_footprint(const rlgl_pool_options *opt, int32_t n, int64_t nnz);

/* The arena is what is left of the workspace after the control records. */
rlgl_status rlgl_pool_create(const rlgl_pool_options *opt, void *dev_workspace, size_t ws_bytes, void *stream,
                             rlgl_pool **out);

/* Checks the request, builds its plan on the host, reserves its footprint and
 * enqueues its upload.  *slot receives the chain's slot.  RLGL_EBUSY when no
 * slot or no arena block is free now (nothing was changed). */
rlgl_status rlgl_pool_admit(rlgl_pool *p, const rlgl_request *req, int32_t *slot);

/* Starts the chains whose upload has landed, runs `iterations` lockstep
 * iterations (one step of every running chain each, at most) on the pool's
 * stream, waits for them, and collects the chains that finished.
 * *running (may be NULL) receives the number of chains still uploading or
 * running.  Equal to rlgl_pool_launch followed by rlgl_pool_wait. */
rlgl_status rlgl_pool_advance(rlgl_pool *p, int32_t iterations, int32_t *running);

/* The two halves of rlgl_pool_advance, so that the host can admit requests
 * while the iterations run: rlgl_pool_launch enqueues them and returns at
 * once (RLGL_EINVAL if a launch is still in flight); rlgl_pool_wait waits for
 * them and collects the chains that finished (it returns at once when nothing
 * is in flight).  Between the two, rlgl_pool_admit, _poll, _result and
 * _release may be called; a chain admitted then joins at the next launch. */
rlgl_status rlgl_pool_launch(rlgl_pool *p, int32_t iterations);
rlgl_status rlgl_pool_wait(rlgl_pool *p, int32_t *running);

/* Writes up to max_slots slots of chains finished since the last call into
 * slots (host) and returns their number (or a negative rlgl_status). */
int32_t rlgl_pool_poll(rlgl_pool *p, int32_t *slots, int32_t max_slots);

/* Outcome of a finished chain and its pi_hat (device, n doubles, valid until
 * the slot is released).  start_us/end_us are device wall-clock times since
 * the pool was created.  RLGL_EBUSY while the chain runs. */
rlgl_status rlgl_pool_result(rlgl_pool *p, int32_t slot, rlgl_chain_result *result, const double **dev_pi);

/* Frees a finished chain's slot and arena block.  RLGL_EBUSY while the chain
 * is uploading or running. */
rlgl_status rlgl_pool_release(rlgl_pool *p, int32_t slot);

/* Waits for the pool's work and frees its host resources. */
void rlgl_pool_destroy(rlgl_pool *p);

#ifdef __cplusplus
}
#endif

#endif /* RLGL_H */
