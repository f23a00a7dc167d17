/*
 * cpapr.h - C ABI of the MI355X (gfx950) CP-APR MU library.
 *
 * CP-APR with multiplicative updates fits a nonnegative rank-R Kruskal model
 * M = [lambda; A(1) .. A(N)] to a sparse count tensor X (Algorithm 1 of
 * Anderson, Teranishi, Dunlavy, Choi, "Analyzing the Performance Portability
 * of Tensor Decomposition", arXiv:2307.03276). Its hot path is
 *
 *     Phi(n) = (X_(n) ./ max(B Pi, eps)) Pi^T                  (Algorithm 2)
 *
 * computed one nonzero at a time (Section 3.1): pi_k[r] = prod_{m != n}
 * A(m)[i_m(k), r]; m_k = B[i_n(k), :] . pi_k; s_k = x_k / max(m_k, eps);
 * Phi[i_n(k), :] += s_k * pi_k. Phi feeds the MU step B <- B .* Phi, the
 * inner loop and the KKT test on min(B, 1 - Phi).
 *
 * Conventions (every entry point):
 *   - Layout: matrices are row-major I x R doubles (a row is R contiguous
 *     words). Coordinates are 0-based int32; idx[m * nnz + k] is nonzero k's
 *     mode-m coordinate.
 *   - Memory: pointers documented "device" are HIP device memory on the
 *     current device; "host" pointers are ordinary host memory. The caller
 *     owns every buffer. The library never allocates device memory: a plan
 *     lives in a caller-provided workspace sized by
 *     cpapr_plan_workspace_size().
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream). cpapr_phi is stream-ordered and returns without waiting.
 *     Functions that fill host results (plan creation, mu_inner, pqnr_inner,
 *     solve, loglik, batch status) wait for the stream before returning.
 *   - Errors: 0 on success, a negative CPAPR_E* code otherwise, with a
 *     message from cpapr_last_error() (thread-local). No C++ exception
 *     crosses this boundary. Non-convergence is not an error.
 *   - Limits: 2 <= N <= CPAPR_MAX_MODES, 1 <= R <= CPAPR_MAX_RANK,
 *     0 <= nnz < 2^31, 1 <= I_n < 2^31, I_n * R < 2^32 (factor row offsets
 *     are stored as 32-bit element offsets).
 */
#ifndef CPAPR_H
#define CPAPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPAPR_MAX_MODES 8
#define CPAPR_MAX_RANK 256
#define CPAPR_MAX_LMAX 4096

enum {
    CPAPR_OK = 0,
    CPAPR_EINVAL = -1,      /* bad argument (null pointer, size, mode, rank) */
    CPAPR_EINDEX = -2,      /* a coordinate lies outside [0, I_m) */
    CPAPR_EVALUE = -3,      /* a tensor value is not finite and > 0 */
    CPAPR_EWORKSPACE = -4,  /* workspace missing, misaligned or too small */
    CPAPR_EHIP = -5,        /* a HIP runtime call failed */
    CPAPR_EUNSUPPORTED = -6 /* size outside the documented limits */
};

/* Precision. FP64: factors gathered as stored. MIXED: Phi's gathers read FP32
 * copies of the other factors (half the gathered bytes), widened to FP64 as
 * they are loaded; every product, sum, B, Phi, lambda and the KKT test stay
 * FP64. */
enum { CPAPR_FP64 = 0, CPAPR_MIXED = 1 };

/* Phi kernel variants. SEGMENTED: mode-sorted nonzeros, in-register and
 * in-workgroup segmented reduction, atomics only for rows that cross a tile
 * boundary. ATOMIC: the per-nonzero atomic scatter of the paper's GPU kernel
 * (Algorithm 3), kept for comparison. XR: SEGMENTED with the per-nonzero dot
 * products reduced across the lane group by a reduce-scatter through LDS
 * (one sum and one division per nonzero in one lane), for 8 or 16 lanes per
 * nonzero and up to 8 gathered words per lane; other shapes run SEGMENTED.
 * AUTO picks SEGMENTED. */
enum { CPAPR_VARIANT_AUTO = 0, CPAPR_VARIANT_SEGMENTED = 1, CPAPR_VARIANT_ATOMIC = 2, CPAPR_VARIANT_XR = 3 };

/* Order of the nonzeros inside a row of the mode-n sorted copy (Phi's sum over
 * a row is order-free). ROW: input order (a stable sort by i_n). ROW_COL: by
 * the coordinate of the largest other mode (the first such mode on ties), so
 * long rows sweep that factor in order: a stable sort by the 32-bit key
 * (i_n << k) | (j >> d), where j is that coordinate, b_n and b_j the bit widths
 * of the two modes' sizes (ceil(log2 I)), k = min(b_j, 32 - b_n) and
 * d = b_j - k; when b_n + b_j > 32, runs of 2^d consecutive values of j keep
 * input order. */
enum { CPAPR_SORT_ROW = 0, CPAPR_SORT_ROW_COL = 1 };

/* Inner solver of each mode. MU: the multiplicative update of Algorithm 1.
 * PQNR: projected quasi-Newton solves of the row subproblems (the variant the
 * paper names in its Background): each row b of B = A(n) Lambda minimises
 * sum(b) - sum_k x_k log(max(b . pi_k, eps)) over b >= 0 by L-BFGS steps (3
 * pairs) over the variables not held at zero, with a projected backtracking
 * line search (sufficient decrease 1e-4, trials that bring a model value to
 * the floor eps rejected, 4 trials, then the MU step and the pairs dropped);
 * rows stop independently
 * when max|min(b, 1 - phi)| < tol. The outer loop, S shift included, is
 * Algorithm 1's. PQNR runs in FP64 only (precision CPAPR_FP64) and needs
 * R <= 256.
 *
 * PDNR: projected damped Newton solves of the same row subproblems (the
 * Background's other row-wise variant). Each iteration forms the row's exact
 * Hessian H = sum_k x_k / max(b . pi_k, eps)^2 pi_k pi_k^T in one pass over the
 * nonzeros, holds entries with b_r <= 1e-10 and g_r > 0 at the bound, solves
 * (H_FF + mu t I) d_F = -g_F on the other entries (t = trace(H_FF) / |F|,
 * Cholesky), and runs the same projected line search; mu starts at 1e-3 and
 * moves by a factor 4 with the ratio of actual to predicted decrease (within
 * [1e-8, 1e8]). FP64 only, R <= 64, not with deterministic = 1. */
enum { CPAPR_METHOD_MU = 0, CPAPR_METHOD_PQNR = 1, CPAPR_METHOD_PDNR = 2 };

/* Sparse count tensor in coordinate format (the paper's I[n][j], X[j]). */
typedef struct cpapr_coo {
    int32_t nmodes;      /* N */
    const int64_t* dims; /* host [N]: I_1..I_N */
    int64_t nnz;         /* number of stored entries; duplicates are allowed */
    const int32_t* idx;  /* device [N * nnz], 0-based */
    const double* vals;  /* device [nnz], finite and > 0 */
} cpapr_coo;

/* Algorithm parameters. */
typedef struct cpapr_params {
    int32_t kmax;      /* outer iterations (Algorithm 1), >= 1 */
    int32_t lmax;      /* inner iterations per mode, 1..CPAPR_MAX_LMAX */
    double tol;        /* KKT tolerance tau; <= 0: fixed kmax x lmax schedule */
    double eps;        /* divisor floor of Algorithm 2 (1e-10) */
    double kappa;      /* inadmissible-zero shift (0.01) */
    double kappa_tol;  /* entries below this count as zero (1e-10) */
    int32_t precision; /* CPAPR_FP64 or CPAPR_MIXED */
    int32_t variant;   /* CPAPR_VARIANT_* */
    int32_t group;     /* lanes per nonzero (0 = launch-policy model; else 4, 8, 16, 32 or 64) */
    int32_t chunk;     /* nonzeros per lane group per tile (0 = launch-policy model) */
    int32_t sort;      /* CPAPR_SORT_*: order of the nonzeros inside each row of a mode */
    int32_t method;    /* CPAPR_METHOD_*: inner solver of cpapr_solve */
    int32_t deterministic; /* 1: rows crossing a tile boundary are summed in a fixed order by a
                              second small kernel instead of with atomics, so single-plan
                              results repeat bit for bit (same plan and launch shape); needs
                              tiles of >= 128 nonzeros and the SEGMENTED variant; batches keep
                              atomics. 0: atomics (the default). */
} cpapr_params;

/* Result summary of cpapr_mu_inner / cpapr_solve (host). */
typedef struct cpapr_stats {
    int32_t outer_iters;  /* outer iterations run */
    int32_t converged;    /* 1 if an outer sweep made no update (tol > 0) */
    int64_t inner_iters;  /* MU updates performed, summed over modes */
    double kkt_violation; /* largest last-seen max|min(B, 1-Phi)| over modes of the final sweep */
    double loglik;        /* Poisson log-likelihood of the result (solve only) */
    int64_t phi_evals;    /* Phi computations performed (an inner loop stopped by the KKT test
                             computes one Phi more than it updates) */
    int64_t row_steps;    /* PQNR / PDNR: steps taken, summed over rows and modes (MU: 0) */
    int64_t trial_evals;  /* PQNR / PDNR: line-search passes over the nonzeros (MU: 0) */
} cpapr_stats;

typedef struct cpapr_plan cpapr_plan;

/* Fill *p with the defaults: kmax 10, lmax 10, tol 1e-4, eps 1e-10,
 * kappa 0.01, kappa_tol 1e-10, FP64, AUTO, group 0, chunk 0, sort ROW_COL,
 * method MU, deterministic 0. */
void cpapr_params_default(cpapr_params* p);

/* Bytes of device workspace a plan for X at rank R and parameters p needs
 * (written to *bytes). X->idx and X->vals may be NULL here. */
int cpapr_plan_workspace_size(const cpapr_coo* X, int32_t R, const cpapr_params* p, size_t* bytes);

/* Build a plan: checks every coordinate and value on the device, then sorts
 * the nonzeros by each mode's coordinate into N stable, physically permuted
 * copies kept in the workspace (the paper's sort-by-mode strategy: sorting
 * once per mode at the start, Section 3.1). ws (device, 256-byte aligned,
 * ws_bytes >= cpapr_plan_workspace_size) must outlive the plan; X's buffers
 * may be freed once this returns. Waits for `stream`. *out receives the plan. */
int cpapr_plan_create(const cpapr_coo* X, int32_t R, const cpapr_params* p, void* ws,
                      size_t ws_bytes, void* stream, cpapr_plan** out);
int cpapr_plan_destroy(cpapr_plan* plan);

/* Change the Phi launch shape of an existing plan (lanes per nonzero `group`:
 * 0 = launch-policy model, else 4, 8, 16, 32 or 64; nonzeros per lane group
 * per tile `chunk`: 0 = launch-policy model, else 1..65536). Host-only; used
 * by the autotuner to time shapes without re-sorting. Returns
 * CPAPR_EUNSUPPORTED for shapes with no kernel at this rank and mode count. */
int cpapr_plan_set_shape(cpapr_plan* plan, int32_t group, int32_t chunk);

/* The Phi launch shape a plan uses: lanes per nonzero and nonzeros per lane
 * group per tile. With group or chunk 0 (params or cpapr_plan_set_shape) they
 * come from a launch-policy model of the tensor (the kind of heuristic the
 * paper names as future work in Section 4): 512-nonzero tiles, smaller ones
 * (down to 64 nonzeros, 16 lanes per nonzero) when the tensor has fewer than
 * about 512,000 nonzeros; for 17 <= R <= 32 and up to four modes 16 lanes x 2
 * columns on 256-nonzero tiles in FP64 and 8 lanes x 4 columns on
 * 1024-nonzero tiles with FP32-stored factors; otherwise lanes by rank
 * (4 up to R = 4, 8 up to R = 32, then 16 or 64). Host-only. */
int cpapr_plan_shape(const cpapr_plan* plan, int32_t* group, int32_t* chunk);

/* Number of nonempty rows (segments) of mode `mode` (host query). */
int64_t cpapr_plan_segments(const cpapr_plan* plan, int32_t mode);

/* Phi(n) (Algorithm 2) for mode `mode` of the plan's tensor.
 *   B   device [I_n x R], nonnegative.
 *   A   host array of N device pointers to A(m) [I_m x R]; A[mode] is unused.
 *   eps divisor floor, > 0.
 *   Phi device [I_n x R], overwritten (rows without nonzeros become 0).
 * In CPAPR_MIXED the other factors are first rounded to FP32 copies in the
 * workspace and gathered from there (half the bytes); they are widened to FP64
 * as they are loaded, so products, sums and Phi are FP64.
 * Stream-ordered; does not wait. */
int cpapr_phi(cpapr_plan* plan, int32_t mode, const double* B, const double* const* A, double eps,
              double* Phi, void* stream);

/* Transient Phi(n) (Algorithm 2) of a COO tensor without a plan, for a caller
 * that needs Phi once. The nonzeros of mode `mode` are checked (coordinates in
 * range, values finite and > 0), sorted by their mode-n coordinate into the
 * caller's workspace (Section 3.1's sort by mode, for this mode only) and
 * reduced by the plan path's Phi kernel with its default launch shape.
 *   X   the tensor (device idx / vals, host dims), nnz >= 0.
 *   R   rank, 1..CPAPR_MAX_RANK.
 *   B   device [I_mode x R], nonnegative.
 *   A   host array of N device pointers to A(m) [I_m x R]; A[mode] is unused.
 *   eps divisor floor, > 0.
 *   Phi device [I_mode x R], overwritten (rows without nonzeros become 0).
 *   ws  device, 256-byte aligned, ws_bytes >= cpapr_phi_coo_workspace_size;
 *       its contents are scratch.
 * FP64 only. Waits for `stream` before returning, so ws may be reused or freed
 * at once. Errors: CPAPR_EINDEX / CPAPR_EVALUE for bad entries,
 * CPAPR_EWORKSPACE for a missing, misaligned or small workspace. */
int cpapr_phi_coo_workspace_size(const cpapr_coo* X, int32_t mode, int32_t R, size_t* bytes);
int cpapr_phi_coo(const cpapr_coo* X, int32_t mode, int32_t R, const double* B, const double* const* A, double eps,
                  double* Phi, void* ws, size_t ws_bytes, void* stream);

/* Device scratch that cpapr_phi_coo_noalloc keeps in the library's static
 * device memory, per GPU it runs on, until the process ends. */
#define CPAPR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* cpapr_phi_coo for callers that cannot allocate device memory (code that
 * must not call hipMalloc: serving loops, harnesses that forbid it). Same
 * arguments, checks and result as cpapr_phi_coo, with no workspace: the
 * scratch is a static device array of CPAPR_NOALLOC_SCRATCH_BYTES on each GPU
 * (a 3-way tensor of about 1.8M nonzeros fits). A tensor whose transient
 * workspace (cpapr_phi_coo_workspace_size) is larger is refused with
 * CPAPR_EUNSUPPORTED before any device work. Calls no hipMalloc, hipFree or
 * other allocating routine. All calls on one GPU share its array: calls that
 * overlap on a GPU (from other threads, on any stream) race; a call waits for
 * its stream before returning, so calls made one after another are safe.
 * Not for graph capture (it waits for the stream). FP64 only. */
int cpapr_phi_coo_noalloc(const cpapr_coo* X, int32_t mode, int32_t R, const double* B, const double* const* A,
                          double eps, double* Phi, void* stream);

/* MU inner loop of Algorithm 1 for one mode, params lmax / tol / eps of the plan:
 * for l < lmax: Phi = phi(B); viol = max|min(B, 1 - Phi)|; stop if tol > 0 and
 * viol < tol; else B <- B .* Phi.
 *   B        device [I_n x R], in/out.
 *   A        host array of N device pointers (A[mode] unused).
 *   Phi_last device [I_n x R], out: the last Phi computed.
 *   out      host, may be NULL: inner_iters = updates made, kkt_violation =
 *            last violation, outer_iters = 0.
 * The loop's stop decision stays on the device; waits for the stream once. */
int cpapr_mu_inner(cpapr_plan* plan, int32_t mode, double* B, const double* const* A,
                   double* Phi_last, cpapr_stats* out, void* stream);

/* PQNR row solves of one mode (see CPAPR_METHOD_PQNR): up to params.lmax
 * iterations for every row of B (device, I_mode x R, in/out, the row
 * subproblems' starting point, e.g. A(mode) Lambda) with the other factors A
 * (device, columns summing to one). Every iteration is one Phi pass for the
 * gradients and one line-search pass over the nonzeros that evaluates the four
 * trial steps at once (R < 4: up to four passes, one per trial), all ordered on
 * `stream` with stops decided on the device. out (host, may be NULL):
 * inner_iters = most steps taken by a row, row_steps = steps summed over rows,
 * kkt_violation = largest last violation over rows, converged = every row met
 * tol, phi_evals / trial_evals = passes run. The plan must have been created
 * with method CPAPR_METHOD_PQNR (its workspace holds the row state);
 * otherwise CPAPR_EINVAL. */
int cpapr_pqnr_inner(cpapr_plan* plan, int32_t mode, double* B, const double* const* A, cpapr_stats* out,
                     void* stream);

/* PDNR row solves of one mode (see CPAPR_METHOD_PDNR): the same arguments,
 * results and stream behaviour as cpapr_pqnr_inner; every iteration is one
 * pass over the nonzeros that forms each active row's Phi row and Hessian (the
 * phi_evals count) and the same line-search pass(es). The plan must have been
 * created with method CPAPR_METHOD_PDNR; otherwise CPAPR_EINVAL. Workspace:
 * (R*R + 5R) doubles and 7 scalars per row of the largest mode on top of the
 * MU plan's. */
int cpapr_pdnr_inner(cpapr_plan* plan, int32_t mode, double* B, const double* const* A, cpapr_stats* out,
                     void* stream);

/* Per-row outcome of the last cpapr_pqnr_inner / cpapr_pdnr_inner call on this
 * plan, which must have been for `mode` (the row state is that of the mode
 * solved last): steps (device [I_mode] int32, may be NULL) receives the steps
 * each row took; viol (device [I_mode] doubles, may be NULL) the violation
 * max_r |min(b_r, 1 - phi_r)| of its last KKT test, which for a row that
 * stopped is the value found below tol. Stream-ordered device-to-device
 * copies. CPAPR_EINVAL for an MU plan. */
int cpapr_row_stats(cpapr_plan* plan, int32_t mode, int32_t* steps, double* viol, void* stream);

/* Full CP-APR MU (Algorithm 1) with the plan's parameters.
 *   lambda device [R], in/out.  A host array of N device pointers, in/out.
 * From the second outer iteration on, entries with A(n)[i,r] < kappa_tol whose
 * previous Phi(n)[i,r] > 1 are raised by kappa before B = (A(n)+S) diag(lambda)
 * is formed; after the inner loop lambda = column sums of B and A(n) = B
 * diag(lambda)^-1 (zero columns stay zero). With tol > 0 the solve stops after
 * an outer sweep with no update. out (host, may be NULL) receives the stats,
 * including the log-likelihood of the result. Waits for the stream at most
 * once per outer iteration (tol > 0) or once at the end (tol <= 0). */
int cpapr_solve(cpapr_plan* plan, double* lambda, double* const* A, cpapr_stats* out, void* stream);

/* Poisson log-likelihood sum_k x_k log(max(m_k, eps)) - sum_r lambda_r
 * prod_m sum_i A(m)[i,r], with m_k the model value at nonzero k (the constant
 * -sum log x_k! is omitted). lambda device [R]; A host array of N device
 * pointers; *out host. Waits for the stream. */
int cpapr_loglik(cpapr_plan* plan, const double* lambda, const double* const* A, double eps,
                 double* out, void* stream);

/* MTTKRP for CP-ALS (the paper's Eqs. 10-12): M[i_n, :] = sum over nonzeros in
 * row i_n of x_k * prod_{m != n} A(m)[i_m, :]. Same sorted engine as Phi
 * without the divide. M device [I_n x R], overwritten. Stream-ordered. */
int cpapr_mttkrp(cpapr_plan* plan, int32_t mode, const double* const* A, double* M, void* stream);

/* ---- Batched Phi over many plans (work items) in persistent launches ----
 *
 * A batch is a set of slots; each slot is one Phi(n) work item: a plan, a mode
 * and its operands (B, the factors, the Phi output). cpapr_batch_run computes
 * Phi for every set slot with one list-driven fill/conversion launch and one
 * launch per shape class (lane group, rank block, number of other modes,
 * precision) present, all reading their work lists from device memory. With
 * use_graph the sequence is captured once into a hipGraph and replayed until
 * a commit changes what the graph baked in (see cpapr_batch_create2). Caller-provided
 * workspace; the library allocates no device memory. Slots of one batch must
 * write disjoint Phi buffers; a plan may appear in several slots. */
typedef struct cpapr_batch cpapr_batch;

/* Device workspace bytes for up to max_slots slots totalling up to max_tiles
 * workgroup tiles (a slot of nnz nonzeros takes ceil(nnz / 512) tiles at the
 * default chunk; cpapr_batch_tiles gives the exact count for a plan). */
int cpapr_batch_workspace_size(int32_t max_slots, int64_t max_tiles, size_t* bytes);
/* Tiles one slot of this plan takes in a batch (at its batch shape); -1 if
 * plan is NULL. */
int64_t cpapr_batch_tiles(const cpapr_plan* plan);
/* The launch shape of this plan's slots in a batch. A plan whose shape is the
 * launch-policy model's (group and chunk 0 at creation or in the last
 * cpapr_plan_set_shape) takes, in a batch, the model's shape for a tensor
 * large enough to fill the device by itself: the batch's slots share each
 * launch and fill the device together, so the small tiles the model gives a
 * small tensor launched alone (to make enough workgroups) only cost there.
 * A plan with a shape set by the caller keeps it. */
int cpapr_plan_batch_shape(const cpapr_plan* plan, int32_t* group, int32_t* chunk);
int cpapr_batch_create(int32_t max_slots, int64_t max_tiles, void* ws, size_t ws_bytes, cpapr_batch** out);
/* As cpapr_batch_create, with flags. By default (flags 0, what
 * cpapr_batch_create uses) each shape class is one launch with a workgroup per
 * tile, so the hardware dispatcher balances the uneven tiles; a captured graph
 * is re-captured whenever the tile counts change. CPAPR_BATCH_PERSISTENT runs
 * each class as one persistent launch sized to the device that claims tiles
 * dynamically and whose graph survives any commit with the same shape classes
 * (on MI355X about 1.5x slower per nonzero: each tile's descriptor loads are
 * serialised inside a workgroup instead of overlapped across workgroups). */
#define CPAPR_BATCH_PERSISTENT 1
/* CPAPR_BATCH_SKIP_HELD: held slots (cpapr_batch_hold) are left out of the
 * launches altogether (no tiles, no fill, no MU work) instead of being passed
 * over by the kernels; a change of the held set then takes effect at the next
 * cpapr_batch_commit (a run before it fails as uncommitted), and a captured
 * graph is re-captured when the tile counts change. For callers that run a
 * small subset of many slots per round. */
#define CPAPR_BATCH_SKIP_HELD 2
int cpapr_batch_create2(int32_t max_slots, int64_t max_tiles, int32_t flags, void* ws, size_t ws_bytes,
                        cpapr_batch** out);
int cpapr_batch_destroy(cpapr_batch* batch);

/* Set slot `slot` (host-side only). B device [I_mode x R]; A host array of the
 * plan's N device factor pointers (A[mode] unused); Phi device [I_mode x R],
 * overwritten by cpapr_batch_run. The plan must stay alive while set. flags:
 * CPAPR_BATCH_F32_CURRENT = the plan's FP32 factor copies already hold A
 * (mixed precision; see cpapr_plan_sync_f32), so runs skip the conversion. */
#define CPAPR_BATCH_F32_CURRENT 1
int cpapr_batch_set(cpapr_batch* batch, int32_t slot, cpapr_plan* plan, int32_t mode, const double* B,
                    const double* const* A, double* Phi, int32_t flags);
int cpapr_batch_clear(cpapr_batch* batch, int32_t slot);

/* Upload the work lists of the set slots to the device (waits for `stream`).
 * Required after cpapr_batch_set/clear and before cpapr_batch_run. */
int cpapr_batch_commit(cpapr_batch* batch, void* stream);

/* Phi for every set slot (stream-ordered, no host wait). use_graph != 0:
 * replay the captured hipGraph (capturing it first when needed). */
int cpapr_batch_run(cpapr_batch* batch, int32_t use_graph, void* stream);

/* One MU inner step for every set slot whose inner loop has not stopped, after
 * cpapr_batch_run: viol = max |min(B, 1 - Phi)| per slot; B <- B .* Phi
 * unless the slot plan's tol > 0 and viol < tol, which stops the slot (the
 * inner-loop test of cpapr_mu_inner). Stream-ordered. */
int cpapr_batch_mu(cpapr_batch* batch, void* stream);

/* The whole MU inner loop of Algorithm 1 for every set slot at once: lmax x
 * {Phi, KKT, update}, where a slot that stops (viol < tol) does no further
 * work and keeps its last Phi. Equivalent, per slot, to cpapr_mu_inner.
 * use_graph != 0 replays a captured hipGraph of the whole sequence.
 * Stream-ordered; read the outcome with cpapr_batch_status. */
int cpapr_batch_inner(cpapr_batch* batch, int32_t lmax, int32_t use_graph, void* stream);

/* Per-slot hold flags for the following cpapr_batch_run / cpapr_batch_inner
 * calls (host array of max_slots entries: nonzero = hold). A held slot does no
 * work in those runs: its Phi, B and factors are left as they are and
 * cpapr_batch_status reports it as stopped with no updates. Lets a caller run
 * a subset of its slots (e.g. the requests with the least remaining work).
 * Without CPAPR_BATCH_SKIP_HELD the batch's shape is unchanged, so a captured
 * graph stays valid and the held slots' tiles are launched and exit at once;
 * with it, a changed held set needs a cpapr_batch_commit. All slots run by
 * default. Waits for `stream`. */
int cpapr_batch_hold(cpapr_batch* batch, const int32_t* hold, void* stream);

/* Per-slot outcome since the last cpapr_batch_run / cpapr_batch_inner (host
 * arrays of max_slots entries; entries of unset slots are unspecified): last
 * KKT violation, MU updates made, and whether the slot's loop stopped on the
 * KKT test. Waits for `stream`. */
int cpapr_batch_status(cpapr_batch* batch, double* viol, int32_t* updates, int32_t* done, void* stream);

/* The per-mode steps of Algorithm 1 around the inner loop, for callers that
 * interleave many solves (cpapr_solve runs the same steps):
 * cpapr_mode_begin: from the second outer iteration on (outer_iter > 1,
 *   phi_prev != NULL) raise entries of A_mode below kappa_tol whose previous
 *   Phi exceeds 1 by kappa; then B = A_mode diag(lambda).
 * cpapr_mode_end: lambda = column sums of B; A_mode = B diag(lambda)^-1 (and
 *   the plan's FP32 copy of A_mode in mixed precision).
 * Device pointers: lambda [R], A_mode / phi_prev / B [I_mode x R].
 * Stream-ordered. */
int cpapr_mode_begin(cpapr_plan* plan, int32_t mode, int32_t outer_iter, const double* lambda, double* A_mode,
                     const double* phi_prev, double* B, void* stream);
int cpapr_mode_end(cpapr_plan* plan, int32_t mode, const double* B, double* lambda, double* A_mode, void* stream);

/* The same steps for many solves in one host call (a serving loop advancing
 * every request of a round): for item i in order, cpapr_mode_end(plans[i],
 * end_mode[i], B[i], lambda[i], A[i][end_mode[i]]) when end_mode[i] >= 0,
 * then cpapr_mode_begin(plans[i], begin_mode[i], outer_iter[i], lambda[i],
 * A[i][begin_mode[i]], phi_prev[i], B[i]) when begin_mode[i] >= 0. Host
 * arrays of `count` entries; A[i] is a host array of that plan's N device
 * factor pointers; phi_prev may be NULL (no shift) or hold NULL entries.
 * Stops at the first failing item and returns its error (earlier items'
 * launches stay queued). Stream-ordered. */
int cpapr_modes_advance(int32_t count, cpapr_plan* const* plans, const int32_t* end_mode, const int32_t* begin_mode,
                        const int32_t* outer_iter, double* const* lambda, double* const* const* A, double* const* B,
                        const double* const* phi_prev, void* stream);

/* Mixed precision: refresh the plan's FP32 copies of all N factors from A
 * (host array of N device pointers). No-op in FP64. Stream-ordered. */
int cpapr_plan_sync_f32(cpapr_plan* plan, const double* const* A, void* stream);

/* Kernel timing for measurement: while enabled, every Phi, MTTKRP and PDNR
 * Hessian-pass kernel launch is bracketed by HIP events on its stream (up to
 * `capacity` launches).
 * cpapr_prof_enable_sampled brackets only every `every`-th launch after the
 * call (the 1st, the every+1-th, ...): each event pair holds the stream for a
 * few microseconds on either side of its kernel, so sampling keeps the timed
 * work close to an unobserved run. cpapr_prof_read waits for the recorded
 * events and writes, per recorded launch, the mode and the kernel's duration
 * in milliseconds; returns the number of launches written (<= cap) or a
 * negative error. Not thread-safe. */
int cpapr_prof_enable(int32_t capacity);
int cpapr_prof_enable_sampled(int32_t capacity, int32_t every);
int cpapr_prof_disable(void);
int cpapr_prof_read(int32_t* modes, float* ms, int32_t cap);

const char* cpapr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CPAPR_H */
