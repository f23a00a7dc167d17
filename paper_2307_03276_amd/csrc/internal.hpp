// Internal declarations shared by the HIP translation units of libcpapr.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/cpapr.h"

namespace cpapr {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64s); the PDNR row kernels use one wave per row
constexpr int kXcds = 8;     // MI355X: 8 accelerator complex dies, each with its own L2

struct Error {
    int code;
    std::string msg;
};

// Slots of the KKT max-reduction: blocks spread their atomics over kViolSlots
// addresses, one per 128-byte line, because same-address device atomics
// serialise; consumers take the max over the slots.
constexpr int kViolSlots = 64;
constexpr int kViolStride = 16;  // u64 words per slot (128 bytes)

// Device-side state block of one inner loop (lives in the plan workspace).
struct DevState {
    unsigned long long viol[2][kViolSlots * kViolStride];  // per-parity slots, ordered bits of doubles >= 0
    double last_viol[CPAPR_MAX_MODES];                      // last KKT violation seen per mode
    int done;                                               // inner loop of the current mode has stopped
    int updates;                                            // MU updates in the current inner loop
    int sweep_updates;                                      // MU updates in the current outer sweep
    int pad;
    long long total_updates;                                // MU updates since the last reset
    long long phi_evals;                                    // Phi computations since the last reset
    double ll;                                              // log-likelihood result
    long long row_steps;                                    // row solves: steps summed over rows since the last reset
    long long trial_evals;                                  // row solves: line-search passes since the last reset
    int pq_all_done;                                        // row solves: no row of the current mode is active
    int pq_idle;                                            // row solves: no row is in a line search
};

// PQNR (projected quasi-Newton row solves): constants shared by every kernel.
constexpr int kPqnrMem = 3;          // curvature pairs kept per row
constexpr int kPqnrTrials = 4;       // backtracking trials before the MU step
constexpr double kPqnrSigma = 1e-4;  // sufficient-decrease constant
constexpr double kPqnrCurv = 1e-10;  // pair kept when s.y > kPqnrCurv |s| |y|

// PQNR state of the mode being solved (rows x R matrices, per-row scalars).
struct PqnrState {
    double* G;      // gradient 1 - Phi at the current b
    double* Gp;     // gradient before the last step
    double* Dd;     // search direction
    double* Dt;     // trial step (after a step: the step taken)
    double* T;      // line-search sums (column 0 of each row)
    double* S;      // kPqnrMem x (rows x R) steps of the kept pairs
    double* Y;      // kPqnrMem x (rows x R) gradient changes of the kept pairs
    double* alpha;  // per row: current trial length
    double* gdel;   // per row: g . trial step
    double* viol;   // per row: last KKT violation
    int32_t* status;  // per row: 0 active, 1 in a line search, 3 converged
    int32_t* trials;  // per row: rejected trials in this line search
    int32_t* steps;   // per row: steps taken
    int32_t* npairs;  // per row: kept pairs
    int32_t* head;    // per row: ring position of the next pair
    int64_t stride;   // rows of every matrix (largest mode)
};

// PDNR (projected damped Newton row solves): constants shared by every kernel.
constexpr int kPdnrMaxRank = 64;       // one wave per row: lane r holds row r of the Newton system
constexpr int kPdnrTrials = 4;         // backtracking trials before the MU step
constexpr double kPdnrSigma = 1e-4;    // sufficient-decrease constant
constexpr double kPdnrHeld = 1e-10;    // entries at or below this with g > 0 are held at the bound
constexpr double kPdnrMu0 = 1e-3;      // damping at the start of an inner loop (times trace(H_FF) / |F|)
constexpr double kPdnrMuMin = 1e-8;
constexpr double kPdnrMuMax = 1e8;
constexpr double kPdnrMuStep = 4.0;    // damping growth / shrink factor

// PDNR state of the mode being solved.
struct PdnrState {
    double* HP;         // rows x (R*R + R): Hessian (row-major) then the Phi row, accumulated per pass
    int64_t hp_stride;  // R*R + R
    double* G;          // gradient 1 - Phi at the current b
    double* Dd;         // search direction
    double* Dt;         // trial step (after a step: the step taken)
    double* T;          // line-search sums (column 0 of each row)
    double* mu;         // per row: damping
    double* alpha;      // per row: current trial length
    double* gdel;       // per row: g . trial step
    double* viol;       // per row: last KKT violation
    int32_t* status;    // per row: 0 active, 1 in a line search, 3 converged
    int32_t* trials;    // per row: rejected trials in this line search
    int32_t* steps;     // per row: steps taken
};

struct PlanMode {
    int32_t* rows;  // [nnz] sorted mode-n coordinates
    uint32_t* cofs;  // [(N-1) * nnz] the other modes' factor row offsets (coordinate x R), ascending m
    double* vals;   // [nnz]
    // [nnz] the same nonzeros as 16-byte records {row, offset 0, offset 1 (0 for
    // N = 2), value as FP32}: one load per staged nonzero instead of N + 1.
    // Only for N <= 3 and when every value is exact in FP32 (counts up to
    // 2^24); nullptr otherwise.
    int4* pk;
    int64_t segments;
};

constexpr int kMaxOther = CPAPR_MAX_MODES - 1;

// Operands of one Phi launch over one sorted copy (kernel argument).
struct PhiArgs {
    const int32_t* rows;
    const uint32_t* cofs;
    const double* vals;
    const int4* pk;        // packed records of the same nonzeros (nullptr: read the arrays above)
    const void* fac[kMaxOther];
    const double* B;
    double* Phi;
    const int* done;
    const double* D;       // trial step matrix (line-search pass only)
    const int32_t* live;   // line-search pass: rows with live[row] == 1 are evaluated, the others skipped
    double* det_part;      // deterministic mode: [2 x tiles x R] partial rows of the tile ends (head, tail)
    int32_t* det_rows;     // deterministic mode: [tiles x 2] their row ids (-1: none)
    int64_t det_tiles;     // tiles the partial buffers hold
    int64_t nnz;
    int R;
    int NM1;
    int L;
    int o32;               // 1: every gathered factor is below 4 GiB (32-bit byte offsets)
    double eps;
};

// One work item of a batched launch: operands and its first tile in the
// class's tile space.
struct alignas(16) BatchSlot {
    PhiArgs args;
    int64_t tile_begin;
    int32_t slot;  // caller's slot id (index of its done flag)
    int32_t pad;
};

// One list entry of the batched fill / conversion kernel.
struct alignas(16) BatchCopy {
    const double* src;
    void* dst;
    int64_t n;
    int64_t begin;  // offset in the concatenated element space
    int32_t op;     // 0: zero FP64 dst; 1: dst (FP32) = src (FP64)
    int32_t slot;   // op 0: skipped while this slot's done flag is set; -1: never skipped
};

// One list entry of the batched KKT / MU update kernels (one per slot).
struct alignas(16) BatchMu {
    double* B;
    const double* Phi;
    int64_t n;      // elements (I_mode x R)
    int64_t begin;  // offset in the concatenated element space
    double tol;     // the slot plan's KKT tolerance
    int32_t slot;
    int32_t pad;
};

constexpr int kMuSpread = 8;  // per-slot KKT maxima are spread over this many cache lines

// Dynamic tile claiming of the persistent batched Phi kernel.
constexpr int kBatchSubs = 64;      // tile sub-ranges per shape class (8 per XCD)
constexpr int kBatchClaim = 4;      // tiles claimed per atomic
constexpr int kCounterStride = 32;  // u32 words between counters (one 128-byte line each)
constexpr int kBatchClassesMax = 64;
constexpr int kBatchCounters = kBatchClassesMax * kBatchSubs;

}  // namespace cpapr

struct cpapr_plan {
    int32_t N;
    int64_t nnz;
    int32_t R;
    int64_t dims[CPAPR_MAX_MODES];
    cpapr_params params;
    cpapr::PlanMode mode[CPAPR_MAX_MODES];
    float* f32[CPAPR_MAX_MODES];      // FP32 factor copies (mixed precision)
    double* B;                        // [maxI x R] solve work matrix
    double* phi_prev[CPAPR_MAX_MODES];  // [I_m x R] last Phi per mode (solve)
    double* partial;                  // [kPartials x R] column-sum / reduction partials
    double* llpart;                   // [loglik_partials(nnz)] log-likelihood partials, one per tile
    double* colsums;                  // [N x R]
    cpapr::DevState* state;
    char* ws;
    size_t ws_bytes;
    int group, chunk;                 // resolved launch shape of the Phi kernel
    bool shape_auto;                  // group and chunk both from the launch-policy model
    cpapr::PqnrState pq;              // PQNR row-solve state (method CPAPR_METHOD_PQNR only)
    cpapr::PdnrState pd;              // PDNR row-solve state (method CPAPR_METHOD_PDNR only)
    double* det_part;                 // deterministic mode: tile-end partial rows (nullptr: atomics)
    int32_t* det_rows;                // deterministic mode: their row ids
    int64_t det_tiles;                // tiles the buffers hold (launches with more tiles are refused)
};

namespace cpapr {

constexpr int kPartials = 512;   // blocks of the two-level deterministic column sums

// ---- plan construction (sort.hip) ----
int64_t sort_scratch_bytes(int64_t nnz, int N);
// Validates coordinates/values, then builds the sorted copies of every mode
// (only >= 0: of that mode alone).
Error build_sorted(cpapr_plan* P, const cpapr_coo* X, char* scratch, hipStream_t s, int only = -1);

// ---- Phi (phi.hip) ----
// Whether a Phi kernel exists for this lane group, rank block and mode count.
bool phi_shape_supported(int group, int rpl, int nmodes_other);
// Resolve the lane-group size for rank R (the `group` parameter, 0 = automatic).
int resolve_group(int R, int requested, int nm1);
int resolve_chunk(int group, int requested);
int model_group(const cpapr_plan* P);             // launch-policy model: lanes per nonzero
int model_chunk(const cpapr_plan* P, int group);  // launch-policy model: nonzeros per lane group per tile
// Shape of this plan's slots in a batched launch: the model's shape for a
// tensor large enough to fill the device when the plan's shape is the model's,
// else the plan's own shape.
void batch_shape(const cpapr_plan* P, int* group, int* chunk);
// Deterministic mode: tiles the partial buffers are sized for (tiles of >= 128 nonzeros).
inline int64_t det_tile_capacity(int64_t nnz) { return nnz / 128 + 2; }
// Rank columns per lane (1, 2 or 4) for rank R on `group` lanes; -1 if R > 4 * group.
int rank_block(int R, int group);
Error launch_phi(const cpapr_plan* P, int mode, const double* B, const void* const* fac, bool mixed,
                 double eps, double* Phi, const int* done, hipStream_t s);
Error launch_mttkrp(const cpapr_plan* P, int mode, const double* const* A, double* M, hipStream_t s);

// ---- batched Phi (phi.hip; host side in batch.hip) ----
int batch_class_count();
int batch_class_of(int G, int RPL, int NM1, bool mixed);  // -1: no batched kernel for this shape
// counters: [kBatchCounters * kCounterStride] u32 in device memory.
// grid_tiles > 0: launch one workgroup per tile (that many) instead of the
// persistent kernel.
Error launch_phi_batch(int cls, const BatchSlot* slots, const int32_t* tile_map, const int64_t* class_off,
                       const int64_t* class_ntiles, const int32_t* slot_done, unsigned int* counters,
                       int* grid_cache, int64_t grid_tiles, hipStream_t s);
Error launch_batch_elementwise(const BatchCopy* items, const int32_t* nitems_dev, const int64_t* total_dev,
                               const int32_t* slot_done, unsigned int* counters, int grid, hipStream_t s);
PhiArgs phi_args(const cpapr_plan* P, int mode, const double* B, const void* const* fac, double eps, double* Phi);
// Per-slot state of the batched inner loop, all [max_slots]: done flag, MU
// updates made, last KKT violation.
struct BatchState {
    int32_t* done;
    int32_t* updates;
    double* viol;
    int32_t* hold;  // 1: the slot sits out the run (its done flag starts set)
};
// viol_spread: [kMuSpread * max_slots] u64 (slot s, spread j at j * max_slots + s).
Error launch_batch_mu(const BatchMu* items, const int32_t* nitems_dev, const int64_t* total_dev, int max_slots,
                      unsigned long long* viol_spread, BatchState st, int grid, hipStream_t s);
Error launch_batch_reset(BatchState st, int max_slots, hipStream_t s);

// ---- elementwise and reduction kernels (mu.hip) ----
Error launch_fill(double* p, int64_t n, double v, const int* done, hipStream_t s);
// Per-row sums of the likelihood-term changes along the trial steps D (m = B pi,
// dm = D pi; see delta_term) into column 0 of `out` (the other columns get 0),
// for rows with live[row] == 1 only; skipped when *skip != 0.
Error launch_delta(const cpapr_plan* P, int mode, const double* B, const double* D, const int32_t* live,
                   const void* const* fac, double eps, double* out, const int* skip, hipStream_t s);
// The same for the four trial steps max(b + alpha d, 0) - b, alpha = 1, 1/2,
// 1/4, 1/8, along the directions D, in one pass: trial k's sum in column k of
// `out`, the other columns 0. Needs R >= 4.
Error launch_delta4(const cpapr_plan* P, int mode, const double* B, const double* D, const int32_t* live,
                    const void* const* fac, double eps, double* out, const int* skip, hipStream_t s);

// ---- PQNR row solves (pqnr.hip) ----
size_t pqnr_bytes(int64_t maxI, int R);
void pqnr_bind(PqnrState* q, char* base, int64_t maxI, int R);
// One PQNR inner loop (lmax iterations) for the rows of `mode`; B in/out.
// `phi` (I_mode x R) receives every Phi pass, so it ends with the last Phi
// computed. Leaves per-mode stats in the device state (updates = most steps of
// a row, row_steps, last_viol[mode]).
Error enqueue_pqnr_inner(cpapr_plan* P, int mode, double* B, const void* const* fac, double* phi, hipStream_t s);

// ---- PDNR row solves (pdnr.hip) ----
size_t pdnr_bytes(int64_t maxI, int R);
void pdnr_bind(PdnrState* d, char* base, int64_t maxI, int R);
// One PDNR inner loop (lmax iterations) for the rows of `mode`; B in/out,
// `phi` as for PQNR, the same per-mode stats in the device state.
Error enqueue_pdnr_inner(cpapr_plan* P, int mode, double* B, const void* const* fac, double* phi, hipStream_t s);
Error launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);
Error launch_reset_state(DevState* st, bool new_sweep, bool all, hipStream_t s);
Error launch_kkt(const double* B, const double* Phi, int64_t n, DevState* st, int l, hipStream_t s);
// tol <= 0: the KKT violation and the update in one pass (the violation reaches
// last_viol one launch later; launch_kkt_fold after the last iteration).
Error launch_mu_fused(double* B, double* Phi, int64_t n, DevState* st, int l, int mode, bool zero_phi, hipStream_t s);
Error launch_kkt_fold(DevState* st, int l, int mode, hipStream_t s);
Error launch_mu_update(double* B, double* Phi, int64_t n, DevState* st, int l, int mode, double tol, bool zero_phi,
                       hipStream_t s);
Error launch_shift_scale(double* A, const double* phi_prev, const double* lam, double* B, int64_t I, int R,
                         double kappa, double kappa_tol, bool shift, hipStream_t s);
Error launch_colsum(const double* M, int64_t I, int R, double* partial, double* out, hipStream_t s);
Error launch_normalize(const double* B, const double* lam, double* A, float* A32, int64_t I, int R,
                       hipStream_t s);
Error launch_loglik(const cpapr_plan* P, const double* lam, const double* const* A, double eps,
                    hipStream_t s);
// Sum of x_k log(max(m_k, eps)) over the nonzeros of the mode-0 copy into
// `partial` (one entry per tile; returns the number of tiles in *nparts), where
// m_k = B[i_0(k), :] . pi_k and B = A(0) diag(lambda).
Error launch_loglik_terms(const cpapr_plan* P, const double* B, const double* const* A, double eps, double* partial,
                          int* nparts, hipStream_t s);
int64_t loglik_partials(int64_t nnz);

// ---- transient Phi without a plan (api.hip) ----
// Workspace bytes of a transient Phi for N modes and nnz nonzeros.
size_t transient_bytes(int N, int64_t nnz);
// Validate X and `mode`, sort the mode into `ws`, run Phi; waits for the stream.
Error phi_transient(const cpapr_coo* X, int32_t mode, int32_t R, const double* B, const double* const* A,
                    double eps, double* Phi, char* ws, size_t ws_bytes, hipStream_t s);
// Argument checks of a transient Phi that touch no device memory.
Error check_transient(const cpapr_coo* X, int32_t mode, int32_t R, bool need_data);

// ---- error message of the last failing entry point (api.hip, thread-local) ----
void set_last_error(const std::string& msg);

// ---- profiling hooks (api.hip) ----
void prof_begin(int mode, hipStream_t s);
void prof_end(hipStream_t s);

}  // namespace cpapr

#define CPAPR_HIP(call)                                                                 \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::cpapr::Error{CPAPR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define CPAPR_LAUNCHED()                                                                \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return ::cpapr::Error{CPAPR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)}; \
    } while (0)
