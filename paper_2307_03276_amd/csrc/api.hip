// C ABI entry points (include/cpapr.h): argument checks, the workspace layout
// of a plan, and the host-side sequencing of Algorithm 1's kernels. Every step
// of the computation runs in the HIP kernels of sort.hip, phi.hip and mu.hip.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "internal.hpp"

using cpapr::Error;

namespace {

thread_local std::string g_error;

int fail(int code, const std::string& msg)
{
    g_error = msg;
    return code;
}

int report(const Error& e)
{
    if (e.code) g_error = e.msg;
    return e.code;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---- kernel timing (measurement only) ----
struct Prof {
    bool on = false;
    int cap = 0;
    int count = 0;
    int every = 1;      // record every `every`-th launch
    int64_t seen = 0;   // launches since enable
    bool open = false;
    std::vector<hipEvent_t> start, stop;
    std::vector<int> mode;
} g_prof;

Error check_coo(const cpapr_coo* X, int32_t R, bool need_data)
{
    if (!X) return {CPAPR_EINVAL, "X is NULL"};
    if (X->nmodes < 2 || X->nmodes > CPAPR_MAX_MODES) return {CPAPR_EINVAL, "nmodes must be in [2, 8]"};
    if (!X->dims) return {CPAPR_EINVAL, "dims is NULL"};
    for (int m = 0; m < X->nmodes; ++m)
        if (X->dims[m] < 1 || X->dims[m] > 0x7fffffffLL) return {CPAPR_EUNSUPPORTED, "each dim must be in [1, 2^31)"};
    if (X->nnz < 0) return {CPAPR_EINVAL, "nnz < 0"};
    if (X->nnz > 0x7fffffffLL) return {CPAPR_EUNSUPPORTED, "nnz must be < 2^31"};
    if (need_data && X->nnz > 0 && (!X->idx || !X->vals)) return {CPAPR_EINVAL, "idx or vals is NULL"};
    if (R < 1 || R > CPAPR_MAX_RANK) return {CPAPR_EUNSUPPORTED, "R must be in [1, 256]"};
    for (int m = 0; m < X->nmodes; ++m)
        if (X->dims[m] * (int64_t)R > 0xffffffffLL)
            return {CPAPR_EUNSUPPORTED, "each factor must have fewer than 2^32 entries (I_m * R)"};
    return {CPAPR_OK, ""};
}

Error check_params(const cpapr_params* p, int32_t R, int nmodes)
{
    if (!p) return {CPAPR_EINVAL, "params is NULL"};
    if (p->kmax < 1) return {CPAPR_EINVAL, "kmax must be >= 1"};
    if (p->lmax < 1 || p->lmax > CPAPR_MAX_LMAX) return {CPAPR_EINVAL, "lmax must be in [1, 4096]"};
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return {CPAPR_EINVAL, "eps must be finite and > 0"};
    if (!(p->kappa >= 0.0) || !(p->kappa_tol >= 0.0)) return {CPAPR_EINVAL, "kappa and kappa_tol must be >= 0"};
    if (p->precision != CPAPR_FP64 && p->precision != CPAPR_MIXED) return {CPAPR_EINVAL, "unknown precision"};
    if (p->variant < CPAPR_VARIANT_AUTO || p->variant > CPAPR_VARIANT_XR) return {CPAPR_EINVAL, "unknown variant"};
    if (p->variant == CPAPR_VARIANT_ATOMIC && p->precision == CPAPR_MIXED)
        return {CPAPR_EUNSUPPORTED, "the atomic variant is FP64 only"};
    const int g = cpapr::resolve_group(R, p->group, nmodes - 1);
    if (g != 4 && g != 8 && g != 16 && g != 32 && g != 64) return {CPAPR_EINVAL, "group must be 0, 4, 8, 16, 32 or 64"};
    if (cpapr::rank_block(R, g) < 0) return {CPAPR_EUNSUPPORTED, "rank too large for this lane group (R > 4 * group)"};
    if (!cpapr::phi_shape_supported(g, cpapr::rank_block(R, g), nmodes - 1))
        return {CPAPR_EUNSUPPORTED, "no Phi kernel for this lane group and rank block at this mode count"};
    if (p->chunk < 0 || p->chunk > 65536) return {CPAPR_EINVAL, "chunk must be in [0, 65536]"};
    if (p->sort != CPAPR_SORT_ROW && p->sort != CPAPR_SORT_ROW_COL) return {CPAPR_EINVAL, "unknown sort"};
    if (p->method != CPAPR_METHOD_MU && p->method != CPAPR_METHOD_PQNR && p->method != CPAPR_METHOD_PDNR)
        return {CPAPR_EINVAL, "unknown method"};
    if (p->deterministic != 0 && p->deterministic != 1) return {CPAPR_EINVAL, "deterministic must be 0 or 1"};
    if (p->deterministic && p->variant == CPAPR_VARIANT_ATOMIC)
        return {CPAPR_EUNSUPPORTED, "the atomic variant is not deterministic"};
    if (p->method == CPAPR_METHOD_PQNR && p->precision != CPAPR_FP64)
        return {CPAPR_EUNSUPPORTED, "PQNR runs in FP64 only"};
    if (p->method == CPAPR_METHOD_PDNR) {
        if (p->precision != CPAPR_FP64) return {CPAPR_EUNSUPPORTED, "PDNR runs in FP64 only"};
        if (R > cpapr::kPdnrMaxRank) return {CPAPR_EUNSUPPORTED, "PDNR supports R <= 64"};
        if (p->deterministic) return {CPAPR_EUNSUPPORTED, "PDNR's Hessian pass is not deterministic"};
    }
    return {CPAPR_OK, ""};
}

// Workspace layout. Region 1 (kept): the sorted copies of every mode and the
// FP32 factor copies. Region 2 (shared): the sort's temporaries during plan
// creation, afterwards the solve's B, previous Phi per mode, reduction
// partials, column sums and the device state block.
struct Layout {
    size_t mode_rows[CPAPR_MAX_MODES], mode_cidx[CPAPR_MAX_MODES], mode_vals[CPAPR_MAX_MODES];
    size_t mode_pk[CPAPR_MAX_MODES];  // packed records (N <= 3), size 0 otherwise
    size_t f32[CPAPR_MAX_MODES];
    size_t region2;
    size_t B, phi_prev[CPAPR_MAX_MODES], partial, llpart, colsums, state, pqnr, pdnr, det_part, det_rows;
    size_t total;
};

Layout layout(int N, int64_t nnz, const int64_t* dims, int R, bool mixed, int method, bool det)
{
    Layout L{};
    size_t off = 0;
    for (int n = 0; n < N; ++n) {
        L.mode_rows[n] = off;
        off += align256((size_t)nnz * 4);
        L.mode_cidx[n] = off;
        off += align256((size_t)nnz * 4 * (N - 1));
        L.mode_vals[n] = off;
        off += align256((size_t)nnz * 8);
        L.mode_pk[n] = off;
        if (N <= 3) off += align256((size_t)nnz * 16);
    }
    for (int n = 0; n < N; ++n) {
        L.f32[n] = off;
        if (mixed) off += align256((size_t)dims[n] * R * 4);
    }
    L.region2 = off;
    int64_t maxI = 0;
    for (int n = 0; n < N; ++n) maxI = std::max(maxI, dims[n]);
    size_t s = 0;
    L.B = off + s;
    s += align256((size_t)maxI * R * 8);
    for (int n = 0; n < N; ++n) {
        L.phi_prev[n] = off + s;
        s += align256((size_t)dims[n] * R * 8);
    }
    L.partial = off + s;
    s += align256((size_t)cpapr::kPartials * R * 8);
    L.llpart = off + s;
    s += align256((size_t)cpapr::loglik_partials(nnz) * 8);
    L.colsums = off + s;
    s += align256((size_t)N * R * 8);
    L.state = off + s;
    s += align256(sizeof(cpapr::DevState));
    L.pqnr = off + s;
    if (method == CPAPR_METHOD_PQNR) s += cpapr::pqnr_bytes(maxI, R);
    L.pdnr = off + s;
    if (method == CPAPR_METHOD_PDNR) s += cpapr::pdnr_bytes(maxI, R);
    const int64_t cap = cpapr::det_tile_capacity(nnz);
    L.det_part = off + s;
    if (det) s += align256((size_t)2 * cap * R * 8);
    L.det_rows = off + s;
    if (det) s += align256((size_t)2 * cap * 4);
    s = std::max(s, (size_t)cpapr::sort_scratch_bytes(nnz, N));
    L.total = off + s;
    return L;
}

Error check_plan_call(const cpapr_plan* P, int32_t mode)
{
    if (!P) return {CPAPR_EINVAL, "plan is NULL"};
    if (mode < 0 || mode >= P->N) return {CPAPR_EINVAL, "mode out of range"};
    return {CPAPR_OK, ""};
}

Error check_factors(const cpapr_plan* P, const double* const* A, int skip)
{
    if (!A) return {CPAPR_EINVAL, "factor array is NULL"};
    for (int m = 0; m < P->N; ++m)
        if (m != skip && !A[m]) return {CPAPR_EINVAL, "a factor pointer is NULL"};
    return {CPAPR_OK, ""};
}

// Factor pointers the Phi kernel gathers from: the caller's FP64 matrices, or
// (mixed precision) FP32 copies refreshed here.
Error phi_factors(cpapr_plan* P, int mode, const double* const* A, const void** fac, hipStream_t s)
{
    const bool mixed = P->params.precision == CPAPR_MIXED;
    for (int m = 0; m < P->N; ++m) {
        if (m == mode) {
            fac[m] = nullptr;
            continue;
        }
        if (mixed) {
            Error e = cpapr::launch_to_f32(A[m], P->f32[m], P->dims[m] * (int64_t)P->R, s);
            if (e.code) return e;
            fac[m] = P->f32[m];
        } else {
            fac[m] = A[m];
        }
    }
    return {CPAPR_OK, ""};
}

// One inner loop (Algorithm 1): zero Phi, then lmax x {Phi, KKT, MU update},
// all gated by the device-side `done` flag. No host synchronisation. With a
// fixed schedule (tol <= 0) nothing depends on the violation before the
// update, so KKT and update are one pass over B and Phi.
Error enqueue_inner(cpapr_plan* P, int mode, double* B, const void* const* fac, double* Phi, hipStream_t s)
{
    const int64_t n = P->dims[mode] * (int64_t)P->R;
    const bool mixed = P->params.precision == CPAPR_MIXED;
    const bool fused = !(P->params.tol > 0.0);
    const int* done = &P->state->done;
    Error e = cpapr::launch_fill(Phi, n, 0.0, done, s);
    if (e.code) return e;
    const int lmax = P->params.lmax;
    for (int l = 0; l < lmax; ++l) {
        e = cpapr::launch_phi(P, mode, B, fac, mixed, P->params.eps, Phi, done, s);
        if (e.code) return e;
        // the update clears Phi for the next Phi launch, except after the last one
        if (fused) {
            e = cpapr::launch_mu_fused(B, Phi, n, P->state, l, mode, l + 1 < lmax, s);
        } else {
            e = cpapr::launch_kkt(B, Phi, n, P->state, l, s);
            if (e.code) return e;
            e = cpapr::launch_mu_update(B, Phi, n, P->state, l, mode, P->params.tol, l + 1 < lmax, s);
        }
        if (e.code) return e;
    }
    if (fused && lmax > 0) return cpapr::launch_kkt_fold(P->state, lmax - 1, mode, s);
    return {CPAPR_OK, ""};
}

struct HostState {
    double last_viol[CPAPR_MAX_MODES];
    int done, updates, sweep_updates;
    long long total_updates, phi_evals, row_steps, trial_evals;
    double ll;
};

Error read_state(const cpapr_plan* P, HostState* h, hipStream_t s)
{
    cpapr::DevState* d = P->state;
    CPAPR_HIP(hipMemcpyAsync(h->last_viol, d->last_viol, sizeof(h->last_viol), hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipMemcpyAsync(&h->done, &d->done, sizeof(int) * 3, hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipMemcpyAsync(&h->total_updates, &d->total_updates, sizeof(long long), hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipMemcpyAsync(&h->phi_evals, &d->phi_evals, sizeof(long long), hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipMemcpyAsync(&h->row_steps, &d->row_steps, sizeof(long long), hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipMemcpyAsync(&h->trial_evals, &d->trial_evals, sizeof(long long), hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipMemcpyAsync(&h->ll, &d->ll, sizeof(double), hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipStreamSynchronize(s));
    return {CPAPR_OK, ""};
}

}  // namespace

namespace cpapr {

void set_last_error(const std::string& msg) { g_error = msg; }

void prof_begin(int mode, hipStream_t s)
{
    if (!g_prof.on) return;
    if (g_prof.seen++ % g_prof.every != 0 || g_prof.count >= g_prof.cap) return;
    if (hipEventRecord(g_prof.start[g_prof.count], s) == hipSuccess) {
        g_prof.mode[g_prof.count] = mode;
        g_prof.open = true;
    }
}

void prof_end(hipStream_t s)
{
    if (!g_prof.on || !g_prof.open) return;
    g_prof.open = false;
    if (hipEventRecord(g_prof.stop[g_prof.count], s) == hipSuccess) g_prof.count++;
}

// Workspace of a transient Phi (no plan): the sorted copy of the one mode,
// then the scratch of its sort.
struct TransientLayout {
    size_t rows, cidx, vals, scratch, total;
};

TransientLayout transient_layout(int N, int64_t nnz)
{
    TransientLayout L{};
    size_t off = 0;
    L.rows = off;
    off += align256((size_t)nnz * 4);
    L.cidx = off;
    off += align256((size_t)nnz * 4 * (N - 1));
    L.vals = off;
    off += align256((size_t)nnz * 8);
    L.scratch = off;
    off += (size_t)cpapr::sort_scratch_bytes(nnz, N);
    L.total = off;
    return L;
}

size_t transient_bytes(int N, int64_t nnz) { return transient_layout(N, nnz).total; }

Error check_transient(const cpapr_coo* X, int32_t mode, int32_t R, bool need_data)
{
    Error e = check_coo(X, R, need_data);
    if (e.code) return e;
    if (mode < 0 || mode >= X->nmodes) return {CPAPR_EINVAL, "mode out of range"};
    return {CPAPR_OK, ""};
}

// Transient Phi of mode `mode` of X: validate and sort the mode's nonzeros
// into `ws` (a one-mode plan kept on the host stack), then the plan's Phi
// launch. Waits for the stream.
Error phi_transient(const cpapr_coo* X, int32_t mode, int32_t R, const double* B, const double* const* A,
                    double eps, double* Phi, char* ws, size_t ws_bytes, hipStream_t s)
{
    Error e = check_transient(X, mode, R, true);
    if (e.code) return e;
    if (!B || !Phi || !A) return {CPAPR_EINVAL, "B, A or Phi is NULL"};
    for (int m = 0; m < X->nmodes; ++m)
        if (m != mode && !A[m]) return {CPAPR_EINVAL, "a factor pointer is NULL"};
    if (!(eps > 0.0) || !std::isfinite(eps)) return {CPAPR_EINVAL, "eps must be finite and > 0"};
    const TransientLayout L = transient_layout(X->nmodes, X->nnz);
    if (!ws) return {CPAPR_EWORKSPACE, "workspace is NULL"};
    if (((uintptr_t)ws & 255) != 0) return {CPAPR_EWORKSPACE, "workspace must be 256-byte aligned"};
    if (ws_bytes < L.total) return {CPAPR_EWORKSPACE, "workspace too small"};
    cpapr_plan P{};
    P.N = X->nmodes;
    P.nnz = X->nnz;
    P.R = R;
    for (int m = 0; m < P.N; ++m) P.dims[m] = X->dims[m];
    cpapr_params_default(&P.params);
    P.ws = ws;
    P.ws_bytes = ws_bytes;
    P.group = cpapr::model_group(&P);
    P.mode[mode].rows = (int32_t*)(ws + L.rows);
    P.mode[mode].cofs = (uint32_t*)(ws + L.cidx);
    P.mode[mode].vals = (double*)(ws + L.vals);
    e = cpapr::build_sorted(&P, X, ws + L.scratch, s, mode);
    if (e.code) return e;
    P.chunk = cpapr::model_chunk(&P, P.group);
    const void* fac[CPAPR_MAX_MODES];
    for (int m = 0; m < P.N; ++m) fac[m] = A[m];
    e = cpapr::launch_fill(Phi, X->dims[mode] * (int64_t)R, 0.0, nullptr, s);
    if (e.code) return e;
    e = cpapr::launch_phi(&P, mode, B, fac, false, eps, Phi, nullptr, s);
    if (e.code) return e;
    CPAPR_HIP(hipStreamSynchronize(s));
    return {CPAPR_OK, ""};
}

}  // namespace cpapr

extern "C" {

void cpapr_params_default(cpapr_params* p)
{
    if (!p) return;
    p->kmax = 10;
    p->lmax = 10;
    p->tol = 1e-4;
    p->eps = 1e-10;
    p->kappa = 0.01;
    p->kappa_tol = 1e-10;
    p->precision = CPAPR_FP64;
    p->variant = CPAPR_VARIANT_AUTO;
    p->group = 0;
    p->chunk = 0;
    p->sort = CPAPR_SORT_ROW_COL;
    p->method = CPAPR_METHOD_MU;
    p->deterministic = 0;
}

const char* cpapr_last_error(void) { return g_error.c_str(); }

int cpapr_plan_workspace_size(const cpapr_coo* X, int32_t R, const cpapr_params* p, size_t* bytes)
{
    try {
        Error e = check_coo(X, R, false);
        if (e.code) return report(e);
        e = check_params(p, R, X->nmodes);
        if (e.code) return report(e);
        if (!bytes) return fail(CPAPR_EINVAL, "bytes is NULL");
        *bytes = layout(X->nmodes, X->nnz, X->dims, R, p->precision == CPAPR_MIXED, p->method,
                        p->deterministic != 0).total;
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_plan_create(const cpapr_coo* X, int32_t R, const cpapr_params* p, void* ws, size_t ws_bytes,
                      void* stream, cpapr_plan** out)
{
    try {
        if (!out) return fail(CPAPR_EINVAL, "out is NULL");
        *out = nullptr;
        Error e = check_coo(X, R, true);
        if (e.code) return report(e);
        e = check_params(p, R, X->nmodes);
        if (e.code) return report(e);
        const bool mixed = p->precision == CPAPR_MIXED;
        const Layout L = layout(X->nmodes, X->nnz, X->dims, R, mixed, p->method, p->deterministic != 0);
        if (!ws) return fail(CPAPR_EWORKSPACE, "workspace is NULL");
        if (((uintptr_t)ws & 255) != 0) return fail(CPAPR_EWORKSPACE, "workspace must be 256-byte aligned");
        if (ws_bytes < L.total) return fail(CPAPR_EWORKSPACE, "workspace too small");

        cpapr_plan* P = new (std::nothrow) cpapr_plan();
        if (!P) return fail(CPAPR_EINVAL, "out of host memory");
        char* w = (char*)ws;
        P->N = X->nmodes;
        P->nnz = X->nnz;
        P->R = R;
        for (int m = 0; m < P->N; ++m) P->dims[m] = X->dims[m];
        P->params = *p;
        P->ws = w;
        P->ws_bytes = ws_bytes;
        P->group = p->group ? cpapr::resolve_group(R, p->group, X->nmodes - 1) : cpapr::model_group(P);
        P->chunk = cpapr::resolve_chunk(P->group, p->chunk);  // replaced by the model below if 0
        for (int n = 0; n < P->N; ++n) {
            P->mode[n].rows = (int32_t*)(w + L.mode_rows[n]);
            P->mode[n].cofs = (uint32_t*)(w + L.mode_cidx[n]);
            P->mode[n].vals = (double*)(w + L.mode_vals[n]);
            P->mode[n].pk = P->N <= 3 && X->nnz > 0 ? (int4*)(w + L.mode_pk[n]) : nullptr;
            P->f32[n] = mixed ? (float*)(w + L.f32[n]) : nullptr;
            P->phi_prev[n] = (double*)(w + L.phi_prev[n]);
        }
        P->B = (double*)(w + L.B);
        P->partial = (double*)(w + L.partial);
        P->llpart = (double*)(w + L.llpart);
        P->colsums = (double*)(w + L.colsums);
        P->state = (cpapr::DevState*)(w + L.state);
        P->det_part = p->deterministic ? (double*)(w + L.det_part) : nullptr;
        P->det_rows = p->deterministic ? (int32_t*)(w + L.det_rows) : nullptr;
        P->det_tiles = cpapr::det_tile_capacity(X->nnz);
        int64_t maxI = 0;
        for (int m = 0; m < P->N; ++m) maxI = std::max(maxI, P->dims[m]);
        if (p->method == CPAPR_METHOD_PQNR) cpapr::pqnr_bind(&P->pq, w + L.pqnr, maxI, R);
        if (p->method == CPAPR_METHOD_PDNR) cpapr::pdnr_bind(&P->pd, w + L.pdnr, maxI, R);

        hipStream_t s = (hipStream_t)stream;
        e = cpapr::build_sorted(P, X, w + L.region2, s);
        if (e.code) {
            delete P;
            return report(e);
        }
        if (p->chunk == 0) P->chunk = cpapr::model_chunk(P, P->group);
        P->shape_auto = p->group == 0 && p->chunk == 0;
        if (P->det_part != nullptr && (int64_t)(cpapr::kBlock / P->group) * P->chunk < 128) {
            delete P;
            return fail(CPAPR_EUNSUPPORTED, "deterministic mode needs tiles of at least 128 nonzeros");
        }
        e = cpapr::launch_reset_state(P->state, true, true, s);
        if (e.code) {
            delete P;
            return report(e);
        }
        if (hipStreamSynchronize(s) != hipSuccess) {
            delete P;
            return fail(CPAPR_EHIP, "stream synchronisation failed");
        }
        *out = P;
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_plan_destroy(cpapr_plan* plan)
{
    delete plan;
    return CPAPR_OK;
}

int cpapr_plan_set_shape(cpapr_plan* plan, int32_t group, int32_t chunk)
{
    if (!plan) return fail(CPAPR_EINVAL, "plan is NULL");
    cpapr_params p = plan->params;
    p.group = group;
    p.chunk = chunk;
    Error e = check_params(&p, plan->R, plan->N);
    if (e.code) return report(e);
    const int new_group = group ? cpapr::resolve_group(plan->R, group, plan->N - 1) : cpapr::model_group(plan);
    const int new_chunk = chunk > 0 ? chunk : cpapr::model_chunk(plan, new_group);
    if (plan->det_part != nullptr && (int64_t)(cpapr::kBlock / new_group) * new_chunk < 128)
        return fail(CPAPR_EUNSUPPORTED, "deterministic mode needs tiles of at least 128 nonzeros");
    plan->params = p;
    plan->group = new_group;
    plan->chunk = new_chunk;
    plan->shape_auto = group == 0 && chunk == 0;
    return CPAPR_OK;
}

int cpapr_plan_shape(const cpapr_plan* plan, int32_t* group, int32_t* chunk)
{
    if (!plan) return fail(CPAPR_EINVAL, "plan is NULL");
    if (group) *group = plan->group;
    if (chunk) *chunk = plan->chunk;
    return CPAPR_OK;
}

int64_t cpapr_plan_segments(const cpapr_plan* plan, int32_t mode)
{
    if (!plan || mode < 0 || mode >= plan->N) return -1;
    return plan->mode[mode].segments;
}

int cpapr_phi(cpapr_plan* plan, int32_t mode, const double* B, const double* const* A, double eps, double* Phi,
              void* stream)
{
    try {
        Error e = check_plan_call(plan, mode);
        if (e.code) return report(e);
        e = check_factors(plan, A, mode);
        if (e.code) return report(e);
        if (!B || !Phi) return fail(CPAPR_EINVAL, "B or Phi is NULL");
        if (!(eps > 0.0) || !std::isfinite(eps)) return fail(CPAPR_EINVAL, "eps must be finite and > 0");
        hipStream_t s = (hipStream_t)stream;
        const void* fac[CPAPR_MAX_MODES];
        e = phi_factors(plan, mode, A, fac, s);
        if (e.code) return report(e);
        e = cpapr::launch_fill(Phi, plan->dims[mode] * (int64_t)plan->R, 0.0, nullptr, s);
        if (e.code) return report(e);
        e = cpapr::launch_phi(plan, mode, B, fac, plan->params.precision == CPAPR_MIXED, eps, Phi, nullptr, s);
        return report(e);
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_phi_coo_workspace_size(const cpapr_coo* X, int32_t mode, int32_t R, size_t* bytes)
{
    try {
        Error e = cpapr::check_transient(X, mode, R, false);
        if (e.code) return report(e);
        if (!bytes) return fail(CPAPR_EINVAL, "bytes is NULL");
        *bytes = cpapr::transient_layout(X->nmodes, X->nnz).total;
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_phi_coo(const cpapr_coo* X, int32_t mode, int32_t R, const double* B, const double* const* A, double eps,
                  double* Phi, void* ws, size_t ws_bytes, void* stream)
{
    try {
        return report(cpapr::phi_transient(X, mode, R, B, A, eps, Phi, (char*)ws, ws_bytes, (hipStream_t)stream));
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_mu_inner(cpapr_plan* plan, int32_t mode, double* B, const double* const* A, double* Phi_last,
                   cpapr_stats* out, void* stream)
{
    try {
        Error e = check_plan_call(plan, mode);
        if (e.code) return report(e);
        e = check_factors(plan, A, mode);
        if (e.code) return report(e);
        if (!B || !Phi_last) return fail(CPAPR_EINVAL, "B or Phi_last is NULL");
        hipStream_t s = (hipStream_t)stream;
        const void* fac[CPAPR_MAX_MODES];
        e = phi_factors(plan, mode, A, fac, s);
        if (e.code) return report(e);
        e = cpapr::launch_reset_state(plan->state, true, true, s);
        if (e.code) return report(e);
        e = enqueue_inner(plan, mode, B, fac, Phi_last, s);
        if (e.code) return report(e);
        HostState h{};
        e = read_state(plan, &h, s);
        if (e.code) return report(e);
        if (out) {
            out->outer_iters = 0;
            out->converged = h.done;
            out->inner_iters = h.updates;
            out->kkt_violation = h.last_viol[mode];
            out->loglik = NAN;
            out->phi_evals = h.phi_evals;
            out->row_steps = 0;
            out->trial_evals = 0;
        }
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

namespace {

// Row-solve inner loop of one mode (PQNR or PDNR) behind the two entry points.
int rows_inner(cpapr_plan* plan, int32_t method, int32_t mode, double* B, const double* const* A,
               cpapr_stats* out, void* stream)
{
    try {
        Error e = check_plan_call(plan, mode);
        if (e.code) return report(e);
        if (plan->params.method != method)
            return fail(CPAPR_EINVAL, method == CPAPR_METHOD_PQNR ? "the plan was not created for PQNR"
                                                                  : "the plan was not created for PDNR");
        e = check_factors(plan, A, mode);
        if (e.code) return report(e);
        if (!B) return fail(CPAPR_EINVAL, "B is NULL");
        hipStream_t s = (hipStream_t)stream;
        const void* fac[CPAPR_MAX_MODES];
        e = phi_factors(plan, mode, A, fac, s);
        if (e.code) return report(e);
        e = cpapr::launch_reset_state(plan->state, true, true, s);
        if (e.code) return report(e);
        e = method == CPAPR_METHOD_PQNR ? cpapr::enqueue_pqnr_inner(plan, mode, B, fac, plan->phi_prev[mode], s)
                                        : cpapr::enqueue_pdnr_inner(plan, mode, B, fac, plan->phi_prev[mode], s);
        if (e.code) return report(e);
        HostState h{};
        e = read_state(plan, &h, s);
        if (e.code) return report(e);
        if (out) {
            out->outer_iters = 0;
            out->converged = h.done;
            out->inner_iters = h.updates;
            out->kkt_violation = h.last_viol[mode];
            out->loglik = NAN;
            out->phi_evals = h.phi_evals;
            out->row_steps = h.row_steps;
            out->trial_evals = h.trial_evals;
        }
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

}  // namespace

int cpapr_pqnr_inner(cpapr_plan* plan, int32_t mode, double* B, const double* const* A, cpapr_stats* out,
                     void* stream)
{
    return rows_inner(plan, CPAPR_METHOD_PQNR, mode, B, A, out, stream);
}

int cpapr_pdnr_inner(cpapr_plan* plan, int32_t mode, double* B, const double* const* A, cpapr_stats* out,
                     void* stream)
{
    return rows_inner(plan, CPAPR_METHOD_PDNR, mode, B, A, out, stream);
}

int cpapr_row_stats(cpapr_plan* plan, int32_t mode, int32_t* steps, double* viol, void* stream)
{
    try {
        Error e = check_plan_call(plan, mode);
        if (e.code) return report(e);
        const int32_t* s_src = nullptr;
        const double* v_src = nullptr;
        if (plan->params.method == CPAPR_METHOD_PQNR) {
            s_src = plan->pq.steps;
            v_src = plan->pq.viol;
        } else if (plan->params.method == CPAPR_METHOD_PDNR) {
            s_src = plan->pd.steps;
            v_src = plan->pd.viol;
        } else {
            return fail(CPAPR_EINVAL, "the plan was not created for row solves (PQNR or PDNR)");
        }
        const int64_t rows = plan->dims[mode];
        hipStream_t s = (hipStream_t)stream;
        if (steps && rows > 0)
            if (hipMemcpyAsync(steps, s_src, (size_t)rows * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(CPAPR_EHIP, "hipMemcpyAsync of the row steps failed");
        if (viol && rows > 0)
            if (hipMemcpyAsync(viol, v_src, (size_t)rows * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(CPAPR_EHIP, "hipMemcpyAsync of the row violations failed");
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_solve(cpapr_plan* plan, double* lambda, double* const* A, cpapr_stats* out, void* stream)
{
    try {
        if (!plan) return fail(CPAPR_EINVAL, "plan is NULL");
        Error e = check_factors(plan, (const double* const*)A, -1);
        if (e.code) return report(e);
        if (!lambda) return fail(CPAPR_EINVAL, "lambda is NULL");
        cpapr_plan* P = plan;
        hipStream_t s = (hipStream_t)stream;
        const int N = P->N, R = P->R;
        const bool mixed = P->params.precision == CPAPR_MIXED;
        const double tol = P->params.tol;
        const void* fac[CPAPR_MAX_MODES];
        for (int m = 0; m < N; ++m) {
            if (mixed) {
                e = cpapr::launch_to_f32(A[m], P->f32[m], P->dims[m] * (int64_t)R, s);
                if (e.code) return report(e);
                fac[m] = P->f32[m];
            } else {
                fac[m] = A[m];
            }
        }
        e = cpapr::launch_reset_state(P->state, true, true, s);
        if (e.code) return report(e);
        int k = 1, converged = 0;
        for (; k <= P->params.kmax; ++k) {
            for (int n = 0; n < N; ++n) {
                const int64_t In = P->dims[n];
                e = cpapr::launch_reset_state(P->state, n == 0, false, s);
                if (e.code) return report(e);
                const int32_t method = P->params.method;
                e = cpapr::launch_shift_scale(A[n], P->phi_prev[n], lambda, P->B, In, R, P->params.kappa,
                                              P->params.kappa_tol, k > 1, s);
                if (e.code) return report(e);
                e = method == CPAPR_METHOD_PQNR   ? cpapr::enqueue_pqnr_inner(P, n, P->B, fac, P->phi_prev[n], s)
                    : method == CPAPR_METHOD_PDNR ? cpapr::enqueue_pdnr_inner(P, n, P->B, fac, P->phi_prev[n], s)
                                                  : enqueue_inner(P, n, P->B, fac, P->phi_prev[n], s);
                if (e.code) return report(e);
                e = cpapr::launch_colsum(P->B, In, R, P->partial, lambda, s);
                if (e.code) return report(e);
                e = cpapr::launch_normalize(P->B, lambda, A[n], mixed ? P->f32[n] : nullptr, In, R, s);
                if (e.code) return report(e);
            }
            if (tol > 0.0) {
                int sweep = 0;
                if (hipMemcpyAsync(&sweep, &P->state->sweep_updates, sizeof(int), hipMemcpyDeviceToHost, s) !=
                        hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return fail(CPAPR_EHIP, "reading the sweep status failed");
                if (sweep == 0) {
                    converged = 1;
                    break;
                }
            }
        }
        if (k > P->params.kmax) k = P->params.kmax;
        e = cpapr::launch_loglik(P, lambda, (const double* const*)A, P->params.eps, s);
        if (e.code) return report(e);
        HostState h{};
        e = read_state(P, &h, s);
        if (e.code) return report(e);
        if (out) {
            out->outer_iters = k;
            out->converged = converged;
            out->inner_iters = h.total_updates;
            double kkt = 0.0;
            for (int n = 0; n < N; ++n) kkt = std::max(kkt, h.last_viol[n]);
            out->kkt_violation = kkt;
            out->loglik = h.ll;
            out->phi_evals = h.phi_evals;
            out->row_steps = h.row_steps;
            out->trial_evals = h.trial_evals;
        }
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_mode_begin(cpapr_plan* plan, int32_t mode, int32_t outer_iter, const double* lambda, double* A_mode,
                     const double* phi_prev, double* B, void* stream)
{
    Error e = check_plan_call(plan, mode);
    if (e.code) return report(e);
    if (!lambda || !A_mode || !B) return fail(CPAPR_EINVAL, "lambda, A_mode or B is NULL");
    const bool shift = outer_iter > 1 && phi_prev != nullptr;
    return report(cpapr::launch_shift_scale(A_mode, phi_prev, lambda, B, plan->dims[mode], plan->R, plan->params.kappa,
                                            plan->params.kappa_tol, shift, (hipStream_t)stream));
}

int cpapr_mode_end(cpapr_plan* plan, int32_t mode, const double* B, double* lambda, double* A_mode, void* stream)
{
    Error e = check_plan_call(plan, mode);
    if (e.code) return report(e);
    if (!lambda || !A_mode || !B) return fail(CPAPR_EINVAL, "lambda, A_mode or B is NULL");
    hipStream_t s = (hipStream_t)stream;
    e = cpapr::launch_colsum(B, plan->dims[mode], plan->R, plan->partial, lambda, s);
    if (e.code) return report(e);
    float* a32 = plan->params.precision == CPAPR_MIXED ? plan->f32[mode] : nullptr;
    return report(cpapr::launch_normalize(B, lambda, A_mode, a32, plan->dims[mode], plan->R, s));
}

int cpapr_modes_advance(int32_t count, cpapr_plan* const* plans, const int32_t* end_mode, const int32_t* begin_mode,
                        const int32_t* outer_iter, double* const* lambda, double* const* const* A, double* const* B,
                        const double* const* phi_prev, void* stream)
{
    if (count < 0) return fail(CPAPR_EINVAL, "count must be >= 0");
    if (count > 0 && (!plans || !end_mode || !begin_mode || !outer_iter || !lambda || !A || !B))
        return fail(CPAPR_EINVAL, "an item array is NULL");
    for (int32_t i = 0; i < count; ++i) {
        cpapr_plan* P = plans[i];
        if (!P || !A[i]) return fail(CPAPR_EINVAL, "item " + std::to_string(i) + ": plan or factor array is NULL");
        const int e0 = end_mode[i], b0 = begin_mode[i];
        if ((e0 >= 0 && e0 >= P->N) || (b0 >= 0 && b0 >= P->N))
            return fail(CPAPR_EINVAL, "item " + std::to_string(i) + ": mode out of range");
        if (e0 >= 0) {
            const int rc = cpapr_mode_end(P, e0, B[i], lambda[i], A[i][e0], stream);
            if (rc != CPAPR_OK) return rc;
        }
        if (b0 >= 0) {
            const int rc = cpapr_mode_begin(P, b0, outer_iter[i], lambda[i], A[i][b0], phi_prev ? phi_prev[i] : nullptr,
                                            B[i], stream);
            if (rc != CPAPR_OK) return rc;
        }
    }
    return CPAPR_OK;
}

int cpapr_plan_sync_f32(cpapr_plan* plan, const double* const* A, void* stream)
{
    if (!plan) return fail(CPAPR_EINVAL, "plan is NULL");
    if (plan->params.precision != CPAPR_MIXED) return CPAPR_OK;
    Error e = check_factors(plan, A, -1);
    if (e.code) return report(e);
    for (int m = 0; m < plan->N; ++m) {
        e = cpapr::launch_to_f32(A[m], plan->f32[m], plan->dims[m] * (int64_t)plan->R, (hipStream_t)stream);
        if (e.code) return report(e);
    }
    return CPAPR_OK;
}

int cpapr_loglik(cpapr_plan* plan, const double* lambda, const double* const* A, double eps, double* out,
                 void* stream)
{
    try {
        if (!plan) return fail(CPAPR_EINVAL, "plan is NULL");
        Error e = check_factors(plan, A, -1);
        if (e.code) return report(e);
        if (!lambda || !out) return fail(CPAPR_EINVAL, "lambda or out is NULL");
        if (!(eps > 0.0)) return fail(CPAPR_EINVAL, "eps must be > 0");
        hipStream_t s = (hipStream_t)stream;
        e = cpapr::launch_loglik(plan, lambda, A, eps, s);
        if (e.code) return report(e);
        HostState h{};
        e = read_state(plan, &h, s);
        if (e.code) return report(e);
        *out = h.ll;
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_mttkrp(cpapr_plan* plan, int32_t mode, const double* const* A, double* M, void* stream)
{
    try {
        Error e = check_plan_call(plan, mode);
        if (e.code) return report(e);
        e = check_factors(plan, A, mode);
        if (e.code) return report(e);
        if (!M) return fail(CPAPR_EINVAL, "M is NULL");
        return report(cpapr::launch_mttkrp(plan, mode, A, M, (hipStream_t)stream));
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_prof_enable(int32_t capacity) { return cpapr_prof_enable_sampled(capacity, 1); }

int cpapr_prof_enable_sampled(int32_t capacity, int32_t every)
{
    if (capacity < 1 || capacity > (1 << 20)) return fail(CPAPR_EINVAL, "capacity must be in [1, 2^20]");
    if (every < 1) return fail(CPAPR_EINVAL, "every must be >= 1");
    cpapr_prof_disable();
    g_prof.start.resize(capacity);
    g_prof.stop.resize(capacity);
    g_prof.mode.assign(capacity, -1);
    for (int i = 0; i < capacity; ++i) {
        if (hipEventCreate(&g_prof.start[i]) != hipSuccess || hipEventCreate(&g_prof.stop[i]) != hipSuccess) {
            g_prof.cap = i;
            cpapr_prof_disable();
            return fail(CPAPR_EHIP, "hipEventCreate failed");
        }
    }
    g_prof.cap = capacity;
    g_prof.count = 0;
    g_prof.every = every;
    g_prof.seen = 0;
    g_prof.open = false;
    g_prof.on = true;
    return CPAPR_OK;
}

int cpapr_prof_disable(void)
{
    for (int i = 0; i < g_prof.cap; ++i) {
        hipEventDestroy(g_prof.start[i]);
        hipEventDestroy(g_prof.stop[i]);
    }
    g_prof.start.clear();
    g_prof.stop.clear();
    g_prof.mode.clear();
    g_prof.cap = 0;
    g_prof.count = 0;
    g_prof.on = false;
    return CPAPR_OK;
}

int cpapr_prof_read(int32_t* modes, float* ms, int32_t cap)
{
    if (!modes || !ms || cap < 0) return fail(CPAPR_EINVAL, "bad arguments");
    const int n = std::min(cap, g_prof.count);
    for (int i = 0; i < n; ++i) {
        if (hipEventSynchronize(g_prof.stop[i]) != hipSuccess) return fail(CPAPR_EHIP, "hipEventSynchronize failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, g_prof.start[i], g_prof.stop[i]) != hipSuccess)
            return fail(CPAPR_EHIP, "hipEventElapsedTime failed");
        modes[i] = g_prof.mode[i];
        ms[i] = t;
    }
    return n;
}

}  // extern "C"
