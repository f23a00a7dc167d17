// Batched Phi: host side of the slot lists, their device copies, and the
// launch / hipGraph sequence (kernels in phi.hip).
//
// Device work lists: one BatchSlot per set slot (operands + first tile in its
// shape class), a tile -> slot map per class, per-class offsets and tile
// counts, and the fill / conversion list. Kernels read all of them from
// device memory, so a captured graph replays correctly after a commit that
// keeps the same set of shape classes.
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using cpapr::BatchCopy;
using cpapr::BatchSlot;
using cpapr::Error;

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kMaxClasses = cpapr::kBatchClassesMax;

struct HostSlot {
    bool set = false;
    int flags = 0;
    cpapr_plan* plan = nullptr;
    int mode = 0;
    const double* B = nullptr;
    const double* A[CPAPR_MAX_MODES] = {};
    double* Phi = nullptr;
};

struct Layout {
    size_t slots, tile_map, class_off, class_ntiles, copies, ncopies, copy_total;
    size_t mu, nmu, mu_total, viol, st_done, st_updates, st_viol, st_hold, counters, total;
};

Layout layout(int max_slots, int64_t max_tiles)
{
    Layout L{};
    size_t off = 0;
    L.slots = off;
    off += align256(sizeof(BatchSlot) * (size_t)max_slots);
    L.tile_map = off;
    off += align256(4 * (size_t)std::max<int64_t>(max_tiles, 1));
    L.class_off = off;
    off += align256(8 * kMaxClasses);
    L.class_ntiles = off;
    off += align256(8 * kMaxClasses);
    L.copies = off;
    off += align256(sizeof(BatchCopy) * (size_t)max_slots * CPAPR_MAX_MODES);
    L.ncopies = off;
    off += 256;
    L.copy_total = off;
    off += 256;
    L.mu = off;
    off += align256(sizeof(cpapr::BatchMu) * (size_t)max_slots);
    L.nmu = off;
    off += 256;
    L.mu_total = off;
    off += 256;
    L.viol = off;
    off += align256(8 * (size_t)cpapr::kMuSpread * max_slots);
    L.st_done = off;
    off += align256(4 * (size_t)max_slots);
    L.st_updates = off;
    off += align256(4 * (size_t)max_slots);
    L.st_viol = off;
    off += align256(8 * (size_t)max_slots);
    L.st_hold = off;
    off += align256(4 * (size_t)max_slots);
    L.counters = off;
    off += align256(4 * (size_t)cpapr::kBatchCounters * cpapr::kCounterStride);
    L.total = off;
    return L;
}

// Tiles of one slot of this plan (at its batch shape).
int64_t plan_tiles(const cpapr_plan* P)
{
    int G, L;
    cpapr::batch_shape(P, &G, &L);
    return cdiv(P->nnz, (int64_t)(cpapr::kBlock / G) * L);
}

int slot_class(const cpapr_plan* P)
{
    int G, L;
    cpapr::batch_shape(P, &G, &L);
    return cpapr::batch_class_of(G, cpapr::rank_block(P->R, G), P->N - 1, P->params.precision == CPAPR_MIXED);
}

}  // namespace

struct cpapr_batch {
    int max_slots;
    int64_t max_tiles;
    char* ws;
    Layout L;
    BatchSlot* d_slots;
    int32_t* d_tile_map;
    int64_t* d_class_off;
    int64_t* d_class_ntiles;
    BatchCopy* d_copies;
    int32_t* d_ncopies;
    int64_t* d_copy_total;
    cpapr::BatchMu* d_mu;
    int32_t* d_nmu;
    int64_t* d_mu_total;
    unsigned long long* d_viol;
    unsigned int* d_counters;
    cpapr::BatchState st;
    std::vector<HostSlot> slots;
    std::vector<int32_t> hold;          // per slot: 1 = sits out the next runs (uploaded by commit and hold)
    bool committed = false;
    std::vector<int> classes;           // classes with work at the last commit
    std::vector<int64_t> class_tiles;   // their tile counts (grid launches)
    bool persistent = true;
    bool skip_held = false;             // held slots are left out of the launches at commit
    int grid_cache[kMaxClasses] = {};   // persistent grid per class
    int copy_grid = 0;
    struct Graph {
        hipGraphExec_t exec = nullptr;
        std::vector<int> classes;  // classes captured
        std::vector<int64_t> tiles;  // per-class tile counts captured (grid launches)
        int lmax = 0;              // inner iterations captured (0: Phi only)
    } graph_run, graph_inner;
};

namespace {

int fail(int code, const std::string& msg)
{
    cpapr::set_last_error(msg);
    return code;
}

int report(const Error& e)
{
    if (e.code) cpapr::set_last_error(e.msg);
    return e.code;
}

Error ensure_grids(cpapr_batch* b)
{
    if (b->copy_grid <= 0) {
        int dev = 0, cus = 0;
        CPAPR_HIP(hipGetDevice(&dev));
        CPAPR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        b->copy_grid = 4 * std::max(1, cus);
    }
    return {CPAPR_OK, ""};
}

// Phi for every slot whose done flag is clear: zero their Phi (and refresh FP32
// factor copies), then one persistent launch per shape class.
Error enqueue_phi(cpapr_batch* b, const std::vector<int>& classes, hipStream_t s)
{
    Error e = ensure_grids(b);
    if (e.code) return e;
    e = cpapr::launch_batch_elementwise(b->d_copies, b->d_ncopies, b->d_copy_total, b->st.done, b->d_counters,
                                        b->copy_grid, s);
    if (e.code) return e;
    for (int c : classes) {
        const int64_t grid_tiles = b->persistent ? 0 : b->class_tiles[c];
        e = cpapr::launch_phi_batch(c, b->d_slots, b->d_tile_map, b->d_class_off, b->d_class_ntiles, b->st.done,
                                    b->d_counters, &b->grid_cache[c], grid_tiles, s);
        if (e.code) return e;
    }
    return {CPAPR_OK, ""};
}

Error enqueue_mu(cpapr_batch* b, hipStream_t s)
{
    Error e = ensure_grids(b);
    if (e.code) return e;
    return cpapr::launch_batch_mu(b->d_mu, b->d_nmu, b->d_mu_total, b->max_slots, b->d_viol, b->st, b->copy_grid, s);
}

// lmax == 0: clear the per-slot state and compute Phi for every slot.
// lmax > 0: clear it and run lmax x {Phi, KKT, MU update} with per-slot stops.
Error enqueue_sequence(cpapr_batch* b, int lmax, hipStream_t s)
{
    Error e = cpapr::launch_batch_reset(b->st, b->max_slots, s);
    if (e.code) return e;
    if (lmax == 0) return enqueue_phi(b, b->classes, s);
    for (int l = 0; l < lmax; ++l) {
        e = enqueue_phi(b, b->classes, s);
        if (e.code) return e;
        e = enqueue_mu(b, s);
        if (e.code) return e;
    }
    return {CPAPR_OK, ""};
}

// Run a sequence directly, or replay it from a graph captured for the current
// set of shape classes (capturing, after one direct run, when needed).
int run_sequence(cpapr_batch* b, cpapr_batch::Graph& g, int lmax, bool use_graph, hipStream_t s)
{
    if (!use_graph) return report(enqueue_sequence(b, lmax, s));
    bool covered = g.exec != nullptr && g.lmax == lmax;
    for (int c : b->classes)
        if (std::find(g.classes.begin(), g.classes.end(), c) == g.classes.end()) covered = false;
    if (!b->persistent && g.tiles != b->class_tiles) covered = false;  // grid sizes are baked into the graph
    if (covered) {
        if (hipGraphLaunch(g.exec, s) != hipSuccess) return fail(CPAPR_EHIP, "hipGraphLaunch failed");
        return CPAPR_OK;
    }
    if (s == nullptr) return fail(CPAPR_EINVAL, "graph capture needs a non-null stream");
    if (g.exec) {
        hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
    }
    // One direct run first: it computes this call's result and performs the
    // occupancy queries and lazy kernel loading outside the capture.
    Error e = enqueue_sequence(b, lmax, s);
    if (e.code) return report(e);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(CPAPR_EHIP, "hipStreamBeginCapture failed");
    e = enqueue_sequence(b, lmax, s);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (e.code) {
        if (graph) hipGraphDestroy(graph);
        return report(e);
    }
    if (ec != hipSuccess || !graph) return fail(CPAPR_EHIP, "hipStreamEndCapture failed");
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        g.exec = nullptr;
        return fail(CPAPR_EHIP, "hipGraphInstantiate failed");
    }
    g.classes = b->classes;
    g.tiles = b->class_tiles;
    g.lmax = lmax;
    return CPAPR_OK;
}

}  // namespace

extern "C" {

int cpapr_batch_workspace_size(int32_t max_slots, int64_t max_tiles, size_t* bytes)
{
    if (max_slots < 1 || max_tiles < 0 || max_tiles > 0x7fffffffLL || !bytes)
        return fail(CPAPR_EINVAL, "max_slots must be >= 1, max_tiles in [0, 2^31), bytes not NULL");
    *bytes = layout(max_slots, max_tiles).total;
    return CPAPR_OK;
}

int64_t cpapr_batch_tiles(const cpapr_plan* plan)
{
    if (!plan) return -1;
    return plan_tiles(plan);
}

int cpapr_plan_batch_shape(const cpapr_plan* plan, int32_t* group, int32_t* chunk)
{
    if (!plan) return fail(CPAPR_EINVAL, "plan is NULL");
    int G, L;
    cpapr::batch_shape(plan, &G, &L);
    if (group) *group = G;
    if (chunk) *chunk = L;
    return CPAPR_OK;
}

int cpapr_batch_create(int32_t max_slots, int64_t max_tiles, void* ws, size_t ws_bytes, cpapr_batch** out)
{
    return cpapr_batch_create2(max_slots, max_tiles, 0, ws, ws_bytes, out);
}

int cpapr_batch_create2(int32_t max_slots, int64_t max_tiles, int32_t flags, void* ws, size_t ws_bytes,
                        cpapr_batch** out)
{
    try {
        if (!out) return fail(CPAPR_EINVAL, "out is NULL");
        *out = nullptr;
        if (max_slots < 1 || max_tiles < 0 || max_tiles > 0x7fffffffLL)
            return fail(CPAPR_EINVAL, "max_slots must be >= 1 and max_tiles in [0, 2^31)");
        const Layout L = layout(max_slots, max_tiles);
        if (!ws || ((uintptr_t)ws & 255)) return fail(CPAPR_EWORKSPACE, "workspace missing or not 256-byte aligned");
        if (ws_bytes < L.total) return fail(CPAPR_EWORKSPACE, "workspace too small");
        cpapr_batch* b = new (std::nothrow) cpapr_batch();
        if (!b) return fail(CPAPR_EINVAL, "out of host memory");
        if (flags & ~(CPAPR_BATCH_PERSISTENT | CPAPR_BATCH_SKIP_HELD)) {
            delete b;
            return fail(CPAPR_EINVAL, "unknown batch flags");
        }
        b->persistent = (flags & CPAPR_BATCH_PERSISTENT) != 0;
        b->skip_held = (flags & CPAPR_BATCH_SKIP_HELD) != 0;
        b->max_slots = max_slots;
        b->max_tiles = max_tiles;
        b->ws = (char*)ws;
        b->L = L;
        b->d_slots = (BatchSlot*)(b->ws + L.slots);
        b->d_tile_map = (int32_t*)(b->ws + L.tile_map);
        b->d_class_off = (int64_t*)(b->ws + L.class_off);
        b->d_class_ntiles = (int64_t*)(b->ws + L.class_ntiles);
        b->d_copies = (BatchCopy*)(b->ws + L.copies);
        b->d_ncopies = (int32_t*)(b->ws + L.ncopies);
        b->d_copy_total = (int64_t*)(b->ws + L.copy_total);
        b->d_mu = (cpapr::BatchMu*)(b->ws + L.mu);
        b->d_nmu = (int32_t*)(b->ws + L.nmu);
        b->d_mu_total = (int64_t*)(b->ws + L.mu_total);
        b->d_viol = (unsigned long long*)(b->ws + L.viol);
        b->st.done = (int32_t*)(b->ws + L.st_done);
        b->st.updates = (int32_t*)(b->ws + L.st_updates);
        b->st.viol = (double*)(b->ws + L.st_viol);
        b->st.hold = (int32_t*)(b->ws + L.st_hold);
        b->d_counters = (unsigned int*)(b->ws + L.counters);
        b->slots.resize(max_slots);
        b->hold.assign(max_slots, 0);
        *out = b;
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_batch_destroy(cpapr_batch* batch)
{
    if (!batch) return CPAPR_OK;
    if (batch->graph_run.exec) hipGraphExecDestroy(batch->graph_run.exec);
    if (batch->graph_inner.exec) hipGraphExecDestroy(batch->graph_inner.exec);
    delete batch;
    return CPAPR_OK;
}

int cpapr_batch_set(cpapr_batch* batch, int32_t slot, cpapr_plan* plan, int32_t mode, const double* B,
                    const double* const* A, double* Phi, int32_t flags)
{
    if (!batch || !plan) return fail(CPAPR_EINVAL, "batch or plan is NULL");
    if (slot < 0 || slot >= batch->max_slots) return fail(CPAPR_EINVAL, "slot out of range");
    if (mode < 0 || mode >= plan->N) return fail(CPAPR_EINVAL, "mode out of range");
    if (!B || !Phi || !A) return fail(CPAPR_EINVAL, "B, A or Phi is NULL");
    for (int m = 0; m < plan->N; ++m)
        if (m != mode && !A[m]) return fail(CPAPR_EINVAL, "a factor pointer is NULL");
    if (plan->params.variant == CPAPR_VARIANT_ATOMIC) return fail(CPAPR_EUNSUPPORTED, "batches run the segmented kernel");
    if (slot_class(plan) < 0)
        return fail(CPAPR_EUNSUPPORTED, "no batched kernel for this plan's shape (lane group 4, 8 or 16; N <= 4)");
    if (flags & ~CPAPR_BATCH_F32_CURRENT) return fail(CPAPR_EINVAL, "unknown flags");
    HostSlot& h = batch->slots[slot];
    h.set = true;
    h.flags = flags;
    h.plan = plan;
    h.mode = mode;
    h.B = B;
    for (int m = 0; m < CPAPR_MAX_MODES; ++m) h.A[m] = m < plan->N ? A[m] : nullptr;
    h.Phi = Phi;
    batch->committed = false;
    return CPAPR_OK;
}

int cpapr_batch_clear(cpapr_batch* batch, int32_t slot)
{
    if (!batch) return fail(CPAPR_EINVAL, "batch is NULL");
    if (slot < 0 || slot >= batch->max_slots) return fail(CPAPR_EINVAL, "slot out of range");
    batch->slots[slot] = HostSlot();
    batch->committed = false;
    return CPAPR_OK;
}

int cpapr_batch_commit(cpapr_batch* batch, void* stream)
{
    try {
        if (!batch) return fail(CPAPR_EINVAL, "batch is NULL");
        cpapr_batch* b = batch;
        hipStream_t s = (hipStream_t)stream;
        const int ncls = cpapr::batch_class_count();
        std::vector<std::vector<int>> by_class(ncls);
        for (int i = 0; i < b->max_slots; ++i) {
            const HostSlot& h = b->slots[i];
            if (!h.set || (b->skip_held && b->hold[i])) continue;
            const cpapr_plan* P = h.plan;
            const int c = slot_class(P);
            if (c < 0) return fail(CPAPR_EUNSUPPORTED, "slot with an unsupported shape");
            by_class[c].push_back(i);
        }
        std::vector<BatchSlot> hs;
        std::vector<int32_t> tmap;
        std::vector<int64_t> coff(kMaxClasses, 0), cnt(kMaxClasses, 0);
        std::vector<BatchCopy> copies;
        int64_t copy_total = 0;
        std::vector<int> classes;
        for (int c = 0; c < ncls; ++c) {
            coff[c] = (int64_t)tmap.size();
            int64_t tiles = 0;
            for (int i : by_class[c]) {
                const HostSlot& h = b->slots[i];
                const cpapr_plan* P = h.plan;
                const bool mixed = P->params.precision == CPAPR_MIXED;
                const void* fac[CPAPR_MAX_MODES] = {};
                for (int m = 0; m < P->N; ++m) {
                    if (m == h.mode) continue;
                    if (mixed) {
                        if (!(h.flags & CPAPR_BATCH_F32_CURRENT)) {
                            BatchCopy cp{h.A[m], P->f32[m], P->dims[m] * (int64_t)P->R, copy_total, 1, -1};
                            copies.push_back(cp);
                            copy_total += cp.n;
                        }
                        fac[m] = P->f32[m];
                    } else {
                        fac[m] = h.A[m];
                    }
                }
                BatchCopy z{nullptr, h.Phi, P->dims[h.mode] * (int64_t)P->R, copy_total, 0, i};
                copies.push_back(z);
                copy_total += z.n;
                BatchSlot bs{};
                bs.args = cpapr::phi_args(P, h.mode, h.B, fac, P->params.eps, h.Phi);
                int G;
                cpapr::batch_shape(P, &G, &bs.args.L);
                bs.tile_begin = tiles;
                bs.slot = i;
                const int64_t nt = plan_tiles(P);
                const int32_t idx = (int32_t)hs.size();
                hs.push_back(bs);
                for (int64_t q = 0; q < nt; ++q) tmap.push_back(idx);
                tiles += nt;
                if ((int64_t)tmap.size() > b->max_tiles) return fail(CPAPR_EWORKSPACE, "more tiles than max_tiles");
            }
            cnt[c] = tiles;
            if (tiles > 0) classes.push_back(c);
        }
        const int32_t ncopies = (int32_t)copies.size();
        std::vector<cpapr::BatchMu> mus;
        int64_t mu_total = 0;
        for (int i = 0; i < b->max_slots; ++i) {
            const HostSlot& h = b->slots[i];
            if (!h.set || (b->skip_held && b->hold[i])) continue;
            const cpapr_plan* P = h.plan;
            cpapr::BatchMu mu{const_cast<double*>(h.B), h.Phi, P->dims[h.mode] * (int64_t)P->R, mu_total,
                              P->params.tol, i, 0};
            mus.push_back(mu);
            mu_total += mu.n;
        }
        const int32_t nmu = (int32_t)mus.size();
        if (!mus.empty() && hipMemcpyAsync(b->d_mu, mus.data(), sizeof(cpapr::BatchMu) * mus.size(),
                                           hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(CPAPR_EHIP, "upload of the MU list failed");
        if (hipMemcpyAsync(b->d_nmu, &nmu, 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(b->d_mu_total, &mu_total, 8, hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(CPAPR_EHIP, "upload of MU list sizes failed");
        if (!hs.empty()) {
            if (hipMemcpyAsync(b->d_slots, hs.data(), sizeof(BatchSlot) * hs.size(), hipMemcpyHostToDevice, s) !=
                hipSuccess)
                return fail(CPAPR_EHIP, "upload of batch slots failed");
        }
        if (!tmap.empty() &&
            hipMemcpyAsync(b->d_tile_map, tmap.data(), 4 * tmap.size(), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(CPAPR_EHIP, "upload of the tile map failed");
        if (hipMemcpyAsync(b->d_class_off, coff.data(), 8 * kMaxClasses, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(b->d_class_ntiles, cnt.data(), 8 * kMaxClasses, hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(CPAPR_EHIP, "upload of class tables failed");
        if (!copies.empty() && hipMemcpyAsync(b->d_copies, copies.data(), sizeof(BatchCopy) * copies.size(),
                                              hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(CPAPR_EHIP, "upload of the fill list failed");
        if (hipMemcpyAsync(b->d_ncopies, &ncopies, 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(b->d_copy_total, &copy_total, 8, hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(CPAPR_EHIP, "upload of list sizes failed");
        if (hipMemcpyAsync(b->st.hold, b->hold.data(), 4 * (size_t)b->max_slots, hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return fail(CPAPR_EHIP, "upload of the hold flags failed");
        if (hipStreamSynchronize(s) != hipSuccess) return fail(CPAPR_EHIP, "stream synchronisation failed");
        b->classes = classes;
        b->class_tiles.assign(cnt.begin(), cnt.end());
        b->committed = true;
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_batch_hold(cpapr_batch* batch, const int32_t* hold, void* stream)
{
    try {
        if (!batch) return fail(CPAPR_EINVAL, "batch is NULL");
        if (!hold) return fail(CPAPR_EINVAL, "hold is NULL");
        bool changed = false;
        for (int i = 0; i < batch->max_slots; ++i) {
            const int32_t v = hold[i] != 0;
            changed = changed || v != batch->hold[i];
            batch->hold[i] = v;
        }
        // left out of the launches: the held set takes effect at the next commit
        if (batch->skip_held && changed) batch->committed = false;
        hipStream_t s = (hipStream_t)stream;
        if (hipMemcpyAsync(batch->st.hold, batch->hold.data(), 4 * (size_t)batch->max_slots, hipMemcpyHostToDevice,
                           s) != hipSuccess)
            return fail(CPAPR_EHIP, "upload of the hold flags failed");
        if (hipStreamSynchronize(s) != hipSuccess) return fail(CPAPR_EHIP, "stream synchronisation failed");
        return CPAPR_OK;
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_batch_mu(cpapr_batch* batch, void* stream)
{
    if (!batch) return fail(CPAPR_EINVAL, "batch is NULL");
    if (!batch->committed) return fail(CPAPR_EINVAL, "batch not committed since the last change");
    return report(enqueue_mu(batch, (hipStream_t)stream));
}

int cpapr_batch_status(cpapr_batch* batch, double* viol, int32_t* updates, int32_t* done, void* stream)
{
    if (!batch || !viol || !updates || !done) return fail(CPAPR_EINVAL, "batch or an output array is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)batch->max_slots;
    if (hipMemcpyAsync(viol, batch->st.viol, 8 * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(updates, batch->st.updates, 4 * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(done, batch->st.done, 4 * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(CPAPR_EHIP, "reading the batch status failed");
    return CPAPR_OK;
}

int cpapr_batch_run(cpapr_batch* batch, int32_t use_graph, void* stream)
{
    try {
        if (!batch) return fail(CPAPR_EINVAL, "batch is NULL");
        if (!batch->committed) return fail(CPAPR_EINVAL, "batch not committed since the last change");
        return run_sequence(batch, batch->graph_run, 0, use_graph != 0, (hipStream_t)stream);
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

int cpapr_batch_inner(cpapr_batch* batch, int32_t lmax, int32_t use_graph, void* stream)
{
    try {
        if (!batch) return fail(CPAPR_EINVAL, "batch is NULL");
        if (lmax < 1 || lmax > CPAPR_MAX_LMAX) return fail(CPAPR_EINVAL, "lmax must be in [1, 4096]");
        if (!batch->committed) return fail(CPAPR_EINVAL, "batch not committed since the last change");
        return run_sequence(batch, batch->graph_inner, lmax, use_graph != 0, (hipStream_t)stream);
    } catch (...) {
        return fail(CPAPR_EINVAL, "unexpected exception");
    }
}

}  // extern "C"
