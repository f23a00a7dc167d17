// Kernels around Phi in Algorithm 1: the MU step B <- B .* Phi, the KKT
// violation max |min(B, 1 - Phi)|, the inadmissible-zero shift and
// B = (A + S) Lambda, lambda = e^T B with A = B Lambda^-1, FP32 factor copies,
// and the Poisson log-likelihood.
//
// The inner loop's stop decision never leaves the device: the KKT kernel
// max-reduces the violation into a per-iteration slot; the update kernel reads
// it, and when it is below tol raises a `done` flag that every later kernel of
// the same inner loop checks before doing any work. The host enqueues lmax
// iterations without waiting.
//
// All reductions are two-level with a fixed partition and a fixed order, so
// their results are bitwise reproducible run to run.
#include <algorithm>

#include "internal.hpp"

namespace cpapr {
namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline unsigned grid_for(int64_t n, int64_t cap = 4096)
{
    int64_t g = cdiv(n, kBlock);
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

__global__ __launch_bounds__(kBlock) void fill_kernel(double* p, int64_t n, double v, const int* done)
{
    if (done != nullptr && *done) return;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                                        int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        dst[i] = (float)src[i];
}

__global__ __launch_bounds__(kBlock) void reset_state_kernel(DevState* st, int new_sweep, int all)
{
    for (int i = threadIdx.x; i < 2 * kViolSlots * kViolStride; i += kBlock) (&st->viol[0][0])[i] = 0ull;
    if (threadIdx.x == 0) {
        st->done = 0;
        st->updates = 0;
        if (new_sweep) st->sweep_updates = 0;
        if (all) {
            st->total_updates = 0;
            st->phi_evals = 0;
            st->row_steps = 0;
            st->trial_evals = 0;
            for (int m = 0; m < CPAPR_MAX_MODES; ++m) st->last_viol[m] = 0.0;
        }
    }
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Max over entries of |min(B, 1 - Phi)|, folded into the slots of parity l & 1
// (ordered bit patterns of nonnegative doubles, so u64 max is double max).
__global__ __launch_bounds__(kBlock) void kkt_kernel(const double* __restrict__ B, const double* __restrict__ Phi,
                                                     int64_t n, DevState* st, int l)
{
    if (st->done) return;
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double b = B[i], q = 1.0 - Phi[i];
        v = fmax(v, fabs(b < q ? b : q));
    }
    __shared__ double red[kBlock / 64];
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0) st->phi_evals += 1;  // this iteration's Phi was computed
        double m = red[0];
        for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, red[w]);
        const int slot = blockIdx.x % kViolSlots;
        atomicMax(&st->viol[l & 1][slot * kViolStride], (unsigned long long)__double_as_longlong(m));
    }
}

// B <- B .* Phi unless the KKT test says stop. Every block folds the slots to
// the same violation; only block 0 records it, raises `done` and clears the
// other parity's slots for the next iteration. Other blocks of this launch
// that see `done` early skip work they would have skipped anyway. With
// zero_phi the consumed Phi is cleared for the next iteration's accumulation
// (never on a stop, so the last Phi survives).
__global__ __launch_bounds__(kBlock) void mu_update_kernel(double* __restrict__ B, double* __restrict__ Phi,
                                                           int64_t n, DevState* st, int l, int mode, double tol,
                                                           int zero_phi)
{
    if (st->done) return;
    __shared__ double viol_sh;
    if (threadIdx.x < 64) {
        double v = __longlong_as_double((long long)st->viol[l & 1][threadIdx.x * kViolStride]);
        v = wave_max(v);
        if (threadIdx.x == 0) viol_sh = v;
    }
    __syncthreads();
    const double viol = viol_sh;
    const bool stop = tol > 0.0 && viol < tol;
    if (blockIdx.x == 0) {
        if (threadIdx.x < kViolSlots) st->viol[(l + 1) & 1][threadIdx.x * kViolStride] = 0ull;
        if (threadIdx.x == 0) {
            st->last_viol[mode] = viol;
            if (stop) {
                st->done = 1;
            } else {
                st->updates += 1;
                st->sweep_updates += 1;
                st->total_updates += 1;
            }
        }
    }
    if (stop) return;
    if (zero_phi) {
        for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
            B[i] *= Phi[i];
            Phi[i] = 0.0;
        }
    } else {
        for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
            B[i] *= Phi[i];
    }
}

// A fixed schedule (tol <= 0) takes no stop decision, so iteration l's KKT
// violation (before the update) and the update go through the entries in one
// pass: B <- B .* Phi (Phi cleared for the next accumulation with zero_phi)
// while the block maxima of |min(B, 1 - Phi)| fold into the slots of parity
// l & 1. Block 0 folds the previous iteration's slots (complete: that launch
// has finished) into last_viol and clears them for iteration l + 1; after the
// last iteration kkt_fold_kernel folds its slots. Counters as kkt_kernel and
// mu_update_kernel keep them.
__global__ __launch_bounds__(kBlock) void mu_fused_kernel(double* __restrict__ B, double* __restrict__ Phi, int64_t n,
                                                          DevState* st, int l, int mode, int zero_phi)
{
    if (st->done) return;
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        const int prev = (l + 1) & 1;
        if (l > 0) {
            double v = __longlong_as_double((long long)st->viol[prev][threadIdx.x * kViolStride]);
            v = wave_max(v);
            if (threadIdx.x == 0) st->last_viol[mode] = v;
        }
        if (threadIdx.x < kViolSlots) st->viol[prev][threadIdx.x * kViolStride] = 0ull;
        if (threadIdx.x == 0) {
            st->phi_evals += 1;
            st->updates += 1;
            st->sweep_updates += 1;
            st->total_updates += 1;
        }
    }
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double b = B[i], p = Phi[i], q = 1.0 - p;
        v = fmax(v, fabs(b < q ? b : q));
        B[i] = b * p;
        if (zero_phi) Phi[i] = 0.0;
    }
    __shared__ double red[kBlock / 64];
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, red[w]);
        atomicMax(&st->viol[l & 1][(blockIdx.x % kViolSlots) * kViolStride], (unsigned long long)__double_as_longlong(m));
    }
}

// The last iteration's violation of a fused loop: fold its slots into
// last_viol and clear them.
__global__ __launch_bounds__(64) void kkt_fold_kernel(DevState* st, int l, int mode)
{
    if (st->done) return;
    double v = __longlong_as_double((long long)st->viol[l & 1][threadIdx.x * kViolStride]);
    v = wave_max(v);
    if (threadIdx.x == 0) st->last_viol[mode] = v;
    if (threadIdx.x < kViolSlots) st->viol[l & 1][threadIdx.x * kViolStride] = 0ull;
}

// A(n) += kappa where A < kappa_tol and the previous Phi > 1 (from the second
// outer iteration on), then B = A(n) diag(lambda).
__global__ __launch_bounds__(kBlock) void shift_scale_kernel(double* __restrict__ A,
                                                             const double* __restrict__ phi_prev,
                                                             const double* __restrict__ lam, double* __restrict__ B,
                                                             int64_t n, int R, double kappa, double kappa_tol,
                                                             int shift)
{
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
        double a = A[e];
        if (shift && a < kappa_tol && phi_prev[e] > 1.0) {
            a += kappa;
            A[e] = a;
        }
        B[e] = a * lam[e % R];
    }
}

// Column sums, level 1: block b sums rows [b*rpb, (b+1)*rpb) with Q = 256/R
// threads per column, then reduces the Q partials in order.
__global__ __launch_bounds__(kBlock) void colsum_partial_kernel(const double* __restrict__ M, int64_t I, int R,
                                                                int64_t rpb, double* __restrict__ partial)
{
    __shared__ double sm[kBlock];
    const int Q = kBlock / R;
    const int t = threadIdx.x;
    const int c = t % R, q = t / R;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = min(r0 + rpb, I);
    double s = 0.0;
    if (q < Q)
        for (int64_t i = r0 + q; i < r1; i += Q) s += M[i * R + c];
    sm[t] = q < Q ? s : 0.0;
    __syncthreads();
    if (t < R) {
        double tot = 0.0;
        for (int qq = 0; qq < Q; ++qq) tot += sm[qq * R + t];
        partial[(int64_t)blockIdx.x * R + t] = tot;
    }
}

// Column sums, level 2: Q = 256/R threads per column each sum a fixed stride of
// the partials, then one thread per column adds the Q results in order.
__global__ __launch_bounds__(kBlock) void colsum_final_kernel(const double* __restrict__ partial, int nparts, int R,
                                                              double* __restrict__ out)
{
    __shared__ double sm[kBlock];
    const int Q = kBlock / R;
    const int t = threadIdx.x;
    const int c = t % R, q = t / R;
    double s = 0.0;
    if (q < Q)
        for (int b = q; b < nparts; b += Q) s += partial[(int64_t)b * R + c];
    sm[t] = q < Q ? s : 0.0;
    __syncthreads();
    if (t < R) {
        double tot = 0.0;
        for (int qq = 0; qq < Q; ++qq) tot += sm[qq * R + t];
        out[t] = tot;
    }
}

__global__ __launch_bounds__(kBlock) void normalize_kernel(const double* __restrict__ B,
                                                           const double* __restrict__ lam, double* __restrict__ A,
                                                           float* __restrict__ A32, int64_t n, int R)
{
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
        const double l = lam[e % R];
        const double a = l > 0.0 ? B[e] / l : 0.0;
        A[e] = a;
        if (A32) A32[e] = (float)a;
    }
}

__global__ __launch_bounds__(kBlock) void loglik_final_kernel(const double* __restrict__ partial, int nparts,
                                                              const double* __restrict__ lam,
                                                              const double* __restrict__ colsums, int N, int R,
                                                              DevState* st)
{
    __shared__ double sm[kBlock];
    double part = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) part += partial[b];
    sm[threadIdx.x] = part;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < kBlock; ++q) s += sm[q];
    double mass = 0.0;
    for (int r = 0; r < R; ++r) {
        double p = lam[r];
        for (int m = 0; m < N; ++m) p *= colsums[(int64_t)m * R + r];
        mass += p;
    }
    st->ll = s - mass;
}

// Locate the first list item whose range contains element e0 (items sorted by begin).
template <typename Item>
__device__ __forceinline__ int first_item(const Item* items, int nitems, int64_t e0)
{
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (items[mid].begin <= e0) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void batch_clear_kernel(unsigned long long* viol, int n)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) viol[i] = 0ull;
}

__global__ __launch_bounds__(kBlock) void batch_reset_kernel(BatchState st, int n)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        st.done[i] = st.hold != nullptr ? st.hold[i] : 0;  // a held slot does no work in this run
        st.updates[i] = 0;
        st.viol[i] = 0.0;
    }
}

// Per slot: max over its entries of |min(B, 1 - Phi)|. Workgroup b takes a
// contiguous range of the concatenated element space; its maxima go to one of
// kMuSpread line-separated words of each slot it touches.
__global__ __launch_bounds__(kBlock) void batch_kkt_kernel(const BatchMu* __restrict__ items,
                                                           const int32_t* __restrict__ nitems_dev,
                                                           const int64_t* __restrict__ total_dev, int max_slots,
                                                           unsigned long long* viol, const int32_t* __restrict__ done)
{
    __shared__ double red[kBlock / 64];
    const int nitems = *nitems_dev;
    const int64_t total = *total_dev;
    const int64_t per = ((total + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int64_t e0 = blockIdx.x * per, e1 = min(e0 + per, total);
    if (e0 >= e1) return;
    for (int it = first_item(items, nitems, e0); it < nitems && items[it].begin < e1; ++it) {
        const BatchMu m = items[it];
        if (done[m.slot]) continue;  // block-uniform
        const int64_t a0 = max(e0, m.begin) - m.begin, a1 = min(e1, m.begin + m.n) - m.begin;
        double v = 0.0;
        for (int64_t i = a0 + threadIdx.x; i < a1; i += kBlock) {
            const double b = m.B[i], q = 1.0 - m.Phi[i];
            v = fmax(v, fabs(b < q ? b : q));
        }
        v = wave_max(v);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double w = red[0];
            for (int q = 1; q < kBlock / 64; ++q) w = fmax(w, red[q]);
            const int j = blockIdx.x % kMuSpread;
            atomicMax(&viol[(int64_t)j * max_slots + m.slot], (unsigned long long)__double_as_longlong(w));
        }
        __syncthreads();
    }
}

// Per slot: B <- B .* Phi unless tol > 0 and its violation < tol, which stops
// the slot's inner loop (done flag). The workgroup whose range holds a slot's
// first element records the violation, the decision and the update count.
// Blocks of this launch that see a flag raised by it skip work they would have
// skipped anyway (a raised flag means no update).
__global__ __launch_bounds__(kBlock) void batch_update_kernel(const BatchMu* __restrict__ items,
                                                              const int32_t* __restrict__ nitems_dev,
                                                              const int64_t* __restrict__ total_dev, int max_slots,
                                                              const unsigned long long* __restrict__ viol,
                                                              BatchState st)
{
    const int nitems = *nitems_dev;
    const int64_t total = *total_dev;
    const int64_t per = ((total + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int64_t e0 = blockIdx.x * per, e1 = min(e0 + per, total);
    if (e0 >= e1) return;
    for (int it = first_item(items, nitems, e0); it < nitems && items[it].begin < e1; ++it) {
        const BatchMu m = items[it];
        if (st.done[m.slot]) continue;
        double v = 0.0;
        for (int j = 0; j < kMuSpread; ++j)
            v = fmax(v, __longlong_as_double((long long)viol[(int64_t)j * max_slots + m.slot]));
        const bool upd = !(m.tol > 0.0 && v < m.tol);
        if (threadIdx.x == 0 && m.begin >= e0) {
            st.viol[m.slot] = v;
            if (upd)
                st.updates[m.slot] += 1;
            else
                st.done[m.slot] = 1;
        }
        if (!upd) continue;
        const int64_t a0 = max(e0, m.begin) - m.begin, a1 = min(e1, m.begin + m.n) - m.begin;
        for (int64_t i = a0 + threadIdx.x; i < a1; i += kBlock) m.B[i] *= m.Phi[i];
    }
}

}  // namespace

Error launch_batch_mu(const BatchMu* items, const int32_t* nitems_dev, const int64_t* total_dev, int max_slots,
                      unsigned long long* viol_spread, BatchState st, int grid, hipStream_t s)
{
    batch_clear_kernel<<<32, kBlock, 0, s>>>(viol_spread, kMuSpread * max_slots);
    CPAPR_LAUNCHED();
    batch_kkt_kernel<<<grid, kBlock, 0, s>>>(items, nitems_dev, total_dev, max_slots, viol_spread, st.done);
    CPAPR_LAUNCHED();
    batch_update_kernel<<<grid, kBlock, 0, s>>>(items, nitems_dev, total_dev, max_slots, viol_spread, st);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_batch_reset(BatchState st, int max_slots, hipStream_t s)
{
    batch_reset_kernel<<<std::max(1, std::min(64, (max_slots + kBlock - 1) / kBlock)), kBlock, 0, s>>>(st, max_slots);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_fill(double* p, int64_t n, double v, const int* done, hipStream_t s)
{
    if (n <= 0) return {CPAPR_OK, ""};
    fill_kernel<<<grid_for(n, 8192), kBlock, 0, s>>>(p, n, v, done);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return {CPAPR_OK, ""};
    to_f32_kernel<<<grid_for(n, 8192), kBlock, 0, s>>>(src, dst, n);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_reset_state(DevState* st, bool new_sweep, bool all, hipStream_t s)
{
    reset_state_kernel<<<1, kBlock, 0, s>>>(st, new_sweep ? 1 : 0, all ? 1 : 0);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_kkt(const double* B, const double* Phi, int64_t n, DevState* st, int l, hipStream_t s)
{
    kkt_kernel<<<grid_for(n, 2048), kBlock, 0, s>>>(B, Phi, n, st, l);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_mu_update(double* B, double* Phi, int64_t n, DevState* st, int l, int mode, double tol, bool zero_phi,
                       hipStream_t s)
{
    mu_update_kernel<<<grid_for(n, 4096), kBlock, 0, s>>>(B, Phi, n, st, l, mode, tol, zero_phi ? 1 : 0);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_mu_fused(double* B, double* Phi, int64_t n, DevState* st, int l, int mode, bool zero_phi, hipStream_t s)
{
    mu_fused_kernel<<<grid_for(n, 4096), kBlock, 0, s>>>(B, Phi, n, st, l, mode, zero_phi ? 1 : 0);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_kkt_fold(DevState* st, int l, int mode, hipStream_t s)
{
    kkt_fold_kernel<<<1, 64, 0, s>>>(st, l, mode);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_shift_scale(double* A, const double* phi_prev, const double* lam, double* B, int64_t I, int R,
                         double kappa, double kappa_tol, bool shift, hipStream_t s)
{
    const int64_t n = I * R;
    shift_scale_kernel<<<grid_for(n, 4096), kBlock, 0, s>>>(A, phi_prev, lam, B, n, R, kappa, kappa_tol,
                                                            shift ? 1 : 0);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_colsum(const double* M, int64_t I, int R, double* partial, double* out, hipStream_t s)
{
    int64_t nparts = cdiv(I, 64);
    if (nparts > kPartials) nparts = kPartials;
    if (nparts < 1) nparts = 1;
    const int64_t rpb = cdiv(I, nparts);
    colsum_partial_kernel<<<(unsigned)nparts, kBlock, 0, s>>>(M, I, R, rpb, partial);
    CPAPR_LAUNCHED();
    colsum_final_kernel<<<1, kBlock, 0, s>>>(partial, (int)nparts, R, out);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_normalize(const double* B, const double* lam, double* A, float* A32, int64_t I, int R, hipStream_t s)
{
    const int64_t n = I * R;
    normalize_kernel<<<grid_for(n, 4096), kBlock, 0, s>>>(B, lam, A, A32, n, R);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_loglik(const cpapr_plan* P, const double* lam, const double* const* A, double eps, hipStream_t s)
{
    const int N = P->N, R = P->R;
    for (int m = 0; m < N; ++m) {
        Error e = launch_colsum(A[m], P->dims[m], R, P->partial, P->colsums + (int64_t)m * R, s);
        if (e.code) return e;
    }
    // m_k = sum_r lambda_r prod_m A(m)[i_m, r] = B[i_0, :] . pi_k with B = A(0) diag(lambda):
    // the Phi engine's dot product on the mode-0 copy.
    Error e = launch_shift_scale(const_cast<double*>(A[0]), nullptr, lam, P->B, P->dims[0], R, 0.0, 0.0, false, s);
    if (e.code) return e;
    int nparts = 0;
    e = launch_loglik_terms(P, P->B, A, eps, P->llpart, &nparts, s);
    if (e.code) return e;
    loglik_final_kernel<<<1, kBlock, 0, s>>>(P->llpart, nparts, lam, P->colsums, N, R, P->state);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

}  // namespace cpapr
