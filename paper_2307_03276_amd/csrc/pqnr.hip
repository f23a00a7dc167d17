// PQNR: projected quasi-Newton solves of the row subproblems of one mode.
//
// The paper lists this CP-APR variant beside MU in its Background: every row
// of B = A(n) Lambda is its own subproblem, converging independently of the
// other rows. With the other factors' columns summing to one, row i minimises
//   f_i(b) = sum_r b_r - sum_{k in row i} x_k log(max(b . pi_k, eps)),  b >= 0,
// whose gradient is g = 1 - (row i of Phi), Phi from Algorithm 2. So the Phi
// engine supplies every gradient, and a second pass over the nonzeros (the
// line-search kind of the Phi tile code) supplies f_i(b + delta) - f_i(b) for
// the trial steps of every row still in a line search at once (the other rows'
// nonzeros are skipped, gathers included).
//
// One inner iteration for all rows of the mode, with no host round trip:
//   Phi pass            -> gradients (skipped once every row has converged)
//   pqnr_begin_kernel   -> KKT test, curvature pair, direction, first trial
//   kPqnrTrials x { line-search pass (skipped when no row searches),
//                   pqnr_accept_kernel: accept, shorten the step, or take the MU step }
// A lane group of RG lanes owns one row: its R columns are spread over the
// lanes (coalesced row access) and dot products are group reductions.
//
// Row rules (the same as the oracle's, which documents them): KKT viol =
// max |min(b, g)|, stop when tau > 0 and viol < tau; keep (s, y) when
// s.y > kPqnrCurv |s| |y| (at most kPqnrMem); bound set b_r == 0 and g_r > 0;
// two-loop L-BFGS direction on the free set with the newest usable pair's
// scaling, else the MU direction -b .* g; projected backtracking from
// alpha = 1 with sufficient decrease kPqnrSigma, rejecting trials that bring
// a model value of the row down to the floor eps (they leave the objective's
// domain); after kPqnrTrials rejected trials the MU step b + (-b .* g), and the
// row's pairs are dropped.
#include <algorithm>

#include "internal.hpp"

namespace cpapr {
namespace {

constexpr int kCpl = 4;  // columns per lane at most (R <= 4 * RG, RG <= 64)

enum : int32_t { kActive = 0, kSearching = 1, kConverged = 3 };

template <int RG>
__device__ __forceinline__ double rg_sum(double v)
{
#pragma unroll
    for (int off = RG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int RG>
__device__ __forceinline__ double rg_max(double v)
{
#pragma unroll
    for (int off = RG / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

struct RowArgs {
    double* B;
    const double* buf;  // Phi (begin) or line-search sums (accept)
    int64_t rows;
    int R;
    double tau;
    PqnrState q;
    DevState* st;
};

__global__ __launch_bounds__(kBlock) void pqnr_reset_kernel(PqnrState q, int64_t rows, DevState* st)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kBlock) {
        q.status[i] = kActive;
        q.trials[i] = 0;
        q.steps[i] = 0;
        q.npairs[i] = 0;
        q.head[i] = 0;
        q.viol[i] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq_all_done = rows == 0 ? 1 : 0;
        st->pq_idle = 1;
    }
}

// Before the rows decide: assume every row done / no row searching; rows that
// keep working clear the flags. Counts the Phi pass that just ran, if any.
__global__ void pqnr_flags_kernel(DevState* st, int before_begin)
{
    if (threadIdx.x == 0) {
        if (before_begin) {
            if (!st->pq_all_done) st->phi_evals += 1;
            st->pq_all_done = 1;
        } else {
            if (!st->pq_idle) st->trial_evals += 1;
        }
        st->pq_idle = 1;
    }
}

// Trial step for length alpha along the stored direction; returns g . delta.
template <int RG>
__device__ __forceinline__ double make_trial(const RowArgs& a, int64_t i, int lane, double alpha, const double (&b)[kCpl],
                                             const double (&g)[kCpl])
{
    double gd = 0.0;
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = lane + j * RG;
        if (c < a.R) {
            const double d = a.q.Dd[i * a.R + c];
            const double nb = b[j] + alpha * d;
            const double delta = (nb > 0.0 ? nb : 0.0) - b[j];
            a.q.Dt[i * a.R + c] = delta;
            gd += g[j] * delta;
        }
    }
    return rg_sum<RG>(gd);
}

template <int RG>
__global__ __launch_bounds__(kBlock) void pqnr_begin_kernel(RowArgs a)
{
    constexpr int RPB = kBlock / RG;
    const int lane = threadIdx.x % RG;
    const int64_t i = (int64_t)blockIdx.x * RPB + threadIdx.x / RG;
    if (i >= a.rows) return;
    const int32_t status = a.q.status[i];
    if (status == kConverged) return;
    const int R = a.R;
    const PqnrState& q = a.q;
    double b[kCpl], g[kCpl];
    bool fr[kCpl];
    double viol = 0.0;
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = lane + j * RG;
        b[j] = g[j] = 0.0;
        fr[j] = false;
        if (c < R) {
            b[j] = a.B[i * R + c];
            g[j] = 1.0 - a.buf[i * R + c];
            q.G[i * R + c] = g[j];
            viol = fmax(viol, fabs(b[j] < g[j] ? b[j] : g[j]));
            fr[j] = !(b[j] == 0.0 && g[j] > 0.0);
        }
    }
    viol = rg_max<RG>(viol);
    if (lane == 0) q.viol[i] = viol;
    if (a.tau > 0.0 && viol < a.tau) {
        if (lane == 0) q.status[i] = kConverged;
        return;
    }
    if (lane == 0) a.st->pq_all_done = 0;

    // curvature pair from the previous step
    int np = q.npairs[i], hd = q.head[i];
    if (q.steps[i] > 0) {
        double sy = 0.0, ss = 0.0, yy = 0.0;
        double sv[kCpl], yv[kCpl];
#pragma unroll
        for (int j = 0; j < kCpl; ++j) {
            const int c = lane + j * RG;
            sv[j] = yv[j] = 0.0;
            if (c < R) {
                sv[j] = q.Dt[i * R + c];
                yv[j] = g[j] - q.Gp[i * R + c];
                sy += sv[j] * yv[j];
                ss += sv[j] * sv[j];
                yy += yv[j] * yv[j];
            }
        }
        sy = rg_sum<RG>(sy);
        ss = rg_sum<RG>(ss);
        yy = rg_sum<RG>(yy);
        if (sy > kPqnrCurv * sqrt(ss * yy)) {
#pragma unroll
            for (int j = 0; j < kCpl; ++j) {
                const int c = lane + j * RG;
                if (c < R) {
                    q.S[(int64_t)hd * q.stride * R + i * R + c] = sv[j];
                    q.Y[(int64_t)hd * q.stride * R + i * R + c] = yv[j];
                }
            }
            hd = (hd + 1) % kPqnrMem;
            np = np < kPqnrMem ? np + 1 : np;
            if (lane == 0) {
                q.head[i] = hd;
                q.npairs[i] = np;
            }
        }
    }

    // direction: two-loop recursion over the free set, else the MU direction
    double d[kCpl];
    bool use_mu = true;
    if (np > 0) {
        double qv[kCpl], al[kPqnrMem], syv[kPqnrMem];
#pragma unroll
        for (int j = 0; j < kCpl; ++j) qv[j] = fr[j] ? g[j] : 0.0;
        double gamma = 0.0;
        bool usable = false;
#pragma unroll
        for (int c2 = 0; c2 < kPqnrMem; ++c2) {  // newest to oldest
            if (c2 >= np) break;
            const int jp = (hd - 1 - c2 + 2 * kPqnrMem) % kPqnrMem;
            const double* Sj = q.S + (int64_t)jp * q.stride * R + i * R;
            const double* Yj = q.Y + (int64_t)jp * q.stride * R + i * R;
            double sy = 0.0, yy = 0.0, sq = 0.0;
#pragma unroll
            for (int j = 0; j < kCpl; ++j) {
                const int c = lane + j * RG;
                if (c < R && fr[j]) {
                    sy += Sj[c] * Yj[c];
                    yy += Yj[c] * Yj[c];
                    sq += Sj[c] * qv[j];
                }
            }
            sy = rg_sum<RG>(sy);
            yy = rg_sum<RG>(yy);
            sq = rg_sum<RG>(sq);
            syv[c2] = sy;
            al[c2] = 0.0;
            if (sy <= 0.0) continue;
            if (!usable) gamma = yy > 0.0 ? sy / yy : 0.0;
            usable = true;
            al[c2] = sq / sy;
#pragma unroll
            for (int j = 0; j < kCpl; ++j) {
                const int c = lane + j * RG;
                if (c < R && fr[j]) qv[j] -= al[c2] * Yj[c];
            }
        }
        if (usable && gamma > 0.0) {
#pragma unroll
            for (int j = 0; j < kCpl; ++j) qv[j] *= gamma;
#pragma unroll
            for (int c2 = kPqnrMem - 1; c2 >= 0; --c2) {  // oldest to newest
                if (c2 >= np || syv[c2] <= 0.0) continue;
                const int jp = (hd - 1 - c2 + 2 * kPqnrMem) % kPqnrMem;
                const double* Sj = q.S + (int64_t)jp * q.stride * R + i * R;
                const double* Yj = q.Y + (int64_t)jp * q.stride * R + i * R;
                double yq = 0.0;
#pragma unroll
                for (int j = 0; j < kCpl; ++j) {
                    const int c = lane + j * RG;
                    if (c < R && fr[j]) yq += Yj[c] * qv[j];
                }
                const double beta = rg_sum<RG>(yq) / syv[c2];
#pragma unroll
                for (int j = 0; j < kCpl; ++j) {
                    const int c = lane + j * RG;
                    if (c < R && fr[j]) qv[j] += (al[c2] - beta) * Sj[c];
                }
            }
            double gd = 0.0;
#pragma unroll
            for (int j = 0; j < kCpl; ++j) {
                d[j] = fr[j] ? -qv[j] : 0.0;
                gd += g[j] * d[j];
            }
            use_mu = !(rg_sum<RG>(gd) < 0.0);
        }
    }
    if (use_mu)
#pragma unroll
        for (int j = 0; j < kCpl; ++j) d[j] = -b[j] * g[j];
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = lane + j * RG;
        if (c < R) q.Dd[i * R + c] = d[j];
    }
    const double gd = make_trial<RG>(a, i, lane, 1.0, b, g);
    if (lane == 0) {
        q.alpha[i] = 1.0;
        q.gdel[i] = gd;
        q.trials[i] = 0;
        q.status[i] = kSearching;
        a.st->pq_idle = 0;
    }
}

template <int RG>
__global__ __launch_bounds__(kBlock) void pqnr_accept_kernel(RowArgs a)
{
    constexpr int RPB = kBlock / RG;
    const int lane = threadIdx.x % RG;
    const int64_t i = (int64_t)blockIdx.x * RPB + threadIdx.x / RG;
    if (i >= a.rows) return;
    if (a.q.status[i] != kSearching) return;
    const int R = a.R;
    const PqnrState& q = a.q;
    double b[kCpl], g[kCpl], lin = 0.0;
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = lane + j * RG;
        b[j] = g[j] = 0.0;
        if (c < R) {
            b[j] = a.B[i * R + c];
            g[j] = q.G[i * R + c];
            lin += q.Dt[i * R + c];
        }
    }
    lin = rg_sum<RG>(lin);
    const double gdel = q.gdel[i];
    const double df = lin - a.buf[i * R];
    const bool accept = gdel < 0.0 && df <= kPqnrSigma * gdel;
    const int t = q.trials[i] + 1;
    if (!accept && t < kPqnrTrials) {
        const double alpha = q.alpha[i] * 0.5;
        const double gd = make_trial<RG>(a, i, lane, alpha, b, g);
        if (lane == 0) {
            q.alpha[i] = alpha;
            q.gdel[i] = gd;
            q.trials[i] = t;
            a.st->pq_idle = 0;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = lane + j * RG;
        if (c < R) {
            const double delta = accept ? q.Dt[i * R + c] : -b[j] * g[j];  // else the MU step
            a.B[i * R + c] = b[j] + delta;
            q.Dt[i * R + c] = delta;
            q.Gp[i * R + c] = g[j];
        }
    }
    if (lane == 0) {
        q.steps[i] += 1;
        q.status[i] = kActive;
        if (!accept) q.npairs[i] = 0;  // the pairs led to no sufficient decrease: drop them
    }
}

// The same decision for all trials at once (R >= 4): the line-search pass has
// summed the four trials alpha = 1, 1/2, 1/4, 1/8 into columns 0-3, and the
// first acceptable one is taken, as the trial-by-trial rounds would.
template <int RG>
__global__ __launch_bounds__(kBlock) void pqnr_accept4_kernel(RowArgs a)
{
    static_assert(kPqnrTrials == 4, "the fused line-search pass evaluates four trials");
    constexpr int RPB = kBlock / RG;
    const int lane = threadIdx.x % RG;
    const int64_t i = (int64_t)blockIdx.x * RPB + threadIdx.x / RG;
    if (i >= a.rows) return;
    if (a.q.status[i] != kSearching) return;
    const int R = a.R;
    const PqnrState& q = a.q;
    double b[kCpl], g[kCpl], d[kCpl], step[kCpl];
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = lane + j * RG;
        b[j] = g[j] = d[j] = step[j] = 0.0;
        if (c < R) {
            b[j] = a.B[i * R + c];
            g[j] = q.G[i * R + c];
            d[j] = q.Dd[i * R + c];
        }
    }
    bool accept = false;
    double alpha = 1.0;
#pragma unroll
    for (int k = 0; k < kPqnrTrials; ++k, alpha *= 0.5) {
        double dl[kCpl], gd = 0.0, lin = 0.0;
#pragma unroll
        for (int j = 0; j < kCpl; ++j) {
            const int c = lane + j * RG;
            dl[j] = 0.0;
            if (c < R) {
                const double nb = b[j] + alpha * d[j];
                dl[j] = (nb > 0.0 ? nb : 0.0) - b[j];
                gd += g[j] * dl[j];
                lin += dl[j];
            }
        }
        gd = rg_sum<RG>(gd);
        lin = rg_sum<RG>(lin);
        const double df = lin - a.buf[i * R + k];
        if (!accept && gd < 0.0 && df <= kPqnrSigma * gd) {
            accept = true;
#pragma unroll
            for (int j = 0; j < kCpl; ++j) step[j] = dl[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = lane + j * RG;
        if (c < R) {
            const double delta = accept ? step[j] : -b[j] * g[j];  // else the MU step
            a.B[i * R + c] = b[j] + delta;
            q.Dt[i * R + c] = delta;
            q.Gp[i * R + c] = g[j];
        }
    }
    if (lane == 0) {
        q.steps[i] += 1;
        q.status[i] = kActive;
        if (!accept) q.npairs[i] = 0;
    }
}

// Per-mode results: most steps of a row, steps summed, largest last violation.
__global__ __launch_bounds__(kBlock) void pqnr_stats_kernel(PqnrState q, int64_t rows, int mode, DevState* st)
{
    __shared__ long long ssum[kBlock / 64];
    __shared__ int smax[kBlock / 64];
    __shared__ double svio[kBlock / 64];
    long long sum = 0;
    int mx = 0;
    double vio = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += kBlock) {
        sum += q.steps[i];
        mx = max(mx, (int)q.steps[i]);
        vio = fmax(vio, q.viol[i]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        mx = max(mx, __shfl_xor(mx, off));
        vio = fmax(vio, __shfl_xor(vio, off));
    }
    if ((threadIdx.x & 63) == 0) {
        ssum[threadIdx.x >> 6] = sum;
        smax[threadIdx.x >> 6] = mx;
        svio[threadIdx.x >> 6] = vio;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            sum += ssum[w];
            mx = max(mx, smax[w]);
            vio = fmax(vio, svio[w]);
        }
        st->updates = mx;
        st->sweep_updates += mx;
        st->total_updates += mx;
        st->row_steps += sum;
        st->last_viol[mode] = vio;
        st->done = st->pq_all_done;
    }
}

int row_group(int R)
{
    int rg = 4;
    while (rg < R && rg < 64) rg *= 2;
    return rg;
}

template <typename F>
Error by_group(int rg, F&& f)
{
    switch (rg) {
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 32: return f(std::integral_constant<int, 32>{});
        default: return f(std::integral_constant<int, 64>{});
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t pqnr_bytes(int64_t maxI, int R)
{
    const size_t mat = align256((size_t)maxI * R * 8);
    return mat * (5 + 2 * kPqnrMem) + 3 * align256((size_t)maxI * 8) + 5 * align256((size_t)maxI * 4);
}

void pqnr_bind(PqnrState* q, char* base, int64_t maxI, int R)
{
    const size_t mat = align256((size_t)maxI * R * 8);
    char* p = base;
    auto take = [&](size_t n) {
        char* r = p;
        p += n;
        return r;
    };
    q->G = (double*)take(mat);
    q->Gp = (double*)take(mat);
    q->Dd = (double*)take(mat);
    q->Dt = (double*)take(mat);
    q->T = (double*)take(mat);
    q->S = (double*)take(mat * kPqnrMem);
    q->Y = (double*)take(mat * kPqnrMem);
    q->alpha = (double*)take(align256((size_t)maxI * 8));
    q->gdel = (double*)take(align256((size_t)maxI * 8));
    q->viol = (double*)take(align256((size_t)maxI * 8));
    q->status = (int32_t*)take(align256((size_t)maxI * 4));
    q->trials = (int32_t*)take(align256((size_t)maxI * 4));
    q->steps = (int32_t*)take(align256((size_t)maxI * 4));
    q->npairs = (int32_t*)take(align256((size_t)maxI * 4));
    q->head = (int32_t*)take(align256((size_t)maxI * 4));
    q->stride = maxI;
}

Error enqueue_pqnr_inner(cpapr_plan* P, int mode, double* B, const void* const* fac, double* phi, hipStream_t s)
{
    const int64_t rows = P->dims[mode];
    const int R = P->R;
    if (R > 4 * 64) return {CPAPR_EUNSUPPORTED, "PQNR supports R <= 256"};
    const int64_t n = rows * (int64_t)R;
    DevState* st = P->state;
    const int* all_done = &st->pq_all_done;
    const int* idle = &st->pq_idle;
    const int rg = row_group(R);
    const int64_t blocks64 = (rows + (kBlock / rg) - 1) / (kBlock / rg);
    if (blocks64 > 0x7fffffff) return {CPAPR_EUNSUPPORTED, "too many rows"};
    const dim3 grid((unsigned)std::max<int64_t>(blocks64, 1));
    const int rgrid = (int)std::min<int64_t>(std::max<int64_t>((rows + kBlock - 1) / kBlock, 1), 4096);
    pqnr_reset_kernel<<<rgrid, kBlock, 0, s>>>(P->pq, rows, st);
    CPAPR_LAUNCHED();
    RowArgs ra{B, phi, rows, R, P->params.tol, P->pq, st};   // begin reads Phi
    RowArgs rt{B, P->pq.T, rows, R, P->params.tol, P->pq, st};  // accept reads the line-search sums
    for (int l = 0; l < P->params.lmax; ++l) {
        Error e = launch_fill(phi, n, 0.0, all_done, s);
        if (e.code) return e;
        e = launch_phi(P, mode, B, fac, false, P->params.eps, phi, all_done, s);
        if (e.code) return e;
        pqnr_flags_kernel<<<1, 64, 0, s>>>(st, 1);
        CPAPR_LAUNCHED();
        e = by_group(rg, [&](auto RG) -> Error {
            pqnr_begin_kernel<decltype(RG)::value><<<grid, kBlock, 0, s>>>(ra);
            CPAPR_LAUNCHED();
            return {CPAPR_OK, ""};
        });
        if (e.code) return e;
        if (R >= kPqnrTrials) {  // all trials in one line-search pass
            e = launch_fill(P->pq.T, n, 0.0, idle, s);
            if (e.code) return e;
            e = launch_delta4(P, mode, B, P->pq.Dd, P->pq.status, fac, P->params.eps, P->pq.T, idle, s);
            if (e.code) return e;
            pqnr_flags_kernel<<<1, 64, 0, s>>>(st, 0);
            CPAPR_LAUNCHED();
            e = by_group(rg, [&](auto RG) -> Error {
                pqnr_accept4_kernel<decltype(RG)::value><<<grid, kBlock, 0, s>>>(rt);
                CPAPR_LAUNCHED();
                return {CPAPR_OK, ""};
            });
            if (e.code) return e;
            continue;
        }
        for (int t = 0; t < kPqnrTrials; ++t) {  // R < 4: one pass per trial
            e = launch_fill(P->pq.T, n, 0.0, idle, s);
            if (e.code) return e;
            e = launch_delta(P, mode, B, P->pq.Dt, P->pq.status, fac, P->params.eps, P->pq.T, idle, s);
            if (e.code) return e;
            pqnr_flags_kernel<<<1, 64, 0, s>>>(st, 0);
            CPAPR_LAUNCHED();
            e = by_group(rg, [&](auto RG) -> Error {
                pqnr_accept_kernel<decltype(RG)::value><<<grid, kBlock, 0, s>>>(rt);
                CPAPR_LAUNCHED();
                return {CPAPR_OK, ""};
            });
            if (e.code) return e;
        }
    }
    pqnr_stats_kernel<<<1, kBlock, 0, s>>>(P->pq, rows, mode, st);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

}  // namespace cpapr
