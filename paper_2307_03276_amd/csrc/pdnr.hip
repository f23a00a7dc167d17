// PDNR: projected damped Newton solves of the row subproblems of one mode.
//
// The second row-wise CP-APR variant of the paper's Background. Every row b of
// B = A(n) Lambda minimises the same objective as in PQNR,
//   f_i(b) = sum_r b_r - sum_{k in row i} x_k log(max(b . pi_k, eps)),  b >= 0,
// with gradient g = 1 - (row i of Phi) and, here, its exact Hessian
//   H = sum_k x_k / max(m_k, eps)^2  pi_k pi_k^T,   m_k = b . pi_k.
//
// One inner iteration for all rows of the mode, with no host round trip:
//   pdnr_hess_kernel    -> Phi row and H of every active row (one pass over the
//                          mode-sorted nonzeros on the matrix cores; skipped once
//                          every row has converged)
//   pdnr_begin_kernel   -> KKT test, held set, damped Newton direction (Cholesky of
//                          the free block, one wave per row), first trial
//   line-search pass    -> the Phi engine's four-trial kind: f(b + delta) - f(b)
//                          for alpha = 1, 1/2, 1/4, 1/8 at once
//   pdnr_accept4_kernel -> the first acceptable trial (damping from the ratio of
//                          actual to predicted decrease) or the MU step
// (R < 4: kPdnrTrials rounds of a one-trial pass and pdnr_accept_kernel, which
// accepts, shortens the step or takes the MU step.)
//
// Row rules (the oracle documents the same ones): stop when tau > 0 and
// max|min(b, g)| < tau; entries with g_r > 0 and b_r <= kPdnrHeld are held
// (d_r = -g_r); on the free set F solve (H_FF + mu t I) d_F = -g_F with
// t = trace(H_FF) / |F|; the MU direction -b .* g when t is not > 0, a pivot
// is not > 0 or g.d >= 0; projected backtracking from alpha = 1 with
// sufficient decrease kPdnrSigma, trials that bring a model value of the row
// to the floor eps rejected; after kPdnrTrials rejected trials the MU step and
// mu grows. An accepted step sets rho = actual / predicted decrease of the
// quadratic model (-(g.delta + delta^T H delta / 2)): rho < 1/4 grows mu,
// rho > 3/4 shrinks it (factor kPdnrMuStep, within [kPdnrMuMin, kPdnrMuMax]).
//
// H and the Phi row live together in one accumulation row of R*R + R doubles
// per matrix row. The Hessian pass adds into it (plain stores for rows that lie
// inside one wave's range, atomics for rows at range ends); the row kernels clear
// it once the row's line search is over, so it is zero again for the next pass
// (and stays zero for converged rows, whose nonzeros the pass skips).
#include <algorithm>

#include "internal.hpp"

namespace cpapr {
namespace {

enum : int32_t { kActive = 0, kSearching = 1, kConverged = 3 };

constexpr int kHessWaves = kBlock / 64;  // waves per workgroup of the Hessian pass
constexpr int kHessTile = 512;           // nonzeros per wave

// Lane `src`'s value of v (src uniform across the wave).
__device__ __forceinline__ double lane_value(double v, int src)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffu), src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u & 0xffffffffu), CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over aligned segments of W lanes, every lane receiving its segment's
// total (called with the whole wave active). DPP controls: quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror, row_mirror; then lane ^ 16, lane ^ 32.
template <int W>
__device__ __forceinline__ double seg_sum(double v)
{
    if constexpr (W >= 2) v += dpp<0xB1>(v);
    if constexpr (W >= 4) v += dpp<0x4E>(v);
    if constexpr (W >= 8) v += dpp<0x141>(v);
    if constexpr (W >= 16) v += dpp<0x140>(v);
    if constexpr (W >= 32) v += __shfl_xor(v, 16);
    if constexpr (W >= 64) v += __shfl_xor(v, 32);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return seg_sum<64>(v); }

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct HessArgs {
    const int32_t* rows;
    const uint32_t* cofs;
    const double* vals;
    const double* fac[kMaxOther];
    const double* B;
    const int32_t* status;
    double* HP;
    const int* skip;
    int64_t nnz;
    int64_t hp_stride;
    int R;
    int NM1;
    double eps;
};

// v_mfma_f64_16x16x4_f64 computes D = A B + C for A 16 x 4 and B 4 x 16 with one
// double per lane for A and B and four for C and D: A[i][k] comes from lane
// i + 16k, B[k][j] from lane j + 16k, and D[i][j] is element i / 4 of lane
// j + 16 (i % 4) (checked on gfx950 with lane-coded operands).
typedef double f64x4 __attribute__((ext_vector_type(4)));

// H and Phi rows of the active rows: per row, H = sum_k w_k pi_k pi_k^T is a
// rank-n_i update, which the matrix cores take four nonzeros at a time. A wave
// owns kHessTile consecutive nonzeros in rounds of four, one per 16-lane slot
// q: lane s of slot q gathers columns 16t + s (t < NT) of its nonzero's pi and
// b, the slot reduces m = b . pi, and forms x / m (the Phi scale) and w = x / m^2.
// Then lane (s, q) holds exactly A[s][q] = w_q pi_q[16ta + s] and B[q][s] =
// pi_q[16tb + s] of the 16 x 16 block (ta, tb) of H, so one MFMA per block adds
// the round's four outer products. A round whose nonzeros belong to several
// rows runs once per row, with the other slots' A set to zero. Phi's row is
// summed per slot and across the slots at the flush. NMAX bounds the other
// modes' count (exact for 1-3 other modes).
template <int RM, int NMAX>
__device__ __forceinline__ void hess_tiles(const HessArgs& a)
{
    constexpr int NT = RM / 16;  // 16-column blocks of the rank
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = lane & 15, q = lane >> 4;
    const int64_t p0 = ((int64_t)blockIdx.x * kHessWaves + wv) * kHessTile;
    const int64_t p1 = min(p0 + kHessTile, a.nnz);
    if (p0 >= p1) return;  // the whole wave; no workgroup barriers below
    const int R = a.R;
    f64x4 acc[NT][NT];
    double ph[NT];
    auto zero = [&]() {
#pragma unroll
        for (int ta = 0; ta < NT; ++ta) {
            ph[ta] = 0.0;
#pragma unroll
            for (int tb = 0; tb < NT; ++tb) acc[ta][tb] = f64x4{0.0, 0.0, 0.0, 0.0};
        }
    };
    zero();
    int cur = -1, nseg = 0;
    int brow = -1;  // row whose B columns bv holds (a slot's rows repeat across rounds)
    double bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bv[t] = 0.0;

    auto flush = [&](bool atomic) {
        double* base = a.HP + (int64_t)cur * a.hp_stride;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * ta + 4 * v + q, c = 16 * tb + s;
                    if (r < R && c < R) {
                        if (atomic)
                            unsafeAtomicAdd(base + r * R + c, acc[ta][tb][v]);
                        else
                            base[r * R + c] = acc[ta][tb][v];
                    }
                }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            double tot = ph[t];
            tot += __shfl_xor(tot, 16);
            tot += __shfl_xor(tot, 32);
            const int c = 16 * t + s;
            if (q == 0 && c < R) {
                if (atomic)
                    unsafeAtomicAdd(base + R * R + c, tot);
                else
                    base[R * R + c] = tot;
            }
        }
    };

    for (int64_t base = p0; base < p1; base += 64) {
        const int cnt = (int)min((int64_t)64, p1 - base);
        int myrow = -1;  // -1: past the range, or a converged row (skipped)
        int myc[NMAX];
        double myx = 0.0;
#pragma unroll
        for (int m = 0; m < NMAX; ++m) myc[m] = 0;
        if (lane < cnt) {
            myrow = a.rows[base + lane];
            if (a.status[myrow] == kConverged) myrow = -1;
#pragma unroll
            for (int m = 0; m < NMAX; ++m)
                if (m < a.NM1) myc[m] = (int)a.cofs[(int64_t)m * a.nnz + base + lane];
            myx = a.vals[base + lane];
        }
        for (int u0 = 0; u0 < cnt; u0 += 4) {
            const int u = u0 + q;  // this slot's nonzero (<= 63: u0 steps by 4)
            const int row = __shfl(myrow, u);
            const double x = __shfl(myx, u);
            int c[NMAX];
#pragma unroll
            for (int m = 0; m < NMAX; ++m) c[m] = __shfl(myc[m], u);
            double pi[NT];
            if (row != brow) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int col = 16 * t + s;
                    bv[t] = row >= 0 && col < R ? a.B[(int64_t)row * R + col] : 0.0;
                }
                brow = row;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                pi[t] = 0.0;
                const int col = 16 * t + s;
                if (row >= 0 && col < R) {
                    double p = a.fac[0][(uint64_t)(uint32_t)c[0] + col];
#pragma unroll
                    for (int m = 1; m < NMAX; ++m)
                        if (m < a.NM1) p *= a.fac[m][(uint64_t)(uint32_t)c[m] + col];
                    pi[t] = p;
                }
            }
            double mk = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) mk = __builtin_fma(bv[t], pi[t], mk);
            mk = seg_sum<16>(mk);
            const double mm = mk > a.eps ? mk : a.eps;
            const double sc = x / mm;
            const double w = sc / mm;
            int rk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) rk[k] = __builtin_amdgcn_readlane(row, 16 * k);
            // runs of equal rows among the four slots, in order
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int r = rk[k];
                if (r < 0 || (k > 0 && rk[k - 1] == r)) continue;
                int k2 = k + 1;
#pragma unroll
                for (int j = k + 1; j < 4; ++j)
                    if (k2 == j && rk[j] == r) k2 = j + 1;
                if (r != cur) {
                    if (cur >= 0) flush(nseg == 1);
                    cur = r;
                    ++nseg;
                    zero();
                }
                const bool mine = q >= k && q < k2;
#pragma unroll
                for (int ta = 0; ta < NT; ++ta) {
                    const double av = mine ? w * pi[ta] : 0.0;
#pragma unroll
                    for (int tb = 0; tb < NT; ++tb)
                        acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, pi[tb], acc[ta][tb], 0, 0, 0);
                    if (mine) ph[ta] = __builtin_fma(sc, pi[ta], ph[ta]);
                }
            }
        }
    }
    if (cur >= 0) flush(true);
}

// Up to R = 32 the registers are capped for four waves per SIMD (-15 % at
// R = 32 against the compiler's three); at R = 64 the accumulators alone take
// 128 registers, so that kernel is left uncapped.
template <int RM, int NMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void pdnr_hess_kernel(HessArgs a)
{
    if (*a.skip) return;
    hess_tiles<RM, NMAX>(a);
}

template <int NMAX>
__global__ __launch_bounds__(kBlock) void pdnr_hess_kernel_r64(HessArgs a)
{
    if (*a.skip) return;
    hess_tiles<64, NMAX>(a);
}

struct RowArgs {
    double* B;
    double* phi;  // receives the Phi row of every row that is evaluated
    int64_t rows;
    int R;
    double tau;
    PdnrState d;
    DevState* st;
};

__global__ __launch_bounds__(kBlock) void pdnr_reset_kernel(PdnrState d, int64_t rows, DevState* st)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kBlock) {
        d.status[i] = kActive;
        d.trials[i] = 0;
        d.steps[i] = 0;
        d.mu[i] = kPdnrMu0;
        d.viol[i] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq_all_done = rows == 0 ? 1 : 0;
        st->pq_idle = 1;
    }
}

// Before the rows decide: assume every row done / no row searching; rows that
// keep working clear the flags. Counts the pass that just ran, if any.
__global__ void pdnr_flags_kernel(DevState* st, int before_begin)
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

__device__ __forceinline__ void clear_row(double* hp, int64_t n, int lane)
{
    for (int64_t e = lane; e < n; e += 64) hp[e] = 0.0;
}

// Trial step of length alpha along the stored direction; returns g . delta.
__device__ __forceinline__ double make_trial(const RowArgs& a, int64_t i, int lane, double alpha, double b, double g)
{
    double gd = 0.0;
    if (lane < a.R) {
        const double nb = b + alpha * a.d.Dd[i * a.R + lane];
        const double delta = (nb > 0.0 ? nb : 0.0) - b;
        a.d.Dt[i * a.R + lane] = delta;
        gd = g * delta;
    }
    return wave_sum(gd);
}

// Waves per workgroup of the begin kernel (its LDS: RM x (RM + 1) doubles per
// wave). One: four per workgroup measured no faster.
template <int RM>
constexpr int begin_waves() { return 1; }

// One wave per row; lane i holds row i of the free-set matrix in registers
// (RM >= R columns, the unused ones an identity block) and the columns of its
// Cholesky factor go through the wave's LDS.
template <int RM>
__global__ __launch_bounds__(64 * begin_waves<RM>()) void pdnr_begin_kernel(RowArgs a)
{
    __shared__ double lcol_all[begin_waves<RM>()][RM][RM + 1];  // lcol[k][j] = L[j][k]; padded against bank conflicts
    const int lane = threadIdx.x & 63;
    auto& lcol = lcol_all[threadIdx.x >> 6];
    const int64_t i = (int64_t)blockIdx.x * begin_waves<RM>() + (threadIdx.x >> 6);
    if (i >= a.rows || a.d.status[i] == kConverged) return;
    const int R = a.R;
    const bool on = lane < R;
    double* hp = a.d.HP + i * a.d.hp_stride;
    double b = 0.0, g = 0.0;
    if (on) {
        b = a.B[i * R + lane];
        const double ph = hp[(int64_t)R * R + lane];
        g = 1.0 - ph;
        a.phi[i * R + lane] = ph;
        a.d.G[i * R + lane] = g;
    }
    const double viol = wave_max(on ? fabs(b < g ? b : g) : 0.0);
    if (lane == 0) a.d.viol[i] = viol;
    if (a.tau > 0.0 && viol < a.tau) {
        if (lane == 0) a.d.status[i] = kConverged;
        clear_row(hp, a.d.hp_stride, lane);
        return;
    }
    if (lane == 0) a.st->pq_all_done = 0;

    const bool fre = on && !(g > 0.0 && b <= kPdnrHeld);
    const unsigned long long fmask = __ballot(fre);
    const int nf = __popcll(fmask);
    double d = -g;  // held entries (and every entry when no entry is free)
    bool newton = nf == 0;
    if (nf > 0) {
        const double trace = wave_sum(fre ? hp[(int64_t)lane * R + lane] : 0.0);
        if (trace > 0.0) {
            const double damp = a.d.mu[i] * (trace / nf);
            double M[RM];
#pragma unroll
            for (int j = 0; j < RM; ++j) {
                const bool fj = j < R && ((fmask >> j) & 1ull);
                M[j] = fre ? (fj ? hp[(int64_t)lane * R + j] : 0.0) + (j == lane ? damp : 0.0) : (j == lane ? 1.0 : 0.0);
            }
            // Right-looking Cholesky: at step k lane k's diagonal becomes L[k][k],
            // lanes below it take L[lane][k] and update their row's later columns.
            bool ok = true;
#pragma unroll
            for (int k = 0; k < RM; ++k) {
                const double piv = lane_value(M[k], k);
                if (!(piv > 0.0)) {
                    ok = false;
                    break;
                }
                const double lkk = sqrt(piv);
                const double lik = lane == k ? lkk : M[k] / lkk;
                M[k] = lik;
                if (lane < RM) lcol[k][lane] = lik;
                wave_sync();
#pragma unroll
                for (int j = k + 1; j < RM; ++j) M[j] = __builtin_fma(-lik, lcol[k][j], M[j]);
            }
            if (ok) {
                // L y = -g_F (rows of L in registers), then L^T d_F = y (columns from LDS)
                double z = fre ? -g : 0.0;
#pragma unroll
                for (int j = 0; j < RM; ++j) {
                    const double yj = lane_value(z, j) / lane_value(M[j], j);
                    if (lane > j)
                        z = __builtin_fma(-M[j], yj, z);
                    else if (lane == j)
                        z = yj;
                }
#pragma unroll
                for (int j = RM - 1; j >= 0; --j) {
                    const double dj = lane_value(z, j) / lane_value(M[j], j);
                    if (lane < j)
                        z = __builtin_fma(-lcol[lane][j], dj, z);
                    else if (lane == j)
                        z = dj;
                }
                if (fre) d = z;
                newton = true;
            }
        }
    }
    if (newton) newton = wave_sum(on ? g * d : 0.0) < 0.0;
    if (!newton) d = -b * g;
    if (on) a.d.Dd[i * R + lane] = d;
    const double gd = make_trial(a, i, lane, 1.0, b, g);
    if (lane == 0) {
        a.d.alpha[i] = 1.0;
        a.d.gdel[i] = gd;
        a.d.trials[i] = 0;
        a.d.status[i] = kSearching;
        a.st->pq_idle = 0;
    }
}

// max over aligned 16-lane segments (whole wave active)
__device__ __forceinline__ double seg16_max(double v)
{
    v = fmax(v, dpp<0xB1>(v));
    v = fmax(v, dpp<0x4E>(v));
    v = fmax(v, dpp<0x141>(v));
    return fmax(v, dpp<0x140>(v));
}

// R <= 16: four rows per wave, one per 16-lane segment, with the same steps
// as pdnr_begin_kernel (lane s of a segment holds row s of its row's system).
// Segments stay in step: a segment that has nothing left to do keeps
// computing on neutral values and discards the result, so every shuffle and
// segment reduction runs with the whole wave active.
__global__ __launch_bounds__(64) void pdnr_begin16_kernel(RowArgs a)
{
    constexpr int RM = 16;
    __shared__ double lcol_all[4][RM][RM + 1];  // per segment: lcol[k][j] = L[j][k]
    const int lane = threadIdx.x;
    const int q = lane >> 4, s = lane & 15, sb = lane & ~15;
    auto& lcol = lcol_all[q];
    const int64_t i = (int64_t)blockIdx.x * 4 + q;
    const int R = a.R;
    bool live = i < a.rows && a.d.status[i] != kConverged;
    const bool on = live && s < R;
    double* hp = a.d.HP + (live ? i : 0) * a.d.hp_stride;
    double b = 0.0, g = 0.0;
    if (on) {
        b = a.B[i * R + s];
        const double ph = hp[(int64_t)R * R + s];
        g = 1.0 - ph;
        a.phi[i * R + s] = ph;
        a.d.G[i * R + s] = g;
    }
    const double viol = seg16_max(on ? fabs(b < g ? b : g) : 0.0);
    if (live && s == 0) a.d.viol[i] = viol;
    if (live && a.tau > 0.0 && viol < a.tau) {
        if (s == 0) a.d.status[i] = kConverged;
        for (int64_t e = s; e < a.d.hp_stride; e += 16) hp[e] = 0.0;
        live = false;
    }
    if (live && s == 0) a.st->pq_all_done = 0;

    const bool fre = live && s < R && !(g > 0.0 && b <= kPdnrHeld);
    const unsigned fmask = (unsigned)((__ballot(fre) >> sb) & 0xFFFFull);
    const int nf = __popc(fmask);
    const double trace = seg_sum<16>(fre ? hp[(int64_t)s * R + s] : 0.0);
    const bool chol = live && nf > 0 && trace > 0.0;
    const double damp = chol ? a.d.mu[i] * (trace / nf) : 0.0;
    double M[RM];
#pragma unroll
    for (int j = 0; j < RM; ++j) {
        const bool fj = j < R && ((fmask >> j) & 1u);
        M[j] = fre ? (fj ? hp[(int64_t)s * R + j] : 0.0) + (j == s ? damp : 0.0) : (j == s ? 1.0 : 0.0);
    }
    bool ok = chol;
#pragma unroll
    for (int k = 0; k < RM; ++k) {
        const double piv = __shfl(M[k], sb + k);
        ok = ok && piv > 0.0;
        const double lkk = sqrt(piv > 0.0 ? piv : 1.0);
        const double lik = s == k ? lkk : M[k] / lkk;
        M[k] = lik;
        lcol[k][s] = lik;
        wave_sync();
#pragma unroll
        for (int j = k + 1; j < RM; ++j) M[j] = __builtin_fma(-lik, lcol[k][j], M[j]);
    }
    double z = fre ? -g : 0.0;
#pragma unroll
    for (int j = 0; j < RM; ++j) {
        const double yj = __shfl(z, sb + j) / __shfl(M[j], sb + j);
        if (s > j)
            z = __builtin_fma(-M[j], yj, z);
        else if (s == j)
            z = yj;
    }
#pragma unroll
    for (int j = RM - 1; j >= 0; --j) {
        const double dj = __shfl(z, sb + j) / __shfl(M[j], sb + j);
        if (s < j)
            z = __builtin_fma(-lcol[s][j], dj, z);
        else if (s == j)
            z = dj;
    }
    double d = -g;  // held entries (and every entry when no entry is free)
    if (ok && fre) d = z;
    const bool newton0 = live && (nf == 0 || ok);
    const bool newton = newton0 && seg_sum<16>(on ? g * d : 0.0) < 0.0;
    if (!newton) d = -b * g;
    double delta = 0.0;
    if (on) {
        a.d.Dd[i * R + s] = d;
        const double nb = b + d;
        delta = (nb > 0.0 ? nb : 0.0) - b;
        a.d.Dt[i * R + s] = delta;
    }
    const double gd = seg_sum<16>(g * delta);
    if (live && s == 0) {
        a.d.alpha[i] = 1.0;
        a.d.gdel[i] = gd;
        a.d.trials[i] = 0;
        a.d.status[i] = kSearching;
        a.st->pq_idle = 0;
    }
}

// Value of lane src of v's SEG-lane segment (sb: the segment's first lane; the
// whole wave active).
template <int SEG>
__device__ __forceinline__ double seg_value(double v, int sb, int src)
{
    if constexpr (SEG == 64)
        return lane_value(v, src);
    else
        return __shfl(v, sb + src);
}

// End of a row's line search (lane s of the row's SEG-lane segment holds entry
// s; `live`: the segment has a row that searched): the accepted step, or the
// MU step if none was; the damping update from the ratio of actual to
// predicted decrease; the accumulation row cleared.
template <int SEG>
__device__ __forceinline__ void finish_step(const RowArgs& a, int64_t i, int s, int sb, bool live, bool accept,
                                            double b, double g, double delta, double gdel, double df)
{
    const int R = a.R;
    const bool on = live && s < R;
    double* hp = a.d.HP + (live ? i : 0) * a.d.hp_stride;
    double mu = live ? a.d.mu[i] : 0.0;
    // predicted decrease of the quadratic model along the step (used if accepted)
    double hd = 0.0;
    for (int r = 0; r < R; ++r) {
        const double dr = seg_value<SEG>(delta, sb, r);
        if (on) hd = __builtin_fma(hp[(int64_t)r * R + s], dr, hd);
    }
    const double quad = seg_sum<SEG>(on ? delta * hd : 0.0);
    if (accept) {
        const double pred = -(gdel + 0.5 * quad);
        const double rho = pred > 0.0 ? -df / pred : 0.0;
        if (rho < 0.25)
            mu = fmin(mu * kPdnrMuStep, kPdnrMuMax);
        else if (rho > 0.75)
            mu = fmax(mu / kPdnrMuStep, kPdnrMuMin);
    } else {
        delta = -b * g;  // the MU step
        mu = fmin(mu * kPdnrMuStep, kPdnrMuMax);
    }
    if (on) {
        a.B[i * R + s] = b + delta;
        a.d.Dt[i * R + s] = delta;
    }
    if (live) {
        for (int64_t e = s; e < a.d.hp_stride; e += SEG) hp[e] = 0.0;
        if (s == 0) {
            a.d.mu[i] = mu;
            a.d.steps[i] += 1;
            a.d.status[i] = kActive;
        }
    }
}

// One wave per row: the line-search decision for the current trial.
__global__ __launch_bounds__(kBlock) void pdnr_accept_kernel(RowArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (i >= a.rows || a.d.status[i] != kSearching) return;
    const int R = a.R;
    const bool on = lane < R;
    double b = 0.0, g = 0.0, delta = 0.0;
    if (on) {
        b = a.B[i * R + lane];
        g = a.d.G[i * R + lane];
        delta = a.d.Dt[i * R + lane];
    }
    const double lin = wave_sum(delta);
    const double gdel = a.d.gdel[i];
    const double df = lin - a.d.T[i * R];
    const bool accept = gdel < 0.0 && df <= kPdnrSigma * gdel;
    const int t = a.d.trials[i] + 1;
    if (!accept && t < kPdnrTrials) {
        const double alpha = a.d.alpha[i] * 0.5;
        const double gd = make_trial(a, i, lane, alpha, b, g);
        if (lane == 0) {
            a.d.alpha[i] = alpha;
            a.d.gdel[i] = gd;
            a.d.trials[i] = t;
            a.st->pq_idle = 0;
        }
        return;
    }
    finish_step<64>(a, i, lane, 0, true, accept, b, g, delta, gdel, df);
}

// The same decision for all trials at once (R >= 4): the line-search pass has
// summed the four trials alpha = 1, 1/2, 1/4, 1/8 into columns 0-3, and the
// first acceptable one is taken, as the trial-by-trial rounds would. A row per
// SEG-lane segment: SEG = 64 with four waves per workgroup, or SEG = 16 (R <= 16)
// with four rows per wave.
template <int SEG>
__global__ __launch_bounds__(SEG == 64 ? kBlock : 64) void pdnr_accept4_kernel(RowArgs a)
{
    static_assert(kPdnrTrials == 4, "the fused line-search pass evaluates four trials");
    const int lane = threadIdx.x & 63;
    const int s = lane & (SEG - 1), sb = lane & ~(SEG - 1);
    const int64_t i = (int64_t)blockIdx.x * 4 + (SEG == 64 ? (threadIdx.x >> 6) : (lane >> 4));
    const bool live = i < a.rows && a.d.status[i] == kSearching;
    if (SEG == 64 && !live) return;  // a whole wave
    const int R = a.R;
    const bool on = live && s < R;
    double b = 0.0, g = 0.0, d = 0.0;
    if (on) {
        b = a.B[i * R + s];
        g = a.d.G[i * R + s];
        d = a.d.Dd[i * R + s];
    }
    bool accept = false;
    double delta = 0.0, gdel = 0.0, df = 0.0;
    double alpha = 1.0;
#pragma unroll
    for (int k = 0; k < kPdnrTrials; ++k, alpha *= 0.5) {
        double dl = 0.0;
        if (on) {
            const double nb = b + alpha * d;
            dl = (nb > 0.0 ? nb : 0.0) - b;
        }
        const double gd = seg_sum<SEG>(g * dl);
        const double dfk = seg_sum<SEG>(dl) - (live ? a.d.T[i * R + k] : 0.0);
        if (live && !accept && gd < 0.0 && dfk <= kPdnrSigma * gd) {
            accept = true;
            delta = dl;
            gdel = gd;
            df = dfk;
        }
    }
    finish_step<SEG>(a, i, s, sb, live, accept, b, g, delta, gdel, df);
}

// Per-mode results: most steps of a row, steps summed, largest last violation.
__global__ __launch_bounds__(kBlock) void pdnr_stats_kernel(PdnrState d, int64_t rows, int mode, DevState* st)
{
    __shared__ long long ssum[kBlock / 64];
    __shared__ int smax[kBlock / 64];
    __shared__ double svio[kBlock / 64];
    long long sum = 0;
    int mx = 0;
    double vio = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += kBlock) {
        sum += d.steps[i];
        mx = max(mx, (int)d.steps[i]);
        vio = fmax(vio, d.viol[i]);
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

int rank_tile(int R) { return R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64; }

template <typename F>
Error by_tile(int rm, F&& f)
{
    switch (rm) {
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 32: return f(std::integral_constant<int, 32>{});
        default: return f(std::integral_constant<int, 64>{});
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t pdnr_bytes(int64_t maxI, int R)
{
    const size_t mat = align256((size_t)maxI * R * 8);
    const size_t hp = align256((size_t)maxI * ((size_t)R * R + R) * 8);
    return hp + 4 * mat + 4 * align256((size_t)maxI * 8) + 3 * align256((size_t)maxI * 4);
}

void pdnr_bind(PdnrState* d, char* base, int64_t maxI, int R)
{
    const size_t mat = align256((size_t)maxI * R * 8);
    char* p = base;
    auto take = [&](size_t n) {
        char* r = p;
        p += n;
        return r;
    };
    d->hp_stride = (int64_t)R * R + R;
    d->HP = (double*)take(align256((size_t)maxI * d->hp_stride * 8));
    d->G = (double*)take(mat);
    d->Dd = (double*)take(mat);
    d->Dt = (double*)take(mat);
    d->T = (double*)take(mat);
    d->mu = (double*)take(align256((size_t)maxI * 8));
    d->alpha = (double*)take(align256((size_t)maxI * 8));
    d->gdel = (double*)take(align256((size_t)maxI * 8));
    d->viol = (double*)take(align256((size_t)maxI * 8));
    d->status = (int32_t*)take(align256((size_t)maxI * 4));
    d->trials = (int32_t*)take(align256((size_t)maxI * 4));
    d->steps = (int32_t*)take(align256((size_t)maxI * 4));
}

Error enqueue_pdnr_inner(cpapr_plan* P, int mode, double* B, const void* const* fac, double* phi, hipStream_t s)
{
    const int64_t rows = P->dims[mode];
    const int R = P->R;
    if (R > kPdnrMaxRank) return {CPAPR_EUNSUPPORTED, "PDNR supports R <= 64"};
    if (rows > 0x7fffffff) return {CPAPR_EUNSUPPORTED, "too many rows"};
    const int64_t n = rows * (int64_t)R;
    DevState* st = P->state;
    const int* all_done = &st->pq_all_done;
    const int* idle = &st->pq_idle;
    const int rm = rank_tile(R);
    const dim3 agrid((unsigned)std::max<int64_t>((rows + kBlock / 64 - 1) / (kBlock / 64), 1));
    const int64_t hwaves = (P->nnz + kHessTile - 1) / kHessTile;
    const dim3 hgrid((unsigned)std::max<int64_t>((hwaves + kHessWaves - 1) / kHessWaves, 1));
    if ((hwaves + kHessWaves - 1) / kHessWaves > 0x7fffffff) return {CPAPR_EUNSUPPORTED, "too many nonzeros"};

    HessArgs h{};
    const PlanMode& pm = P->mode[mode];
    h.rows = pm.rows;
    h.cofs = pm.cofs;
    h.vals = pm.vals;
    int j = 0;
    for (int m = 0; m < P->N; ++m)
        if (m != mode) h.fac[j++] = (const double*)fac[m];
    h.B = B;
    h.status = P->pd.status;
    h.HP = P->pd.HP;
    h.skip = all_done;
    h.nnz = P->nnz;
    h.hp_stride = P->pd.hp_stride;
    h.R = R;
    h.NM1 = P->N - 1;
    h.eps = P->params.eps;

    const int zgrid = (int)std::min<int64_t>(std::max<int64_t>((rows + kBlock - 1) / kBlock, 1), 4096);
    pdnr_reset_kernel<<<zgrid, kBlock, 0, s>>>(P->pd, rows, st);
    CPAPR_LAUNCHED();
    Error e = launch_fill(P->pd.HP, rows * P->pd.hp_stride, 0.0, nullptr, s);
    if (e.code) return e;
    RowArgs ra{B, phi, rows, R, P->params.tol, P->pd, st};
    for (int l = 0; l < P->params.lmax; ++l) {
        prof_begin(mode, s);
        e = by_tile(std::max(rm, 16), [&](auto RM) -> Error {
            constexpr int T = decltype(RM)::value < 16 ? 16 : decltype(RM)::value;
            if constexpr (T == 64) {
                switch (h.NM1) {
                    case 1: pdnr_hess_kernel_r64<1><<<hgrid, kBlock, 0, s>>>(h); break;
                    case 2: pdnr_hess_kernel_r64<2><<<hgrid, kBlock, 0, s>>>(h); break;
                    case 3: pdnr_hess_kernel_r64<3><<<hgrid, kBlock, 0, s>>>(h); break;
                    default: pdnr_hess_kernel_r64<kMaxOther><<<hgrid, kBlock, 0, s>>>(h); break;
                }
            } else {
                switch (h.NM1) {
                    case 1: pdnr_hess_kernel<T, 1><<<hgrid, kBlock, 0, s>>>(h); break;
                    case 2: pdnr_hess_kernel<T, 2><<<hgrid, kBlock, 0, s>>>(h); break;
                    case 3: pdnr_hess_kernel<T, 3><<<hgrid, kBlock, 0, s>>>(h); break;
                    default: pdnr_hess_kernel<T, kMaxOther><<<hgrid, kBlock, 0, s>>>(h); break;
                }
            }
            CPAPR_LAUNCHED();
            return {CPAPR_OK, ""};
        });
        prof_end(s);
        if (e.code) return e;
        pdnr_flags_kernel<<<1, 64, 0, s>>>(st, 1);
        CPAPR_LAUNCHED();
        if (rm <= 16) {
            pdnr_begin16_kernel<<<dim3((unsigned)std::max<int64_t>((rows + 3) / 4, 1)), 64, 0, s>>>(ra);
            CPAPR_LAUNCHED();
        } else {
            e = by_tile(rm, [&](auto RM) -> Error {
                constexpr int W = begin_waves<decltype(RM)::value>();
                const dim3 bgrid((unsigned)std::max<int64_t>((rows + W - 1) / W, 1));
                pdnr_begin_kernel<decltype(RM)::value><<<bgrid, 64 * W, 0, s>>>(ra);
                CPAPR_LAUNCHED();
                return {CPAPR_OK, ""};
            });
        }
        if (e.code) return e;
        if (R >= kPdnrTrials) {  // all trials in one line-search pass
            e = launch_fill(P->pd.T, n, 0.0, idle, s);
            if (e.code) return e;
            e = launch_delta4(P, mode, B, P->pd.Dd, P->pd.status, fac, P->params.eps, P->pd.T, idle, s);
            if (e.code) return e;
            pdnr_flags_kernel<<<1, 64, 0, s>>>(st, 0);
            CPAPR_LAUNCHED();
            if (R <= 16)
                pdnr_accept4_kernel<16><<<dim3((unsigned)std::max<int64_t>((rows + 3) / 4, 1)), 64, 0, s>>>(ra);
            else
                pdnr_accept4_kernel<64><<<agrid, kBlock, 0, s>>>(ra);
            CPAPR_LAUNCHED();
            continue;
        }
        for (int t = 0; t < kPdnrTrials; ++t) {  // R < 4: one pass per trial
            e = launch_fill(P->pd.T, n, 0.0, idle, s);
            if (e.code) return e;
            e = launch_delta(P, mode, B, P->pd.Dt, P->pd.status, fac, P->params.eps, P->pd.T, idle, s);
            if (e.code) return e;
            pdnr_flags_kernel<<<1, 64, 0, s>>>(st, 0);
            CPAPR_LAUNCHED();
            pdnr_accept_kernel<<<agrid, kBlock, 0, s>>>(ra);
            CPAPR_LAUNCHED();
        }
    }
    pdnr_stats_kernel<<<1, kBlock, 0, s>>>(P->pd, rows, mode, st);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

}  // namespace cpapr
