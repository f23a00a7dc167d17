// Phi(n) = (X_(n) ./ max(B Pi, eps)) Pi^T  (Algorithm 2), one nonzero at a time.
//
// Work decomposition (gfx950, wave64):
//  * A lane group of G lanes owns one nonzero at a time; each lane holds RPL
//    consecutive rank columns (rank blocking: R <= G * RPL). A wave runs 64/G
//    nonzeros side by side.
//  * Nonzeros are pre-sorted by the mode-n coordinate (plan). A workgroup takes
//    a tile of consecutive sorted nonzeros; each of its lane groups walks a
//    contiguous sub-chunk of `chunk` nonzeros sequentially, keeping the Phi row
//    being built in registers. This is the paper's CPU "atomic mitigation"
//    idea (Algorithm 4: accumulate locally while the row is unchanged) mapped to
//    lane groups: a row that starts and ends inside the sub-chunk is owned by
//    the group and written with a plain store.
//  * A sub-chunk's first and last rows may continue in the neighbouring
//    sub-chunks; their partial rows go to LDS and are merged in order across
//    the workgroup. After the merge only rows that cross the tile boundary are
//    written with FP64 atomics (the paper's atomic update strategy, Section 3.1,
//    now confined to tile ends); every other row is a plain store.
//  * The dot product B[i,:] . pi_k is an all-reduce across the lane group with
//    DPP row permutations (xor-1, xor-2, half-mirror, mirror) and, for 32/64
//    lanes, ds_swizzle / ds_bpermute; every lane ends with the same bits.
//  * Tiles are mapped XCD-aware: consecutive tiles (which share B and Phi rows)
//    are given to the same XCD so their rows stay in one L2.
//
// Mixed precision: the other factors are stored (and gathered) as FP32, which
// halves the gathered bytes, and widened to FP64 as they are loaded; products,
// sums and Phi are FP64. (Compensated FP32 arithmetic was the earlier design:
// it made the kernel issue-bound and slower than FP64; widening runs at the
// FP64 kernel's speed at R = 16 and 19-29 % faster at R = 32.)
//
// The same tile code serves several kinds of pass over the nonzeros: Phi,
// MTTKRP (Eqs. 10-12: x_k pi_k scattered), the log-likelihood terms (summed
// per tile) and the line-search sums of the row solves (per-row changes of
// the likelihood along one or four trial steps).
#include <algorithm>
#include <type_traits>

#include "internal.hpp"

namespace cpapr {
namespace {

__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int q = nb / kXcds, rmd = nb % kXcds;
    const int xcd = bid % kXcds, local = bid / kXcds;
    return (xcd < rmd ? xcd * (q + 1) : rmd * (q + 1) + (xcd - rmd) * q) + local;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// lane ^ 16 inside each 32-lane half (ds_swizzle bitmask mode: and 0x1f, xor 0x10)
__device__ __forceinline__ double xor16_f64(double v)
{
    int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double xor32_f64(double v)
{
    const int addr = ((int)(threadIdx.x & 63) ^ 32) << 2;
    int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// DPP controls: quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140.
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    if constexpr (G >= 2) v += dpp_f64<0xB1>(v);
    if constexpr (G >= 4) v += dpp_f64<0x4E>(v);
    if constexpr (G >= 8) v += dpp_f64<0x141>(v);
    if constexpr (G >= 16) v += dpp_f64<0x140>(v);
    if constexpr (G >= 32) v += xor16_f64(v);
    if constexpr (G >= 64) v += xor32_f64(v);
    return v;
}


// Per-lane accumulator of one Phi row slice (FP64 in both precisions: FP32-stored
// factors are widened as they are loaded).
struct Acc {
    double v;
    __device__ void zero() { v = 0.0; }
    __device__ void add(double s, double pi) { v = __builtin_fma(s, pi, v); }
    __device__ double value() const { return v; }
};

// q = x / m for normal, finite m > 0 (m is clamped to eps > 0 before): the
// hardware reciprocal estimate, one Newton step r <- r + r(1 - m r), then
// q = x r. The Newton step squares the estimate's relative error e, so q is
// off by about e^2 plus the roundings: at most 10.2 x 2^-52 measured over 1e6
// quotients (an estimate good to about 2^-24), a few ulps. A residual step
// q + r(x - m q), which would bring it within an ulp, measured 3 % of the Phi
// kernel's time; a few ulps per quotient are far below the rounding of the
// row sums the quotients feed and the 1e-12 parity gate. The IEEE division
// sequence's scaling for denormal and huge operands is not needed in this
// range.
__device__ __forceinline__ double div_pos(double x, double m)
{
    double r = __builtin_amdgcn_rcp(m);
    r = __builtin_fma(r, __builtin_fma(-m, r, 1.0), r);
    return x * r;
}

// What the segmented kernel computes per nonzero and where it goes.
constexpr int kPhi = 0;     // s_k = x_k / max(m_k, eps); Phi[i_n] += s_k pi_k
constexpr int kMttkrp = 1;  // s_k = x_k;                  M[i_n]  += s_k pi_k
constexpr int kLoglik = 2;  // x_k log(max(m_k, eps)) summed per tile (no scatter)
constexpr int kDelta = 3;   // x_k log(max(m_k + dm_k, eps) / max(m_k, eps)) summed per row (column 0)
constexpr int kDelta4 = 4;  // the same for the four trial steps max(b + alpha d, 0) - b, alpha = 1, 1/2, 1/4, 1/8 (columns 0-3)
constexpr int kTrials4 = 4;

// The change of the likelihood term of one nonzero along a trial step d of its
// row, m = b . pi and dm = d . pi: x log1p(dm / m) when neither end is at the
// floor (accurate for small steps, unlike a difference of two logarithms);
// -infinity when the step brings m from above eps down to eps or below (the
// trial leaves the domain of the row objective and must be rejected); from a
// point already at the floor, the difference of the clamped logarithms.
// Returns true with the ratio dm / m in *ratio for the common case (the caller
// batches the logarithms), false with the whole term in *term otherwise.
template <int G, int RPL>
__device__ __forceinline__ bool delta_ratio(const double (&b)[RPL], const double (&d)[RPL], const double (&pi)[RPL],
                                            double x, double eps, double* ratio, double* term)
{
    double m = 0.0, dm = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; ++c) {
        m = __builtin_fma(b[c], pi[c], m);
        dm = __builtin_fma(d[c], pi[c], dm);
    }
    m = group_sum<G>(m);
    dm = group_sum<G>(dm);
    const double m1 = m + dm;
    if (m > eps && m1 > eps) {
        *ratio = div_pos(dm, m);
        return true;
    }
    *term = m > eps ? -__builtin_inf() : x * (log(m1 > eps ? m1 : eps) - log(eps));
    return false;
}

// One nonzero's dot product and scale: s_k for Phi, x_k for MTTKRP, the
// likelihood term for Loglik.
template <int G, int RPL, int KIND>
__device__ __forceinline__ double nonzero_scale(const double (&b)[RPL], const double (&pi)[RPL], double x, double eps)
{
    if constexpr (KIND == kMttkrp) {
        return x;
    } else {
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < RPL; ++c) d = __builtin_fma(b[c], pi[c], d);
        d = group_sum<G>(d);
        // max(m, eps) as one v_max (m is never NaN: values and factors are finite)
        if constexpr (KIND == kLoglik) return x * log(__builtin_fmax(d, eps));
        return div_pos(x, __builtin_fmax(d, eps));
    }
}

// The nonzero stream (records or coordinate / value arrays) is read once per
// launch: non-temporal loads keep it from displacing reused factor rows in L2
// (used where one load instruction reads whole or half cache lines).
template <typename T>
__device__ __forceinline__ T stream_load(const T* p)
{
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ int4 stream_load(const int4* p)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = __builtin_nontemporal_load((const v4i*)p);
    return make_int4(v.x, v.y, v.z, v.w);
}

// Staged nonzero: its row, the other modes' coordinates and its value. A lane
// group loads G consecutive nonzeros cooperatively (coalesced) into its slice
// of LDS and then reads them back one at a time as broadcasts.
template <int NM1>
struct alignas(8) Staged {
    int row;
    uint32_t c[NM1];  // factor row offsets (coordinate x R)
    double x;
};

// Nonzeros whose factor rows are gathered before any of them is consumed, so
// that U x NM1 gathers are in flight per lane group.
template <int NM1, int RPL>
constexpr int gather_depth()
{
    return NM1 * RPL <= 2 ? 4 : (NM1 * RPL <= 4 ? 2 : 1);
}

// LDS of one workgroup tile: head/tail partial rows, their row ids, and the
// staged nonzeros of every lane group.
template <int G, int RPL, int NM1>
struct TileShared {
    static constexpr int NG = kBlock / G;
    static constexpr int BATCH = G >= 8 ? G : 8;  // nonzeros staged per lane group per round
    double part[2 * NG][G * RPL];
    int prow[2 * NG];
    Staged<NM1> stage[NG * BATCH];
};

// Ordered merge of the head/tail partial rows a tile's lane groups left in
// LDS; rows crossing the tile boundary go out with atomics (or, in the
// deterministic mode, as kept partials), all others with plain stores. Called
// by every thread of the workgroup after a barrier.
template <int G, int RPL>
__device__ __forceinline__ void tile_merge(const PhiArgs& a, int64_t tile, int64_t tile_start, int64_t tile_end,
                                           const double (*part)[G * RPL], const int* prow)
{
    constexpr int NG = kBlock / G;
    constexpr int W = G * RPL;
    const int t = threadIdx.x;
    const int R = a.R;
    const int64_t nnz = a.nnz;
    if (t < R && t < W) {
        const int prev_row = tile_start > 0 ? a.rows[tile_start - 1] : -1;
        const int next_row = tile_end < nnz ? a.rows[tile_end] : -1;
        int run = -1;
        double v = 0.0;
        // Deterministic mode: the tile-end rows' partials are kept (head: the row
        // continuing from the previous tile; tail: a row starting here and
        // continuing) and summed in tile order by det_fixup_kernel.
        double* det = a.det_part;
        if (det != nullptr && t == 0) {
            a.det_rows[2 * tile] = -1;
            a.det_rows[2 * tile + 1] = -1;
        }
        auto emit = [&](int row, double val) {
            double* dst = a.Phi + (int64_t)row * R + t;
            if (row == prev_row || row == next_row) {
                if (det == nullptr) {
                    unsafeAtomicAdd(dst, val);
                } else {
                    const int side = row == prev_row ? 0 : 1;
                    det[((int64_t)side * a.det_tiles + tile) * R + t] = val;
                    if (t == 0) a.det_rows[2 * tile + side] = row;
                }
            } else {
                *dst = val;
            }
        };
        for (int e = 0; e < 2 * NG; ++e) {
            const int re = prow[e];
            if (re < 0) continue;
            if (re == run) {
                v += part[e][t];
            } else {
                if (run >= 0) emit(run, v);
                run = re;
                v = part[e][t];
            }
        }
        if (run >= 0) emit(run, v);
    }
}

// One workgroup tile of consecutive sorted nonzeros (tile index `tile` of the
// operand set `a`).
// O32: every gathered factor is smaller than 4 GiB, so a row's address is the
// factor's base plus a 32-bit byte offset (one VALU add, and the loads take the
// base from scalar registers).
template <int G, int RPL, int NM1, bool MIXED, int KIND, bool O32 = false>
__device__ __forceinline__ void phi_tile(const PhiArgs& a, int64_t tile, TileShared<G, RPL, NM1>& sh)
{
    using T = double;  // arithmetic: FP64 in both precisions
    using L = typename std::conditional<MIXED, float, double>::type;  // the factors as stored
    constexpr int NG = kBlock / G;
    constexpr int U = gather_depth<NM1, RPL>();
    constexpr int BATCH = TileShared<G, RPL, NM1>::BATCH;
    constexpr int EPL = BATCH / G;  // staged entries loaded by each lane
    auto& part = sh.part;
    auto& prow = sh.prow;
    auto& stage = sh.stage;

    const int t = threadIdx.x;
    const int g = t / G;
    const int lane = t % G;
    const int R = a.R;
    const int64_t nnz = a.nnz;
    const int64_t tile_start = (int64_t)tile * NG * a.L;
    const int64_t tile_end = min(tile_start + (int64_t)NG * a.L, nnz);
    const int64_t p0 = tile_start + (int64_t)g * a.L;
    const int64_t p1 = min(p0 + (int64_t)a.L, nnz);

    if (lane == 0) {
        prow[2 * g] = -1;
        prow[2 * g + 1] = -1;
    }

    // Each lane owns the rank columns [lane*RPL, lane*RPL + RPL) that are < R,
    // but always reads a window of RPL contiguous, in-row columns starting at
    // colbase (shifted left for lanes at or past the end of the row). One
    // address per gathered row, no selects in the hot loop; slots the lane
    // does not own get B = 0 (no contribution to the dot product) and are
    // never stored.
    const int colbase = min(lane * RPL, R - RPL);
    bool own[RPL];
#pragma unroll
    for (int c = 0; c < RPL; ++c) own[c] = colbase + c >= lane * RPL && colbase + c < R;

    int cur = -1;
    int nseg = 0;
    double ll = 0.0;  // likelihood terms of this lane group (Loglik)
    Acc acc[RPL];
    T b[RPL];
    constexpr bool LS = KIND == kDelta || KIND == kDelta4;  // a line-search pass
    constexpr int NTR = KIND == kDelta4 ? kTrials4 : 1;      // trial steps it evaluates
    double dv[RPL];  // the row's trial step (kDelta) or search direction (kDelta4)
    double dk[NTR][RPL];  // kDelta4: the row's trial steps
    // Line-search pass: the log1p terms of a row are batched over the lane
    // group, lane j holding the ratios and value of the row's j-th pending
    // nonzero; one log1p per lane and trial and one group sum then cover G
    // nonzeros.
    int pend = 0;
    double pr[NTR], px = 0.0;
#pragma unroll
    for (int k = 0; k < NTR; ++k) pr[k] = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; ++c) {
        acc[c].zero();
        b[c] = (T)0;
        dv[c] = 0.0;
#pragma unroll
        for (int k = 0; k < NTR; ++k) dk[k][c] = 0.0;
    }
    // kDelta4: trial k's sum goes to column k (owned by lane k / RPL; R >= 4)
    auto add_trial = [&](int k, double v) {
        if constexpr (KIND == kDelta4) {
#pragma unroll
            for (int c = 0; c < RPL; ++c)
                if (own[c] && colbase + c == k) acc[c].v += v;
        }
    };

    // Flush kinds: 0 = head partial (LDS), 1 = tail partial (LDS), 2 = owned row (store).
    auto flush = [&](int row, int kind) {
        if (kind == 2) {
            double* dst = a.Phi + (int64_t)row * R + colbase;
#pragma unroll
            for (int c = 0; c < RPL; ++c)
                if (own[c]) dst[c] = acc[c].value();
        } else {
            const int e = 2 * g + kind;
#pragma unroll
            for (int c = 0; c < RPL; ++c)
                if (own[c]) part[e][colbase + c] = acc[c].value();
            if (lane == 0) prow[e] = row;
        }
    };

    auto drain = [&]() {
        if constexpr (KIND == kDelta) {
            if (pend > 0) {
                double v = lane < pend ? px * log1p(pr[0]) : 0.0;
                v = group_sum<G>(v);
                if (lane == 0) acc[0].v += v;
                pend = 0;
            }
        } else if constexpr (KIND == kDelta4) {
            if (pend > 0) {
#pragma unroll 1  // one log1p body in the code (fewer live registers)
                for (int k = 0; k < NTR; ++k) {
                    double v = lane < pend ? px * log1p(pr[k]) : 0.0;
                    add_trial(k, group_sum<G>(v));
                }
                pend = 0;
            }
        }
    };

    const L* fac[NM1];
#pragma unroll
    for (int m = 0; m < NM1; ++m) fac[m] = (const L*)a.fac[m];
    Staged<NM1>* my = stage + g * BATCH;

    // Metadata of the next round is loaded into registers while the current
    // round is processed (coalesced: lane j of the group takes entries j, j+G, ...).
    Staged<NM1> pre[EPL];
    // With packed records (up to two other modes, values exact in FP32) a
    // staged nonzero is one 16-byte load instead of NM1 + 2: the gather path's
    // address and data units work per lane and load instruction, and the
    // metadata loads were a fifth of them.
    const bool packed = NM1 <= 2 && a.pk != nullptr;
    auto load_meta = [&](int64_t base) {
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int64_t p = base + k * G + lane;
            if (p < p1) {
                if (packed) {
                    const int4 q = stream_load(a.pk + p);
                    pre[k].row = q.x;
                    pre[k].c[0] = (uint32_t)q.y;
                    if constexpr (NM1 == 2) pre[k].c[NM1 - 1] = (uint32_t)q.z;
                    pre[k].x = (double)__int_as_float(q.w);
                } else {
                    // non-temporal only where a group's load covers at least half a
                    // 128-byte line of each array: 8 lanes read a quarter line of the
                    // 4-byte arrays and come back to it three times, re-fetching it
                    // once it has been let go (measured 13 % slower)
                    if constexpr (G >= 16) {
                        pre[k].row = stream_load(a.rows + p);
#pragma unroll
                        for (int m = 0; m < NM1; ++m) pre[k].c[m] = stream_load(a.cofs + (int64_t)m * nnz + p);
                        pre[k].x = stream_load(a.vals + p);
                    } else {
                        pre[k].row = a.rows[p];
#pragma unroll
                        for (int m = 0; m < NM1; ++m) pre[k].c[m] = a.cofs[(int64_t)m * nnz + p];
                        pre[k].x = a.vals[p];
                    }
                }
                // line-search pass: a row not in a line search is staged as ~row
                // (negative), so the skip costs no load in the gather loop
                if constexpr (LS)
                    if (a.live[pre[k].row] != 1) pre[k].row = ~pre[k].row;
            }
        }
    };
    if (p0 < p1) load_meta(p0);

    for (int64_t base = p0; base < p1; base += BATCH) {
        const int cnt = (int)min((int64_t)BATCH, p1 - base);
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            if (k * G + lane < cnt) my[k * G + lane] = pre[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (base + BATCH < p1) load_meta(base + BATCH);

        for (int q0 = 0; q0 < cnt; q0 += U) {
            int rowu[U];
            double xu[U];
            L fu[U][NM1][RPL];
            bool liveu[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q0 + u < cnt) {
                    const Staged<NM1> e = my[q0 + u];
                    // line-search pass: rows not in a line search contribute nothing
                    liveu[u] = !LS || e.row >= 0;
                    rowu[u] = liveu[u] ? e.row : ~e.row;
                    xu[u] = e.x;
                    if (liveu[u]) {
#pragma unroll
                        for (int m = 0; m < NM1; ++m) {
                            const L* f = O32 ? (const L*)((const char*)fac[m] +
                                                          (uint32_t)((e.c[m] + (uint32_t)colbase) * (uint32_t)sizeof(L)))
                                             : fac[m] + (uint64_t)e.c[m] + colbase;
#pragma unroll
                            for (int c = 0; c < RPL; ++c) fu[u][m][c] = f[c];
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // line-search pass: nonzeros of rows not in a line search are
                // passed over as if absent (no row change, no B load, no flush)
                if (q0 + u < cnt && (!LS || liveu[u])) {
                    const int row = rowu[u];
                    T pi[RPL];
#pragma unroll
                    for (int c = 0; c < RPL; ++c) {
                        pi[c] = fu[u][0][c];
#pragma unroll
                        for (int m = 1; m < NM1; ++m) pi[c] *= fu[u][m][c];
                    }
                    if (row != cur) {
                        if constexpr (LS) drain();
                        if constexpr (KIND != kLoglik)
                            if (cur >= 0) flush(cur, nseg == 1 ? 0 : 2);
                        cur = row;
                        ++nseg;
#pragma unroll
                        for (int c = 0; c < RPL; ++c) acc[c].zero();
                        if constexpr (KIND != kMttkrp) {
                            const double* brow = a.B + (int64_t)row * R + colbase;
#pragma unroll
                            for (int c = 0; c < RPL; ++c) b[c] = own[c] ? (T)brow[c] : (T)0;
                        }
                        if constexpr (LS) {
                            const double* drow = a.D + (int64_t)row * R + colbase;
#pragma unroll
                            for (int c = 0; c < RPL; ++c) dv[c] = own[c] ? drow[c] : 0.0;
                        }
                        if constexpr (KIND == kDelta4) {
                            double alpha = 1.0;
#pragma unroll
                            for (int k = 0; k < NTR; ++k, alpha *= 0.5)
#pragma unroll
                                for (int c = 0; c < RPL; ++c) {
                                    const double nb = (double)b[c] + alpha * dv[c];
                                    dk[k][c] = (nb > 0.0 ? nb : 0.0) - (double)b[c];
                                }
                        }
                    }
                    if constexpr (KIND == kDelta) {
                        static_assert(!MIXED, "the line-search pass is FP64");
                        double ratio, term;
                        if (delta_ratio<G, RPL>(b, dv, pi, xu[u], a.eps, &ratio, &term)) {
                            if (lane == pend) {
                                pr[0] = ratio;
                                px = xu[u];
                            }
                            if (++pend == G) drain();
                        } else if (lane == 0) {
                            acc[0].v += term;
                        }
                    } else if constexpr (KIND == kDelta4) {
                        static_assert(!MIXED, "the line-search pass is FP64");
                        // m = b . pi and dm_k = delta_k . pi, then as delta_ratio for each trial
                        double m = 0.0, dm[NTR];
#pragma unroll
                        for (int k = 0; k < NTR; ++k) dm[k] = 0.0;
#pragma unroll
                        for (int c = 0; c < RPL; ++c) {
                            m = __builtin_fma(b[c], pi[c], m);
#pragma unroll
                            for (int k = 0; k < NTR; ++k) dm[k] = __builtin_fma(dk[k][c], pi[c], dm[k]);
                        }
                        m = group_sum<G>(m);
                        double ratios[NTR];
#pragma unroll
                        for (int k = 0; k < NTR; ++k) {
                            dm[k] = group_sum<G>(dm[k]);
                            const double m1 = m + dm[k];
                            if (m > a.eps && m1 > a.eps) {
                                ratios[k] = div_pos(dm[k], m);
                            } else {
                                ratios[k] = 0.0;  // log1p(0) adds nothing at the drain
                                add_trial(k, m > a.eps ? -__builtin_inf()
                                                       : xu[u] * (log(m1 > a.eps ? m1 : a.eps) - log(a.eps)));
                            }
                        }
                        if (lane == pend) {
#pragma unroll
                            for (int k = 0; k < NTR; ++k) pr[k] = ratios[k];
                            px = xu[u];
                        }
                        if (++pend == G) drain();
                    } else {
                        const double s = nonzero_scale<G, RPL, KIND>(b, pi, xu[u], a.eps);
                        if constexpr (KIND == kLoglik) {
                            ll += s;
                        } else {
#pragma unroll
                            for (int c = 0; c < RPL; ++c) acc[c].add(s, pi[c]);
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if constexpr (KIND == kLoglik) {
        if (lane == 0) part[2 * g][0] = ll;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int q = 0; q < NG; ++q) sum += part[2 * q][0];
            a.Phi[tile] = sum;  // one partial per tile, reduced in order later
        }
        return;
    }
    if constexpr (LS) drain();
    if (cur >= 0) flush(cur, nseg == 1 ? 0 : 1);
    __syncthreads();

    tile_merge<G, RPL>(a, tile, tile_start, tile_end, part, prow);
}

// Nonzeros per lane group per round of the reduce-scatter Phi tile.
#ifndef CPAPR_XR_Q
#define CPAPR_XR_Q 4
#endif

// LDS of one reduce-scatter tile: the merge rows and staged nonzeros of the
// plain tile, plus per lane group the Q x G partial dot products of a round
// (padded by two words so that rows of different groups start on different
// banks) and the round's Q scales.
template <int G, int RPL, int NM1, int Q>
struct XrShared {
    static constexpr int NG = kBlock / G;
    static constexpr int BATCH = G;  // nonzeros staged per lane group per batch
    static constexpr int RSTR = Q * G + 2;
    double part[2 * NG][G * RPL];
    int prow[2 * NG];
    Staged<NM1> stage[NG * BATCH];
    double red[NG * RSTR];
    double sv[NG * Q];
};

// Phi over one tile, the dot products reduced across the lane group by a
// reduce-scatter instead of an all-reduce per nonzero. A lane group takes Q
// consecutive nonzeros of its sub-chunk per round: every lane gathers its rank
// slice of the Q pi rows and forms its Q partial dot products; the partials go
// to LDS, where lane q of the group sums the G partials of nonzero q (a fixed
// order) and forms the one scale s_q = x_q / max(m_q, eps) for it; the Q scales
// are read back by every lane and scattered into the register Phi row as in
// the plain tile. Per round that is one sum of G terms and one division per
// nonzero in one lane instead of a log2(G)-step all-reduce and a division in
// all G lanes, and Q nonzeros' gathers in flight per lane group.
template <int G, int RPL, int NM1, bool MIXED, int Q>
__device__ __forceinline__ void phi_tile_xr(const PhiArgs& a, int64_t tile, XrShared<G, RPL, NM1, Q>& sh)
{
    using L = typename std::conditional<MIXED, float, double>::type;
    constexpr int NG = kBlock / G;
    constexpr int BATCH = XrShared<G, RPL, NM1, Q>::BATCH;
    constexpr int RSTR = XrShared<G, RPL, NM1, Q>::RSTR;
    static_assert(BATCH % Q == 0 && Q <= G, "a batch holds whole rounds; one divider lane per nonzero");
    auto& part = sh.part;
    auto& prow = sh.prow;

    const int t = threadIdx.x;
    const int g = t / G;
    const int lane = t % G;
    const int R = a.R;
    const int64_t nnz = a.nnz;
    const int64_t tile_start = (int64_t)tile * NG * a.L;
    const int64_t tile_end = min(tile_start + (int64_t)NG * a.L, nnz);
    const int64_t p0 = tile_start + (int64_t)g * a.L;
    const int64_t p1 = min(p0 + (int64_t)a.L, nnz);
    double* red = sh.red + g * RSTR;
    double* sv = sh.sv + g * Q;
    Staged<NM1>* my = sh.stage + g * BATCH;

    if (lane == 0) {
        prow[2 * g] = -1;
        prow[2 * g + 1] = -1;
    }
    const int colbase = min(lane * RPL, R - RPL);
    bool own[RPL];
#pragma unroll
    for (int c = 0; c < RPL; ++c) own[c] = colbase + c >= lane * RPL && colbase + c < R;

    int cur = -1;
    int nseg = 0;
    double acc[RPL], bcur[RPL];
#pragma unroll
    for (int c = 0; c < RPL; ++c) acc[c] = bcur[c] = 0.0;

    auto flush = [&](int row, int kind) {
        if (kind == 2) {
            double* dst = a.Phi + (int64_t)row * R + colbase;
#pragma unroll
            for (int c = 0; c < RPL; ++c)
                if (own[c]) dst[c] = acc[c];
        } else {
            const int e = 2 * g + kind;
#pragma unroll
            for (int c = 0; c < RPL; ++c)
                if (own[c]) part[e][colbase + c] = acc[c];
            if (lane == 0) prow[e] = row;
        }
    };

    const L* fac[NM1];
#pragma unroll
    for (int m = 0; m < NM1; ++m) fac[m] = (const L*)a.fac[m];

    // metadata of the next batch in registers while the current one is processed
    Staged<NM1> pre;
    auto load_meta = [&](int64_t base) {
        const int64_t p = base + lane;
        if (p < p1) {
            pre.row = a.rows[p];
#pragma unroll
            for (int m = 0; m < NM1; ++m) pre.c[m] = a.cofs[(int64_t)m * nnz + p];
            pre.x = a.vals[p];
        }
    };
    if (p0 < p1) load_meta(p0);

    for (int64_t base = p0; base < p1; base += BATCH) {
        const int cnt = (int)min((int64_t)BATCH, p1 - base);
        if (lane < cnt) my[lane] = pre;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (base + BATCH < p1) load_meta(base + BATCH);

        for (int q0 = 0; q0 < cnt; q0 += Q) {
            const int nq = min(Q, cnt - q0);
            // gathers of the round's pi rows, and the B rows of rows starting here
            L fu[Q][NM1][RPL];
            double bq[Q][RPL];
            int rowq[Q];
            bool newr[Q];
            int prev = cur;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                newr[q] = false;
                rowq[q] = prev;
                if (q < nq) {
                    const Staged<NM1> e = my[q0 + q];
                    rowq[q] = e.row;
                    newr[q] = e.row != prev;
                    prev = e.row;
#pragma unroll
                    for (int m = 0; m < NM1; ++m) {
                        const L* f = fac[m] + (uint64_t)e.c[m] + colbase;
#pragma unroll
                        for (int c = 0; c < RPL; ++c) fu[q][m][c] = f[c];
                    }
                    if (newr[q]) {
                        const double* brow = a.B + (int64_t)e.row * R + colbase;
#pragma unroll
                        for (int c = 0; c < RPL; ++c) bq[q][c] = own[c] ? brow[c] : 0.0;
                    }
                }
            }
            // pi rows and this lane's partial dot products
            double pi[Q][RPL];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (newr[q]) {
#pragma unroll
                    for (int c = 0; c < RPL; ++c) bcur[c] = bq[q][c];
                }
                if (q < nq) {
                    double d = 0.0;
#pragma unroll
                    for (int c = 0; c < RPL; ++c) {
                        double v = (double)fu[q][0][c];
#pragma unroll
                        for (int m = 1; m < NM1; ++m) v *= (double)fu[q][m][c];
                        pi[q][c] = v;
                        d = __builtin_fma(bcur[c], v, d);
                    }
                    red[q * G + lane] = d;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // lane q: the whole dot product of nonzero q and its scale
            if (lane < nq) {
                double m = 0.0;
#pragma unroll
                for (int j = 0; j < G; ++j) m += red[lane * G + j];
                sv[lane] = div_pos(my[q0 + lane].x, m > a.eps ? m : a.eps);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double s[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) s[q] = sv[q];
            // scatter into the register Phi row; a row change flushes the previous row
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (q < nq) {
                    if (newr[q]) {
                        if (cur >= 0) flush(cur, nseg == 1 ? 0 : 2);
                        cur = rowq[q];
                        ++nseg;
#pragma unroll
                        for (int c = 0; c < RPL; ++c) acc[c] = 0.0;
                    }
#pragma unroll
                    for (int c = 0; c < RPL; ++c) acc[c] = __builtin_fma(s[q], pi[q][c], acc[c]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (cur >= 0) flush(cur, nseg == 1 ? 0 : 1);
    __syncthreads();
    tile_merge<G, RPL>(a, tile, tile_start, tile_end, part, prow);
}

template <int G, int RPL, int NM1, bool MIXED>
__global__ __launch_bounds__(kBlock) void phi_xr_kernel(PhiArgs a)
{
    __shared__ XrShared<G, RPL, NM1, CPAPR_XR_Q> sh;
    if (a.done != nullptr && *a.done) return;
    phi_tile_xr<G, RPL, NM1, MIXED, CPAPR_XR_Q>(a, xcd_remap(blockIdx.x, gridDim.x), sh);
}

template <int G, int RPL, int NM1, bool MIXED, int KIND, bool O32 = false>
__global__ __launch_bounds__(kBlock) void phi_seg_kernel(PhiArgs a)
{
    __shared__ TileShared<G, RPL, NM1> sh;
    if (a.done != nullptr && *a.done) return;
    phi_tile<G, RPL, NM1, MIXED, KIND, O32>(a, xcd_remap(blockIdx.x, gridDim.x), sh);
}

// The four-trial line-search pass with its registers capped for four waves per
// SIMD, used for up to two rank columns per lane (at 8 lanes x 2 columns the
// compiler's choice gives three waves with 139 registers; capped, -5 % per
// pass). With four columns per lane the cap spills 130-220 bytes per lane and
// costs 1.6x, so those shapes keep the plain kernel.
template <int G, int RPL, int NM1, bool MIXED, int KIND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void phi_ls4_kernel(PhiArgs a)
{
    __shared__ TileShared<G, RPL, NM1> sh;
    if (a.done != nullptr && *a.done) return;
    phi_tile<G, RPL, NM1, MIXED, KIND>(a, xcd_remap(blockIdx.x, gridDim.x), sh);
}

// Persistent Phi over a batch of operand sets of one shape class. The grid is
// sized to the device; the tile count and the tile -> slot map are read from
// device memory (so a captured graph stays valid when the batch changes).
// Tiles are handed out dynamically: the class's tile space is cut into
// kBatchSubs contiguous sub-ranges (kBatchSubs / 8 per XCD, so neighbouring
// tiles, which share B and Phi rows, stay in one L2), each with its own
// counter on its own cache line; a workgroup claims kBatchClaim tiles at a
// time from its home sub-range, then from the following ones. Tile costs vary
// a lot (a tile inside one heavy row does one flush, a tile in a sparse tail
// many), which is why a static split loses to dynamic claiming.
template <int G, int RPL, int NM1, bool MIXED>
__global__ __launch_bounds__(kBlock) void phi_batch_kernel(const BatchSlot* __restrict__ slots,
                                                           const int32_t* __restrict__ tile_map,
                                                           const int64_t* __restrict__ class_off,
                                                           const int64_t* __restrict__ class_ntiles,
                                                           const int32_t* __restrict__ slot_done,
                                                           unsigned int* __restrict__ counters, int cls)
{
    __shared__ TileShared<G, RPL, NM1> sh;
    __shared__ unsigned int claimed;
    const int64_t total = class_ntiles[cls];
    const int32_t* __restrict__ tile_slot = tile_map + class_off[cls];
    unsigned int* ctr_base = counters + (int64_t)cls * kBatchSubs * kCounterStride;
    const int b = blockIdx.x;
    const int home = (b % kXcds) * (kBatchSubs / kXcds) + (b / kXcds) % (kBatchSubs / kXcds);
    for (int k = 0; k < kBatchSubs; ++k) {
        const int sub = (home + k) % kBatchSubs;
        const int64_t lo = sub * total / kBatchSubs, hi = (sub + 1) * total / kBatchSubs;
        const unsigned int len = (unsigned int)(hi - lo);
        unsigned int* ctr = ctr_base + (int64_t)sub * kCounterStride;
        while (true) {
            if (threadIdx.x == 0) {
                unsigned int c = len;
                if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < len)
                    c = atomicAdd(ctr, (unsigned int)kBatchClaim);
                claimed = c;
            }
            __syncthreads();
            const unsigned int c = claimed;
            __syncthreads();
            if (c >= len) break;
            const int64_t t1 = min(lo + (int64_t)c + kBatchClaim, hi);
            for (int64_t tt = lo + c; tt < t1; ++tt) {
                const int si = tile_slot[tt];
                if (slot_done[slots[si].slot]) continue;  // this slot's inner loop has stopped
                const PhiArgs a = slots[si].args;
                __syncthreads();  // LDS of the previous tile is no longer read
                phi_tile<G, RPL, NM1, MIXED, kPhi>(a, tt - slots[si].tile_begin, sh);
            }
        }
    }
}

// Non-persistent variant: one workgroup per tile of the class (grid size from
// the host's commit), tiles spread XCD-aware like the single-plan kernel; the
// hardware dispatcher balances the uneven tiles and overlaps each tile's
// prologue with other workgroups' work.
template <int G, int RPL, int NM1, bool MIXED>
__global__ __launch_bounds__(kBlock) void phi_batch_grid_kernel(const BatchSlot* __restrict__ slots,
                                                                const int32_t* __restrict__ tile_map,
                                                                const int64_t* __restrict__ class_off,
                                                                const int32_t* __restrict__ slot_done, int cls)
{
    __shared__ TileShared<G, RPL, NM1> sh;
    const int64_t tt = xcd_remap(blockIdx.x, gridDim.x);
    const int si = tile_map[class_off[cls] + tt];
    if (slot_done[slots[si].slot]) return;
    const PhiArgs a = slots[si].args;
    phi_tile<G, RPL, NM1, MIXED, kPhi>(a, tt - slots[si].tile_begin, sh);
}

// List-driven fills / conversions for a batch: op 0 zeroes dst (FP64), op 1
// rounds src (FP64) into dst (FP32). Workgroup b takes a contiguous element range
// of the concatenated lists and walks the items it spans.
__global__ __launch_bounds__(kBlock) void batch_elementwise_kernel(const BatchCopy* __restrict__ items,
                                                                   const int32_t* __restrict__ nitems_dev,
                                                                   const int64_t* __restrict__ total_dev,
                                                                   const int32_t* __restrict__ slot_done,
                                                                   unsigned int* __restrict__ counters, int ncounters)
{
    // the tile counters of the Phi launches that follow start from zero
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < ncounters; i += gridDim.x * kBlock)
        counters[(int64_t)i * kCounterStride] = 0u;
    const int nitems = *nitems_dev;
    const int64_t total = *total_dev;
    const int64_t per = ((total + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int64_t e0 = blockIdx.x * per, e1 = min(e0 + per, total);
    if (e0 >= e1) return;
    int lo = 0, hi = nitems - 1;  // last item with begin <= e0
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (items[mid].begin <= e0) lo = mid; else hi = mid - 1;
    }
    for (int it = lo; it < nitems && items[it].begin < e1; ++it) {
        const BatchCopy c = items[it];
        const int64_t a0 = max(e0, c.begin) - c.begin, a1 = min(e1, c.begin + c.n) - c.begin;
        if (c.op == 0 && c.slot >= 0 && slot_done[c.slot]) continue;  // keep a stopped slot's last Phi
        if (c.op == 0) {
            double* d = (double*)c.dst;
            for (int64_t i = a0 + threadIdx.x; i < a1; i += kBlock) d[i] = 0.0;
        } else {
            float* d = (float*)c.dst;
            for (int64_t i = a0 + threadIdx.x; i < a1; i += kBlock) d[i] = (float)c.src[i];
        }
    }
}

// The paper's GPU kernel shape (Algorithm 3): one lane group per nonzero and an
// atomic add of every Phi entry it touches. Kept as a comparison variant.
template <int G, int RPL>
__global__ __launch_bounds__(kBlock) void phi_atomic_kernel(PhiArgs a)
{
    constexpr int NG = kBlock / G;
    if (a.done != nullptr && *a.done) return;
    const int t = threadIdx.x;
    const int g = t / G;
    const int lane = t % G;
    const int R = a.R;
    bool valid[RPL];
#pragma unroll
    for (int c = 0; c < RPL; ++c) valid[c] = lane * RPL + c < R;
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t p = (int64_t)blockIdx.x * NG + g; p < a.nnz; p += stride) {
        const int row = a.rows[p];
        const double x = a.vals[p];
        double pi[RPL], b[RPL];
#pragma unroll
        for (int c = 0; c < RPL; ++c) pi[c] = valid[c] ? 1.0 : 0.0;
        for (int m = 0; m < a.NM1; ++m) {
            const double* f = (const double*)a.fac[m] + (uint64_t)a.cofs[(int64_t)m * a.nnz + p] + lane * RPL;
#pragma unroll
            for (int c = 0; c < RPL; ++c)
                if (valid[c]) pi[c] *= f[c];
        }
        const double* brow = a.B + (int64_t)row * R + lane * RPL;
#pragma unroll
        for (int c = 0; c < RPL; ++c) b[c] = valid[c] ? brow[c] : 0.0;
        const double s = nonzero_scale<G, RPL, kPhi>(b, pi, x, a.eps);
        double* dst = a.Phi + (int64_t)row * R + lane * RPL;
#pragma unroll
        for (int c = 0; c < RPL; ++c)
            if (valid[c]) unsafeAtomicAdd(dst + c, s * pi[c]);
    }
}

// Deterministic mode: a row that starts in tile t and continues is the sum of
// tile t's tail partial and the head partials of the following tiles it
// covers, added in a fixed order (threads strided over the tiles, then a fixed
// tree); the row is written with a plain store.
__global__ __launch_bounds__(kBlock) void det_fixup_kernel(const int32_t* __restrict__ rows, int64_t nnz,
                                                           int64_t tile_nnz, int64_t tiles, int R,
                                                           const double* __restrict__ part,
                                                           const int32_t* __restrict__ det_rows, int64_t cap,
                                                           double* __restrict__ Phi, const int* done)
{
    __shared__ double red[kBlock];
    if (done != nullptr && *done) return;
    const int64_t t = blockIdx.x;
    const int r = det_rows[2 * t + 1];
    if (r < 0) return;
    // the run of row r ends at the first position after tile t holding a larger row
    int64_t lo = (t + 1) * tile_nnz, hi = nnz;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (rows[mid] > r)
            hi = mid;
        else
            lo = mid + 1;
    }
    const int64_t t1 = min((lo - 1) / tile_nnz, tiles - 1);  // last tile holding row r
    int rp = 1;
    while (rp < R) rp *= 2;
    const int c = threadIdx.x % rp;
    const int j = threadIdx.x / rp;
    const int lanes = kBlock / rp;
    for (int c0 = 0; c0 < R; c0 += rp) {
        double v = 0.0;
        if (c0 + c < R)
            for (int64_t k = t + 1 + j; k <= t1; k += lanes) v += part[k * R + c0 + c];  // head partials
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = lanes / 2; w > 0; w >>= 1) {
            if (j < w) red[threadIdx.x] += red[threadIdx.x + w * rp];
            __syncthreads();
        }
        if (j == 0 && c0 + c < R)
            Phi[(int64_t)r * R + c0 + c] = part[(cap + t) * R + c0 + c] + red[threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void zero_kernel(double* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = 0.0;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <int NM1, bool MIXED, int KIND>
Error dispatch_seg_n(int G, int RPL, const PhiArgs& a, dim3 grid, hipStream_t s)
{
#define CPAPR_SEG_CASE(GG, RR)                                                        \
    if (G == GG && RPL == RR) {                                                       \
        if constexpr (KIND == kDelta4 && RR <= 2)                                     \
            phi_ls4_kernel<GG, RR, NM1, MIXED, KIND><<<grid, kBlock, 0, s>>>(a);      \
        else if constexpr (KIND == kPhi)                                              \
            if (a.o32)                                                                \
                phi_seg_kernel<GG, RR, NM1, MIXED, KIND, true><<<grid, kBlock, 0, s>>>(a); \
            else                                                                      \
                phi_seg_kernel<GG, RR, NM1, MIXED, KIND><<<grid, kBlock, 0, s>>>(a);  \
        else                                                                          \
            phi_seg_kernel<GG, RR, NM1, MIXED, KIND><<<grid, kBlock, 0, s>>>(a);      \
        CPAPR_LAUNCHED();                                                             \
        return {CPAPR_OK, ""};                                                        \
    }
    CPAPR_SEG_CASE(4, 1)
    CPAPR_SEG_CASE(8, 1)
    CPAPR_SEG_CASE(16, 1)
    CPAPR_SEG_CASE(32, 1)
    CPAPR_SEG_CASE(64, 1)
    CPAPR_SEG_CASE(64, 2)
    CPAPR_SEG_CASE(64, 4)
    CPAPR_SEG_CASE(8, 2)
    CPAPR_SEG_CASE(16, 2)
    if constexpr (NM1 <= 3) {
        CPAPR_SEG_CASE(8, 4)
        CPAPR_SEG_CASE(16, 4)
    }
    if constexpr (NM1 <= 3 && KIND != kLoglik) {
        CPAPR_SEG_CASE(4, 2)
        CPAPR_SEG_CASE(4, 4)
        CPAPR_SEG_CASE(32, 2)
        CPAPR_SEG_CASE(32, 4)
    }
#undef CPAPR_SEG_CASE
    return {CPAPR_EUNSUPPORTED, "no Phi kernel for this lane-group / rank-block shape and mode count"};
}

// Shapes the reduce-scatter tile is built for: 8 or 16 lanes per nonzero, up
// to 8 gathered words per lane and nonzero (its Q rounds keep them in
// registers).
bool xr_shape_supported(int G, int RPL, int NM1) { return (G == 8 || G == 16) && NM1 * RPL <= 8; }

template <bool MIXED>
Error dispatch_xr(int G, int RPL, const PhiArgs& a, hipStream_t s)
{
    const int NG = kBlock / G;
    const int64_t tiles = cdiv(a.nnz, (int64_t)NG * a.L);
    if (tiles <= 0) return {CPAPR_OK, ""};
    if (tiles > 0x7fffffff) return {CPAPR_EUNSUPPORTED, "too many tiles"};
    const dim3 grid((unsigned)tiles);
#define CPAPR_XR_CASE(GG, RR, NN)                                                     \
    if (G == GG && RPL == RR && a.NM1 == NN) {                                        \
        phi_xr_kernel<GG, RR, NN, MIXED><<<grid, kBlock, 0, s>>>(a);                  \
        CPAPR_LAUNCHED();                                                             \
        return {CPAPR_OK, ""};                                                        \
    }
#define CPAPR_XR_N(GG, RR) CPAPR_XR_CASE(GG, RR, 1) CPAPR_XR_CASE(GG, RR, 2) CPAPR_XR_CASE(GG, RR, 3) \
    CPAPR_XR_CASE(GG, RR, 4)
    CPAPR_XR_N(8, 1)
    CPAPR_XR_N(8, 2)
    CPAPR_XR_N(16, 1)
    CPAPR_XR_N(16, 2)
    CPAPR_XR_CASE(8, 4, 1)
    CPAPR_XR_CASE(8, 4, 2)
    CPAPR_XR_CASE(16, 4, 1)
    CPAPR_XR_CASE(16, 4, 2)
#undef CPAPR_XR_N
#undef CPAPR_XR_CASE
    return {CPAPR_EUNSUPPORTED, "no reduce-scatter Phi kernel for this shape"};
}

template <bool MIXED, int KIND>
Error dispatch_seg(int G, int RPL, const PhiArgs& a, hipStream_t s)
{
    const int NG = kBlock / G;
    const int64_t tiles = cdiv(a.nnz, (int64_t)NG * a.L);
    if (tiles <= 0) return {CPAPR_OK, ""};
    if (tiles > 0x7fffffff) return {CPAPR_EUNSUPPORTED, "too many tiles"};
    const dim3 grid((unsigned)tiles);
    switch (a.NM1) {
        case 1: return dispatch_seg_n<1, MIXED, KIND>(G, RPL, a, grid, s);
        case 2: return dispatch_seg_n<2, MIXED, KIND>(G, RPL, a, grid, s);
        case 3: return dispatch_seg_n<3, MIXED, KIND>(G, RPL, a, grid, s);
        case 4: return dispatch_seg_n<4, MIXED, KIND>(G, RPL, a, grid, s);
        case 5: return dispatch_seg_n<5, MIXED, KIND>(G, RPL, a, grid, s);
        case 6: return dispatch_seg_n<6, MIXED, KIND>(G, RPL, a, grid, s);
        case 7: return dispatch_seg_n<7, MIXED, KIND>(G, RPL, a, grid, s);
        default: return {CPAPR_EUNSUPPORTED, "unsupported number of modes"};
    }
}

Error dispatch_atomic(int G, int RPL, const PhiArgs& a, hipStream_t s)
{
    const int NG = kBlock / G;
    int64_t blocks = cdiv(a.nnz, (int64_t)NG);
    if (blocks > 65536) blocks = 65536;
    if (blocks <= 0) return {CPAPR_OK, ""};
#define CPAPR_AT_CASE(GG, RR)                                                         \
    if (G == GG && RPL == RR) {                                                       \
        phi_atomic_kernel<GG, RR><<<(unsigned)blocks, kBlock, 0, s>>>(a);             \
        CPAPR_LAUNCHED();                                                             \
        return {CPAPR_OK, ""};                                                        \
    }
    CPAPR_AT_CASE(4, 1)
    CPAPR_AT_CASE(4, 2)
    CPAPR_AT_CASE(4, 4)
    CPAPR_AT_CASE(8, 1)
    CPAPR_AT_CASE(8, 2)
    CPAPR_AT_CASE(8, 4)
    CPAPR_AT_CASE(16, 1)
    CPAPR_AT_CASE(16, 2)
    CPAPR_AT_CASE(16, 4)
    CPAPR_AT_CASE(32, 1)
    CPAPR_AT_CASE(32, 2)
    CPAPR_AT_CASE(32, 4)
    CPAPR_AT_CASE(64, 1)
    CPAPR_AT_CASE(64, 2)
    CPAPR_AT_CASE(64, 4)
#undef CPAPR_AT_CASE
    return {CPAPR_EUNSUPPORTED, "no atomic Phi kernel for this shape"};
}

PhiArgs make_args(const cpapr_plan* P, int mode, const double* B, const void* const* fac, double eps,
                  double* Phi, const int* done)
{
    PhiArgs a{};
    const PlanMode& pm = P->mode[mode];
    a.rows = pm.rows;
    a.cofs = pm.cofs;
    a.vals = pm.vals;
    a.pk = pm.pk;
    int j = 0;
    for (int m = 0; m < P->N; ++m)
        if (m != mode) a.fac[j++] = fac[m];
    a.B = B;
    a.Phi = Phi;
    a.done = done;
    a.nnz = P->nnz;
    a.R = P->R;
    a.NM1 = P->N - 1;
    a.L = P->chunk;
    a.eps = eps;
    const uint64_t word = P->params.precision == CPAPR_MIXED ? 4 : 8;
    a.o32 = 1;
    for (int m = 0; m < P->N; ++m)
        if (m != mode && (uint64_t)P->dims[m] * (uint64_t)P->R * word > 0xffffffffull) a.o32 = 0;
    return a;
}

Error zero_matrix(double* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return {CPAPR_OK, ""};
    int64_t g = cdiv(n, kBlock);
    if (g > 8192) g = 8192;
    zero_kernel<<<(unsigned)g, kBlock, 0, s>>>(p, n);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

}  // namespace

// Default launch shapes, from a sweep of lanes per nonzero and chunk on the
// 3-way 20M-nonzero Zipf workload (R = 8, 10, 16, 32): fewer lanes per
// nonzero with more rank columns per lane win because the kernel is bound by
// instruction issue, and the per-nonzero dot all-reduce and FP64 divide are
// shared by more nonzeros per wave.
int resolve_group(int R, int requested, int nm1)
{
    if (requested != 0) return requested;
    if (R <= 4) return 4;
    if (R <= 8) return 8;
    if (R <= 16) return 8;
    if (R <= 32) return nm1 <= 3 ? 8 : 16;
    if (R <= 64) return nm1 <= 3 ? 16 : 64;
    return 64;
}

bool phi_shape_supported(int group, int rpl, int nmodes_other)
{
    if (nmodes_other < 1 || nmodes_other > kMaxOther) return false;
    if (group != 4 && group != 8 && group != 16 && group != 32 && group != 64) return false;
    if (rpl != 1 && rpl != 2 && rpl != 4) return false;
    if (rpl == 1 || group == 64) return true;
    if (nmodes_other <= 3) return true;
    return rpl == 2 && (group == 8 || group == 16);  // N >= 5: the default shapes only
}

int rank_block(int R, int group)
{
    const int need = (R + group - 1) / group;
    if (need <= 1) return 1;
    if (need <= 2) return 2;
    if (need <= 4) return 4;
    return -1;
}

int resolve_chunk(int group, int requested)
{
    if (requested > 0) return requested;
    // 512 nonzeros per workgroup tile
    return 512 / (kBlock / group);
}

// Launch-policy model: the Phi launch shape from the tensor, in place of a
// measured search (the paper leaves such a heuristic as future work, Section
// 4). Fitted to sweeps of lanes per nonzero x nonzeros per lane group on every
// mode of 3- and 4-way tensors from 1e4 to 1e8 nonzeros, uniform and Zipf, R =
// 8..32, both precisions, timed as kernel durations with the launches queued
// back to back. What decides is the nonzero count (tiles enough to fill the
// device), the rank and the precision; the modes of one tensor, and uniform
// against Zipf rows at equal size, preferred the same shape.
//  * a large tensor's shape: 512-nonzero tiles with lanes by rank, except
//    17 <= R <= 32 with up to four modes: 16 lanes x 2 columns on 256-nonzero
//    tiles in FP64, 8 lanes x 4 columns on 1024-nonzero tiles with FP32-stored
//    factors (half the gathered words per lane); and 5 <= R <= 16 with packed
//    nonzero records (one load per staged nonzero): 1024-nonzero tiles, the
//    tile's merge and row flushes weighing more against the cheaper nonzeros
//    (-10 % at zipf3 against 512);
//  * a tensor too small to give ~900 such tiles (3.5 per compute unit) takes
//    tiles of the largest power of two <= nnz / 900 (at least 32): up to 128
//    nonzeros on 16 lanes (shorter per-nonzero chains, the launch being
//    latency-bound); at 256 or 512 lanes by rank (at 256 16 lanes for
//    9 <= R <= 16 with FP32-stored factors). Fewer tiles leave the last round of workgroups on
//    part of the device (measured: 780 tiles 5-13 % slower than 1560 of half
//    the size; 980 within 2 % of the best);
//  * the deterministic mode keeps tiles of at least 128 nonzeros;
//  * in a batch the slots of all tensors share one launch per shape class and
//    fill the device together, so a slot takes the large tensor's shape of its
//    rank and precision whatever its own size.
namespace {
struct ModelIn {
    int64_t nnz;
    int R, nm1;
    bool mixed, det, packed;
};

ModelIn model_in(const cpapr_plan* P)
{
    return {P->nnz, P->R, P->N - 1, P->params.precision == CPAPR_MIXED, P->params.deterministic != 0,
            P->mode[0].pk != nullptr};
}

bool group16_ok(const ModelIn& m)
{
    const int rpl = rank_block(m.R, 16);
    return rpl > 0 && phi_shape_supported(16, rpl, m.nm1);
}

// (tile nonzeros, lanes per nonzero)
void model_shape(const ModelIn& m, int* tile, int* group)
{
    const int g0 = resolve_group(m.R, 0, m.nm1);
    int tb = 512, gb = g0;  // a large tensor's shape
    if (m.R > 16 && m.R <= 32 && m.nm1 <= 3) {
        if (m.mixed) {
            tb = 1024;
        } else if (group16_ok(m)) {
            tb = 256;
            gb = 16;
        }
    } else if (m.packed && m.R > 4 && m.R <= 16) {
        tb = 1024;  // one load per staged nonzero: the tile's fixed costs weigh more
    }
    int64_t t = 32;  // the largest power of two <= nnz / 900, up to the large tensor's tile
    while (t < tb && 2 * t * 900 <= m.nnz) t *= 2;
    if (m.det && t < 128) t = 128;
    if (t >= tb) {
        *tile = tb;
        *group = gb;
    } else if (t <= 128) {
        *tile = (int)t;
        *group = group16_ok(m) ? 16 : g0;
    } else {
        *tile = (int)t;
        *group = t == 256 && m.mixed && m.R > 8 && m.R <= 16 && group16_ok(m) ? 16 : g0;
    }
}
}  // namespace

int model_group(const cpapr_plan* P)
{
    int t, g;
    model_shape(model_in(P), &t, &g);
    return g;
}

int model_chunk(const cpapr_plan* P, int group)
{
    int t, g;
    model_shape(model_in(P), &t, &g);
    return std::max(1, t / (kBlock / group));
}

void batch_shape(const cpapr_plan* P, int* group, int* chunk)
{
    if (!P->shape_auto) {
        *group = P->group;
        *chunk = P->chunk;
        return;
    }
    ModelIn m = model_in(P);
    m.nnz = int64_t(1) << 40;  // the batch fills the device, not this slot
    m.det = false;             // batched launches take no tile-end buffers
    int t;
    model_shape(m, &t, group);
    *chunk = std::max(1, t / (kBlock / *group));
}

// Deterministic mode: attach the plan's tile-end buffers to a single-plan launch.
// G: lanes per nonzero of the launch (the plan's unless a pass picks its own).
Error attach_det(const cpapr_plan* P, PhiArgs& a, int G = 0)
{
    if (P->det_part == nullptr) return {CPAPR_OK, ""};
    const int64_t tiles = cdiv(a.nnz, (int64_t)(kBlock / (G ? G : P->group)) * a.L);
    if (tiles > P->det_tiles) return {CPAPR_EUNSUPPORTED, "deterministic mode: tiles smaller than 128 nonzeros"};
    a.det_part = P->det_part;
    a.det_rows = P->det_rows;
    a.det_tiles = P->det_tiles;
    return {CPAPR_OK, ""};
}

Error launch_det_fixup(const cpapr_plan* P, int mode, const PhiArgs& a, double* out, const int* done, hipStream_t s,
                       int G = 0)
{
    if (a.det_part == nullptr) return {CPAPR_OK, ""};
    const int64_t tile_nnz = (int64_t)(kBlock / (G ? G : P->group)) * a.L;
    const int64_t tiles = cdiv(a.nnz, tile_nnz);
    if (tiles <= 0) return {CPAPR_OK, ""};
    det_fixup_kernel<<<(unsigned)tiles, kBlock, 0, s>>>(P->mode[mode].rows, a.nnz, tile_nnz, tiles, P->R, a.det_part,
                                                        a.det_rows, a.det_tiles, out, done);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

Error launch_phi(const cpapr_plan* P, int mode, const double* B, const void* const* fac, bool mixed,
                 double eps, double* Phi, const int* done, hipStream_t s)
{
    const int G = P->group;
    const int RPL = rank_block(P->R, G);
    PhiArgs a = make_args(P, mode, B, fac, eps, Phi, done);
    if (P->params.variant == CPAPR_VARIANT_ATOMIC) {
        if (mixed) return {CPAPR_EUNSUPPORTED, "the atomic variant is FP64 only"};
        prof_begin(mode, s);
        Error e = dispatch_atomic(G, RPL, a, s);
        prof_end(s);
        return e;
    }
    Error e = attach_det(P, a);
    if (e.code) return e;
    prof_begin(mode, s);
    if (P->params.variant == CPAPR_VARIANT_XR && xr_shape_supported(G, RPL, a.NM1))
        e = mixed ? dispatch_xr<true>(G, RPL, a, s) : dispatch_xr<false>(G, RPL, a, s);
    else
        e = mixed ? dispatch_seg<true, kPhi>(G, RPL, a, s) : dispatch_seg<false, kPhi>(G, RPL, a, s);
    prof_end(s);
    if (e.code) return e;
    return launch_det_fixup(P, mode, a, Phi, done, s);
}

Error launch_delta(const cpapr_plan* P, int mode, const double* B, const double* D, const int32_t* live,
                   const void* const* fac, double eps, double* out, const int* skip, hipStream_t s)
{
    const int G = P->group;
    const int RPL = rank_block(P->R, G);
    PhiArgs a = make_args(P, mode, B, fac, eps, out, skip);
    a.D = D;
    a.live = live;
    Error e = attach_det(P, a);
    if (e.code) return e;
    e = dispatch_seg<false, kDelta>(G, RPL, a, s);
    if (e.code) return e;
    return launch_det_fixup(P, mode, a, out, skip, s);
}

Error launch_delta4(const cpapr_plan* P, int mode, const double* B, const double* D, const int32_t* live,
                    const void* const* fac, double eps, double* out, const int* skip, hipStream_t s)
{
    if (P->R < kTrials4) return {CPAPR_EUNSUPPORTED, "the four-trial line-search pass needs R >= 4"};
    int G = P->group;
    int RPL = rank_block(P->R, G);
    PhiArgs a = make_args(P, mode, B, fac, eps, out, skip);
    // Four rank columns per lane hold 16 trial-step words per lane: such shapes
    // take twice the lanes per nonzero for this pass, on the same tiles.
    if (RPL == 4 && G <= 32 && phi_shape_supported(2 * G, rank_block(P->R, 2 * G), P->N - 1)) {
        G *= 2;
        RPL = rank_block(P->R, G);
        a.L *= 2;
    }
    a.D = D;
    a.live = live;
    Error e = attach_det(P, a, G);
    if (e.code) return e;
    e = dispatch_seg<false, kDelta4>(G, RPL, a, s);
    if (e.code) return e;
    return launch_det_fixup(P, mode, a, out, skip, s, G);
}

Error launch_mttkrp(const cpapr_plan* P, int mode, const double* const* A, double* M, hipStream_t s)
{
    const int G = P->group;
    const int RPL = rank_block(P->R, G);
    PhiArgs a = make_args(P, mode, nullptr, (const void* const*)A, 0.0, M, nullptr);
    Error e = zero_matrix(M, P->dims[mode] * (int64_t)P->R, s);
    if (e.code) return e;
    e = attach_det(P, a);
    if (e.code) return e;
    prof_begin(mode, s);
    e = dispatch_seg<false, kMttkrp>(G, RPL, a, s);
    prof_end(s);
    if (e.code) return e;
    return launch_det_fixup(P, mode, a, M, nullptr, s);
}

int64_t loglik_partials(int64_t nnz) { return cdiv(nnz, 512) + 1; }

// ---- batched launches ----

namespace {

template <int G, int RPL, int NM1, bool MIXED>
Error batch_launch_t(const BatchSlot* slots, const int32_t* tile_map, const int64_t* class_off,
                     const int64_t* class_ntiles, const int32_t* slot_done, unsigned int* counters, int cls,
                     int* grid_cache, int64_t grid_tiles, hipStream_t s)
{
    if (grid_tiles > 0) {
        if (grid_tiles > 0x7fffffffLL) return {CPAPR_EUNSUPPORTED, "too many tiles in one class"};
        phi_batch_grid_kernel<G, RPL, NM1, MIXED><<<(unsigned)grid_tiles, kBlock, 0, s>>>(slots, tile_map, class_off,
                                                                                         slot_done, cls);
        CPAPR_LAUNCHED();
        return {CPAPR_OK, ""};
    }
    if (*grid_cache <= 0) {
        int per_cu = 0, dev = 0, cus = 0;
        CPAPR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, phi_batch_kernel<G, RPL, NM1, MIXED>,
                                                               kBlock, 0));
        CPAPR_HIP(hipGetDevice(&dev));
        CPAPR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        *grid_cache = std::max(1, per_cu) * std::max(1, cus);
    }
    phi_batch_kernel<G, RPL, NM1, MIXED><<<*grid_cache, kBlock, 0, s>>>(slots, tile_map, class_off, class_ntiles,
                                                                        slot_done, counters, cls);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

struct BatchShape {
    int G, RPL, NM1;
    bool mixed;
};

constexpr BatchShape kBatchShapes[] = {
#define CPAPR_BS(GG, RR)                                                                              \
    {GG, RR, 1, false}, {GG, RR, 2, false}, {GG, RR, 3, false}, {GG, RR, 1, true}, {GG, RR, 2, true}, \
        {GG, RR, 3, true}
    CPAPR_BS(4, 1), CPAPR_BS(8, 1), CPAPR_BS(8, 2), CPAPR_BS(8, 4), CPAPR_BS(16, 1), CPAPR_BS(16, 2), CPAPR_BS(16, 4)
#undef CPAPR_BS
};

}  // namespace

int batch_class_count() { return (int)(sizeof(kBatchShapes) / sizeof(kBatchShapes[0])); }

int batch_class_of(int G, int RPL, int NM1, bool mixed)
{
    for (int c = 0; c < batch_class_count(); ++c) {
        const BatchShape& b = kBatchShapes[c];
        if (b.G == G && b.RPL == RPL && b.NM1 == NM1 && b.mixed == mixed) return c;
    }
    return -1;
}

Error launch_phi_batch(int cls, const BatchSlot* slots, const int32_t* tile_map, const int64_t* class_off,
                       const int64_t* class_ntiles, const int32_t* slot_done, unsigned int* counters,
                       int* grid_cache, int64_t grid_tiles, hipStream_t s)
{
    if (cls < 0 || cls >= batch_class_count()) return {CPAPR_EINVAL, "bad batch class"};
    const BatchShape& b = kBatchShapes[cls];
#define CPAPR_BL(GG, RR, NN, MM)                                                                     \
    if (b.G == GG && b.RPL == RR && b.NM1 == NN && b.mixed == MM)                                    \
        return batch_launch_t<GG, RR, NN, MM>(slots, tile_map, class_off, class_ntiles, slot_done, counters, cls,   \
                                              grid_cache, grid_tiles, s);
#define CPAPR_BL6(GG, RR)                                                                            \
    CPAPR_BL(GG, RR, 1, false) CPAPR_BL(GG, RR, 2, false) CPAPR_BL(GG, RR, 3, false)                 \
    CPAPR_BL(GG, RR, 1, true) CPAPR_BL(GG, RR, 2, true) CPAPR_BL(GG, RR, 3, true)
    CPAPR_BL6(4, 1) CPAPR_BL6(8, 1) CPAPR_BL6(8, 2) CPAPR_BL6(8, 4) CPAPR_BL6(16, 1) CPAPR_BL6(16, 2) CPAPR_BL6(16, 4)
#undef CPAPR_BL6
#undef CPAPR_BL
    return {CPAPR_EUNSUPPORTED, "no batched Phi kernel for this shape"};
}

Error launch_batch_elementwise(const BatchCopy* items, const int32_t* nitems_dev, const int64_t* total_dev,
                               const int32_t* slot_done, unsigned int* counters, int grid, hipStream_t s)
{
    batch_elementwise_kernel<<<grid, kBlock, 0, s>>>(items, nitems_dev, total_dev, slot_done, counters,
                                                     kBatchCounters);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

PhiArgs phi_args(const cpapr_plan* P, int mode, const double* B, const void* const* fac, double eps, double* Phi)
{
    return make_args(P, mode, B, fac, eps, Phi, nullptr);
}

Error launch_loglik_terms(const cpapr_plan* P, const double* B, const double* const* A, double eps, double* partial,
                          int* nparts, hipStream_t s)
{
    // Default shape for this rank (always instantiated), 512 nonzeros per tile.
    const int G = resolve_group(P->R, 0, P->N - 1);
    const int RPL = rank_block(P->R, G);
    PhiArgs a = make_args(P, 0, B, (const void* const*)A, eps, partial, nullptr);
    a.L = resolve_chunk(G, 0);
    const int64_t tiles = cdiv(P->nnz, (int64_t)(kBlock / G) * a.L);
    *nparts = (int)tiles;
    if (tiles == 0) return {CPAPR_OK, ""};
    return dispatch_seg<false, kLoglik>(G, RPL, a, s);
}

}  // namespace cpapr
