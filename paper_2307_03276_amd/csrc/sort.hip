// Plan construction: input validation and the per-mode sort of the nonzeros.
//
// The paper avoids the Phi-row write race by storing the nonzeros of one Phi
// row contiguously, sorting once per mode at the start (Section 3.1, the
// sort-by-mode strategy). SparTen keeps N permutation arrays and reads through
// them; the indirection is the scattered access the paper flags as slow. Here
// each mode instead gets a physically permuted structure-of-arrays copy, so the
// Phi kernel streams coordinates and values in order.
//
// Sort: stable least-significant-digit radix sort of (key, k) pairs with 8-bit
// digits, one pass per digit of the key's width. The key is i_n, or (in the
// ROW_COL order) i_n followed by the high bits of the largest other mode's
// coordinate in one 32-bit word. Each pass is (1) per-tile digit histograms,
// (2) each (tile, digit)'s output offset, scanned over digits and tiles, (3) a stable
// scatter: a tile is ranked in registers (equal digits matched inside a wave
// with ballots, running counts per wave in LDS), reordered by digit in LDS and
// written out in digit runs, so consecutive lanes store to consecutive
// addresses. Stability keeps nonzeros of equal keys in input order, so plans
// and Phi are deterministic.
#include <algorithm>

#include "internal.hpp"

namespace cpapr {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortRounds = 16;                // items per thread per tile
constexpr int kSortTile = kBlock * kSortRounds;  // 4096 keys per tile
constexpr int kScanTiles = 64;                   // tiles per workgroup in the offsets scan
constexpr int kSegPartials = 1024;               // blocks of the segment count

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct DimsArg {
    int64_t d[CPAPR_MAX_MODES];
};

// Nonzero record: the N coordinates (int32 words 0..N-1) and the value (the
// last two words) of one nonzero in 32 bytes (N <= 6) or 64 bytes (N = 7, 8).
// The per-mode gathers through a sort permutation then touch one record per
// nonzero instead of N + 1 separate arrays.
inline int record_words(int N) { return N <= 6 ? 8 : 16; }

// Validates the input and packs it into records in the same pass.
// flags bit 0: coordinate out of range; bit 1: value not finite or <= 0.
template <int RSW>
__global__ __launch_bounds__(kBlock) void validate_pack_kernel(const int32_t* __restrict__ idx,
                                                               const double* __restrict__ vals, int64_t nnz,
                                                               int N, DimsArg dims, int* flags,
                                                               uint4* __restrict__ rec)
{
    int bad = 0;
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kBlock) {
        int32_t w[RSW];
#pragma unroll
        for (int m = 0; m < RSW - 2; ++m) {
            w[m] = 0;
            if (m < N) {
                const int32_t c = idx[(int64_t)m * nnz + k];
                if (c < 0 || (int64_t)c >= dims.d[m]) bad |= 1;
                w[m] = c;
            }
        }
        const double v = vals[k];
        if (!(v > 0.0) || !(v <= 1.7976931348623157e308)) bad |= 2;
        if ((double)(float)v != v) bad |= 4;  // the packed records need values exact in FP32
        __builtin_memcpy(&w[RSW - 2], &v, sizeof(double));
        uint4* r = rec + k * (RSW / 4);
#pragma unroll
        for (int i = 0; i < RSW / 4; ++i) r[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
    }
    if (bad) atomicOr(flags, bad);
}

// Mask of the lanes of this wave whose digit equals this lane's (8 ballots);
// lanes with valid == false match nothing.
__device__ __forceinline__ unsigned long long digit_peers(int d, bool valid)
{
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const unsigned long long ones = __ballot((d >> b) & 1);
        m &= ((d >> b) & 1) ? ones : ~ones;
    }
    return m;
}

__device__ __forceinline__ unsigned long long lanes_below()
{
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Digit histogram of one 4096-key tile, written tile-major: counts[tile * 256 + d].
// The tile's keys are loaded first (all loads in flight), then counted with
// one LDS add each.
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                            int shift, int* __restrict__ counts)
{
    __shared__ int h[kRadix];
    const int t = threadIdx.x;
    h[t] = 0;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    uint32_t key[kSortRounds];
#pragma unroll
    for (int q = 0; q < kSortRounds; ++q) {
        const int64_t e = base + q * kBlock + t;
        key[q] = e < n ? keys[e] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortRounds; ++q)
        if (base + q * kBlock + t < n) atomicAdd(&h[(key[q] >> shift) & (kRadix - 1)], 1);
    __syncthreads();
    counts[(int64_t)blockIdx.x * kRadix + t] = h[t];
}

// Output offsets of a pass: offset(tile, d) = (keys with a smaller digit) +
// (keys with digit d in earlier tiles), in place over the tile-major table, in
// three steps with one thread per digit (every access coalesced across digits):
// per-group column sums over kScanTiles tiles; one walk down the groups (their
// exclusive prefixes per digit) and the scan of the digit totals; the scan
// inside each group.
__global__ __launch_bounds__(kBlock) void offsets_sum_kernel(const int* __restrict__ counts, int ntiles,
                                                             int* __restrict__ part)
{
    const int t0 = blockIdx.x * kScanTiles;
    const int t1 = min(t0 + kScanTiles, ntiles);
    int s = 0;
#pragma unroll 16
    for (int tile = t0; tile < t1; ++tile) s += counts[(int64_t)tile * kRadix + threadIdx.x];
    part[(int64_t)blockIdx.x * kRadix + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void offsets_groups_kernel(int* __restrict__ part, int ngroups,
                                                                int* __restrict__ dbase)
{
    static_assert(kRadix == kBlock, "one digit per thread");
    __shared__ int wsum[kBlock / 64];
    const int d = threadIdx.x;
    const int lane = d & 63;
    int run = 0;
#pragma unroll 16
    for (int g = 0; g < ngroups; ++g) {
        const int v = part[(int64_t)g * kRadix + d];
        part[(int64_t)g * kRadix + d] = run;
        run += v;
    }
    // exclusive scan of the digit totals
    int incl = run;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[d >> 6] = incl;
    __syncthreads();
    int base = incl - run;
    for (int w = 0; w < (d >> 6); ++w) base += wsum[w];
    dbase[d] = base;
}

__global__ __launch_bounds__(kBlock) void offsets_tiles_kernel(int* __restrict__ counts, int ntiles,
                                                               const int* __restrict__ part,
                                                               const int* __restrict__ dbase)
{
    const int t0 = blockIdx.x * kScanTiles;
    const int t1 = min(t0 + kScanTiles, ntiles);
    int run = part[(int64_t)blockIdx.x * kRadix + threadIdx.x] + dbase[threadIdx.x];
#pragma unroll 16
    for (int tile = t0; tile < t1; ++tile) {
        const int64_t i = (int64_t)tile * kRadix + threadIdx.x;
        const int v = counts[i];
        counts[i] = run;
        run += v;
    }
}

// Stable scatter of one tile. Wave w ranks the tile's w-th quarter in rounds
// of 64 consecutive keys: a key's rank among equal digits is its matching lower
// lanes plus the wave's running count of that digit (LDS). The per-wave counts
// then give each key its position in the tile ordered by (digit, input order);
// the tile is rearranged in LDS and written out in that order, the digit's
// global offset (from the scan) minus the digit's start in the tile added to
// the LDS position.
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const uint32_t* __restrict__ keys_in,
                                                               const int32_t* __restrict__ pay_in,
                                                               uint32_t* __restrict__ keys_out,
                                                               int32_t* __restrict__ pay_out, int64_t n,
                                                               int shift, const int* __restrict__ offsets)
{
    constexpr int kWaves = kBlock / 64;
    constexpr int kRounds = kSortTile / kBlock;  // rounds of 64 keys per wave
    static_assert(kRadix == kBlock, "one digit per thread in the per-digit steps");
    __shared__ int wrun[kWaves][kRadix];  // per-wave digit counts, then their exclusive prefix over waves
    __shared__ int dstart[kRadix];        // digit start in the tile's sorted order
    __shared__ int64_t gshift[kRadix];    // global position - tile position, per digit
    __shared__ int wsum[kWaves];
    __shared__ uint32_t skey[kSortTile];
    __shared__ int32_t spay[kSortTile];
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const int lane = t & 63;
    const unsigned long long below = lanes_below();
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wrun[w][t] = 0;
    const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = tbase + (int64_t)wave * (kSortTile / kWaves);
    uint32_t key[kRounds];
    int32_t pay[kRounds];
    int rk[kRounds];
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
        const int64_t e = wbase + q * 64 + lane;
        key[q] = e < n ? keys_in[e] : 0u;
        pay[q] = e < n ? (pay_in ? pay_in[e] : (int32_t)e) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
        const bool valid = wbase + q * 64 + lane < n;
        const int d = (int)((key[q] >> shift) & (kRadix - 1));
        const unsigned long long match = digit_peers(d, valid);
        const int prev = wrun[wave][d];
        rk[q] = prev + __popcll(match & below);
        // every lane has read its digit's count before the group's lowest lane adds to it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid && (match & below) == 0) wrun[wave][d] = prev + __popcll(match);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    // thread t = digit t: prefix over waves, then the digit's start in the tile
    int tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int c = wrun[w][t];
        wrun[w][t] = tot;
        tot += c;
    }
    int incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int start = incl - tot;
    for (int w = 0; w < wave; ++w) start += wsum[w];
    dstart[t] = start;
    gshift[t] = (int64_t)offsets[(int64_t)blockIdx.x * kRadix + t] - start;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
        if (wbase + q * 64 + lane < n) {
            const int d = (int)((key[q] >> shift) & (kRadix - 1));
            const int j = dstart[d] + wrun[wave][d] + rk[q];
            if ((unsigned)j < (unsigned)kSortTile) {  // always true: the counts are this tile's own
                skey[j] = key[q];
                spay[j] = pay[q];
            }
        }
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kSortTile, n - tbase);
    for (int j = t; j < cnt; j += kBlock) {
        const uint32_t k = skey[j];
        const int64_t pos = gshift[(k >> shift) & (kRadix - 1)] + j;
        if (pos >= 0 && pos < n) {  // always true when the histogram scan is consistent
            keys_out[pos] = k;
            pay_out[pos] = spay[j];
        }
    }
}

// Sort keys of the ROW_COL order: i_n in the high bits, the secondary
// coordinate without its `drop` low bits below it (lo_bits = its kept width).
__global__ __launch_bounds__(kBlock) void composite_keys_kernel(const int32_t* __restrict__ hi,
                                                                const int32_t* __restrict__ lo, int64_t nnz,
                                                                int lo_bits, int drop, uint32_t* __restrict__ keys)
{
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kBlock)
        keys[p] = ((uint32_t)hi[p] << lo_bits) | ((uint32_t)lo[p] >> drop);
}

// Write the sorted copy of one mode: row, value and the other modes' factor
// row offsets (coordinate x R), read from the records through the permutation
// (perm == nullptr: identity); with pk also the packed 16-byte records
// {row, offset 0, offset 1 or 0, value as FP32} (N <= 3, values exact in FP32).
template <int RSW>
__global__ __launch_bounds__(kBlock) void gather_sorted_kernel(const uint4* __restrict__ rec, int64_t nnz, int N,
                                                               int mode, const int32_t* __restrict__ perm, int R,
                                                               int32_t* __restrict__ rows,
                                                               uint32_t* __restrict__ cofs,
                                                               double* __restrict__ svals, int4* __restrict__ pk)
{
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kBlock) {
        int64_t k = perm ? perm[p] : p;
        if (k < 0 || k >= nnz) k = p;  // a permutation never leaves [0, nnz); keeps reads in bounds
        int32_t w[RSW];
        const uint4* r = rec + k * (RSW / 4);
#pragma unroll
        for (int i = 0; i < RSW / 4; ++i) {
            const uint4 q = r[i];
            w[4 * i] = (int32_t)q.x;
            w[4 * i + 1] = (int32_t)q.y;
            w[4 * i + 2] = (int32_t)q.z;
            w[4 * i + 3] = (int32_t)q.w;
        }
        double v;
        __builtin_memcpy(&v, &w[RSW - 2], sizeof(double));
        svals[p] = v;
        int j = 0;
        uint32_t off[2] = {0u, 0u};
        int32_t row = 0;
#pragma unroll
        for (int m = 0; m < RSW - 2; ++m) {
            if (m >= N) break;
            if (m == mode) {
                rows[p] = w[m];
                row = w[m];
            } else {
                const uint32_t o = (uint32_t)w[m] * (uint32_t)R;
                cofs[(int64_t)j * nnz + p] = o;
                if (j < 2) off[j] = o;
                ++j;
            }
        }
        if (pk != nullptr) pk[p] = make_int4(row, (int)off[0], (int)off[1], __float_as_int((float)v));
    }
}

// Number of row changes in the sorted row array, two-level: per-block counts,
// then one block adds them (no same-address atomics).
__global__ __launch_bounds__(kBlock) void count_segments_kernel(const int32_t* __restrict__ rows, int64_t nnz,
                                                                unsigned long long* partial)
{
    __shared__ unsigned long long red[kBlock / 64];
    unsigned long long c = 0;
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kBlock)
        c += (p == 0 || rows[p] != rows[p - 1]) ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w];
        partial[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const unsigned long long* __restrict__ partial, int n,
                                                              unsigned long long* out)
{
    __shared__ unsigned long long red[kBlock];
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < n; i += kBlock) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kBlock; ++i) t += red[i];
        *out = t;
    }
}

int grid_for(int64_t n)
{
    int64_t g = cdiv(n, kBlock);
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

Error pass_offsets(int* counts, int ntiles, int* part, hipStream_t s)
{
    const int ngroups = (int)cdiv(ntiles, kScanTiles);
    offsets_sum_kernel<<<ngroups, kBlock, 0, s>>>(counts, ntiles, part);
    CPAPR_LAUNCHED();
    offsets_groups_kernel<<<1, kBlock, 0, s>>>(part, ngroups, part + (int64_t)ngroups * kRadix);
    CPAPR_LAUNCHED();
    offsets_tiles_kernel<<<ngroups, kBlock, 0, s>>>(counts, ntiles, part, part + (int64_t)ngroups * kRadix);
    CPAPR_LAUNCHED();
    return {CPAPR_OK, ""};
}

}  // namespace

int64_t sort_scratch_bytes(int64_t nnz, int N)
{
    const int64_t ntiles = cdiv(nnz > 0 ? nnz : 1, kSortTile);
    const int64_t ncounts = ntiles * kRadix;
    size_t b = 0;
    b += align256((size_t)nnz * 4 * record_words(N));       // nonzero records
    b += 4 * align256((size_t)nnz * 4);                     // keys/payload ping-pong
    b += align256((size_t)ncounts * 4);                     // histogram table
    b += align256((size_t)(cdiv(ntiles, kScanTiles) + 1) * kRadix * 4);  // offsets scan: group sums, digit bases
    b += 256;                                                // flags / counters
    b += align256(kSegPartials * 8);                         // segment-count partials
    return (int64_t)b;
}

Error build_sorted(cpapr_plan* P, const cpapr_coo* X, char* scratch, hipStream_t s, int only)
{
    const int64_t nnz = P->nnz;
    const int N = P->N;
    const int64_t ntiles = cdiv(nnz > 0 ? nnz : 1, kSortTile);
    const int64_t ncounts = ntiles * kRadix;
    char* q = scratch;
    auto take = [&](size_t bytes) {
        char* r = q;
        q += align256(bytes);
        return r;
    };
    const int rsw = record_words(N);
    uint4* rec = (uint4*)take((size_t)nnz * 4 * rsw);
    uint32_t* ka = (uint32_t*)take((size_t)nnz * 4);
    uint32_t* kb = (uint32_t*)take((size_t)nnz * 4);
    int32_t* pa = (int32_t*)take((size_t)nnz * 4);
    int32_t* pb = (int32_t*)take((size_t)nnz * 4);
    int* counts = (int*)take((size_t)ncounts * 4);
    int* part = (int*)take((size_t)(cdiv(ntiles, kScanTiles) + 1) * kRadix * 4);
    int* flags = (int*)take(256);
    unsigned long long* segc = (unsigned long long*)(flags + 8);
    unsigned long long* segpart = (unsigned long long*)take(kSegPartials * 8);

    // flags and segment counters start at zero (plain kernel-free path: a tiny fill)
    CPAPR_HIP(hipMemsetAsync(flags, 0, 256, s));
    if (nnz > 0) {
        DimsArg d{};
        for (int m = 0; m < N; ++m) d.d[m] = P->dims[m];
        if (rsw == 8)
            validate_pack_kernel<8><<<grid_for(nnz), kBlock, 0, s>>>(X->idx, X->vals, nnz, N, d, flags, rec);
        else
            validate_pack_kernel<16><<<grid_for(nnz), kBlock, 0, s>>>(X->idx, X->vals, nnz, N, d, flags, rec);
        CPAPR_LAUNCHED();
    }
    int hflags = 0;
    CPAPR_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipStreamSynchronize(s));
    if (hflags & 1) return {CPAPR_EINDEX, "a coordinate lies outside its mode's range"};
    if (hflags & 2) return {CPAPR_EVALUE, "a tensor value is not finite and positive"};
    if (hflags & 4)  // some value is not exact in FP32: the kernels read the arrays
        for (int n = 0; n < N; ++n) P->mode[n].pk = nullptr;

    for (int n = 0; n < N; ++n) {
        if (only >= 0 && n != only) continue;
        PlanMode& pm = P->mode[n];
        if (nnz == 0) {
            pm.segments = 0;
            continue;
        }
        // LSD passes over the low `bits` bits of the keys in (kin, pin); outputs
        // alternate between (ka, kb) and (pa, pb), never aliasing the inputs.
        const uint32_t* kin = (const uint32_t*)(X->idx + (int64_t)n * nnz);  // validated: >= 0
        const int32_t* pin = nullptr;  // nullptr: identity payload
        auto width = [](int64_t dim) {
            int bits = 0;
            while (bits < 31 && ((int64_t)1 << bits) < dim) ++bits;
            return bits;
        };
        int bits = width(P->dims[n]);
        // ROW_COL: within each row of mode n the nonzeros follow the largest
        // other mode's coordinate, so that mode's factor rows are swept in order
        // inside long rows. Both go into one 32-bit key; when i_n and that
        // coordinate need more bits, the coordinate's low bits are dropped
        // (runs of 2^drop consecutive coordinates keep input order).
        int sec = -1;
        if (P->params.sort == CPAPR_SORT_ROW_COL)
            for (int m = 0; m < N; ++m)
                if (m != n && (sec < 0 || P->dims[m] > P->dims[sec])) sec = m;
        if (sec >= 0) {
            const int sbits = width(P->dims[sec]);
            const int keep = std::min(sbits, 32 - bits);
            composite_keys_kernel<<<grid_for(nnz), kBlock, 0, s>>>(X->idx + (int64_t)n * nnz,
                                                                   X->idx + (int64_t)sec * nnz, nnz, keep,
                                                                   sbits - keep, ka);
            CPAPR_LAUNCHED();
            kin = ka;
            bits += keep;
        }
        for (int ps = 0; ps < (bits + kRadixBits - 1) / kRadixBits; ++ps) {
            const int shift = ps * kRadixBits;
            uint32_t* kout = (kin == ka) ? kb : ka;
            int32_t* pout = (pin == pa) ? pb : pa;
            radix_hist_kernel<<<(int)ntiles, kBlock, 0, s>>>(kin, nnz, shift, counts);
            CPAPR_LAUNCHED();
            Error e = pass_offsets(counts, (int)ntiles, part, s);
            if (e.code) return e;
            radix_scatter_kernel<<<(int)ntiles, kBlock, 0, s>>>(kin, pin, kout, pout, nnz, shift, counts);
            CPAPR_LAUNCHED();
            kin = kout;
            pin = pout;
        }
        if (rsw == 8)
            gather_sorted_kernel<8><<<grid_for(nnz), kBlock, 0, s>>>(rec, nnz, N, n, pin, P->R, pm.rows, pm.cofs,
                                                                     pm.vals, pm.pk);
        else
            gather_sorted_kernel<16><<<grid_for(nnz), kBlock, 0, s>>>(rec, nnz, N, n, pin, P->R, pm.rows, pm.cofs,
                                                                      pm.vals, pm.pk);
        CPAPR_LAUNCHED();
        const int gseg = std::min(grid_for(nnz), kSegPartials);
        count_segments_kernel<<<gseg, kBlock, 0, s>>>(pm.rows, nnz, segpart);
        CPAPR_LAUNCHED();
        sum_partials_kernel<<<1, kBlock, 0, s>>>(segpart, gseg, segc + n);
        CPAPR_LAUNCHED();
    }
    unsigned long long hseg[CPAPR_MAX_MODES] = {};
    CPAPR_HIP(hipMemcpyAsync(hseg, segc, sizeof(unsigned long long) * N, hipMemcpyDeviceToHost, s));
    CPAPR_HIP(hipStreamSynchronize(s));
    for (int n = 0; n < N; ++n)
        if (only < 0 || n == only) P->mode[n].segments = (int64_t)hseg[n];
    return {CPAPR_OK, ""};
}

}  // namespace cpapr
