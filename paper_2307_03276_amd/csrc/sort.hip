// Plan construction: input validation and the per-mode sort of the nonzeros.
//
// The paper avoids the Phi-row write race by storing the nonzeros of one Phi
// row contiguously, sorting once per mode at the start (Section 3.1, the
// sort-by-mode strategy). SparTen keeps N permutation arrays and reads through
// them; the indirection is the scattered access the paper flags as slow. Here
// each mode instead gets a physically permuted structure-of-arrays copy, so the
// Phi kernel streams coordinates and values in order.
//
// Sort: stable least-significant-digit radix sort of (i_n, k) pairs with
// 8-bit digits, one pass per digit of ceil(log2 I_n) bits. Each pass is
// (1) per-tile digit histograms, (2) an exclusive scan of the digit-major
// histogram table, (3) a stable scatter that ranks equal digits inside a wave
// with ballots and across the workgroup's waves through LDS. Stability keeps
// nonzeros of a row in input order, so plans and Phi are deterministic.
#include <algorithm>

#include "internal.hpp"

namespace cpapr {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortRounds = 16;                // items per thread per tile
constexpr int kSortTile = kBlock * kSortRounds;  // 4096 keys per tile
constexpr int kScanChunk = 4096;                 // elements per block in the scan
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

// Digit histogram of one 4096-key tile, written digit-major: counts[d * ntiles + tile].
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const int32_t* __restrict__ keys, int64_t n,
                                                            int shift, int* __restrict__ counts, int ntiles)
{
    __shared__ int h[kRadix];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int q = 0; q < kSortRounds; ++q) {
        int64_t e = base + q * kBlock + t;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    counts[(int64_t)t * ntiles + blockIdx.x] = h[t];
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ int block_exclusive_scan(int v, int* tmp, int& total)
{
    const int t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int add = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += add;
        __syncthreads();
    }
    int incl = tmp[t];
    total = tmp[kBlock - 1];
    __syncthreads();
    return incl - v;
}

// Scan phase 1: sums of kScanChunk-element chunks.
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(const int* __restrict__ a, int64_t n,
                                                             int* __restrict__ sums)
{
    __shared__ int red[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int s = 0;
    for (int q = threadIdx.x; q < kScanChunk; q += kBlock)
        if (base + q < n) s += a[base + q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Scan phase 2: exclusive scan of the chunk sums by one workgroup.
__global__ __launch_bounds__(kBlock) void scan_sums_kernel(int* sums, int nsums)
{
    __shared__ int tmp[kBlock];
    int carry = 0;
    for (int base = 0; base < nsums; base += kBlock) {
        int i = base + threadIdx.x;
        int v = i < nsums ? sums[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, tmp, total);
        if (i < nsums) sums[i] = carry + ex;
        carry += total;
    }
}

// Scan phase 3: exclusive scan inside each chunk, offset by the chunk's prefix.
__global__ __launch_bounds__(kBlock) void scan_chunks_kernel(int* a, int64_t n, const int* __restrict__ sums)
{
    __shared__ int tmp[kBlock];
    constexpr int per = kScanChunk / kBlock;  // consecutive elements per thread
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * per;
    int loc[per];
    int s = 0;
    for (int q = 0; q < per; ++q) {
        loc[q] = base + q < n ? a[base + q] : 0;
        s += loc[q];
    }
    int total;
    int ex = block_exclusive_scan(s, tmp, total) + sums[blockIdx.x];
    for (int q = 0; q < per; ++q) {
        if (base + q < n) a[base + q] = ex;
        ex += loc[q];
    }
}

// Stable scatter of one tile. Items are visited in rounds of 256 consecutive
// keys (round-major, thread-minor = input order). Within a round, lanes of a
// wave with equal digits are matched by 8 ballots; a lane's rank is the number
// of matching lower lanes plus the counts of earlier waves, plus the digit's
// running offset from earlier rounds and from earlier tiles (the scan).
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const int32_t* __restrict__ keys_in,
                                                               const int32_t* __restrict__ pay_in,
                                                               int32_t* __restrict__ keys_out,
                                                               int32_t* __restrict__ pay_out, int64_t n,
                                                               int shift, const int* __restrict__ offsets,
                                                               int ntiles)
{
    constexpr int kWaves = kBlock / 64;
    __shared__ int run[kRadix];
    __shared__ int wcnt[kWaves][kRadix];
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const int lane = t & 63;
    run[t] = offsets[(int64_t)t * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int q = 0; q < kSortRounds; ++q) {
        const int64_t e = base + q * kBlock + t;
        const bool valid = e < n;
        int32_t key = valid ? keys_in[e] : 0;
        int32_t pay = valid ? (pay_in ? pay_in[e] : (int32_t)e) : 0;
        const int d = (key >> shift) & (kRadix - 1);
        for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
        __syncthreads();
        unsigned long long match = __ballot(valid);
        for (int b = 0; b < kRadixBits; ++b) {
            unsigned long long ones = __ballot((d >> b) & 1);
            match &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int rank = __popcll(match & below);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(match);
        __syncthreads();
        if (valid) {
            int64_t pos = (int64_t)run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            if (pos >= 0 && pos < n) {  // always true when the histogram scan is consistent
                keys_out[pos] = key;
                pay_out[pos] = pay;
            }
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kWaves; ++w) add += wcnt[w][t];
        run[t] += add;
        __syncthreads();
    }
}

// keys_out[p] = keys[perm[p]]: a key array in the order of an earlier sort.
__global__ __launch_bounds__(kBlock) void permute_keys_kernel(const int32_t* __restrict__ keys,
                                                              const int32_t* __restrict__ perm, int64_t nnz,
                                                              int32_t* __restrict__ keys_out)
{
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kBlock) {
        int64_t k = perm[p];
        if (k < 0 || k >= nnz) k = p;  // a permutation never leaves [0, nnz); keeps reads in bounds
        keys_out[p] = keys[k];
    }
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

Error exclusive_scan(int* a, int64_t n, int* sums, hipStream_t s)
{
    const int nchunks = (int)cdiv(n, kScanChunk);
    scan_reduce_kernel<<<nchunks, kBlock, 0, s>>>(a, n, sums);
    CPAPR_LAUNCHED();
    scan_sums_kernel<<<1, kBlock, 0, s>>>(sums, nchunks);
    CPAPR_LAUNCHED();
    scan_chunks_kernel<<<nchunks, kBlock, 0, s>>>(a, n, sums);
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
    b += 5 * align256((size_t)nnz * 4);                     // keys/payload ping-pong, secondary order
    b += align256((size_t)ncounts * 4);                     // histogram table
    b += align256((size_t)cdiv(ncounts, kScanChunk) * 4 + 4);  // scan chunk sums
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
    int32_t* ka = (int32_t*)take((size_t)nnz * 4);
    int32_t* kb = (int32_t*)take((size_t)nnz * 4);
    int32_t* pa = (int32_t*)take((size_t)nnz * 4);
    int32_t* pb = (int32_t*)take((size_t)nnz * 4);
    int32_t* secperm = (int32_t*)take((size_t)nnz * 4);  // order by the secondary key, kept for reuse
    int sec_cached = -1;
    int* counts = (int*)take((size_t)ncounts * 4);
    int* sums = (int*)take((size_t)cdiv(ncounts, kScanChunk) * 4 + 4);
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
        const int32_t* kin = nullptr;
        const int32_t* pin = nullptr;  // nullptr: identity payload
        auto passes = [&](int64_t dim) -> Error {
            int bits = 0;
            while (bits < 31 && ((int64_t)1 << bits) < dim) ++bits;
            for (int ps = 0; ps < (bits + kRadixBits - 1) / kRadixBits; ++ps) {
                const int shift = ps * kRadixBits;
                int32_t* kout = (kin == ka) ? kb : ka;
                int32_t* pout = (pin == pa) ? pb : pa;
                radix_hist_kernel<<<(int)ntiles, kBlock, 0, s>>>(kin, nnz, shift, counts, (int)ntiles);
                CPAPR_LAUNCHED();
                Error e = exclusive_scan(counts, ncounts, sums, s);
                if (e.code) return e;
                radix_scatter_kernel<<<(int)ntiles, kBlock, 0, s>>>(kin, pin, kout, pout, nnz, shift, counts,
                                                                    (int)ntiles);
                CPAPR_LAUNCHED();
                kin = kout;
                pin = pout;
            }
            return {CPAPR_OK, ""};
        };
        // Secondary key first (stable LSD order): within each row of mode n the
        // nonzeros then follow the largest other mode's coordinate, so that
        // mode's factor rows are swept in order inside long rows.
        int sec = -1;
        if (P->params.sort == CPAPR_SORT_ROW_COL)
            for (int m = 0; m < N; ++m)
                if (m != n && (sec < 0 || P->dims[m] > P->dims[sec])) sec = m;
        if (sec >= 0 && sec == sec_cached) {
            pin = secperm;  // the same secondary order as the previous mode's: reuse it
        } else if (sec >= 0) {
            kin = X->idx + (int64_t)sec * nnz;
            Error e = passes(P->dims[sec]);
            if (e.code) return e;
            if (pin != nullptr) {
                CPAPR_HIP(hipMemcpyAsync(secperm, pin, (size_t)nnz * 4, hipMemcpyDeviceToDevice, s));
                sec_cached = sec;
            }
        }
        if (sec >= 0) {
            if (pin != nullptr) {  // keys of mode n in the secondary order
                int32_t* kout = (kin == ka) ? kb : ka;
                permute_keys_kernel<<<grid_for(nnz), kBlock, 0, s>>>(X->idx + (int64_t)n * nnz, pin, nnz, kout);
                CPAPR_LAUNCHED();
                kin = kout;
            } else {
                kin = X->idx + (int64_t)n * nnz;
            }
        } else {
            kin = X->idx + (int64_t)n * nnz;
        }
        {
            Error e = passes(P->dims[n]);
            if (e.code) return e;
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
