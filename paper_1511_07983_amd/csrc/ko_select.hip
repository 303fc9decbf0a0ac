// gfx950 kernels of libko beyond the simulator: writing sampled launch orders,
// and selecting the smallest values of large device arrays (the orders a
// surrogate scores best; the makespan at a given rank of a full enumeration).
//
// Selection is radix selection on order-preserving unsigned keys: each pass
// counts, among the keys that share the digits fixed so far, how many fall on
// each value of the next 8-bit digit (workgroup-private LDS counters flushed
// with one atomic per nonzero bin); the host walks the counts to fix that
// digit.  After the last pass the k-th smallest key is known exactly.

#include <hip/hip_runtime.h>

#include "ko_device.h"
#include "ko_orders.h"
#include "ko_select.h"

namespace ko {

// ------------------------------------------------------------------ orders

__global__ __launch_bounds__(256) void sample_orders_kernel(uint32_t n, uint32_t set, uint64_t seed,
                                                            uint64_t first, const uint64_t *indices,
                                                            uint64_t count, uint8_t *orders,
                                                            uint8_t *positions)
{
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count)
        return;
    const uint64_t i = indices ? indices[b] : first + b;
    const uint64_t rank = sampled_rank(seed, set, i, n);
    unrank_thread(rank, n, orders ? orders + b * n : nullptr, positions ? positions + b * n : nullptr);
}

// ------------------------------------------------------------------ keys

// float -> unsigned key with the same order (negative values reversed)
__device__ __forceinline__ uint32_t f32_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_f32(uint32_t k)
{
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
}

// int64 -> unsigned key with the same order
__device__ __forceinline__ uint64_t i64_key(int64_t v) { return (uint64_t)v ^ 0x8000000000000000ull; }

template <typename T>
__device__ __forceinline__ uint64_t key_of(const T *src, uint64_t i);

template <>
__device__ __forceinline__ uint64_t key_of<float>(const float *src, uint64_t i)
{
    return f32_key(src[i]);
}

template <>
__device__ __forceinline__ uint64_t key_of<int64_t>(const int64_t *src, uint64_t i)
{
    return i64_key(src[i]);
}

// bins[d] += #{i : (key_i & mask) == prefix and digit (key_i >> shift) & 255 == d}
template <typename T>
__global__ __launch_bounds__(256) void radix_hist_kernel(const T *src, uint64_t count, uint32_t shift,
                                                         uint64_t mask, uint64_t prefix,
                                                         unsigned long long *bins)
{
    __shared__ uint32_t local[256];
    local[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t k = key_of<T>(src, i);
        if ((k & mask) == prefix)
            atomicAdd(&local[(uint32_t)(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = local[threadIdx.x];
    if (c)
        atomicAdd(&bins[threadIdx.x], (unsigned long long)c);
}

// Candidates of a float top-k: every index whose key is <= the k-th smallest,
// as (key << 32) | index, appended through an atomic cursor (order arbitrary;
// the caller sorts).  Entries beyond `cap` are counted but not written.
__global__ __launch_bounds__(256) void gather_f32_kernel(const float *src, uint64_t count,
                                                         uint32_t kth_key, uint64_t *out, uint64_t cap,
                                                         unsigned long long *cursor)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint32_t k = f32_key(src[i]);
        if (k <= kth_key) {
            const uint64_t slot = atomicAdd(cursor, 1ull);
            if (slot < cap)
                out[slot] = ((uint64_t)k << 32) | i;
        }
    }
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t from, uint64_t to, uint64_t value)
{
    const uint64_t i = from + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < to)
        p[i] = value;
}

// One compare-exchange stage (j, k) of the bitonic sorting network over
// keys[0, n), n a power of two: ascending overall.
__global__ void bitonic_stage_kernel(uint64_t *keys, uint64_t n, uint64_t j, uint64_t k)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t l = i ^ j;
    if (l <= i)
        return;
    const uint64_t a = keys[i], b = keys[l];
    const bool up = (i & k) == 0;
    if (up ? (a > b) : (a < b)) {
        keys[i] = b;
        keys[l] = a;
    }
}

__global__ void unpack_topk_kernel(const uint64_t *keys, uint32_t k, int64_t *idx, float *val)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k)
        return;
    const uint64_t c = keys[i];
    if (idx)
        idx[i] = (int64_t)(c & 0xFFFFFFFFull);
    if (val)
        val[i] = key_f32((uint32_t)(c >> 32));
}

// ------------------------------------------------------------------ sorting
//
// Stable LSD radix sort of (key, index) pairs, 8-bit digits, for the ranking
// curve of a full enumeration: keys are makespans minus their minimum, so a
// set whose makespans span less than 2^24 cycles sorts in three passes.  Each
// pass: count the digits of every tile, scan the digit-major count table, then
// scatter each tile in index order.  Within a tile, elements are ranked 256
// at a time: a wavefront finds the lanes that share a lane's digit with eight
// ballots, and the four wavefronts' counts are chained through LDS, so equal
// digits keep their input order (the pass is stable).

constexpr uint32_t kSortThreads = 256;
constexpr uint32_t kSortItems = 16;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;

// keys[i] = v[i] - min as an unsigned offset, idx[i] = i
__global__ __launch_bounds__(256) void sort_init_kernel(const int64_t *v, uint64_t count, int64_t vmin,
                                                        uint64_t *keys, uint32_t *idx)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        keys[i] = (uint64_t)v[i] - (uint64_t)vmin;
        idx[i] = (uint32_t)i;
    }
}

// minimum and maximum of v as order-preserving unsigned keys: mm[0] becomes
// the complement of the smallest key, mm[1] the largest (both start at 0)
__global__ __launch_bounds__(256) void minmax_i64_kernel(const int64_t *v, uint64_t count,
                                                         unsigned long long *mm)
{
    uint64_t lo = ~0ull, hi = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t k = i64_key(v[i]);
        lo = k < lo ? k : lo;
        hi = k > hi ? k : hi;
    }
    __shared__ uint64_t s_lo[256], s_hi[256];
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (uint32_t h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const uint64_t a = s_lo[threadIdx.x + h], b = s_hi[threadIdx.x + h];
            s_lo[threadIdx.x] = a < s_lo[threadIdx.x] ? a : s_lo[threadIdx.x];
            s_hi[threadIdx.x] = b > s_hi[threadIdx.x] ? b : s_hi[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&mm[0], (unsigned long long)~s_lo[0]);
        atomicMax(&mm[1], (unsigned long long)s_hi[0]);
    }
}

// ------------------------------------------------------------------ statistics

// Combine (min, argmin, max, argmax, counts) of two parts; ties go to the
// smaller index.
__device__ __forceinline__ void stats_merge(Partial &a, const Partial &b)
{
    if (b.min_ms < a.min_ms || (b.min_ms == a.min_ms && b.argmin < a.argmin)) {
        a.min_ms = b.min_ms;
        a.argmin = b.argmin;
    }
    if (b.max_ms > a.max_ms || (b.max_ms == a.max_ms && b.argmax < a.argmax)) {
        a.max_ms = b.max_ms;
        a.argmax = b.argmax;
    }
    a.n_less += b.n_less;
    a.n_equal += b.n_equal;
    a.n_greater += b.n_greater;
    a.count += b.count;
}

__device__ __forceinline__ Partial stats_empty()
{
    Partial p;
    p.min_ms = INT64_MAX;
    p.max_ms = INT64_MIN;
    p.argmin = ~0ull;
    p.argmax = ~0ull;
    p.n_less = p.n_equal = p.n_greater = p.count = 0;
    return p;
}

// Tree over the workgroup's 256 parts in LDS; thread 0 ends with the total.
__device__ __forceinline__ Partial stats_block(Partial mine)
{
    __shared__ Partial part[256];
    part[threadIdx.x] = mine;
    __syncthreads();
    for (uint32_t h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            Partial a = part[threadIdx.x];
            stats_merge(a, part[threadIdx.x + h]);
            part[threadIdx.x] = a;
        }
        __syncthreads();
    }
    return part[0];
}

// One Partial per workgroup over a grid-stride share of v[0, count), counts
// against *ref when ref is not null.
__global__ __launch_bounds__(256) void stats_partial_kernel(const int64_t *v, uint64_t count, const int64_t *ref,
                                                            Partial *parts)
{
    Partial p = stats_empty();
    const bool has_ref = ref != nullptr;
    const int64_t r = has_ref ? *ref : 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const int64_t m = v[i];
        // indices only grow along a thread's share: strict comparisons keep the first
        if (m < p.min_ms) {
            p.min_ms = m;
            p.argmin = i;
        }
        if (m > p.max_ms) {
            p.max_ms = m;
            p.argmax = i;
        }
        if (has_ref) {
            p.n_less += (m < r) ? 1u : 0u;
            p.n_equal += (m == r) ? 1u : 0u;
            p.n_greater += (m > r) ? 1u : 0u;
        }
        p.count++;
    }
    const Partial t = stats_block(p);
    if (threadIdx.x == 0)
        parts[blockIdx.x] = t;
}

// One workgroup: the total of n_parts Partials, written as ko_set_stats
// (the same 64-byte layout; an empty array gives min INT64_MAX, max
// INT64_MIN, indices 0).
__global__ __launch_bounds__(256) void stats_final_kernel(const Partial *parts, uint32_t n_parts, Partial *out)
{
    Partial p = stats_empty();
    for (uint32_t i = threadIdx.x; i < n_parts; i += blockDim.x)
        stats_merge(p, parts[i]);
    Partial t = stats_block(p);
    if (threadIdx.x == 0) {
        if (t.count == 0)
            t.argmin = t.argmax = 0;
        *out = t;
    }
}

// counts[d * n_tiles + t] = elements of tile t whose digit is d
__global__ __launch_bounds__(256) void sort_count_kernel(const uint64_t *keys, uint64_t count, uint32_t shift,
                                                         uint32_t n_tiles, uint32_t *counts)
{
    __shared__ uint32_t local[256];
    local[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (uint32_t r = 0; r < kSortItems; r++) {
        const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
        if (i < count)
            atomicAdd(&local[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(uint64_t)threadIdx.x * n_tiles + blockIdx.x] = local[threadIdx.x];
}

// In-place exclusive prefix sum of counts[0, len) by one workgroup of 1024
// threads: each thread sums a contiguous segment, the segment sums are scanned
// in LDS, and each thread rewrites its segment.
__global__ __launch_bounds__(1024) void sort_scan_kernel(uint32_t *counts, uint64_t len)
{
    __shared__ uint32_t part[1024];
    const uint64_t seg = (len + 1023) / 1024;
    const uint64_t lo = min((uint64_t)threadIdx.x * seg, len), hi = min(lo + seg, len);
    uint32_t sum = 0;
    for (uint64_t i = lo; i < hi; i++)
        sum += counts[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        const uint32_t add = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (uint64_t i = lo; i < hi; i++) {
        const uint32_t c = counts[i];
        counts[i] = run;
        run += c;
    }
}

// Scatter tile blockIdx.x to its digits' places: offsets[d * n_tiles + t] is
// where tile t's first element of digit d goes.  Every thread runs every
// round (no early exit), so the ballots see a full wavefront; lanes past the
// end take part as invalid.
__global__ __launch_bounds__(256) void sort_scatter_kernel(const uint64_t *keys_in, const uint32_t *idx_in,
                                                           uint64_t count, uint32_t shift, uint32_t n_tiles,
                                                           const uint32_t *offsets, uint64_t *keys_out,
                                                           uint32_t *idx_out)
{
    __shared__ uint32_t tile_off[256];   // global place of this tile's next element, per digit
    __shared__ uint32_t wave_cnt[4][256];
    __shared__ uint32_t wave_off[4][256];
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    tile_off[t] = offsets[(uint64_t)t * n_tiles + blockIdx.x];
    for (uint32_t w = 0; w < 4; w++)
        wave_cnt[w][t] = 0;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64u - lane));
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (uint32_t r = 0; r < kSortItems; r++) {
        const uint64_t i = base + (uint64_t)r * kSortThreads + t;
        const bool valid = i < count;
        const uint64_t key = valid ? keys_in[i] : 0ull;
        const uint32_t id = valid ? idx_in[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t same = __ballot(valid);
        for (uint32_t b = 0; b < 8; b++) {
            const uint64_t on = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? on : ~on;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        // the lowest valid lane of each digit group records the group's size
        if (valid && rank == 0)
            wave_cnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        {
            uint32_t run = tile_off[t];
            for (uint32_t w = 0; w < 4; w++) {
                wave_off[w][t] = run;
                run += wave_cnt[w][t];
                wave_cnt[w][t] = 0;
            }
            tile_off[t] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = wave_off[wave][d] + rank;
            keys_out[dst] = key;
            idx_out[dst] = id;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void sort_unpack_kernel(const uint64_t *keys, const uint32_t *idx,
                                                          uint64_t count, int64_t vmin, int64_t *sorted,
                                                          uint64_t *index)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        if (sorted)
            sorted[i] = (int64_t)(keys[i] + (uint64_t)vmin);
        if (index)
            index[i] = idx[i];
    }
}

// ------------------------------------------------------------------ launchers

namespace {
unsigned blocks_for(uint64_t count, uint64_t cap)
{
    uint64_t b = (count + 255) / 256;
    if (b > cap)
        b = cap;
    return (unsigned)(b ? b : 1);
}
}  // namespace

int launch_sample_orders(uint32_t n, uint32_t set, uint64_t seed, uint64_t first,
                         const uint64_t *indices, uint64_t count, uint8_t *orders, uint8_t *positions,
                         void *stream)
{
    if (count == 0)
        return 0;
    hipLaunchKernelGGL(sample_orders_kernel, dim3(blocks_for(count, 1ull << 31)), dim3(256), 0,
                       (hipStream_t)stream, n, set, seed, first, indices, count, orders, positions);
    return (int)hipGetLastError();
}

int launch_radix_hist_f32(const float *src, uint64_t count, uint32_t shift, uint64_t mask,
                          uint64_t prefix, unsigned long long *bins, int grid_cap, void *stream)
{
    hipLaunchKernelGGL(radix_hist_kernel<float>, dim3(blocks_for(count, (uint64_t)grid_cap)), dim3(256),
                       0, (hipStream_t)stream, src, count, shift, mask, prefix, bins);
    return (int)hipGetLastError();
}

int launch_radix_hist_i64(const int64_t *src, uint64_t count, uint32_t shift, uint64_t mask,
                          uint64_t prefix, unsigned long long *bins, int grid_cap, void *stream)
{
    hipLaunchKernelGGL(radix_hist_kernel<int64_t>, dim3(blocks_for(count, (uint64_t)grid_cap)),
                       dim3(256), 0, (hipStream_t)stream, src, count, shift, mask, prefix, bins);
    return (int)hipGetLastError();
}

int launch_gather_f32(const float *src, uint64_t count, uint32_t kth_key, uint64_t *out, uint64_t cap,
                      unsigned long long *cursor, int grid_cap, void *stream)
{
    hipLaunchKernelGGL(gather_f32_kernel, dim3(blocks_for(count, (uint64_t)grid_cap)), dim3(256), 0,
                       (hipStream_t)stream, src, count, kth_key, out, cap, cursor);
    return (int)hipGetLastError();
}

int launch_bitonic_sort_u64(uint64_t *keys, uint64_t used, uint64_t n_pow2, void *stream)
{
    if (n_pow2 > used) {
        hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n_pow2 - used, 1ull << 31)), dim3(256), 0,
                           (hipStream_t)stream, keys, used, n_pow2, ~0ull);
        int e = (int)hipGetLastError();
        if (e)
            return e;
    }
    for (uint64_t k = 2; k <= n_pow2; k <<= 1)
        for (uint64_t j = k >> 1; j > 0; j >>= 1) {
            hipLaunchKernelGGL(bitonic_stage_kernel, dim3(blocks_for(n_pow2, 1ull << 31)), dim3(256), 0,
                               (hipStream_t)stream, keys, n_pow2, j, k);
            int e = (int)hipGetLastError();
            if (e)
                return e;
        }
    return 0;
}

int launch_minmax_i64(const int64_t *v, uint64_t count, unsigned long long *mm, int grid_cap, void *stream)
{
    hipLaunchKernelGGL(minmax_i64_kernel, dim3(blocks_for(count, (uint64_t)grid_cap)), dim3(256), 0,
                       (hipStream_t)stream, v, count, mm);
    return (int)hipGetLastError();
}

int launch_stats_i64(const int64_t *v, uint64_t count, const int64_t *ref, Partial *parts, uint32_t n_parts,
                     void *stats, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(stats_partial_kernel, dim3(n_parts), dim3(256), 0, st, v, count, ref, parts);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(256), 0, st, parts, n_parts,
                       reinterpret_cast<Partial *>(stats));
    return (int)hipGetLastError();
}

uint64_t sort_tiles(uint64_t count) { return (count + kSortTile - 1) / kSortTile; }

int launch_sort_i64(const int64_t *v, uint64_t count, int64_t vmin, uint32_t passes, uint64_t *keys_a,
                    uint32_t *idx_a, uint64_t *keys_b, uint32_t *idx_b, uint32_t *counts, int64_t *sorted,
                    uint64_t *index, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const unsigned g = blocks_for(count, 1ull << 31);
    hipLaunchKernelGGL(sort_init_kernel, dim3(g), dim3(256), 0, st, v, count, vmin, keys_a, idx_a);
    int e = (int)hipGetLastError();
    if (e)
        return e;
    const uint32_t tiles = (uint32_t)sort_tiles(count);
    for (uint32_t p = 0; p < passes; p++) {
        const uint32_t shift = 8u * p;
        hipLaunchKernelGGL(sort_count_kernel, dim3(tiles), dim3(256), 0, st, keys_a, count, shift, tiles, counts);
        if ((e = (int)hipGetLastError()))
            return e;
        hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(1024), 0, st, counts, (uint64_t)tiles * 256u);
        if ((e = (int)hipGetLastError()))
            return e;
        hipLaunchKernelGGL(sort_scatter_kernel, dim3(tiles), dim3(256), 0, st, keys_a, idx_a, count, shift,
                           tiles, counts, keys_b, idx_b);
        if ((e = (int)hipGetLastError()))
            return e;
        uint64_t *tk = keys_a;
        keys_a = keys_b;
        keys_b = tk;
        uint32_t *ti = idx_a;
        idx_a = idx_b;
        idx_b = ti;
    }
    hipLaunchKernelGGL(sort_unpack_kernel, dim3(g), dim3(256), 0, st, keys_a, idx_a, count, vmin, sorted, index);
    return (int)hipGetLastError();
}

int launch_unpack_topk(const uint64_t *keys, uint32_t k, int64_t *idx, float *val, void *stream)
{
    if (k == 0)
        return 0;
    hipLaunchKernelGGL(unpack_topk_kernel, dim3((k + 255) / 256), dim3(256), 0, (hipStream_t)stream, keys,
                       k, idx, val);
    return (int)hipGetLastError();
}

}  // namespace ko
