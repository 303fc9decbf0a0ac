// gfx950 kernels of libko's wave engine: the persistent simulate kernel (one
// wavefront per launch order; the per-order routine is in ko_wave.h), the
// per-set reduction and the histogram.

#include <hip/hip_runtime.h>

#include "ko_wave.h"

namespace ko {

// Persistent kernel: each wavefront repeatedly takes a work item (a chunk of
// consecutive orders of one set), evaluates its orders one by one, writes the
// makespans coalesced (64 per store) and one Partial per item.
// CONT: resident blocks share the chip's memory throughput (ko_wave.h).
template <int S, bool CONT>
__global__ __launch_bounds__(256) void simulate_kernel(SimArgs a, uint32_t gslots)
{
    extern __shared__ uint32_t lds_ring[];
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x >> 6;
    uint32_t *ring = lds_ring + wid * gslots * kWave;

    for (;;) {
        // All lanes execute the fetch (lane 0 adds one, the rest zero) and
        // lane 0's old value is broadcast.  No lane-dependent branch may sit
        // at the top of this loop: the lane-0 branch that stores the Partial
        // at the bottom can then be threaded around it, and lanes 1..63 would
        // re-enter the loop without lane 0 (and without a fetched item).
        const uint64_t raw = uniform64(atomicAdd(a.item_counter, lane == 0 ? 1ull : 0ull));
        const uint64_t limit = a.item_list ? (uint64_t)*a.item_list_count : a.n_items;
        if (raw >= limit)
            break;
        const uint64_t item = a.item_list ? (uint64_t)a.item_list[raw] : raw;
        // the set owning this item: the last set whose first item <= item
        int lo = 0, hi = a.n_sets - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.sets[mid].item_base <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int set = lo;
        const uint32_t n = a.sets[set].n;
        const KernelRec *kr = a.krec + a.sets[set].kbase;
        const uint32_t *sh = CONT ? a.share + a.sets[set].kbase : nullptr;
        const uint64_t first = (item - a.sets[set].item_base) * a.chunk;
        const uint64_t n_orders = a.sets[set].n_orders;
        const uint64_t count = min(a.chunk, n_orders - first);
        const uint64_t out_base = a.sets[set].out_base + first;
        const bool ranked = a.mode == kModeAll || a.mode == kModeRange;
        const uint64_t index0 = ranked ? a.sets[set].rank_lo + first : first;
        const bool has_ref = a.ref != nullptr;
        const int64_t ref = has_ref ? a.ref[set] : 0;

        int64_t mn = INT64_MAX, mx = INT64_MIN;
        uint64_t amn = 0, amx = 0, n_less = 0, n_eq = 0, n_gt = 0;
        uint32_t out_lo = 0, out_hi = 0;
        uint32_t perm = 0;
        if (ranked)
            perm = unrank_lanes(index0, n);

        for (uint64_t i = 0; i < count; i++) {
            if (a.mode == kModeExplicit) {
                const uint8_t *o = a.orders + a.sets[set].list_base + (first + i) * n;
                perm = (lane < n) ? (uint32_t)o[lane] : 0xFFu;
                // must be a permutation of 0..n-1
                const uint64_t seen_any = ballot(lane < n && perm >= n);
                uint32_t seen = 0;
                for (uint32_t j = 0; j < n; j++)
                    seen |= 1u << (read_lane(perm, j) & 31u);
                const uint32_t want = (n >= 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
                if (seen_any || seen != want) {
                    flag_status(a.status, kStatusBadOrder);
                    perm = unrank_lanes(0, n);
                }
            } else if (a.mode == kModeSampled) {
                perm = unrank_lanes(sampled_rank(a.seed, (uint32_t)set, first + i, n), n);
            }
            const int64_t m = simulate_order<S, CONT>(a, kr, sh, n, perm, ring, gslots);
            const uint64_t idx = index0 + i;
            if (m < mn) {
                mn = m;
                amn = idx;
            }
            if (m > mx) {
                mx = m;
                amx = idx;
            }
            if (has_ref) {
                n_less += (m < ref) ? 1u : 0u;
                n_eq += (m == ref) ? 1u : 0u;
                n_gt += (m > ref) ? 1u : 0u;
            }
            const uint32_t slot = (uint32_t)(i & 63u);
            out_lo = (lane == slot) ? (uint32_t)m : out_lo;
            out_hi = (lane == slot) ? (uint32_t)((uint64_t)m >> 32) : out_hi;
            if (a.makespans && (slot == 63u || i + 1 == count)) {
                if (lane <= slot) {
                    const uint64_t v = ((uint64_t)out_hi << 32) | out_lo;
                    a.makespans[out_base + (i & ~63ull) + lane] = (int64_t)v;
                }
            }
            if (ranked && i + 1 < count)
                perm = next_perm_lanes(perm, n);
        }
        if (lane == 0) {
            Partial p;
            p.min_ms = mn;
            p.max_ms = mx;
            p.argmin = amn;
            p.argmax = amx;
            p.n_less = n_less;
            p.n_equal = n_eq;
            p.n_greater = n_gt;
            p.count = count;
            a.partials[item] = p;
        }
    }
}

// Orders the lane kernel spilled: one wavefront per order, taken from an
// atomic cursor over the records; records of work items that are re-run whole
// are skipped.  Writes the makespan into the record and the makespan array.
template <int S, bool CONT>
__global__ __launch_bounds__(256) void spill_kernel(SimArgs a, uint32_t gslots)
{
    extern __shared__ uint32_t lds_ring[];
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x >> 6;
    uint32_t *ring = lds_ring + wid * gslots * kWave;
    for (;;) {
        const uint64_t r = uniform64(atomicAdd(a.item_counter, lane == 0 ? 1ull : 0ull));
        const uint64_t limit = min((uint64_t)*a.spill_count, a.spill_cap);
        if (r >= limit)
            break;
        const SpillRec rec = a.spill[r];
        if ((a.handed_bits[rec.item >> 5] >> (rec.item & 31u)) & 1u)
            continue;
        const SetRec st = a.sets[rec.set];
        const uint32_t n = st.n;
        uint32_t perm;
        if (a.mode == kModeAll || a.mode == kModeRange) {
            perm = unrank_lanes(st.rank_lo + rec.sample, n);
        } else if (a.mode == kModeSampled) {
            perm = unrank_lanes(sampled_rank(a.seed, rec.set, rec.sample, n), n);
        } else {
            const uint8_t *o = a.orders + st.list_base + rec.sample * n;
            perm = (lane < n) ? (uint32_t)o[lane] : 0xFFu;
            const uint64_t bad = ballot(lane < n && perm >= n);
            uint32_t seen = 0;
            for (uint32_t j = 0; j < n; j++)
                seen |= 1u << (read_lane(perm, j) & 31u);
            if (bad || seen != (1u << n) - 1u)
                perm = unrank_lanes(0, n);  // the lane kernel raised the status bit
        }
        const uint32_t *sh = CONT ? a.share + st.kbase : nullptr;
        const int64_t m = simulate_order<S, CONT>(a, a.krec + st.kbase, sh, n, perm, ring, gslots);
        // every lane stores the same values
        a.spill[r].makespan = m;
        if (a.makespans)
            a.makespans[rec.pos] = m;
    }
}

// A set's statistics while they are folded: extremes with their indices
// (ties -> the smaller index) and counts.  Folding is associative and
// commutative, so any reduction tree gives the same result.
struct Fold {
    int64_t mn, mx;
    uint64_t amn, amx, nl, ne, ng, cnt;
};

__device__ inline Fold fold_empty()
{
    return Fold{INT64_MAX, INT64_MIN, 0, 0, 0, 0, 0, 0};
}

__device__ inline void fold_extremes(Fold &f, int64_t mn, uint64_t amn, int64_t mx, uint64_t amx)
{
    if (mn < f.mn || (mn == f.mn && amn < f.amn)) {
        f.mn = mn;
        f.amn = amn;
    }
    if (mx > f.mx || (mx == f.mx && amx < f.amx)) {
        f.mx = mx;
        f.amx = amx;
    }
}

__device__ inline void fold_join(Fold &f, const Fold &o)
{
    fold_extremes(f, o.mn, o.amn, o.mx, o.amx);
    f.nl += o.nl;
    f.ne += o.ne;
    f.ng += o.ng;
    f.cnt += o.cnt;
}

// This thread's share of a set: item partials i = first, first + stride, ...
// and spilled orders likewise.
__device__ inline Fold fold_set(const ReduceArgs &a, int set, uint32_t first, uint32_t stride)
{
    const SetRec st = a.sets[set];
    const uint64_t items = (st.n_orders + a.chunk - 1) / a.chunk;
    Fold f = fold_empty();
    for (uint64_t i = first; i < items; i += stride) {
        const Partial p = a.partials[st.item_base + i];
        fold_extremes(f, p.min_ms, p.argmin, p.max_ms, p.argmax);
        f.nl += p.n_less;
        f.ne += p.n_equal;
        f.ng += p.n_greater;
        f.cnt += p.count;
    }
    if (a.spill) {
        const bool ranked = a.mode == kModeAll || a.mode == kModeRange;
        const int64_t ref = a.ref ? a.ref[set] : 0;
        const uint64_t n_spill = min((uint64_t)*a.spill_count, a.spill_cap);
        for (uint64_t r = first; r < n_spill; r += stride) {
            const SpillRec rec = a.spill[r];
            if (rec.set != (uint32_t)set || ((a.handed_bits[rec.item >> 5] >> (rec.item & 31u)) & 1u))
                continue;
            const int64_t m = rec.makespan;
            const uint64_t idx = ranked ? st.rank_lo + rec.sample : rec.sample;
            fold_extremes(f, m, idx, m, idx);
            if (a.ref) {
                f.nl += (m < ref) ? 1u : 0u;
                f.ne += (m == ref) ? 1u : 0u;
                f.ng += (m > ref) ? 1u : 0u;
            }
        }
    }
    return f;
}

// Fold across the wave (xor butterfly: every lane ends with the wave's fold).
__device__ inline Fold fold_wave(Fold f)
{
    for (int o = 32; o >= 1; o >>= 1) {
        Fold g;
        g.mn = __shfl_xor(f.mn, o);
        g.mx = __shfl_xor(f.mx, o);
        g.amn = __shfl_xor(f.amn, o);
        g.amx = __shfl_xor(f.amx, o);
        g.nl = __shfl_xor(f.nl, o);
        g.ne = __shfl_xor(f.ne, o);
        g.ng = __shfl_xor(f.ng, o);
        g.cnt = __shfl_xor(f.cnt, o);
        fold_join(f, g);
    }
    return f;
}

__device__ inline void fold_store(const ReduceArgs &a, int set, const Fold &f)
{
    Partial *out = reinterpret_cast<Partial *>(a.stats) + set;
    Partial p;
    p.min_ms = f.mn;
    p.max_ms = f.mx;
    p.argmin = (f.cnt == 0) ? 0 : f.amn;
    p.argmax = (f.cnt == 0) ? 0 : f.amx;
    p.n_less = f.nl;
    p.n_equal = f.ne;
    p.n_greater = f.ng;
    p.count = f.cnt;
    *out = p;
}

// One wavefront per set: combine the set's Partials (ties -> smaller index)
// and the set's spilled orders.
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    const uint32_t lane = lane_id();
    // the wave index is uniform across the wave; saying so keeps the early
    // return a scalar branch, so the shuffles below run with all lanes active
    const int set = (int)(blockIdx.x * 4 + uniform(threadIdx.x >> 6));
    if (set >= a.n_sets)
        return;
    const Fold f = fold_wave(fold_set(a, set, lane, kWave));
    if (lane == 0)
        fold_store(a, set, f);
}

// One workgroup of kWideWaves waves per set, for launches with few sets (a
// set of all n! orders has tens of thousands of work items): each wave folds
// its stride of the items and spills, the first wave folds the waves' results.
constexpr int kWideWaves = 16;

__global__ __launch_bounds__(kWideWaves * kWave) void reduce_wide_kernel(ReduceArgs a)
{
    __shared__ Fold part[kWideWaves];
    const uint32_t lane = lane_id();
    const int wave = (int)uniform(threadIdx.x >> 6);
    const int set = (int)blockIdx.x;
    Fold f = fold_wave(fold_set(a, set, threadIdx.x, kWideWaves * kWave));
    if (lane == 0)
        part[wave] = f;
    __syncthreads();
    if (wave != 0)
        return;
    f = lane < (uint32_t)kWideWaves ? part[lane] : fold_empty();
    f = fold_wave(f);
    if (lane == 0)
        fold_store(a, set, f);
}

// Histogram of each set's makespans: LDS-private bins per workgroup when they
// fit (n_bins <= 4096), flushed with one atomic per nonzero bin.
__global__ __launch_bounds__(256) void hist_kernel(HistArgs a)
{
    __shared__ uint32_t bins[4096];
    const uint64_t blk = blockIdx.x;
    int lo = 0, hi = a.n_sets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.block_base[mid] <= blk)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int set = lo;
    const SetRec st = a.sets[set];
    const Partial stats = reinterpret_cast<const Partial *>(a.stats)[set];
    const uint64_t first = (blk - a.block_base[set]) * a.per_block;
    const uint64_t end = min(st.n_orders, first + a.per_block);
    const uint64_t width = (uint64_t)(stats.max_ms - stats.min_ms) + 1ull;
    const bool local = a.n_bins <= 4096;
    uint64_t *hist = a.hist + (uint64_t)set * (uint64_t)a.n_bins;
    if (local) {
        for (int b = threadIdx.x; b < a.n_bins; b += blockDim.x)
            bins[b] = 0;
        __syncthreads();
    }
    for (uint64_t i = first + threadIdx.x; i < end; i += blockDim.x) {
        const uint64_t d = (uint64_t)(a.makespans[st.out_base + i] - stats.min_ms);
        const uint32_t b = (uint32_t)(d * (uint64_t)a.n_bins / width);
        if (local)
            atomicAdd(&bins[b], 1u);
        else
            atomicAdd((unsigned long long *)&hist[b], 1ull);
    }
    if (local) {
        __syncthreads();
        for (int b = threadIdx.x; b < a.n_bins; b += blockDim.x)
            if (bins[b])
                atomicAdd((unsigned long long *)&hist[b], (unsigned long long)bins[b]);
    }
}

__global__ void zero_kernel(uint64_t *p, uint64_t count)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <bool CONT>
int launch_simulate_t(const SimArgs &a, int slots_per_lane, uint32_t group_slots, int grid, void *stream)
{
    const size_t lds = (size_t)4 * group_slots * kWave * sizeof(uint32_t);
    hipStream_t st = (hipStream_t)stream;
    switch (slots_per_lane) {
    case 1:
        hipLaunchKernelGGL((simulate_kernel<1, CONT>), dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    case 2:
        hipLaunchKernelGGL((simulate_kernel<2, CONT>), dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    case 4:
        hipLaunchKernelGGL((simulate_kernel<4, CONT>), dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    default:
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_simulate(const SimArgs &a, int slots_per_lane, uint32_t group_slots, int grid,
                    void *stream)
{
    if (a.share)
        return launch_simulate_t<true>(a, slots_per_lane, group_slots, grid, stream);
    return launch_simulate_t<false>(a, slots_per_lane, group_slots, grid, stream);
}

template <bool CONT>
int launch_spill_t(const SimArgs &a, int slots_per_lane, uint32_t group_slots, int grid, void *stream)
{
    const size_t lds = (size_t)4 * group_slots * kWave * sizeof(uint32_t);
    hipStream_t st = (hipStream_t)stream;
    switch (slots_per_lane) {
    case 1:
        hipLaunchKernelGGL((spill_kernel<1, CONT>), dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    case 2:
        hipLaunchKernelGGL((spill_kernel<2, CONT>), dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    case 4:
        hipLaunchKernelGGL((spill_kernel<4, CONT>), dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    default:
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_spill(const SimArgs &a, int slots_per_lane, uint32_t group_slots, int grid, void *stream)
{
    if (a.share)
        return launch_spill_t<true>(a, slots_per_lane, group_slots, grid, stream);
    return launch_spill_t<false>(a, slots_per_lane, group_slots, grid, stream);
}

// fewer sets than this: a workgroup of kWideWaves waves per set
constexpr int kWideSets = 256;

int launch_reduce(const ReduceArgs &a, void *stream)
{
    if (a.n_sets <= 0)
        return 0;
    if (a.n_sets < kWideSets) {
        hipLaunchKernelGGL(reduce_wide_kernel, dim3((uint32_t)a.n_sets), dim3(kWideWaves * kWave), 0,
                           (hipStream_t)stream, a);
        return (int)hipGetLastError();
    }
    const int grid = (a.n_sets + 3) / 4;
    hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_hist(const HistArgs &a, uint64_t n_blocks, void *stream)
{
    if (n_blocks == 0)
        return 0;
    hipLaunchKernelGGL(hist_kernel, dim3((uint32_t)n_blocks), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_zero_u64(uint64_t *p, uint64_t count, void *stream)
{
    if (count == 0)
        return 0;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, p,
                       count);
    return (int)hipGetLastError();
}

int device_cu_count(int *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return (int)e;
    return (int)hipDeviceGetAttribute(out, hipDeviceAttributeMultiprocessorCount, dev);
}

}  // namespace ko
