// gfx950 kernels of libko: exact makespans of kernel launch orders.
//
// Model (Section 2 and Table 1 of Li, Narayana & El-Ghazawi 2015; the
// readings are those stated in include/ko.h): blocks of all kernels form one
// stream in launch order; the front block goes to the first CU at or after a
// cyclic pointer that has room in registers, LDS, waves and block slots, the
// pointer moves past it, and nothing behind a front block that fits nowhere
// is placed; blocks hold their resources for a fixed duration; all blocks
// ending at a cycle release before placement resumes.
//
// Mapping.  One wavefront evaluates one launch order at a time.  Lane l holds
// the free resources of CUs l, l+64, l+128, l+192 (S slots per lane).  Instead
// of placing one block per step, a "bulk step" places every block that the
// front kernel gets at the current cycle:
//   cap[c] = how many more blocks of kernel k fit on CU c
//          = min over resources of floor(free / use)
// A cyclic sweep from the pointer places one block on each CU with cap >= 1,
// then (second pass) one on each CU with cap >= 2, and so on, because a CU
// that cannot take a block at some point of the sweep cannot take one later in
// the same cycle.  So q blocks land as: min(cap[c], r-1) blocks on every CU,
// plus one more on the first (q - A_{r-1}) CUs of {cap >= r} in pointer order,
// where A_r = sum_c min(cap[c], r) and r is the first pass with A_r >= q.
// The pointer ends just past the last CU that received a block.  The result is
// identical to placing the q blocks one at a time.
//
// The blocks one bulk step places form a "group": they share the kernel and
// the finish cycle.  Per group the wave keeps one packed byte count per CU in
// an LDS ring (one dword per lane per slot) and, in lane g of two VGPRs, the
// cycles left until group g ends and its kernel.  Each event releases at least
// one group, and creates at most one group for the kernel already at the
// front plus one per kernel started at that event, so at most n groups are
// ever alive: the ring never overflows.
//
// Once every block is placed the makespan is the current cycle plus the
// longest remaining group; the drain is not simulated.

#include <hip/hip_runtime.h>

#include "ko_device.h"
#include "ko_orders.h"

namespace ko {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t read_lane(uint32_t v, uint32_t lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Sets status bits from a wave without a lane-dependent branch: every lane
// issues the atomic, only lane 0 with a nonzero operand.  Code between wave
// collectives (ballot, readlane, shuffles) stays free of lane-0-only branches,
// whose reconvergence point the compiler does not guarantee.
__device__ __forceinline__ void flag_status(uint32_t *status, uint32_t bits)
{
    atomicOr(status, lane_id() == 0 ? bits : 0u);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v)
{
    for (int o = 32; o >= 1; o >>= 1)
        v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
    for (int o = 32; o >= 1; o >>= 1)
        v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// floor(fr / u), clamped to at most `clamp` (<= 255).  The quotient estimate
// uses a float reciprocal rounded up by 3 ulps, which makes the truncated
// product never less than the true quotient and at most one more when the
// quotient is below 2^18 (fr < 2^24); one multiply-compare removes the excess.
// When the true quotient is larger than the clamp, the clamp is returned.
__device__ __forceinline__ uint32_t div_clamp(uint32_t fr, uint32_t u, float inv, uint32_t clamp)
{
    uint32_t q = (uint32_t)((float)fr * inv);
    q = min(q, clamp);
    return q - ((__umul24(q, u) > fr) ? 1u : 0u);
}

// Lexicographic rank -> permutation, lane j holding position j.  Digit j of
// the factorial number system is floor(rank / (n-1-j)!) mod (n-j); position j
// takes the digit-th smallest kernel index not used by positions < j.
__device__ uint32_t unrank_lanes(uint64_t rank, uint32_t n)
{
    const uint32_t lane = lane_id();
    uint32_t digit = 0;
    if (lane < n) {
        uint64_t f = kFactorial[n - 1 - lane];
        digit = (uint32_t)((rank / f) % (uint64_t)(n - lane));
    }
    uint32_t avail = (n >= 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
    uint32_t perm = 0xFFu;
    for (uint32_t j = 0; j < n; j++) {
        uint32_t d = read_lane(digit, j);
        uint64_t mem = ballot(lane < 32 && ((avail >> lane) & 1u));
        uint64_t hit = ballot(((mem >> lane) & 1ull) && lanes_below(mem) == d);
        // a digit is always below the count of unused indices; the guard keeps
        // the result a valid kernel index regardless
        uint32_t v = hit ? (uint32_t)__builtin_ctzll(hit) : 0u;
        perm = (lane == j) ? v : perm;
        avail &= ~(1u << v);
    }
    return perm;
}

// Next permutation in lexicographic order (lane j holds position j).  The
// caller never steps past the last permutation.
__device__ uint32_t next_perm_lanes(uint32_t perm, uint32_t n)
{
    const uint32_t lane = lane_id();
    uint32_t nxt = (uint32_t)__shfl_down((int)perm, 1);
    uint64_t asc = ballot(lane + 1 < n && perm < nxt);
    if (asc == 0)
        return perm;
    uint32_t i = 63u - (uint32_t)__builtin_clzll(asc);
    uint32_t pi = read_lane(perm, i);
    uint64_t big = ballot(lane > i && lane < n && perm > pi);
    uint32_t l = 63u - (uint32_t)__builtin_clzll(big);
    uint32_t pl = read_lane(perm, l);
    perm = (lane == i) ? pl : ((lane == l) ? pi : perm);
    uint32_t src = (lane > i && lane < n) ? (i + n - lane) : lane;
    return (uint32_t)__shfl((int)perm, (int)src);
}

// Makespan of the order held in `perm` (lane j = kernel at position j).
// Returns -1 (and sets a status bit) only on an internal inconsistency.
template <int S>
__device__ int64_t simulate_order(const SimArgs &a, const KernelRec *__restrict__ kr, uint32_t n,
                                  uint32_t perm, uint32_t *__restrict__ ring, uint32_t gslots)
{
    const uint32_t lane = lane_id();
    const uint32_t n_cu = a.n_cu;
    uint32_t fr_reg[S], fr_lds[S], fr_wave[S], fr_blk[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        fr_reg[s] = a.cap_reg;
        fr_lds[s] = a.cap_lds;
        fr_wave[s] = a.cap_wave;
        fr_blk[s] = (s * kWave + lane < n_cu) ? a.cap_blk : 0u;
    }
    uint32_t rel = 0xFFFFFFFFu;  // lane g: cycles until group g ends (all ones = free slot)
    uint32_t gk = 0;             // lane g: kernel of group g
    uint64_t t = 0;
    uint32_t ptr = 0, pos = 0;
    uint32_t k = uniform(read_lane(perm, 0));
    uint32_t rem = kr[k].tblk;

    for (;;) {
        // ---- placement at cycle t: one bulk step per kernel reached ----
        while (pos < n) {
            const uint32_t u_reg = kr[k].u_reg, u_lds = kr[k].u_lds, u_wave = kr[k].u_wave;
            const float i_reg = kr[k].inv_reg, i_lds = kr[k].inv_lds, i_wave = kr[k].inv_wave;
            uint32_t cap[S];
#pragma unroll
            for (int s = 0; s < S; s++) {
                uint32_t c = fr_blk[s];
                c = div_clamp(fr_wave[s], u_wave, i_wave, c);
                c = div_clamp(fr_reg[s], u_reg, i_reg, c);
                if (u_lds)
                    c = div_clamp(fr_lds[s], u_lds, i_lds, c);
                cap[s] = c;
            }
            // passes of the sweep: M_r CUs take an r-th block
            uint32_t A = 0, Mprev = 0, r = 0, extra = 0, q = 0;
            for (;;) {
                r++;
                uint32_t M = 0;
#pragma unroll
                for (int s = 0; s < S; s++)
                    M += (uint32_t)__popcll(ballot(cap[s] >= r));
                if (M == 0) {  // every CU is full for this kernel
                    r--;
                    extra = Mprev;
                    q = A;
                    break;
                }
                if (A + M >= rem) {
                    extra = rem - A;
                    q = rem;
                    break;
                }
                A += M;
                Mprev = M;
            }
            if (q == 0)
                break;  // the front block fits nowhere
            uint64_t mask[S];
            uint32_t pc[S], mtot = 0;
#pragma unroll
            for (int s = 0; s < S; s++) {
                mask[s] = ballot(cap[s] >= r);
                pc[s] = (uint32_t)__popcll(mask[s]);
                mtot += pc[s];
            }
            // members of pass r before the pointer (CU index order)
            const uint32_t ps = ptr >> 6, pl = ptr & 63u;
            uint32_t pptr = 0;
#pragma unroll
            for (int s = 0; s < S; s++) {
                if ((uint32_t)s < ps)
                    pptr += pc[s];
                else if ((uint32_t)s == ps)
                    pptr += (uint32_t)__popcll(mask[s] & ((1ull << pl) - 1ull));
            }
            uint32_t cnt[S];
            uint32_t base = 0, last = 0;
#pragma unroll
            for (int s = 0; s < S; s++) {
                const uint32_t c = s * kWave + lane;
                const bool mem = cap[s] >= r;
                // position of this CU among the pass-r members, counted from the pointer
                const uint32_t rank = base + lanes_below(mask[s]) - pptr + (c < ptr ? mtot : 0u);
                const bool take = mem && rank < extra;
                cnt[s] = min(cap[s], r - 1u) + (take ? 1u : 0u);
                const uint64_t lm = ballot(mem && rank == extra - 1u);
                if (lm)
                    last = s * kWave + (uint32_t)__builtin_ctzll(lm);
                base += pc[s];
            }
            ptr = (last + 1u == n_cu) ? 0u : last + 1u;
            uint32_t packed = 0;
#pragma unroll
            for (int s = 0; s < S; s++) {
                fr_reg[s] -= __umul24(cnt[s], u_reg);
                fr_lds[s] -= __umul24(cnt[s], u_lds);
                fr_wave[s] -= __umul24(cnt[s], u_wave);
                fr_blk[s] -= cnt[s];
                packed |= cnt[s] << (8 * s);
            }
            const uint64_t free_slots = ballot(lane < gslots && rel == 0xFFFFFFFFu);
            if (free_slots == 0) {
                flag_status(a.status, kStatusGroupOverflow);
                return -1;
            }
            const uint32_t g = (uint32_t)__builtin_ctzll(free_slots);
            ring[g * kWave + lane] = packed;
            const uint32_t dur = kr[k].dur;
            rel = (lane == g) ? dur : rel;
            gk = (lane == g) ? k : gk;
            rem -= q;
            if (rem)
                break;  // the rest of this kernel waits for a release
            pos++;
            if (pos < n) {
                k = uniform(read_lane(perm, pos));
                rem = kr[k].tblk;
            }
        }
        const bool live = rel != 0xFFFFFFFFu;
        if (pos >= n) {
            // every block is placed: the makespan is set by the longest group left
            return (int64_t)(t + uniform(wave_max(live ? rel : 0u)));
        }
        // ---- next event: the earliest group end ----
        const uint32_t dt = uniform(wave_min(rel));
        if (dt == 0xFFFFFFFFu) {  // nothing running yet the front block does not fit
            flag_status(a.status, kStatusGroupOverflow);
            return -1;
        }
        t += dt;
        rel = live ? rel - dt : rel;
        uint64_t ending = ballot(live && rel == 0u);
        rel = (live && rel == 0u) ? 0xFFFFFFFFu : rel;
        while (ending) {
            const uint32_t g = (uint32_t)__builtin_ctzll(ending);
            ending &= ending - 1ull;
            const uint32_t kg = uniform(read_lane(gk, g));
            const uint32_t u_reg = kr[kg].u_reg, u_lds = kr[kg].u_lds, u_wave = kr[kg].u_wave;
            const uint32_t packed = ring[g * kWave + lane];
#pragma unroll
            for (int s = 0; s < S; s++) {
                const uint32_t c = (packed >> (8 * s)) & 0xFFu;
                fr_reg[s] += __umul24(c, u_reg);
                fr_lds[s] += __umul24(c, u_lds);
                fr_wave[s] += __umul24(c, u_wave);
                fr_blk[s] += c;
            }
        }
    }
}

// Persistent kernel: each wavefront repeatedly takes a work item (a chunk of
// consecutive orders of one set), evaluates its orders one by one, writes the
// makespans coalesced (64 per store) and one Partial per item.
template <int S>
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
            const int64_t m = simulate_order<S>(a, kr, n, perm, ring, gslots);
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

// One wavefront per set: combine the set's Partials (ties -> smaller index).
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    const uint32_t lane = lane_id();
    // the wave index is uniform across the wave; saying so keeps the early
    // return a scalar branch, so the shuffles below run with all lanes active
    const int set = (int)(blockIdx.x * 4 + uniform(threadIdx.x >> 6));
    if (set >= a.n_sets)
        return;
    const SetRec st = a.sets[set];
    const uint64_t items = (st.n_orders + a.chunk - 1) / a.chunk;
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    uint64_t amn = 0, amx = 0, nl = 0, ne = 0, ng = 0, cnt = 0;
    for (uint64_t i = lane; i < items; i += kWave) {
        const Partial p = a.partials[st.item_base + i];
        if (p.min_ms < mn || (p.min_ms == mn && p.argmin < amn)) {
            mn = p.min_ms;
            amn = p.argmin;
        }
        if (p.max_ms > mx || (p.max_ms == mx && p.argmax < amx)) {
            mx = p.max_ms;
            amx = p.argmax;
        }
        nl += p.n_less;
        ne += p.n_equal;
        ng += p.n_greater;
        cnt += p.count;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const int64_t omn = __shfl_xor(mn, o), omx = __shfl_xor(mx, o);
        const uint64_t oamn = __shfl_xor(amn, o), oamx = __shfl_xor(amx, o);
        if (omn < mn || (omn == mn && oamn < amn)) {
            mn = omn;
            amn = oamn;
        }
        if (omx > mx || (omx == mx && oamx < amx)) {
            mx = omx;
            amx = oamx;
        }
        nl += __shfl_xor(nl, o);
        ne += __shfl_xor(ne, o);
        ng += __shfl_xor(ng, o);
        cnt += __shfl_xor(cnt, o);
    }
    if (lane == 0) {
        Partial *out = reinterpret_cast<Partial *>(a.stats) + set;
        Partial p;
        p.min_ms = mn;
        p.max_ms = mx;
        p.argmin = (cnt == 0) ? 0 : amn;
        p.argmax = (cnt == 0) ? 0 : amx;
        p.n_less = nl;
        p.n_equal = ne;
        p.n_greater = ng;
        p.count = cnt;
        *out = p;
    }
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

int launch_simulate(const SimArgs &a, int slots_per_lane, uint32_t group_slots, int grid,
                    void *stream)
{
    const size_t lds = (size_t)4 * group_slots * kWave * sizeof(uint32_t);
    hipStream_t st = (hipStream_t)stream;
    switch (slots_per_lane) {
    case 1:
        hipLaunchKernelGGL(simulate_kernel<1>, dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    case 2:
        hipLaunchKernelGGL(simulate_kernel<2>, dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    case 4:
        hipLaunchKernelGGL(simulate_kernel<4>, dim3(grid), dim3(256), lds, st, a, group_slots);
        break;
    default:
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_reduce(const ReduceArgs &a, void *stream)
{
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
