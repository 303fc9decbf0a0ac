// gfx950 kernel of libko: one launch order per lane, CU states as runs.
//
// Same model as simulate_kernel (Section 2 and Table 1; the readings are
// those stated in include/ko.h) and the same bulk step: at a cycle, the front
// kernel k places every block it gets at once, min(cap[c], r-1) blocks on
// every CU plus one more on the first `extra` CUs of {cap >= r} walking from
// the cyclic pointer, where cap[c] = min over resources of floor(free / use).
//
// What differs is the representation.  Along the CU index, the free resources
// of the CUs form a few runs of identical values: blocks land on contiguous
// stretches swept from the pointer, and CUs that hold the same blocks have the
// same free resources.  Measured over the kernel sets this library is run on
// (n = 4..16, 256 CUs), an order rarely holds more runs than it has kernels.
// So each lane of a wave evaluates its own launch order, holding
//   * the runs in registers: A[j] = free registers << 9 | first CU of run j,
//     B[j] = free LDS << 14 | free waves << 7 | free block slots, and R runs
//     in CU order (the last run ends at N_CU);
//   * up to GC live block groups (the blocks of one bulk step share kernel
//     and finish cycle; at most n are ever alive, see ko_sim.hip): cycles left
//     and a bitmask of the group's entries;
//   * the entries in LDS, one dword per entry (first CU, end CU, blocks per
//     CU, kernel): the group's block counts over maximal stretches of CUs that
//     received the same count.
// A bulk step computes cap per run, the pass r and the cut CU from per-run
// sums, splits the runs at the pointer and just past the cut, subtracts the
// counts run by run and records the group's entries.  A release splits the
// runs at each entry's ends and adds the entry's blocks back over its stretch.
// After both, adjacent runs with equal resources are merged.  Every quantity
// is the one the per-CU kernel computes; only the storage is compressed.
//
// Capacities are fixed per instantiation (RC runs, GC groups, E entries).
// A lane gives up on an order that would exceed one and writes a spill record
// (set, item, order index, makespan slot); spill_kernel then evaluates the
// recorded orders with the wave engine, one wavefront per order, and
// reduce_kernel folds them into their sets' statistics.  Only if the record
// list is full is the whole work item listed and marked, and re-run by
// simulate_kernel, which rewrites its makespans and partial (its records are
// then ignored).  Results never depend on the capacities.
//
// Memory contention (CONT; Section 4, the model of ko_wave.h): a group keeps
// its progress left in units (64 bits) and its blocks' summed memory share;
// every resident block advances at the rate the resident shares allow, so an
// event is the first whole cycle at which a group has its progress, and the
// drain after the last placement is simulated event by event, since each
// release changes the rate.
//
// A lane that finishes an order takes the next one of the work item from a
// cursor in LDS, so the wave keeps all lanes busy until the item runs dry.
// Everything between taking the item and combining the lanes' statistics is
// per-lane code: no ballot, shuffle or readlane, so the compiler's handling of
// the lanes' diverging control flow cannot feed a wave operation with lanes
// switched off.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "ko_device.h"
#include "ko_orders.h"

namespace ko {
namespace {

constexpr uint32_t kFree = 0xFFFFFFFFu;
constexpr int kTab = 16;          // largest set of the lane kernels
constexpr int kTabWords = 11 * kTab;
constexpr int kEntBase = kTabWords + 64;  // the item's order cursor, then the entries

// LDS kernel table, struct of arrays (word offsets)
enum : int { kTUa = 0, kTUb = kTab, kTReg = 2 * kTab, kTLds = 3 * kTab, kTWave = 4 * kTab,
             kTIReg = 5 * kTab, kTILds = 6 * kTab, kTIWave = 7 * kTab, kTDur = 8 * kTab,
             kTBlk = 9 * kTab, kTSh = 10 * kTab };

__device__ __forceinline__ uint32_t lane_no() { return __lane_id(); }

__device__ __forceinline__ uint64_t wave_uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// floor(fr / u) clamped to `clamp`; the reciprocal is rounded up by 3 ulps on
// the host, so the truncated product is the quotient or one more (fr < 2^24).
__device__ __forceinline__ uint32_t quot_clamp(uint32_t fr, uint32_t u, float inv, uint32_t clamp)
{
    uint32_t q = (uint32_t)((float)fr * inv);
    q = min(q, clamp);
    return q - ((__umul24(q, u) > fr) ? 1u : 0u);
}

// floor(x / d) for x < 2^53 and 1 <= d < 2^53: the binary64 quotient is off by
// at most one, and one exact integer comparison each way corrects it.
__device__ __forceinline__ uint64_t div_u53(uint64_t x, uint64_t d)
{
    uint64_t q = (uint64_t)((double)x / (double)d);
    if (q * d > x)
        q--;
    else if (x - q * d >= d)
        q++;
    return q;
}

constexpr double fact_d(int k) { return k <= 1 ? 1.0 : k * fact_d(k - 1); }

// 1 / k! in binary64, k = 0..20 (each k! up to 20! is exact in binary64 up to
// 18!; the reciprocal only seeds the digit, which is then corrected exactly)
static __device__ const double kInvFactorial[21] = {
    1.0 / fact_d(0),  1.0 / fact_d(1),  1.0 / fact_d(2),  1.0 / fact_d(3),  1.0 / fact_d(4),
    1.0 / fact_d(5),  1.0 / fact_d(6),  1.0 / fact_d(7),  1.0 / fact_d(8),  1.0 / fact_d(9),
    1.0 / fact_d(10), 1.0 / fact_d(11), 1.0 / fact_d(12), 1.0 / fact_d(13), 1.0 / fact_d(14),
    1.0 / fact_d(15), 1.0 / fact_d(16), 1.0 / fact_d(17), 1.0 / fact_d(18), 1.0 / fact_d(19),
    1.0 / fact_d(20)};

// Lexicographic rank -> order packed as nibbles (position j in bits 4j..4j+3).
// Digit j is floor(rest / (n-1-j)!): estimated as rest x 1/(n-1-j)! in binary64
// (rest < 16! < 2^53, so the estimate is off by at most one) and corrected with
// one exact integer comparison.  No division, so nothing the compiler turns
// into a wave-wide value.
__device__ uint64_t unrank_nibbles(uint64_t rank, uint32_t n)
{
    uint64_t avail = 0xFEDCBA9876543210ull;  // unused kernel indices, ascending
    uint64_t perm = 0;
    for (uint32_t j = 0; j < n; j++) {
        const uint32_t k = n - 1u - j;
        const uint64_t f = kFactorial[k];
        uint64_t d = (uint64_t)((double)rank * kInvFactorial[k]);
        int64_t rest = (int64_t)rank - (int64_t)(d * f);
        if (rest < 0) {
            d--;
            rest += (int64_t)f;
        } else if (rest >= (int64_t)f) {
            d++;
            rest -= (int64_t)f;
        }
        rank = (uint64_t)rest;
        d = min(d, (uint64_t)k);  // holds for every rank below n!
        const uint32_t sh = 4u * (uint32_t)d;
        perm |= ((avail >> sh) & 15ull) << (4u * j);
        const uint64_t low = avail & ((1ull << sh) - 1ull);
        avail = low | (((avail >> sh) >> 4) << sh);
    }
    return perm;
}

__device__ __forceinline__ uint64_t identity_nibbles(uint32_t n)
{
    const uint64_t all = 0xFEDCBA9876543210ull;
    return n >= 16 ? all : (all & ((1ull << (4u * n)) - 1ull));
}

// Entry masks: 32 bits when a variant holds at most 32 entries per lane.
__device__ __forceinline__ uint32_t lowest_bit(uint32_t m) { return (uint32_t)__builtin_ctz(m); }
__device__ __forceinline__ uint32_t lowest_bit(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

template <int RC, int GC, typename Mask, bool CONT>
struct LaneSim {
    // group progress left: cycles, or (CONT) units of 1/65536 cycle at full rate
    using Rel = typename std::conditional<CONT, uint64_t, uint32_t>::type;
    static constexpr Rel kFreeRel = ~Rel(0);
    uint32_t A[RC], B[RC], cap[RC];
    uint32_t R;
    Rel rel[GC];
    Mask gm[GC];
    uint32_t gsh[CONT ? GC : 1];  // CONT: a group's summed memory share
    uint32_t ush;                 // CONT: summed share of every resident block
    Mask used;
    uint64_t t;
    uint32_t ptr, pos, k, rem;  // the front kernel's parameters are read from the LDS table
    bool ovf;

    __device__ __forceinline__ uint32_t end_of(int j, uint32_t n_cu) const
    {
        return (j + 1 < (int)R) ? (A[(j + 1) % RC] & 511u) : n_cu;
    }

    __device__ __forceinline__ void load_kernel(const uint32_t *tab, uint32_t kk)
    {
        k = kk;
        rem = tab[kTBlk + kk];
    }

    __device__ __forceinline__ void reset(const SimArgs &a)
    {
        A[0] = a.cap_reg << 9;
        B[0] = (a.cap_lds << 14) | (a.cap_wave << 7) | a.cap_blk;
#pragma unroll
        for (int j = 1; j < RC; j++) {
            A[j] = 0;
            B[j] = 0;
        }
#pragma unroll
        for (int j = 0; j < RC; j++)
            cap[j] = 0;
        R = 1;
#pragma unroll
        for (int s = 0; s < GC; s++) {
            rel[s] = kFreeRel;
            gm[s] = 0;
            if constexpr (CONT)
                gsh[s] = 0;
        }
        ush = 0;
        used = 0;
        t = 0;
        ptr = 0;
        pos = 0;
        ovf = false;
    }

    // Make x the first CU of a run (0 < x < n_cu); the new run copies the
    // run it is cut from.
    __device__ __forceinline__ void split(uint32_t x, uint32_t n_cu)
    {
        if (x == 0 || x >= n_cu)
            return;
        uint32_t ins = 0;
        bool exists = false;
#pragma unroll
        for (int j = 0; j < RC; j++) {
            if (j < (int)R) {
                const uint32_t s = A[j] & 511u;
                ins += (s < x) ? 1u : 0u;
                exists = exists || (s == x);
            }
        }
        if (exists)
            return;
        if (R >= (uint32_t)RC) {
            ovf = true;
            return;
        }
#pragma unroll
        for (int j = RC - 1; j >= 1; j--) {
            if (j <= (int)R && (uint32_t)j >= ins) {
                const bool at = (uint32_t)j == ins;
                A[j] = at ? ((A[j - 1] & ~511u) | x) : A[j - 1];
                B[j] = B[j - 1];
                cap[j] = cap[j - 1];
            }
        }
        R++;
    }

    // Merge adjacent runs with equal resources.
    __device__ __forceinline__ void merge()
    {
        uint32_t dup = 0;
#pragma unroll
        for (int j = 1; j < RC; j++)
            if (j < (int)R && (A[j] >> 9) == (A[j - 1] >> 9) && B[j] == B[j - 1])
                dup |= 1u << j;
        while (dup) {
            const uint32_t d = (uint32_t)__builtin_ctz(dup);
#pragma unroll
            for (int j = 1; j + 1 < RC; j++) {
                if ((uint32_t)j >= d && j + 1 < (int)R) {
                    A[j] = A[j + 1];
                    B[j] = B[j + 1];
                }
            }
            R--;
            dup = (dup & ((1u << d) - 1u)) | ((dup >> (d + 1u)) << d);
        }
    }

    // One bulk step of the front kernel at the current cycle.  Returns false
    // when no block of it fits anywhere.
    __device__ __forceinline__ bool bulk_step(uint32_t n_cu, const uint32_t *tab, uint32_t *ent,
                                              uint32_t ecap_mask_bits)
    {
        const uint32_t lane = lane_no();
        const uint32_t u_reg = tab[kTReg + k], u_lds = tab[kTLds + k], u_wave = tab[kTWave + k];
        const float i_reg = __uint_as_float(tab[kTIReg + k]), i_lds = __uint_as_float(tab[kTILds + k]),
                    i_wave = __uint_as_float(tab[kTIWave + k]);
        // read once: the entry stores below are LDS stores the compiler cannot
        // tell apart from the table
        const uint32_t ua = tab[kTUa + k], ub = tab[kTUb + k], dur = tab[kTDur + k];
        const uint32_t shk = CONT ? tab[kTSh + k] : 0u;
        uint32_t T = 0, cmax = 0;
#pragma unroll
        for (int j = 0; j < RC; j++) {
            if (j < (int)R) {
                uint32_t c = B[j] & 127u;
                c = quot_clamp((B[j] >> 7) & 127u, u_wave, i_wave, c);
                c = quot_clamp(A[j] >> 9, u_reg, i_reg, c);
                if (u_lds)
                    c = quot_clamp(B[j] >> 14, u_lds, i_lds, c);
                cap[j] = c;
                T += (end_of(j, n_cu) - (A[j] & 511u)) * c;
                cmax = max(cmax, c);
            }
        }
        if (T == 0)
            return false;
        uint32_t r, extra, q;
        if (T <= rem) {
            r = cmax;
            q = T;
            extra = 0;
#pragma unroll
            for (int j = 0; j < RC; j++)
                if (j < (int)R && cap[j] >= r)
                    extra += end_of(j, n_cu) - (A[j] & 511u);
        } else {
            q = rem;
            uint32_t prev = 0;
            r = 0;
            extra = 0;
            for (;;) {
                r++;
                uint32_t acc = 0;
#pragma unroll
                for (int j = 0; j < RC; j++)
                    if (j < (int)R)
                        acc += (end_of(j, n_cu) - (A[j] & 511u)) * min(cap[j], r);
                if (acc >= rem || r >= cmax) {
                    extra = rem - prev;
                    break;
                }
                prev = acc;
            }
        }
        // the extra-th member of pass r walking cyclically from the pointer
        uint32_t after = 0;
#pragma unroll
        for (int j = 0; j < RC; j++) {
            if (j < (int)R && cap[j] >= r) {
                const uint32_t s = max(A[j] & 511u, ptr), e = end_of(j, n_cu);
                after += (e > s) ? e - s : 0u;
            }
        }
        const bool wrap = extra > after;
        const uint32_t need = wrap ? extra - after : extra;
        uint32_t seen = 0, cut = 0;
#pragma unroll
        for (int j = 0; j < RC; j++) {
            if (j < (int)R && cap[j] >= r) {
                const uint32_t s0 = A[j] & 511u, e0 = end_of(j, n_cu);
                const uint32_t s = wrap ? s0 : max(s0, ptr);
                const uint32_t e = wrap ? min(e0, ptr) : e0;
                if (e > s) {
                    const uint32_t L = e - s;
                    if (seen < need && need <= seen + L)
                        cut = s + (need - seen) - 1u;
                    seen += L;
                }
            }
        }
        const uint32_t p0 = ptr, c1 = cut + 1u;
        ptr = (c1 >= n_cu) ? 0u : c1;
        split(p0, n_cu);
        split(c1, n_cu);
        if (ovf)
            return false;
        constexpr uint32_t kBits = 8 * sizeof(Mask);
        const Mask full = (ecap_mask_bits >= kBits) ? (Mask)~(Mask)0 : (Mask)(((Mask)1 << ecap_mask_bits) - 1);
        Mask mask = 0;
        bool open = false;
        uint32_t es = 0, ec = 0;
#pragma unroll
        for (int j = 0; j < RC; j++) {
            if (j < (int)R) {
                const uint32_t s = A[j] & 511u;
                const bool inside = (p0 <= cut) ? (s >= p0 && s <= cut) : (s >= p0 || s <= cut);
                const uint32_t c = min(cap[j], r - 1u) + ((cap[j] >= r && inside) ? 1u : 0u);
                A[j] -= c * ua;
                B[j] -= c * ub;
                if (open && c != ec) {
                    if (used == full) {
                        ovf = true;
                    } else {
                        const uint32_t e = lowest_bit((Mask)~used);
                        used |= (Mask)1 << e;
                        mask |= (Mask)1 << e;
                        ent[e * kWave + lane] = es | (s << 8) | (ec << 17) | (k << 24);
                    }
                    open = false;
                }
                if (!open && c) {
                    open = true;
                    es = s;
                    ec = c;
                }
            }
        }
        if (open) {
            if (used == full) {
                ovf = true;
            } else {
                const uint32_t e = lowest_bit((Mask)~used);
                used |= (Mask)1 << e;
                mask |= (Mask)1 << e;
                ent[e * kWave + lane] = es | (n_cu << 8) | (ec << 17) | (k << 24);
            }
        }
        if (ovf)
            return false;
        // the first free group slot takes the group (live groups never exceed
        // the set size); written as a search that assigns as it goes, which
        // keeps rel and gm in registers
        bool placed = false;
        const Rel start = CONT ? (Rel)dur << 16 : (Rel)dur;
#pragma unroll
        for (int s = 0; s < GC; s++) {
            const bool take = !placed && rel[s] == kFreeRel;
            rel[s] = take ? start : rel[s];
            gm[s] = take ? mask : gm[s];
            if constexpr (CONT)
                gsh[s] = take ? q * shk : gsh[s];
            placed = placed || take;
        }
        if (!placed) {
            ovf = true;
            return false;
        }
        if constexpr (CONT)
            ush += q * shk;
        merge();
        rem -= q;
        return true;
    }

    // Advance to the earliest group end and release every group ending then.
    // Returns false if nothing is running (cannot happen for a valid set).
    // CONT: advance to the first whole cycle at which a group has its progress
    // (every resident block gains `rate` units per cycle) and end the groups
    // done then.  Returns their entry mask; `none` when nothing is running.
    __device__ __forceinline__ Mask contended_event(uint64_t mem_cap, bool &none)
    {
        uint64_t left = kFreeRel;
#pragma unroll
        for (int s = 0; s < GC; s++)
            left = min(left, (uint64_t)rel[s]);
        none = left == (uint64_t)kFreeRel;
        if (none)
            return 0;
        const uint64_t rate = (uint64_t)ush <= mem_cap ? 65536ull : div_u53(65536ull * mem_cap, ush);
        const uint64_t dt = div_u53(left + rate - 1, rate);
        const uint64_t adv = dt * rate;
        t += dt;
        Mask ending = 0;
#pragma unroll
        for (int s = 0; s < GC; s++) {
            if (rel[s] != kFreeRel) {
                if ((uint64_t)rel[s] <= adv) {
                    ending |= gm[s];
                    ush -= gsh[CONT ? s : 0];
                    rel[s] = kFreeRel;
                    gm[s] = 0;
                    gsh[CONT ? s : 0] = 0;
                } else {
                    rel[s] -= (Rel)adv;
                }
            }
        }
        return ending;
    }

    __device__ __forceinline__ bool advance(uint32_t n_cu, const uint32_t *tab, const uint32_t *ent,
                                            uint64_t mem_cap)
    {
        const uint32_t lane = lane_no();
        Mask ending = 0;
        if constexpr (CONT) {
            bool none;
            ending = contended_event(mem_cap, none);
            if (none)
                return false;
        } else {
            uint32_t dt = kFree;
#pragma unroll
            for (int s = 0; s < GC; s++)
                dt = min(dt, rel[s]);
            if (dt == kFree)
                return false;
            t += dt;
#pragma unroll
            for (int s = 0; s < GC; s++) {
                if (rel[s] != kFree) {
                    rel[s] -= dt;
                    if (rel[s] == 0) {
                        ending |= gm[s];
                        rel[s] = kFree;
                        gm[s] = 0;
                    }
                }
            }
        }
        used &= ~ending;
        while (ending) {
            const uint32_t e = lowest_bit(ending);
            ending &= ending - 1;
            const uint32_t w = ent[e * kWave + lane];
            const uint32_t s = w & 255u, en = (w >> 8) & 511u, c = (w >> 17) & 127u, kk = (w >> 24) & 15u;
            const uint32_t dua = c * tab[kTUa + kk], dub = c * tab[kTUb + kk];
            split(s, n_cu);
            split(en, n_cu);
#pragma unroll
            for (int j = 0; j < RC; j++) {
                if (j < (int)R) {
                    const uint32_t st = A[j] & 511u;
                    if (st >= s && st < en) {
                        A[j] += dua;
                        B[j] += dub;
                    }
                }
            }
        }
        merge();
        return true;
    }

    __device__ __forceinline__ uint32_t max_left() const
    {
        uint32_t m = 0;
#pragma unroll
        for (int s = 0; s < GC; s++)
            m = max(m, rel[s] == kFreeRel ? 0u : (uint32_t)rel[s]);
        return m;
    }
};

// The next order of the item for this lane: index from the LDS cursor, the
// permutation by mode, the lane's state reset.  False when the item is done.
// The cursor is indexed by a zero that passes through an empty asm in a
// vector register, so its address counts as lane-varying: the atomic stays one
// LDS atomic per active lane instead of becoming a compiler-built scan and
// broadcast inside lane-divergent code.
template <int RC, int GC, typename Mask, bool CONT>
__device__ __forceinline__ bool take_order(const SimArgs &a, const SetRec &st, int set, uint64_t first,
                                           uint64_t index0, bool ranked, uint64_t count, const uint32_t *tab,
                                           uint32_t *cursor, LaneSim<RC, GC, Mask, CONT> &L, uint32_t &i,
                                           uint64_t &perm)
{
    uint32_t zero = 0;
    asm volatile("" : "+v"(zero));
    i = atomicAdd(cursor + zero, 1u);
    if ((uint64_t)i >= count)
        return false;
    const uint32_t n = st.n;
    if (ranked) {
        perm = unrank_nibbles(index0 + i, n);
    } else if (a.mode == kModeSampled) {
        perm = unrank_nibbles(sampled_rank(a.seed, (uint32_t)set, first + i, n), n);
    } else {
        const uint8_t *o = a.orders + st.list_base + (first + i) * n;
        uint32_t seen = 0;
        perm = 0;
        for (uint32_t j = 0; j < n; j++) {
            const uint32_t v = o[j];
            seen |= (v < n) ? (1u << v) : 0x80000000u;
            perm |= (uint64_t)(v & 15u) << (4u * j);
        }
        if (seen != (1u << n) - 1u) {
            atomicOr(a.status, kStatusBadOrder);
            perm = identity_nibbles(n);
        }
    }
    L.reset(a);
    L.load_kernel(tab, (uint32_t)(perm & 15ull));
    return true;
}

// Resident waves per SIMD.  The contended variants of up to 10 kernels (192
// VGPRs unconstrained) and the plain 12-kernel variant (213) would run 2 waves;
// asked for 3 (at most 168 VGPRs) the compiler moves a few values to scratch
// (8, 15 and 57 dwords), which costs less than the third wave gains: all 10!
// contended n=10 orders in 17.4 ms instead of 23.1, all 12! orders of an n=12
// set in 3.33 s instead of 4.03, the same makespans.  The others fit 3 waves
// (plain, up to 10 kernels) or would spill too much (the 16-kernel variants).
template <int GC, bool CONT>
constexpr int lane_waves_per_simd()
{
    return ((CONT && GC <= 10) || (!CONT && GC == 12)) ? 3 : 1;
}

template <int RC, int GC, typename Mask, bool CONT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(lane_waves_per_simd<GC, CONT>())))
void simulate_lanes_kernel(SimArgs a, uint32_t ecap)
{
    extern __shared__ uint32_t lane_lds[];
    uint32_t *tab = lane_lds;
    uint32_t *cursor = lane_lds + kTabWords;
    uint32_t *ent = lane_lds + kEntBase;
    const uint32_t lane = lane_no();
    const uint32_t n_cu = a.n_cu;

    for (;;) {
        // every lane issues the fetch (lane 0 adds one); no lane-dependent
        // branch at the top of this loop (see simulate_kernel)
        const uint64_t item = wave_uniform64(atomicAdd(a.item_counter, lane == 0 ? 1ull : 0ull));
        if (item >= a.n_items)
            break;
        int lo = 0, hi = a.n_sets - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.sets[mid].item_base <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int set = lo;
        const SetRec st = a.sets[set];
        const uint32_t n = st.n;
        const KernelRec *kr = a.krec + st.kbase;
        const uint64_t first = (item - st.item_base) * a.chunk;
        const uint64_t count = min(a.chunk, st.n_orders - first);
        const uint64_t out_base = st.out_base + first;
        const bool ranked = a.mode == kModeAll || a.mode == kModeRange;
        const uint64_t index0 = ranked ? st.rank_lo + first : first;
        const bool has_ref = a.ref != nullptr;
        const int64_t ref = has_ref ? a.ref[set] : 0;

        __syncthreads();  // the previous item's table and cursor reads are done
        if (lane < n) {
            const KernelRec q = kr[lane];
            tab[kTUa + lane] = q.u_reg << 9;
            tab[kTUb + lane] = (q.u_lds << 14) | (q.u_wave << 7) | 1u;
            tab[kTReg + lane] = q.u_reg;
            tab[kTLds + lane] = q.u_lds;
            tab[kTWave + lane] = q.u_wave;
            tab[kTIReg + lane] = __float_as_uint(q.inv_reg);
            tab[kTILds + lane] = __float_as_uint(q.inv_lds);
            tab[kTIWave + lane] = __float_as_uint(q.inv_wave);
            tab[kTDur + lane] = q.dur;
            tab[kTBlk + lane] = q.tblk;
            if constexpr (CONT)
                tab[kTSh + lane] = a.share[st.kbase + lane];
        }
        *cursor = 0u;  // every lane stores the same value
        __syncthreads();

        // Each lane takes orders of the item from the LDS cursor until it runs
        // dry and simulates them; nothing in this loop crosses lanes.
        int64_t mn = INT64_MAX, mx = INT64_MIN;
        uint32_t imn = 0, imx = 0, n_less = 0, n_eq = 0, n_gt = 0;
        bool item_ovf = false;
        // One flat loop per lane.  Each pass makes at most one bulk step of the
        // placement at the lane's current cycle; once that placement is over
        // (the front kernel is blocked, or every block is placed) the same pass
        // advances to the next release, or records the finished order and
        // takes the next one.  Lanes therefore move through their orders
        // independently (no lane waits for the wave's longest order), and a
        // pass costs one bulk step whatever the lanes' phases (a new order's
        // first cycle places several kernels, over several passes).
        LaneSim<RC, GC, Mask, CONT> L;
        uint32_t i = 0;
        uint64_t perm = 0;
        bool live = take_order(a, st, set, first, index0, ranked, count, tab, cursor, L, i, perm);
        while (live) {
            // (only the contended drain comes here with every kernel placed)
            if ((!CONT || L.pos < n) && L.bulk_step(n_cu, tab, ent, ecap) && L.rem == 0) {
                L.pos++;
                if (L.pos < n) {
                    // the next kernel may still place blocks at this cycle
                    L.load_kernel(tab, (uint32_t)((perm >> (4u * L.pos)) & 15ull));
                    if (!L.ovf)
                        continue;
                }
            }
            int64_t m = -1;
            bool fin = false;
            if (!L.ovf) {
                const bool drain = L.pos >= n;
                if (!CONT && drain) {
                    // every block is placed: the longest group left sets the makespan
                    m = (int64_t)(L.t + L.max_left());
                    fin = true;
                } else if (!L.advance(n_cu, tab, ent, a.mem_cap)) {
                    // CONT drain: every group has ended (one event per pass, since
                    // each release changes the rate; its releases of runs are
                    // no longer needed but harmless).  Otherwise nothing runs
                    // yet the front block fits nowhere.
                    if (drain)
                        m = (int64_t)L.t;
                    else
                        atomicOr(a.status, kStatusGroupOverflow);
                    fin = true;
                }
            }
            if (L.ovf) {
                // recorded for spill_kernel (the wave engine, one wavefront
                // per order); if the record list is full, the whole item goes
                // to simulate_kernel instead
                uint32_t zero = 0;
                asm volatile("" : "+v"(zero));
                const unsigned long long slot = atomicAdd(a.spill_count + zero, 1ull);
                if (slot < a.spill_cap) {
                    SpillRec r;
                    r.set = (uint32_t)set;
                    r.item = (uint32_t)item;
                    r.sample = first + i;
                    r.pos = out_base + i;
                    r.makespan = 0;
                    a.spill[slot] = r;
                } else {
                    item_ovf = true;
                }
                live = take_order(a, st, set, first, index0, ranked, count, tab, cursor, L, i, perm);
                continue;
            }
            if (!fin)
                continue;
            if (m < mn || (m == mn && i < imn)) {
                mn = m;
                imn = i;
            }
            if (m > mx || (m == mx && i < imx)) {
                mx = m;
                imx = i;
            }
            if (has_ref) {
                n_less += (m < ref) ? 1u : 0u;
                n_eq += (m == ref) ? 1u : 0u;
                n_gt += (m > ref) ? 1u : 0u;
            }
            if (a.makespans)
                a.makespans[out_base + i] = m;
            live = take_order(a, st, set, first, index0, ranked, count, tab, cursor, L, i, perm);
        }

        // combine the lanes' statistics (ties -> smaller index)
        for (int o = 32; o >= 1; o >>= 1) {
            const int64_t omn = __shfl_xor(mn, o), omx = __shfl_xor(mx, o);
            const uint32_t oimn = __shfl_xor(imn, o), oimx = __shfl_xor(imx, o);
            if (omn < mn || (omn == mn && oimn < imn)) {
                mn = omn;
                imn = oimn;
            }
            if (omx > mx || (omx == mx && oimx < imx)) {
                mx = omx;
                imx = oimx;
            }
            n_less += __shfl_xor(n_less, o);
            n_eq += __shfl_xor(n_eq, o);
            n_gt += __shfl_xor(n_gt, o);
        }
        const bool any_ovf = __ballot(item_ovf) != 0;
        if (any_ovf) {
            // listed for simulate_kernel, which rewrites the item's makespans
            // and partial; every lane issues the atomic, lane 0 adds one
            const uint64_t at = wave_uniform64(atomicAdd(a.ovf_count, lane == 0 ? 1ull : 0ull));
            atomicOr(&a.handed_bits[item >> 5], lane == 0 ? 1u << (item & 31u) : 0u);
            if (lane == 0)
                a.ovf_list[at] = (uint32_t)item;
        }
        if (lane == 0) {
            Partial p;
            p.min_ms = mn;
            p.max_ms = mx;
            p.argmin = index0 + imn;
            p.argmax = index0 + imx;
            p.n_less = n_less;
            p.n_equal = n_eq;
            p.n_greater = n_gt;
            p.count = count;
            a.partials[item] = p;
        }
    }
}

template <bool CONT>
int launch_lanes_t(const SimArgs &a, int set_class, uint32_t ecap, size_t lds, int grid, hipStream_t st)
{
    switch (set_class) {
    case 8:
        hipLaunchKernelGGL((simulate_lanes_kernel<12, 8, uint32_t, CONT>), dim3(grid), dim3(64), lds, st, a, ecap);
        break;
    case 10:
        hipLaunchKernelGGL((simulate_lanes_kernel<12, 10, uint32_t, CONT>), dim3(grid), dim3(64), lds, st, a, ecap);
        break;
    case 12:
        hipLaunchKernelGGL((simulate_lanes_kernel<16, 12, uint64_t, CONT>), dim3(grid), dim3(64), lds, st, a, ecap);
        break;
    case 16:
        hipLaunchKernelGGL((simulate_lanes_kernel<20, 16, uint64_t, CONT>), dim3(grid), dim3(64), lds, st, a, ecap);
        break;
    default:
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace

// Lane kernels exist for sets of up to 8, 10, 12 and 16 kernels, with `entries`
// group entries per lane (0 = the class default, at most 64).  Returns
// hipErrorInvalidValue otherwise.
int launch_simulate_lanes(const SimArgs &a, int set_class, uint32_t entries, int grid, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const uint32_t ecap = entries ? entries : lane_entry_cap(set_class);
    if (ecap > (set_class <= 10 ? 32u : 64u))
        return (int)hipErrorInvalidValue;
    const size_t lds = (size_t)(kEntBase + ecap * kWave) * sizeof(uint32_t);
    if (a.share)
        return launch_lanes_t<true>(a, set_class, ecap, lds, grid, st);
    return launch_lanes_t<false>(a, set_class, ecap, lds, grid, st);
}

}  // namespace ko
