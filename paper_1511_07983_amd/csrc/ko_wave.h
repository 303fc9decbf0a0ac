// Device routines of libko's wave engine: exact makespan of one launch order
// per wavefront.  Used by simulate_kernel (ko_sim.hip) and by the lane kernel
// (ko_lanes.hip) for orders that outgrow a lane's capacities.
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
// longest remaining group; the drain is not simulated (except under memory
// contention, below).

#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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

__device__ __forceinline__ uint64_t wave_min64(uint64_t v)
{
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
        v = min(v, ((uint64_t)hi << 32) | lo);
    }
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
static __device__ uint32_t unrank_lanes(uint64_t rank, uint32_t n)
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
static __device__ uint32_t next_perm_lanes(uint32_t perm, uint32_t n)
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

// Memory contention (CONT = true; Section 4's balance of instructions and
// memory accesses across the blocks that run together).  Every resident
// block runs at one common rate: a block of kernel i holds a memory share
// sh[i] (1/1024 units), and while the resident shares add up to U above
// mem_cap (1024 times the memory-bound blocks the chip serves at full speed),
// a cycle brings floor(65536 * mem_cap / U) units of progress instead of
// 65536.  A block needs dur * 65536 units; it ends at the first whole cycle
// at which it has them, and all blocks ending at a cycle release before
// placement resumes.  Because every resident block progresses alike, the
// blocks of one bulk step still end together: a group keeps its progress
// left (64 bits) in lane g and its blocks' summed share in lane g of gsh.
// The drain after the last placement is simulated too, since each release
// changes the rate.

// Makespan of the order held in `perm` (lane j = kernel at position j).
// Returns -1 (and sets a status bit) only on an internal inconsistency.
// sh: memory shares of the set's kernels (CONT only).
template <int S, bool CONT = false>
__device__ int64_t simulate_order(const SimArgs &a, const KernelRec *__restrict__ kr,
                                  const uint32_t *__restrict__ sh, uint32_t n, uint32_t perm,
                                  uint32_t *__restrict__ ring, uint32_t gslots)
{
    using Rel = typename std::conditional<CONT, uint64_t, uint32_t>::type;
    constexpr Rel kFree = ~Rel(0);
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
    // lane g: cycles (CONT: units of progress) until group g ends; all ones = free slot
    Rel rel = kFree;
    uint32_t gk = 0;    // lane g: kernel of group g
    uint32_t gsh = 0;   // CONT, lane g: summed memory share of group g's blocks
    uint32_t used = 0;  // CONT: summed memory share of every resident block
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
            const uint64_t free_slots = ballot(lane < gslots && rel == kFree);
            if (free_slots == 0) {
                flag_status(a.status, kStatusGroupOverflow);
                return -1;
            }
            const uint32_t g = (uint32_t)__builtin_ctzll(free_slots);
            ring[g * kWave + lane] = packed;
            const uint32_t dur = kr[k].dur;
            if constexpr (CONT) {
                const uint32_t share = q * sh[k];
                rel = (lane == g) ? ((uint64_t)dur << 16) : rel;
                gsh = (lane == g) ? share : gsh;
                used += share;
            } else {
                rel = (lane == g) ? dur : rel;
            }
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
        const bool live = rel != kFree;
        uint64_t ending;
        if constexpr (CONT) {
            // ---- next event: the first whole cycle at which a group is done ----
            const uint64_t left = uniform64(wave_min64(rel));
            if (left == kFree) {
                if (pos >= n)
                    return (int64_t)t;  // every block placed and ended
                flag_status(a.status, kStatusGroupOverflow);  // the front block fits nowhere
                return -1;
            }
            const uint64_t rate = (uint64_t)used <= a.mem_cap ? 65536ull : (65536ull * a.mem_cap) / used;
            const uint64_t dt = (left + rate - 1) / rate;
            const uint64_t adv = dt * rate;
            t += dt;
            const bool done = live && rel <= adv;
            ending = ballot(done);
            rel = done ? kFree : (live ? rel - adv : rel);
        } else {
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
            ending = ballot(live && rel == 0u);
            rel = (live && rel == 0u) ? 0xFFFFFFFFu : rel;
        }
        while (ending) {
            const uint32_t g = (uint32_t)__builtin_ctzll(ending);
            ending &= ending - 1ull;
            const uint32_t kg = uniform(read_lane(gk, g));
            if constexpr (CONT)
                used -= uniform(read_lane(gsh, g));
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

}  // namespace ko
