// Round-synchronous execution rounds (Section 2 of Li, Narayana & El-Ghazawi
// 2015): the blocks of a kernel set, in launch order, are split into rounds
// that run one after another.  A round takes blocks from the front of the
// stream, each on the first CU at or after a cyclic pointer that has room
// (registers, LDS, waves, block slots; Table 1), until the front block fits on
// no CU.  The round then lasts as long as its longest block, every CU is freed,
// and the next round starts with that block.  The pointer carries over.  No
// block releases its resources in the middle of a round, so the makespan is
// the sum of the round lengths.
//
// Mapping.  One wavefront per launch order; lane l holds the free resources of
// CUs l, l+64, l+128, l+192 (S slots).  Because nothing is released inside a
// round, the blocks of one kernel that enter a round are placed in one bulk
// step: with cap[c] = blocks of the kernel that CU c can still take, a cyclic
// sweep from the pointer places one block on every CU with cap >= 1, then one
// on every CU with cap >= 2, and so on.  Placing q blocks therefore gives each
// CU min(cap, r-1) blocks plus one more to the first q - A(r-1) CUs of
// {cap >= r} in pointer order, where A(r) = sum of min(cap, r) and r is the
// first pass with A(r) >= q (found pass by pass from ballot popcounts); the
// pointer ends just past the last of them.  A kernel needs one bulk step per
// round it spans.  The first step of a round meets empty CUs with equal caps
// and has a closed form; a step that fills every CU while blocks of its kernel
// remain closes the round without another look at the CUs.  All control flow
// depends on wave-uniform values only, so wave collectives always run with
// every lane; sums and maxima over CUs are DPP reductions within the wave.
#include <hip/hip_runtime.h>

#include "ko_device.h"
#include "ko_rounds.h"
#include "ko_wave.h"

namespace ko {
namespace {

constexpr int kRoundsWaves = 4;          // wavefronts per workgroup
constexpr uint32_t kRoundsGridCap = 4096;
constexpr uint64_t kRankRun = 16;        // consecutive ranks per wavefront in rank mode

// Lane-shifted copy of v through DPP: lanes whose source lies outside their
// row of 16 read 0, lanes in rows left out of RowMask read 0.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, true);
}

// Sum and maximum over the 64 lanes, in every lane.  Shifts by 1, 2, 4 and 8
// within each row of 16 make lane 15 of a row hold the row's total; the row
// broadcasts of lane 15 (into rows 1 and 3) and of lane 31 (into rows 2 and 3)
// then leave the wave's total in lane 63, which is read back as a scalar.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    v += dpp<0x111, 0xf>(v);   // row_shr:1
    v += dpp<0x112, 0xf>(v);   // row_shr:2
    v += dpp<0x114, 0xf>(v);   // row_shr:4
    v += dpp<0x118, 0xf>(v);   // row_shr:8
    v += dpp<0x142, 0xa>(v);   // row_bcast:15
    v += dpp<0x143, 0xc>(v);   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_umax(uint32_t v)
{
    v = max(v, dpp<0x111, 0xf>(v));
    v = max(v, dpp<0x112, 0xf>(v));
    v = max(v, dpp<0x114, 0xf>(v));
    v = max(v, dpp<0x118, 0xf>(v));
    v = max(v, dpp<0x142, 0xa>(v));
    v = max(v, dpp<0x143, 0xc>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// Bits of word s (CUs 64s .. 64s+63) that are at or after CU `from`.
__device__ __forceinline__ uint64_t at_or_after(uint32_t from, int s)
{
    const uint32_t base = 64u * (uint32_t)s;
    if (from <= base)
        return ~0ull;
    if (from >= base + 64u)
        return 0ull;
    return ~0ull << (from - base);
}

// Position of the j-th set bit (1-based) of w, which has at least j: halve
// the window six times, skipping its low half when that holds fewer than j.
__device__ __forceinline__ uint32_t nth_bit(uint64_t w, uint32_t j)
{
    uint32_t pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const uint32_t c = (uint32_t)__popcll(w & ((1ull << width) - 1));
        if (j > c) {
            j -= c;
            w >>= width;
            pos += (uint32_t)width;
        }
    }
    return pos;
}

// CU of the j-th member (1-based) of `mem` among CUs >= from, ascending; the
// caller guarantees there are at least j.  Uniform scalar work.
template <int S>
__device__ uint32_t nth_from(const uint64_t (&mem)[S], uint32_t from, uint32_t j)
{
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint64_t w = mem[s] & at_or_after(from, s);
        const uint32_t pc = (uint32_t)__popcll(w);
        if (j <= pc)
            return 64u * (uint32_t)s + nth_bit(w, j);
        j -= pc;
    }
    return 0;
}

// CU that receives the j-th block of the last pass: the j-th member of `mem`
// counted cyclically from the pointer.
template <int S>
__device__ uint32_t cyclic_nth(const uint64_t (&mem)[S], uint32_t ptr, uint32_t j)
{
    uint32_t upper = 0;
#pragma unroll
    for (int s = 0; s < S; ++s)
        upper += (uint32_t)__popcll(mem[s] & at_or_after(ptr, s));
    return j <= upper ? nth_from<S>(mem, ptr, j) : nth_from<S>(mem, 0, j - upper);
}

template <int S>
__device__ int64_t rounds_order(const RoundsArgs &a, const KernelRec *tab, const uint32_t *c0s, uint32_t mine,
                                uint32_t lane)
{
    const uint32_t n = a.n, ncu = a.n_cu;
    uint32_t fr_reg[S], fr_lds[S], fr_wave[S], fr_blk[S];
    auto reset = [&]() {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            fr_reg[s] = a.cap_reg;
            fr_lds[s] = a.cap_lds;
            fr_wave[s] = a.cap_wave;
            fr_blk[s] = lane + 64u * (uint32_t)s < ncu ? a.cap_blk : 0u;   // absent CUs take nothing
        }
    };
    reset();
    int64_t t = 0;          // start of the open round
    uint32_t longest = 0;   // longest block placed in the open round
    uint32_t ptr = 0;
    bool fresh = true;      // nothing placed since the last reset: every CU empty
    uint32_t seen = 0;      // kernels met so far (a row must be a permutation)
    for (uint32_t pos = 0; pos < n; ++pos) {
        const uint32_t k = read_lane(mine, pos);
        if (k >= n || ((seen >> k) & 1u))
            return -1;
        seen |= 1u << k;
        const KernelRec kr = tab[k];
        uint32_t rem = kr.tblk;
        bool full = false;  // the last step gave every CU all the blocks it can take
        while (rem) {
            if (full) {
                // blocks of this kernel remain and fit nowhere: the round ends
                // with its longest block, and the next one starts empty
                t += longest;
                longest = 0;
                reset();
                fresh = true;
                full = false;
                continue;
            }
            uint32_t tot, q, r, cut;
            if (fresh) {
                // every CU empty: the same cap c0 everywhere, so pass r is
                // ceil(q / n_CU) and the cut lies q - n_CU (r-1) CUs past the
                // pointer
                const uint32_t c0 = c0s[k];
                if (c0 == 0)
                    return -1;   // a block that fits no empty CU (rejected by the host)
                tot = ncu * c0;
                q = min(tot, rem);
                r = div_clamp(q + ncu - 1, ncu, a.inv_ncu, c0);   // ceil(q / n_CU) <= c0
                const uint32_t end = ptr + (q - ncu * (r - 1)) - 1;
                cut = end >= ncu ? end - ncu : end;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const uint32_t c = lane + 64u * (uint32_t)s;
                    const bool in = ptr <= cut ? (c >= ptr && c <= cut) : (c >= ptr || c <= cut);
                    const uint32_t cnt = c < ncu ? (r - 1) + (in ? 1u : 0u) : 0u;
                    fr_reg[s] -= cnt * kr.u_reg;
                    fr_lds[s] -= cnt * kr.u_lds;
                    fr_wave[s] -= cnt * kr.u_wave;
                    fr_blk[s] -= cnt;
                }
                fresh = false;
            } else {
                uint32_t cap[S];
                uint32_t cmax = 0;
                tot = 0;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    uint32_t c = div_clamp(fr_reg[s], kr.u_reg, kr.inv_reg, fr_blk[s]);
                    c = div_clamp(fr_wave[s], kr.u_wave, kr.inv_wave, c);
                    if (kr.u_lds)
                        c = div_clamp(fr_lds[s], kr.u_lds, kr.inv_lds, c);
                    cap[s] = c;
                    tot += c;
                    cmax = max(cmax, c);
                }
                tot = wave_sum(tot);
                if (tot == 0) {
                    // the front block fits nowhere: the round ends with its longest block
                    t += longest;
                    longest = 0;
                    reset();
                    fresh = true;
                    continue;
                }
                q = min(tot, rem);
                uint64_t mem[S];
                if (q == tot) {
                    // every block that fits is placed: each CU gets its cap, and
                    // the last block lands on the last CU of the final pass
                    // (cap == max cap) in pointer order
                    const uint32_t cm = wave_umax(cmax);
                    uint32_t members = 0;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        mem[s] = ballot(cap[s] >= cm);
                        members += (uint32_t)__popcll(mem[s]);
                    }
                    cut = uniform(cyclic_nth<S>(mem, ptr, members));
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        fr_reg[s] -= cap[s] * kr.u_reg;
                        fr_lds[s] -= cap[s] * kr.u_lds;
                        fr_wave[s] -= cap[s] * kr.u_wave;
                        fr_blk[s] -= cap[s];
                    }
                } else {
                    // passes one by one: pass r adds |{cap >= r}| blocks (ballot
                    // popcounts); it ends at the first r with A(r) >= q, which
                    // comes no later than the max cap because A(max cap) = tot > q
                    uint32_t below = 0;
                    r = 0;
                    for (;;) {
                        ++r;
                        uint32_t m = 0;
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            mem[s] = ballot(cap[s] >= r);
                            m += (uint32_t)__popcll(mem[s]);
                        }
                        if (below + m >= q)
                            break;
                        below += m;
                    }
                    cut = uniform(cyclic_nth<S>(mem, ptr, q - below));
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const uint32_t c = lane + 64u * (uint32_t)s;
                        const bool in = ptr <= cut ? (c >= ptr && c <= cut) : (c >= ptr || c <= cut);
                        const uint32_t cnt = min(cap[s], r - 1) + ((cap[s] >= r && in) ? 1u : 0u);
                        fr_reg[s] -= cnt * kr.u_reg;
                        fr_lds[s] -= cnt * kr.u_lds;
                        fr_wave[s] -= cnt * kr.u_wave;
                        fr_blk[s] -= cnt;
                    }
                }
            }
            ptr = cut + 1 == ncu ? 0u : cut + 1;
            longest = max(longest, kr.dur);
            full = q == tot && rem > q;
            rem -= q;
        }
    }
    return t + longest;
}

template <int S>
__global__ __launch_bounds__(64 * kRoundsWaves) void rounds_kernel(RoundsArgs a)
{
    __shared__ KernelRec tab[kMaxSet];
    __shared__ uint32_t c0s[kMaxSet];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kMaxSet; ++i)
            if (i < (int)a.n) {
                tab[i] = a.k[i];
                c0s[i] = a.c0[i];
            }
    }
    __syncthreads();
    const uint32_t lane = lane_id();
    const uint64_t first = (uint64_t)blockIdx.x * kRoundsWaves + uniform(threadIdx.x >> 6);
    const uint64_t stride = (uint64_t)gridDim.x * kRoundsWaves;
    // every lane stores the same makespan: no lane-dependent branch in the loops
    if (a.orders) {
        for (uint64_t i = first; i < a.count; i += stride) {
            const uint32_t mine = lane < a.n ? (uint32_t)a.orders[i * a.n + lane] : 0u;
            a.makespans[i] = rounds_order<S>(a, tab, c0s, mine, lane);
        }
    } else {
        // runs of kRankRun consecutive ranks per wavefront: one unranking, then
        // next-permutation steps (never past the run's last rank, which is < n!)
        const uint64_t runs = (a.count + kRankRun - 1) / kRankRun;
        for (uint64_t g = first; g < runs; g += stride) {
            const uint64_t base = g * kRankRun;
            const uint64_t end = min(base + kRankRun, a.count);
            uint32_t perm = unrank_lanes(a.first + base, a.n);
            for (uint64_t i = base;;) {
                a.makespans[i] = rounds_order<S>(a, tab, c0s, perm, lane);
                if (++i == end)
                    break;
                perm = next_perm_lanes(perm, a.n);
            }
        }
    }
}

}  // namespace

int launch_rounds(const RoundsArgs &a, void *stream)
{
    if (a.count == 0)
        return (int)hipSuccess;
    const uint64_t want = (a.count + kRoundsWaves - 1) / kRoundsWaves;
    const dim3 grid((uint32_t)(want < kRoundsGridCap ? want : kRoundsGridCap));
    const dim3 block(64 * kRoundsWaves);
    hipStream_t s = (hipStream_t)stream;
    switch ((a.n_cu + 63) / 64) {
    case 1: hipLaunchKernelGGL(rounds_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(rounds_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(rounds_kernel<3>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(rounds_kernel<4>, grid, block, 0, s, a); break;
    }
    return (int)hipGetLastError();
}

}  // namespace ko
