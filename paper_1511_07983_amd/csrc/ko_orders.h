// Launch orders on the device: factorials, the counter-based sample of a rank,
// and per-thread unranking.  Shared by the simulate kernel and the order writer
// so that a sampled order means the same permutation everywhere in libko.
//
// Ranks are lexicographic over order sequences (order[j] = kernel launched at
// position j): digit j of the factorial number system, floor(r_j / (n-1-j)!),
// with r_j the remainder left by earlier digits, picks the digit-th smallest
// kernel index not used at positions < j.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ko {

static __device__ const uint64_t kFactorial[21] = {
    1ull, 1ull, 2ull, 6ull, 24ull, 120ull, 720ull, 5040ull, 40320ull, 362880ull, 3628800ull,
    39916800ull, 479001600ull, 6227020800ull, 87178291200ull, 1307674368000ull,
    20922789888000ull, 355687428096000ull, 6402373705728000ull, 121645100408832000ull,
    2432902008176640000ull};

// SplitMix64 (Steele, Lea & Flood 2014) evaluated at counter c: the output
// the generator seeded with `seed` returns on its (c+1)-th call.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Rank of sample i of the set at batch index `set` (SAMPLED mode): the high
// 64 bits of splitmix64_at(seed, set * 2^40 + i) * n!, uniform on [0, n!).
__device__ __forceinline__ uint64_t sampled_rank(uint64_t seed, uint32_t set, uint64_t i, uint32_t n)
{
    const uint64_t x = splitmix64_at(seed, ((uint64_t)set << 40) | i);
    return __umul64hi(x, kFactorial[n]);
}

// One thread unranks `rank` (< n!, n <= 20) and writes the order and/or its
// inverse (pos[k] = position of kernel k); either pointer may be null.
__device__ __forceinline__ void unrank_thread(uint64_t rank, uint32_t n, uint8_t *order, uint8_t *pos)
{
    uint32_t avail = (1u << n) - 1u;
    for (uint32_t j = 0; j < n; j++) {
        const uint64_t f = kFactorial[n - 1u - j];
        const uint32_t d = (uint32_t)(rank / f);
        rank -= (uint64_t)d * f;
        uint32_t m = avail;
        for (uint32_t t = 0; t < d && m; t++)
            m &= m - 1u;
        // m is nonzero for every rank below n!; otherwise fall back to the
        // lowest unused kernel so that the indices written stay below n
        const uint32_t k = (uint32_t)__builtin_ctz(m ? m : avail);
        avail &= ~(1u << k);
        if (order)
            order[j] = (uint8_t)k;
        if (pos)
            pos[k] = (uint8_t)j;
    }
}

}  // namespace ko
