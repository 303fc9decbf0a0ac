"""Oracle: counter-based sampled ranks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sampled orders are drawn uniformly with replacement.  The i-th sample of set
s under seed S has lexicographic rank floor(x * N / 2**64), where N = n! and
x is output number c = (s << 40) | i of the SplitMix64 generator seeded with S
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014; Vigna's public-domain splitmix64): the state after c+1 steps is
S + (c+1) * 0x9E3779B97F4A7C15 (mod 2**64), mixed by
z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
z ^= z >> 31.  The map x -> floor(x * N / 2**64) is Lemire's multiply-shift
range reduction; its bias is below N / 2**64.
"""

from __future__ import annotations

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64_at(seed: int, c: int) -> int:
    z = (seed + (c + 1) * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def sampled_rank(seed: int, set_index: int, i: int, n_orders: int) -> int:
    x = splitmix64_at(seed, (set_index << 40) | i)
    return (x * n_orders) >> 64


def sampled_ranks(seed: int, set_index: int, count: int, n_orders: int):
    return [sampled_rank(seed, set_index, i, n_orders) for i in range(count)]
