"""Oracle: per-set statistics, percentile rank, histogram, Table 3 formulas.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Table 3 reports, for the algorithm's order: the optimal and worst times over
all orders, the percentile rank of the algorithm's time among all orders, the
speedup over the worst order and the deviation from the optimal one.  Figure 1
shows the distribution of times over the permutation space.

Readings:
* ranks are lexicographic over the sequence of input kernel indices; argmin
  and argmax take the smallest index on ties;
* the percentile is reported from exact counts: inclusive (share of orders
  at least as slow as the reference), strict (share strictly slower) and
  mid-rank (strict plus half the ties);
* histogram bins: bin = floor((M - min) * n_bins / (max - min + 1));
* Figure 1's ranking: the makespans of all orders in ascending order, equal
  makespans by smaller rank;
* Section 6's "a gain of at least g over a random order with probability at
  least one half": the largest g for which at least half of all orders have a
  makespan of at least (1 + g) times the algorithm's.
"""

from __future__ import annotations

import numpy as np


def set_stats(makespans, ref=None) -> dict:
    m = np.asarray(makespans, dtype=np.int64)
    out = {
        "min": int(m.min()), "max": int(m.max()),
        "argmin": int(np.argmin(m)), "argmax": int(np.argmax(m)),
        "n_orders": int(m.size),
    }
    if ref is not None:
        out["n_less"] = int(np.count_nonzero(m < ref))
        out["n_equal"] = int(np.count_nonzero(m == ref))
        out["n_greater"] = int(np.count_nonzero(m > ref))
    return out


def percentiles(n_less: int, n_equal: int, n_greater: int) -> dict:
    total = n_less + n_equal + n_greater
    return {
        "inclusive": 100.0 * (n_greater + n_equal) / total,
        "strict": 100.0 * n_greater / total,
        "mid": 100.0 * (n_greater + 0.5 * n_equal) / total,
    }


def histogram(makespans, n_bins: int, lo: int, hi: int) -> np.ndarray:
    m = np.asarray(makespans, dtype=np.int64)
    width = hi - lo + 1
    # exact integer arithmetic (Python ints) so that no product can overflow
    bins = ((m - lo).astype(object) * n_bins // width).astype(np.int64)
    return np.bincount(bins, minlength=n_bins).astype(np.uint64)


def speedup_over_worst(t_worst: float, t_alg: float) -> float:
    return t_worst / t_alg


def deviation_from_optimal(t_opt: float, t_alg: float) -> float:
    return (t_alg - t_opt) / t_opt


def ranking_curve(makespans):
    """Figure 1's ranking curve: (makespans ascending, rank of each), ties by
    smaller rank (a stable sort of the rank-ordered array)."""
    m = np.asarray(makespans, dtype=np.int64)
    idx = np.argsort(m, kind="stable")
    return m[idx], idx


def median_gain(makespans, t_alg: int) -> float:
    """Section 6's gain over a random order reached with probability at least
    one half: over the distinct makespans m, the largest with at least half of
    all orders at m or slower, as m / t_alg - 1."""
    m = np.asarray(makespans, dtype=np.int64)
    n = m.size
    vals, counts = np.unique(m, return_counts=True)  # ascending
    at_or_above = n - np.concatenate([[0], np.cumsum(counts)[:-1]])
    best = int(vals[2 * at_or_above >= n].max())
    return best / float(t_alg) - 1.0
