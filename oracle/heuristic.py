"""Oracle: the launch-order heuristic (Algorithm 1) in binary64 Python floats.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Algorithm 1 ("Concurrent Kernel Launch Order Algorithm") and the
prose of Section 5 ("Proposed Algorithm"):

* ScoreGen(X, Y): zero when the two cannot share an execution round;
  otherwise the leftover fractions of shared memory, registers and warps, in
  that order, each clamped at 0, plus a balance term 1 - |R_comb - R_B| / R_B
  (clamped at 0) that is added only when R_B lies between R_X and R_Y
  (inclusive), i.e. one is memory bound and the other compute bound.
* ProfileCombine(a, b): resources and block counts add; the combined ratio is
  the instruction-weighted harmonic mean (W_a + W_b) / (W_a/R_a + W_b/R_b).
* Main loop: while kernels remain, open a round, seed it with the best-scoring
  pair (placed in decreasing shared-memory order), then keep adding the
  best-scoring kernel that still fits the round, combining profiles as it
  goes; the output is the rounds in the order they were opened.

Points the paper leaves open, and the reading taken for each:

* resource quantities in ScoreGen: with PER_SM_SHARE (default) a kernel's
  footprint is ceil(N_tblk / N_SM) blocks' worth of its per-block usage;
  with PER_BLOCK (flag bit 0) it is one block's worth;
* "fit within an execution round": the summed footprints stay within all four
  per-SM limits (registers, shared memory, warps, blocks);
* the inner "For": repeat until no remaining kernel fits; the candidate list
  and their scores are recomputed after every insertion;
* ties in "highest score": the first in scan order wins (pairs i < j in
  lexicographic order; candidates by lowest index), comparing exact binary64;
* pair order: decreasing shared-memory footprint, the lower index first on a tie;
* "(Sort by N_shm_c, N_shm_comb)": INSERT_UNIT (default) puts the new kernel
  before the whole round when its shared memory exceeds the round's combined
  shared memory, else after it; FULL_SORT (flag bit 1) stably re-sorts the
  round members by decreasing shared memory;
* one kernel left: it forms a round of its own;
* the best pair does not fit (score 0): it is still pushed as the pair, and
  no further kernel can join its round;
* the combined ratio of the growing virtual kernel is combined pairwise with
  each newly added kernel, exactly as for a pair.

Parity against the paper is pinned only by hand-worked examples; the paper
prints no trace of the algorithm.
"""

from __future__ import annotations

PER_BLOCK = 1
FULL_SORT = 2

_REG, _LDS, _WAVE, _BLK = range(4)


class _Profile:
    """Footprint F[4] (reg, lds, wave, blk), instruction weight W, ratio R."""

    __slots__ = ("F", "W", "R")

    def __init__(self, F, W, R):
        self.F = list(F)
        self.W = float(W)
        self.R = float(R)


def _get(obj, name):
    return obj[name] if isinstance(obj, dict) else getattr(obj, name)


def _profiles(gpu, kernels, flags):
    n_cu = int(_get(gpu, "n_cu"))
    wave_size = int(_get(gpu, "wave_size"))
    out = []
    for k in kernels:
        tblk = int(k["n_tblk"])
        waves = int(k["waves_blk"])
        per_block = [int(k["regs_thr"]) * waves * wave_size, int(k["lds_blk"]), waves, 1]
        b = 1 if (flags & PER_BLOCK) else -(-tblk // n_cu)  # ceil(N_tblk / N_SM)
        out.append(_Profile([b * u for u in per_block], b * int(k["n_inst"]),
                            float(int(k["r_milli"])) / 1000.0))
    return out


def _caps(gpu):
    return [int(_get(gpu, "reg_cu")), int(_get(gpu, "lds_cu")),
            int(_get(gpu, "wave_cu")), int(_get(gpu, "blk_cu"))]


def fits(cap, X: _Profile, Y: _Profile) -> bool:
    return all(X.F[x] + Y.F[x] <= cap[x] for x in range(4))


def combined_ratio(X: _Profile, Y: _Profile) -> float:
    """ProfileCombine's R: (W_X + W_Y) / (W_X / R_X + W_Y / R_Y)."""
    return (X.W + Y.W) / (X.W / X.R + Y.W / Y.R)


def score(cap, rb: float, X: _Profile, Y: _Profile) -> float:
    """ScoreGen for one pair."""
    if not fits(cap, X, Y):
        return 0.0
    s = 0.0
    s += max(float(cap[_LDS] - X.F[_LDS] - Y.F[_LDS]) / float(cap[_LDS]), 0.0)
    s += max(float(cap[_REG] - X.F[_REG] - Y.F[_REG]) / float(cap[_REG]), 0.0)
    s += max(float(cap[_WAVE] - X.F[_WAVE] - Y.F[_WAVE]) / float(cap[_WAVE]), 0.0)
    if (X.R <= rb <= Y.R) or (Y.R <= rb <= X.R):
        rc = combined_ratio(X, Y)
        s += max(1.0 - abs(rc - rb) / rb, 0.0)
    return s


def combine(X: _Profile, Y: _Profile) -> _Profile:
    """ProfileCombine: summed footprints and weights, combined ratio."""
    return _Profile([X.F[x] + Y.F[x] for x in range(4)], X.W + Y.W, combined_ratio(X, Y))


def score_matrix(gpu, kernels, flags: int = 0):
    """The n x n ScoreMatrix (upper triangle filled, i < j)."""
    P = _profiles(gpu, kernels, flags)
    cap = _caps(gpu)
    rb = float(int(_get(gpu, "rb_milli"))) / 1000.0
    n = len(P)
    S = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            S[i][j] = score(cap, rb, P[i], P[j])
    return S


def heuristic_order(gpu, kernels, flags: int = 0):
    """Launch order of Algorithm 1.  Returns (order, round_of_position)."""
    P = _profiles(gpu, kernels, flags)
    cap = _caps(gpu)
    rb = float(int(_get(gpu, "rb_milli"))) / 1000.0
    n = len(P)
    if n < 1:
        raise ValueError("empty kernel set")
    S = score_matrix(gpu, kernels, flags)
    remaining = list(range(n))
    order, rounds = [], []
    r = 0
    while remaining:
        if len(remaining) == 1:
            order.append(remaining[0])
            rounds.append(r)
            remaining = []
            break
        best, best_s = None, None
        for ai, i in enumerate(remaining):
            for j in remaining[ai + 1:]:
                if best is None or S[i][j] > best_s:
                    best, best_s = (i, j), S[i][j]
        a, b = best
        if P[b].F[_LDS] > P[a].F[_LDS]:
            a, b = b, a
        members = [a, b]
        remaining.remove(a)
        remaining.remove(b)
        comb = combine(P[a], P[b])
        while True:
            cands = [k for k in remaining if fits(cap, comb, P[k])]
            if not cands:
                break
            c, c_s = None, None
            for k in cands:
                s = score(cap, rb, comb, P[k])
                if c is None or s > c_s:
                    c, c_s = k, s
            if flags & FULL_SORT:
                members.append(c)
                members.sort(key=lambda m: -P[m].F[_LDS])  # stable
            elif P[c].F[_LDS] > comb.F[_LDS]:
                members.insert(0, c)
            else:
                members.append(c)
            comb = combine(comb, P[c])
            remaining.remove(c)
        order.extend(members)
        rounds.extend([r] * len(members))
        r += 1
    return order, rounds

