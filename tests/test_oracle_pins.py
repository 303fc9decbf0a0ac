"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-run the oracle's own formula: each compares it with a
hand-traced example (tests/golden), a closed form, an invariant stated in the
paper, a library routine, or an independent brute-force formulation.
"""

import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import stats as ostats
from oracle.heuristic import FULL_SORT, PER_BLOCK, heuristic_order, score_matrix
from oracle.sampling import sampled_rank, splitmix64_at
from oracle.tick import tick_makespan

pytestmark = pytest.mark.filterwarnings("ignore")


def all_makespans(gpu, ks):
    return oracle.makespans_all(gpu, ks, threads=2)


# ---------------------------------------------------------------- hand traces

def test_e1_hand_trace(golden):
    g = golden("e1_two_cu.json")
    use, dur = oracle.derive(g["gpu"], g["kernels"])
    assert dur.tolist() == g["durations"]
    assert all_makespans(g["gpu"], g["kernels"]).tolist() == g["makespans_by_rank"]
    for flags in range(4):
        assert heuristic_order(g["gpu"], g["kernels"], flags)[0] == g["heuristic_order_all_flags"]
    S = score_matrix(g["gpu"], g["kernels"], PER_BLOCK)
    assert S[0][1] == pytest.approx(g["score_per_block_pair"], abs=1e-12)
    ms = all_makespans(g["gpu"], g["kernels"])
    st = ostats.set_stats(ms, ref=ms[0])
    assert {k: st[k] for k in ("n_less", "n_equal", "n_greater")} == g["counts_for_order_rank0"]
    pct = ostats.percentiles(st["n_less"], st["n_equal"], st["n_greater"])
    assert pct == pytest.approx(g["percentiles_for_order_rank0"])


def test_e2_heuristic_hand_worked(golden):
    g = golden("e2_heuristic.json")
    use, dur = oracle.derive(g["gpu"], g["kernels"])
    assert dur.tolist() == g["durations"]
    assert use.tolist() == g["per_block_use"]
    S = score_matrix(g["gpu"], g["kernels"], PER_BLOCK)
    for key, v in g["pair_scores_per_block_values"].items():
        i, j = map(int, key.split(","))
        assert S[i][j] == pytest.approx(v, abs=5e-7), key
    modes = {"per_sm_share_insert_unit": 0, "per_block_insert_unit": PER_BLOCK,
             "per_sm_share_full_sort": FULL_SORT, "per_block_full_sort": PER_BLOCK | FULL_SORT}
    for name, flags in modes.items():
        order, rounds = heuristic_order(g["gpu"], g["kernels"], flags)
        assert order == g["orders"][name]["order"], name
        assert rounds == g["orders"][name]["rounds"], name


def test_e3_single_kernel_hand_trace(golden):
    g = golden("e3_single_kernel.json")
    assert oracle.makespan(g["gpu"], g["kernels"], [0]) == g["makespan"]
    assert tick_makespan(g["gpu"], g["kernels"], [0]) == g["makespan"]


# ---------------------------------------------------------------- closed forms

def _occupancy(gpu, k):
    waves = int(k["waves_blk"])
    use = [int(k["regs_thr"]) * waves * gpu["wave_size"], int(k["lds_blk"]), waves, 1]
    caps = [gpu["reg_cu"], gpu["lds_cu"], gpu["wave_cu"], gpu["blk_cu"]]
    return min(c // u for c, u in zip(caps, use) if u > 0)


def test_single_kernel_closed_form():
    """One kernel alone: every execution round fills all CUs to the kernel's
    occupancy, so M = ceil(N_tblk / (occ * N_CU)) * d."""
    rng = np.random.default_rng(5)
    for model in (synth.SMALL_MODEL, synth.MI355X_MODEL, synth.GTX580_MODEL):
        gpu = model.as_dict()
        for _ in range(40):
            ks = synth.draw_kernels(rng, 1, 1, 3000)
            _, dur = oracle.derive(gpu, ks)
            occ = _occupancy(gpu, ks[0])
            want = -(-int(ks["n_tblk"][0]) // (occ * gpu["n_cu"])) * int(dur[0])
            assert oracle.makespan(gpu, ks, [0]) == want


def test_no_sharing_when_blocks_fit_one_per_cu():
    """Section 2 / Section 3: with at most N_SM blocks in total no SM is
    shared and the order has no effect: M = max d for every order."""
    rng = np.random.default_rng(7)
    gpu = synth.MI355X_MODEL.as_dict()
    for _ in range(6):
        n = int(rng.integers(2, 6))
        ks = synth.draw_kernels(rng, n, 1, 40)
        while ks["n_tblk"].sum() > gpu["n_cu"]:
            ks["n_tblk"] = np.maximum(1, ks["n_tblk"] // 2)
        _, dur = oracle.derive(gpu, ks)
        assert set(all_makespans(gpu, ks).tolist()) == {int(dur.max())}


def test_one_block_per_cu_equal_durations():
    """Section 3: blocks so heavy that a CU holds one at a time make the
    order irrelevant; with equal durations M = ceil(B / N_SM) * d."""
    rng = np.random.default_rng(11)
    gpu = synth.SMALL_MODEL.as_dict()
    for _ in range(5):
        n = int(rng.integers(2, 6))
        ks = synth.draw_kernels(rng, n, 1, 60)
        ks["lds_blk"] = rng.integers(gpu["lds_cu"] // 2 + 1, gpu["lds_cu"] + 1, size=n)
        ks["n_inst"] = 777
        ks["r_milli"] = gpu["rb_milli"]
        B = int(ks["n_tblk"].sum())
        want = -(-B // gpu["n_cu"]) * 777
        assert set(all_makespans(gpu, ks).tolist()) == {want}


def test_block_count_only_differences_do_not_matter():
    """Section 1 / Section 3: kernels identical except for their block counts
    give the same total time in every order."""
    rng = np.random.default_rng(13)
    for model in (synth.SMALL_MODEL, synth.MI355X_MODEL):
        gpu = model.as_dict()
        for _ in range(3):
            base = synth.draw_kernels(rng, 1, 8, 128)
            n = 6
            ks = np.repeat(base, n)
            ks["n_tblk"] = rng.integers(8, 400, size=n)
            ms = all_makespans(gpu, ks)
            assert ms.min() == ms.max()


def test_area_lower_bound_and_count_identities():
    """Per resource, resident use never exceeds N_CU * cap, so
    M >= max(max d, ceil(sum_i N_tblk_i d_i u_i / (N_CU cap)))."""
    rng = np.random.default_rng(17)
    gpu = synth.SMALL_MODEL.as_dict()
    caps = [gpu["reg_cu"], gpu["lds_cu"], gpu["wave_cu"], gpu["blk_cu"]]
    for _ in range(4):
        ks = synth.draw_kernels(rng, 5, 8, 128)
        use, dur = oracle.derive(gpu, ks)
        lb = int(dur.max())
        for x in range(4):
            area = sum(int(ks["n_tblk"][i]) * int(dur[i]) * int(use[i][x]) for i in range(5))
            lb = max(lb, -(-area // (gpu["n_cu"] * caps[x])))
        ms = all_makespans(gpu, ks)
        assert ms.min() >= lb
        st = ostats.set_stats(ms, ref=int(ms[7]))
        assert st["n_less"] + st["n_equal"] + st["n_greater"] == len(ms)
        assert ostats.histogram(ms, 64, st["min"], st["max"]).sum() == len(ms)


def test_cu_symmetry():
    """m identical CUs running m * c_i blocks per kernel behave like one CU
    running c_i blocks: every sweep gives each CU the same block."""
    rng = np.random.default_rng(19)
    for _ in range(8):
        one = dict(synth.SMALL_MODEL.as_dict(), n_cu=1)
        ks = synth.draw_kernels(rng, 4, 1, 6)
        m = int(rng.integers(2, 9))
        big = dict(one, n_cu=m)
        ks_m = ks.copy()
        ks_m["n_tblk"] = ks["n_tblk"] * m
        for order in itertools.permutations(range(4)):
            assert oracle.makespan(one, ks, order) == oracle.makespan(big, ks_m, order)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(12))
def test_tick_by_tick_matches_event_driven(seed):
    """An independent cycle-by-cycle formulation agrees on every order of
    tiny random sets."""
    rng = np.random.default_rng(100 + seed)
    model = synth.GpuModel(n_cu=int(rng.integers(1, 5)), wave_size=int(rng.integers(1, 5)),
                           wave_cu=int(rng.integers(2, 9)), blk_cu=int(rng.integers(1, 5)),
                           reg_cu=int(rng.integers(16, 200)), lds_cu=int(rng.integers(8, 100)),
                           rb_milli=1000)
    n = int(rng.integers(1, 6))
    ks = synth.random_tiny_set(rng, n, model, tblk_hi=6, inst_hi=12)
    gpu = model.as_dict()
    ev = all_makespans(gpu, ks)
    for r, order in enumerate(itertools.permutations(range(n))):
        assert tick_makespan(gpu, ks, order) == ev[r], (order, ks)


# ---------------------------------------------------------------- ranks

@pytest.mark.parametrize("n", range(1, 8))
def test_lehmer_matches_itertools(n):
    """itertools.permutations emits the lexicographic order."""
    for r, perm in enumerate(itertools.permutations(range(n))):
        assert oracle.unrank(n, r) == list(perm)
        assert oracle.rank(list(perm)) == r


def test_lehmer_large_n_edges():
    for n in (8, 12, 16, 20):
        f = math.factorial(n)
        assert oracle.unrank(n, 0) == list(range(n))
        assert oracle.unrank(n, f - 1) == list(range(n))[::-1]
        for r in (1, f // 3, f // 2 + 7, f - 2):
            assert oracle.rank(oracle.unrank(n, r)) == r


# ---------------------------------------------------------------- report formulas

def test_table3_derived_columns(golden):
    """Speedup over worst = T_worst / T_alg and deviation = (T_alg - T_opt) / T_opt
    reproduce every printed Table 3 entry to its printed digits."""
    t = golden("table3.json")
    for name, row in t["rows"].items():
        opt, worst, alg, pct, speedup, dev, n = row
        decimals = len(str(speedup).split(".")[1])
        assert round(ostats.speedup_over_worst(worst, alg), decimals) == pytest.approx(speedup), name
        d = 100 * ostats.deviation_from_optimal(opt, alg)
        dec = len(str(dev).split(".")[1])
        assert abs(d - dev) <= 0.5 * 10 ** -dec + 1e-12, name
        # the percentile is an exact count over the n orders
        assert any(math.floor(1000 * k / n + 0.5) / 10 == pct for k in range(n + 1)), name
        assert n == (720 if name != "EpBsEsSw-8" else math.factorial(8))


# ---------------------------------------------------------------- sampling

def test_splitmix64_published_vector():
    """First outputs of SplitMix64 seeded with 1234567 (Vigna's reference)."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [splitmix64_at(1234567, i) for i in range(5)] == want


def test_sampled_ranks_uniform():
    n_orders = 24
    counts = np.bincount([sampled_rank(99, 3, i, n_orders) for i in range(24000)],
                         minlength=n_orders)
    assert counts.min() > 0 and len(counts) == n_orders
    chi2 = ((counts - 1000.0) ** 2 / 1000.0).sum()
    assert chi2 < 60  # 23 degrees of freedom; p ~ 4e-5 at 60
    big = math.factorial(20)
    assert all(0 <= sampled_rank(5, 0, i, big) < big for i in range(1000))


# ---------------------------------------------------------------- heuristic properties

def test_heuristic_properties_random():
    rng = np.random.default_rng(23)
    for trial in range(200):
        model = (synth.SMALL_MODEL, synth.MI355X_MODEL, synth.GTX580_MODEL)[trial % 3]
        gpu = model.as_dict()
        n = int(rng.integers(1, 13))
        ks = synth.draw_kernels(rng, n, 1, 200)
        for flags in range(4):
            order, rounds = heuristic_order(gpu, ks, flags)
            assert sorted(order) == list(range(n))
            assert rounds == sorted(rounds)


def test_histogram_bins():
    ms = np.array([10, 10, 11, 13, 20], dtype=np.int64)
    h = ostats.histogram(ms, 4, 10, 20)
    # width 11: bins floor(0*4/11)=0, 0, floor(4/11)=0, floor(12/11)=1, floor(40/11)=3
    assert h.tolist() == [3, 1, 0, 1]


# ---------------------------------------------------------------- surrogate inputs

def test_lower_bound_hand_worked(golden):
    """The area lower bound on E1 (the longest block decides) and on E2 (the
    LDS area decides), worked by hand in tests/golden/features_lb.json."""
    from oracle import features as ofeat
    g = golden("features_lb.json")
    e1, e2 = golden("e1_two_cu.json"), golden("e2_heuristic.json")
    assert ofeat.lower_bound(e1["gpu"], e1["kernels"]) == g["e1"]["lower_bound"] == e1["lower_bound"]
    assert ofeat.lower_bound(e2["gpu"], e2["kernels"]) == g["e2"]["lower_bound"]
    # the bound is a bound: every order of E1 and E2 ends no earlier
    assert min(all_makespans(e1["gpu"], e1["kernels"])) >= g["e1"]["lower_bound"]
    assert min(all_makespans(e2["gpu"], e2["kernels"])) >= g["e2"]["lower_bound"]


def test_features_hand_worked(golden):
    """The 8 per-kernel features of E3's kernel and of E2's kernel 2 (whose
    ratio lies below R_B), worked by hand."""
    from oracle import features as ofeat
    g = golden("features_lb.json")
    e2, e3 = golden("e2_heuristic.json"), golden("e3_single_kernel.json")
    got = ofeat.features(e3["gpu"], e3["kernels"])[0]
    assert got == pytest.approx(g["e3_kernel"]["features"], rel=1e-12, abs=1e-15)
    got = ofeat.features(e2["gpu"], e2["kernels"])[2]
    assert got == pytest.approx(g["e2_k2"]["features"], rel=1e-12, abs=1e-15)


def test_sampled_rank_from_published_outputs(golden):
    """Ranks of the first two SplitMix64 outputs for seed 1234567 under the
    multiply-shift range reduction, worked out in tests/golden/sampled_rank.json."""
    g = golden("sampled_rank.json")
    for s in g["samples"]:
        assert splitmix64_at(g["seed"], s["index"]) == s["x"]
        for n_orders, want in s["ranks"].items():
            assert sampled_rank(g["seed"], g["set"], s["index"], int(n_orders)) == want


def test_ranking_curve_and_median_gain_hand_worked():
    """Figure 1's ranking and Section 6's median gain on arrays small enough
    to work by hand.  [3, 1, 3, 1]: ascending 1, 1, 3, 3 from ranks 1, 3, 0, 2
    (ties by smaller rank).  Median gain of [5, 1, 4, 2, 3] against t_alg = 2:
    3 of 5 orders take >= 3 (at least half), only 2 take >= 4, so the gain is
    3/2 - 1 = 0.5; with [1, 2, 3, 4] two of four take >= 3, again 0.5; with
    every order equal to t_alg it is 0."""
    v, r = ostats.ranking_curve([3, 1, 3, 1])
    assert v.tolist() == [1, 1, 3, 3] and r.tolist() == [1, 3, 0, 2]
    assert ostats.median_gain([5, 1, 4, 2, 3], 2) == 0.5
    assert ostats.median_gain([1, 2, 3, 4], 2) == 0.5
    assert ostats.median_gain([7] * 9, 7) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_median_gain_is_the_half_probability_threshold(seed):
    """The defining property by brute force over every candidate gain: at the
    returned g at least half the orders are >= (1 + g) * t_alg, and at any
    larger makespan threshold fewer than half are."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    m = rng.integers(10, 20, n)
    t_alg = int(rng.integers(8, 15))
    g = ostats.median_gain(m, t_alg)
    thr = round((1 + g) * t_alg)
    assert 2 * int((m >= thr).sum()) >= n
    for v in range(thr + 1, 21):
        assert 2 * int((m >= v).sum()) < n


def test_beam_step_oracle_hand_example():
    """One beam step on n = 4, by hand.  Prefixes [2, 0] and [1, 3] (d = 2):
    their unused kernels are {1, 3} and {0, 2}, so the candidates are
    [2,0,1], [2,0,3], [1,3,0], [1,3,2] in that order, with positions (per
    kernel 0..3): [1,2,0,16], [1,16,0,2], [2,0,16,1], [16,0,2,1].  With
    scores [5, 3, 3, 4] and at most one child per prefix, the survivors are
    candidate 1 (3 < 5) and candidate 2 (3 < 4); the others become +inf."""
    from oracle import beam
    pos, parent, kernel = beam.expand(np.array([[2, 0], [1, 3]]), 4)
    assert pos.tolist() == [[1, 2, 0, 16], [1, 16, 0, 2], [2, 0, 16, 1], [16, 0, 2, 1]]
    assert parent.tolist() == [0, 0, 1, 1] and kernel.tolist() == [1, 3, 0, 2]
    ruled = beam.cap(np.array([5, 3, 3, 4], dtype=np.float32), 2, 1)
    assert ruled.tolist() == [math.inf, 3.0, 3.0, math.inf]
    # ties go to the first candidate of a prefix
    assert beam.cap(np.array([2, 2, 7, 7], dtype=np.float32), 2, 1).tolist() == [2.0, math.inf, 7.0, math.inf]
    assert beam.gather(np.array([[2, 0], [1, 3]]), parent, kernel, [2, 1]).tolist() == [[1, 3, 0], [2, 0, 3]]
    # the empty prefix expands to every kernel at position 0
    pos0, parent0, kernel0 = beam.expand(np.zeros((1, 0), dtype=np.int64), 3)
    assert pos0.tolist() == [[0, 16, 16], [16, 0, 16], [16, 16, 0]] and kernel0.tolist() == [0, 1, 2]


def test_beam_gumbel_noise_is_a_gumbel_variate():
    """The noise maps SplitMix64's top 24 bits u to -log(-log u): pinned by the
    published first SplitMix64 output for seed 1234567 (u = its top 24 bits
    over 2^24) and by the Gumbel law's mean (the Euler-Mascheroni constant)
    and variance (pi^2 / 6) over many counters."""
    from oracle import beam
    x = 6457827717110365317
    u = ((x >> 40) + 0.5) / 2 ** 24
    # float32 steps: within a few float32 ulps of the float64 value
    assert beam.gumbel(1234567, 0) == pytest.approx(-math.log(-math.log(u)), rel=1e-5)
    g = np.array([beam.gumbel(99, c) for c in range(20000)])
    assert abs(g.mean() - 0.5772156649) < 0.03
    assert abs(g.var() - math.pi ** 2 / 6) < 0.08
