"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Makespans, counts, extremes and histograms are integers and must match
bit for bit.  Each case prints its name, workload and sizes before it runs.
"""

import itertools
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import stats as ostats
from oracle.heuristic import heuristic_order as oracle_heuristic
from oracle.sampling import sampled_rank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")

INT64_MAX = (1 << 63) - 1
INT64_MIN = -(1 << 63)


def say(*a):
    print("[gpu-parity]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def run_batch(gpu, sets, spec, *, ref=None, want_makespans=True, want_stats=True, n_bins=0):
    """Evaluate a batch on the GPU.  Returns (makespans, stats records, hist)."""
    kernels = np.concatenate([ko.kernel_array(s) for s in sets])
    offsets = np.zeros(len(sets) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(s) for s in sets])
    per, total = ko.ko_count_orders(offsets, spec)
    dev = torch.device("cuda:0")
    ms = torch.full((max(total, 1),), -7, dtype=torch.int64, device=dev) if want_makespans else None
    st = torch.zeros(8 * len(sets), dtype=torch.int64, device=dev) if want_stats else None
    hist = torch.zeros(len(sets) * n_bins, dtype=torch.int64, device=dev) if n_bins else None
    ref_t = torch.tensor(ref, dtype=torch.int64, device=dev) if ref is not None else None
    ko.ko_simulate_batch(gpu, kernels, offsets, spec, ref_makespan=ref_t, makespans=ms, stats=st,
                         hist=hist, n_bins=n_bins)
    ko.ko_sync()
    out_ms = ms.cpu().numpy()[:total] if want_makespans else None
    out_st = ko.stats_records(st) if want_stats else None
    out_h = hist.cpu().numpy().view(np.uint64).reshape(len(sets), n_bins) if n_bins else None
    return out_ms, out_st, out_h, per


def expect_stats(rec, ms, ref=None, index_base=0):
    want = ostats.set_stats(ms, ref=ref)
    assert rec["min_makespan"] == want["min"]
    assert rec["max_makespan"] == want["max"]
    assert rec["argmin"] == want["argmin"] + index_base
    assert rec["argmax"] == want["argmax"] + index_base
    assert rec["n_orders"] == len(ms)
    if ref is not None:
        assert (rec["n_less"], rec["n_equal"], rec["n_greater"]) == (
            want["n_less"], want["n_equal"], want["n_greater"])


# ------------------------------------------------------------------ tiny workload

def test_tiny_workload_full_enumeration():
    """One set of n=6 on the 16-CU model: all 720 orders, stats, histogram and
    the heuristic order's percentile."""
    w = synth.WORKLOADS[0]
    gpu = w.model.as_dict()
    ks = synth.draw_set(0, 0)
    say("tiny n=6 all orders")
    want = oracle.makespans_all(gpu, ks)
    h_order = oracle_heuristic(gpu, ks)[0]
    ref = oracle.makespan(gpu, ks, h_order)
    ms, st, hist, _ = run_batch(w.model, [ks], ko.OrderSpec.all(), ref=[ref], n_bins=64)
    assert np.array_equal(ms, want)
    expect_stats(st[0], want, ref=ref)
    assert np.array_equal(hist[0], ostats.histogram(want, 64, want.min(), want.max()))
    # the heuristic's rank through the one-call entry point
    assert ko.ko_heuristic_order(w.model, ks) == h_order
    r = ko.ko_rank_percentile(w.model, ks, h_order)
    counts = ostats.set_stats(want, ref=ref)
    assert r["makespan"] == ref
    assert (r["n_less"], r["n_equal"], r["n_greater"], r["n_total"]) == (
        counts["n_less"], counts["n_equal"], counts["n_greater"], 720)
    pct = ostats.percentiles(counts["n_less"], counts["n_equal"], counts["n_greater"])
    assert r["pct_inclusive"] == pytest.approx(pct["inclusive"], abs=1e-9)
    assert r["pct_strict"] == pytest.approx(pct["strict"], abs=1e-9)
    assert r["pct_mid"] == pytest.approx(pct["mid"], abs=1e-9)
    assert (r["min_makespan"], r["max_makespan"]) == (want.min(), want.max())


def test_hand_traced_examples_on_gpu(golden):
    e1 = golden("e1_two_cu.json")
    ms, st, _, _ = run_batch(e1["gpu"], [e1["kernels"]], ko.OrderSpec.all())
    assert ms.tolist() == e1["makespans_by_rank"]
    e3 = golden("e3_single_kernel.json")
    ms, _, _, _ = run_batch(e3["gpu"], [e3["kernels"]], ko.OrderSpec.all())
    assert ms.tolist() == [e3["makespan"]]


# ------------------------------------------------------------------ n=10 workload

def test_full_enum_workload_rank_ranges():
    """The n=10, 256-CU set: rank windows at the start, middle and end of the
    3,628,800 orders, each spanning several work chunks with ragged ends."""
    w = synth.WORKLOADS[1]
    gpu = w.model.as_dict()
    ks = synth.draw_set(1, 0)
    N = math.factorial(10)
    windows = [(0, 1500), (N // 2 - 333, N // 2 + 900), (N - 1217, N)]
    for lo, hi in windows:
        say(f"n=10 ranks [{lo}, {hi})")
        want = oracle.makespans_range(gpu, ks, lo, hi - lo)
        ms, st, _, _ = run_batch(w.model, [ks], ko.OrderSpec.rank_range([[lo, hi]]))
        assert np.array_equal(ms, want), (lo, hi)
        expect_stats(st[0], want, index_base=lo)


def test_full_enum_workload_sampled_and_explicit():
    w = synth.WORKLOADS[1]
    gpu = w.model.as_dict()
    ks = synth.draw_set(1, 0)
    N = math.factorial(10)
    seed = 0xC0FFEE
    say("n=10 sampled 1200")
    ranks = [sampled_rank(seed, 0, i, N) for i in range(1200)]
    want = oracle.makespans_ranks(gpu, ks, ranks)
    ms, st, _, _ = run_batch(w.model, [ks], ko.OrderSpec.sampled([1200], seed))
    assert np.array_equal(ms, want)
    expect_stats(st[0], want)
    say("n=10 explicit 900")
    rng = np.random.default_rng(4)
    orders = np.stack([rng.permutation(10) for _ in range(900)]).astype(np.uint8)
    want = oracle.makespans_orders(gpu, ks, orders.astype(np.int32))
    dev_orders = torch.from_numpy(orders.ravel().copy()).to("cuda:0")
    ref = int(want[17])
    ms, st, _, _ = run_batch(w.model, [ks], ko.OrderSpec.explicit(dev_orders, [900]), ref=[ref])
    assert np.array_equal(ms, want)
    expect_stats(st[0], want, ref=ref)


# ------------------------------------------------------------------ batched workload

def test_batch_workload_many_sets():
    """Sets of the 4096-set batch (n = 4..9): complete enumeration of the
    small sets and rank windows of the large ones, all in one call."""
    w = synth.WORKLOADS[2]
    gpu = w.model.as_dict()
    small, large = [], []
    s = 0
    while len(small) < 24 or len(large) < 4:
        ks = synth.draw_set(2, s)
        (small if len(ks) <= 6 else large).append((s, ks))
        s += 1
    small, large = small[:24], large[:4]
    say(f"batch: {len(small)} small sets (all orders)")
    sets = [k for _, k in small]
    want = [oracle.makespans_all(gpu, k) for k in sets]
    refs = [int(m[len(m) // 3]) for m in want]
    ms, st, hist, per = run_batch(w.model, sets, ko.OrderSpec.all(), ref=refs, n_bins=32)
    off = np.concatenate([[0], np.cumsum(np.asarray(per, dtype=np.int64))])
    for i, m in enumerate(want):
        assert np.array_equal(ms[off[i]:off[i + 1]], m), small[i][0]
        expect_stats(st[i], m, ref=refs[i])
        assert np.array_equal(hist[i], ostats.histogram(m, 32, m.min(), m.max()))
    say(f"batch: {len(large)} large sets (rank windows)")
    sets = [k for _, k in large]
    lohi = []
    for k in sets:
        N = math.factorial(len(k))
        lohi.append([N // 3, N // 3 + 700])
    ms, st, _, per = run_batch(w.model, sets, ko.OrderSpec.rank_range(lohi))
    off = np.concatenate([[0], np.cumsum(np.asarray(per, dtype=np.int64))])
    for i, k in enumerate(sets):
        m = oracle.makespans_range(gpu, k, lohi[i][0], 700)
        assert np.array_equal(ms[off[i]:off[i + 1]], m)
        expect_stats(st[i], m, index_base=lohi[i][0])


# ------------------------------------------------------------------ edge cases

@pytest.mark.parametrize("n_cu", [1, 3, 16, 63, 64, 65, 127, 128, 129, 200, 255, 256])
def test_random_models_all_orders(n_cu):
    """Random small sets on models whose CU count exercises 1, 2 and 4 CU
    slots per lane and partial last slots."""
    rng = np.random.default_rng(1000 + n_cu)
    for trial in range(3):
        model = synth.GpuModel(n_cu=n_cu, wave_size=int(rng.choice([32, 64])),
                               wave_cu=int(rng.integers(4, 65)), blk_cu=int(rng.integers(1, 33)),
                               reg_cu=int(rng.choice([32768, 65536, 131072])),
                               lds_cu=int(rng.choice([49152, 65536, 163840])),
                               rb_milli=int(rng.integers(1000, 12000)))
        n = int(rng.integers(1, 6))
        ks = synth.draw_kernels(rng, n, 1, 3 * n_cu)
        ks["waves_blk"] = np.minimum(ks["waves_blk"], model.wave_cu)
        ks["regs_thr"] = np.minimum(ks["regs_thr"], model.reg_cu // (ks["waves_blk"] * model.wave_size))
        ks["lds_blk"] = np.minimum(ks["lds_blk"], model.lds_cu)
        say(f"random model n_cu={n_cu} blk_cu={model.blk_cu} n={n}")
        gpu = model.as_dict()
        want = oracle.makespans_all(gpu, ks)
        ms, st, _, _ = run_batch(model, [ks], ko.OrderSpec.all())
        assert np.array_equal(ms, want), (trial, ks)
        expect_stats(st[0], want)


def test_tiny_sets_brute_force_models():
    """Very small resource limits (blocks pack 1..8 per CU, many releases)."""
    rng = np.random.default_rng(77)
    for trial in range(20):
        model = synth.GpuModel(n_cu=int(rng.integers(1, 6)), wave_size=int(rng.integers(1, 5)),
                               wave_cu=int(rng.integers(2, 9)), blk_cu=int(rng.integers(1, 5)),
                               reg_cu=int(rng.integers(16, 200)), lds_cu=int(rng.integers(8, 100)),
                               rb_milli=1000)
        n = int(rng.integers(1, 6))
        ks = synth.random_tiny_set(rng, n, model, tblk_hi=9, inst_hi=30)
        want = oracle.makespans_all(model.as_dict(), ks)
        ms, _, _, _ = run_batch(model, [ks], ko.OrderSpec.all())
        assert np.array_equal(ms, want), (trial, model, ks)


def test_single_kernel_and_empty_sampled_set():
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)[:1]
    say("single kernel; a set with zero sampled orders")
    want = oracle.makespan(w.model.as_dict(), ks, [0])
    ms, st, _, _ = run_batch(w.model, [ks, synth.draw_set(1, 0)[:3]], ko.OrderSpec.sampled([5, 0], 9))
    assert ms.tolist() == [want] * 5
    assert st[1]["n_orders"] == 0
    assert st[1]["min_makespan"] == INT64_MAX and st[1]["max_makespan"] == INT64_MIN


def test_twenty_kernels_sampled():
    """The largest set size: 20 kernels, sampled ranks."""
    rng = np.random.default_rng(20)
    model = synth.MI355X_MODEL
    ks = synth.draw_kernels(rng, 20, 64, 2048)
    N = math.factorial(20)
    ranks = [sampled_rank(3, 0, i, N) for i in range(64)]
    say("n=20 sampled 64")
    want = oracle.makespans_ranks(model.as_dict(), ks, ranks)
    ms, _, _, _ = run_batch(model, [ks], ko.OrderSpec.sampled([64], 3))
    assert np.array_equal(ms, want)


def test_deterministic_repeat():
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    say("repeat determinism")
    a, sa, _, _ = run_batch(w.model, [ks], ko.OrderSpec.rank_range([[123456, 223456]]))
    b, sb, _, _ = run_batch(w.model, [ks], ko.OrderSpec.rank_range([[123456, 223456]]))
    assert np.array_equal(a, b) and np.array_equal(sa, sb)


def test_explicit_non_permutation_reports_device_status():
    """A malformed explicit order (kernel index repeated) is reported as a
    device status error by the next synchronisation, and the next call runs
    cleanly again."""
    w = synth.WORKLOADS[0]
    ks = synth.draw_set(0, 0)
    bad = torch.tensor([0, 1, 2, 3, 4, 4], dtype=torch.uint8, device="cuda:0")
    kernels = ko.kernel_array(ks)
    ms = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    ko.ko_simulate_batch(w.model, kernels, [0, 6], ko.OrderSpec.explicit(bad, [1]), makespans=ms)
    with pytest.raises(ko.KoError) as e:
        ko.ko_sync()
    assert e.value.code == ko.KO_EHIP
    ms2, _, _, _ = run_batch(w.model, [ks], ko.OrderSpec.rank_range([[0, 10]]))
    assert np.array_equal(ms2, oracle.makespans_range(w.model.as_dict(), ks, 0, 10))


# ------------------------------------------------------------------ full size

def oracle_threads():
    """The oracle's worker threads: every host core, at most the 16 that one
    GPU's share of a box holds."""
    return min(16, oracle.default_threads())


def test_full_size_n10_all_orders_against_oracle():
    """All 3,628,800 orders of the n=10 set in the configuration the benchmark
    times, element by element against the oracle's full enumeration (Section
    6's exhaustive evaluation); extremes, argmin/argmax ranks, the histogram
    and Algorithm 1's rank counts all come from the oracle's array."""
    w = synth.WORKLOADS[1]
    gpu = w.model.as_dict()
    ks = synth.draw_set(1, 0)
    N = math.factorial(10)
    h_order = ko.ko_heuristic_order(w.model, ks)
    assert h_order == oracle_heuristic(gpu, ks)[0]
    ref = oracle.makespan(gpu, ks, h_order)
    say("n=10 all 3,628,800 orders: oracle")
    want = oracle.makespans_all(gpu, ks, threads=oracle_threads())
    say("n=10 all 3,628,800 orders: GPU")
    ms, st, hist, _ = run_batch(w.model, [ks], ko.OrderSpec.all(), ref=[ref], n_bins=1024)
    assert len(ms) == N
    bad = np.flatnonzero(ms != want)
    assert bad.size == 0, f"{bad.size} makespans differ, first at rank {bad[:1]}"
    o = ostats.set_stats(want, ref=ref)
    rec = st[0]
    assert rec["n_orders"] == N
    assert (rec["min_makespan"], rec["max_makespan"]) == (o["min"], o["max"])
    assert (rec["argmin"], rec["argmax"]) == (o["argmin"], o["argmax"])
    assert (rec["n_less"], rec["n_equal"], rec["n_greater"]) == (o["n_less"], o["n_equal"], o["n_greater"])
    assert np.array_equal(hist[0], ostats.histogram(want, 1024, o["min"], o["max"]))
    r = ko.ko_rank_percentile(w.model, ks, h_order)
    assert r["makespan"] == ref
    assert (r["n_less"], r["n_equal"], r["n_greater"]) == (o["n_less"], o["n_equal"], o["n_greater"])
    # Figure 1's ranking curve (device sort) and Section 6's median gain
    say("n=10 ranking curve")
    curve, ranks = ko.ranking_curve(torch.from_numpy(ms).to("cuda:0"))
    want_curve, want_ranks = ostats.ranking_curve(want)
    assert np.array_equal(curve.cpu().numpy(), want_curve)
    assert np.array_equal(ranks.cpu().numpy(), want_ranks)
    assert ko.median_gain(torch.from_numpy(ms).to("cuda:0"), ref) == ostats.median_gain(want, ref)


def test_batch_sets_n7_to_n9_full_enumeration_against_oracle():
    """A stratified subset of the 4096-set batch: the first six sets of each
    size n = 7, 8 and 9 in one call, every order of each set element by
    element against the oracle, with Algorithm 1's order as each set's
    reference (Table 3's percentile) and per-set statistics from the oracle."""
    w = synth.WORKLOADS[2]
    gpu = w.model.as_dict()
    picked = {7: [], 8: [], 9: []}
    s = 0
    while any(len(v) < 6 for v in picked.values()):
        ks = synth.draw_set(2, s)
        if len(ks) in picked and len(picked[len(ks)]) < 6:
            picked[len(ks)].append((s, ks))
        s += 1
    sets = [ks for n in (7, 8, 9) for _, ks in picked[n]]
    say("batch sets", [i for n in (7, 8, 9) for i, _ in picked[n]], "n = 7, 8, 9: oracle")
    refs, wants = [], []
    for ks in sets:
        refs.append(oracle.makespan(gpu, ks, oracle_heuristic(gpu, ks)[0]))
        wants.append(oracle.makespans_all(gpu, ks, threads=oracle_threads()))
    say("batch sets n = 7, 8, 9: GPU")
    ms, st, hist, per = run_batch(w.model, sets, ko.OrderSpec.all(), ref=refs, n_bins=256)
    off = 0
    for i, (ks, want, ref) in enumerate(zip(sets, wants, refs)):
        got = ms[off:off + len(want)]
        off += len(want)
        assert per[i] == len(want) == math.factorial(len(ks))
        assert np.array_equal(got, want), f"set {i} (n={len(ks)})"
        o = ostats.set_stats(want, ref=ref)
        rec = st[i]
        assert (rec["min_makespan"], rec["max_makespan"], rec["argmin"], rec["argmax"]) == \
            (o["min"], o["max"], o["argmin"], o["argmax"])
        assert (rec["n_less"], rec["n_equal"], rec["n_greater"]) == (o["n_less"], o["n_equal"], o["n_greater"])
        assert np.array_equal(hist[i], ostats.histogram(want, 256, o["min"], o["max"]))
    assert off == len(ms)


@pytest.mark.parametrize("workload,n_samples", [(13, 65536), (4, 16384)])
def test_rank_percentile_sampled_against_oracle(workload, n_samples):
    """Percentile of Algorithm 1's order over sampled orders (Section 6's
    random order choice), the only percentile there is for n = 16: the counts
    equal the oracle's over the same counter-based sample ranks."""
    w = synth.WORKLOADS[workload]
    gpu = w.model.as_dict()
    ks = synth.draw_set(workload, 0)
    n = len(ks)
    seed = 0x5EED0000 + n
    order = oracle_heuristic(gpu, ks)[0]
    ref = oracle.makespan(gpu, ks, order)
    ranks = np.array([sampled_rank(seed, 0, i, math.factorial(n)) for i in range(n_samples)],
                     dtype=np.uint64)
    say(f"sampled percentile n={n}, {n_samples} samples: oracle")
    want = oracle.makespans_ranks(gpu, ks, ranks, threads=oracle_threads())
    say(f"sampled percentile n={n}: GPU")
    r = ko.ko_rank_percentile(w.model, ks, order, n_samples=n_samples, seed=seed)
    assert r["makespan"] == ref
    assert r["n_total"] == n_samples
    assert (r["min_makespan"], r["max_makespan"]) == (int(want.min()), int(want.max()))
    assert (r["n_less"], r["n_equal"], r["n_greater"]) == \
        (int((want < ref).sum()), int((want == ref).sum()), int((want > ref).sum()))
    o = ostats.percentiles(int((want < ref).sum()), int((want == ref).sum()), int((want > ref).sum()))
    assert r["pct_inclusive"] == pytest.approx(o["inclusive"], abs=1e-9)


# ------------------------------------------------------------------ degenerate cases

def test_identical_kernels_every_order_ties():
    """A set of identical kernels: every launch order is the same sequence of
    blocks, so all n! makespans are equal (and equal the oracle's)."""
    w = synth.WORKLOADS[1]
    k0 = synth.draw_set(1, 3)[:1]
    ks = np.concatenate([k0] * 7)
    say("identical kernels n=7")
    ms, st, hist, _ = run_batch(w.model, [ks], ko.OrderSpec.all(), ref=[0], n_bins=8)
    want = oracle.makespan(w.model.as_dict(), ks, list(range(7)))
    assert np.all(ms == want) and len(ms) == math.factorial(7)
    rec = st[0]
    assert rec["min_makespan"] == rec["max_makespan"] == want
    assert rec["argmin"] == 0 and rec["argmax"] == 0
    assert int(hist[0][0]) == math.factorial(7) and int(hist[0][1:].sum()) == 0


def test_blocks_on_distinct_cus_make_order_irrelevant():
    """Total blocks <= N_CU with one block per CU: every block starts at
    cycle 0 on its own CU, so the makespan is the longest block duration for
    every order."""
    model = synth.MI355X_MODEL
    rng = np.random.default_rng(5)
    ks = synth.draw_kernels(rng, 6, 10, 40)  # 6 kernels x <= 40 blocks <= 240 CUs
    assert int(ks["n_tblk"].sum()) <= model.n_cu
    say("blocks on distinct CUs")
    ms, _, _, _ = run_batch(model, [ks], ko.OrderSpec.all())
    _, dur = oracle.derive(model.as_dict(), ks)
    assert np.all(ms == int(max(dur)))
