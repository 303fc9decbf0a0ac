"""GPU tests of the lane engine: one launch order per lane, CU states as runs.

The lane engine and the wave engine evaluate the same model with different
storage, so they must agree bit for bit: makespans, per-set statistics and
histograms, on every workload and order mode.  Makespans are also checked
against the CPU oracle on sampled orders.  With the per-lane entry capacity cut
down, work items overflow and are handed to the wave engine; results must not
change.  Each case prints its name and sizes before it runs.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle.sampling import sampled_rank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")
kb = pytest.importorskip("paper_1511_07983_amd.batch")

DEV = "cuda:0"


def say(*a):
    print("[lanes-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def run(model, sets, spec, engine, *, ref=None, n_bins=0, lane_entries=0, chunk_log2=0):
    kernels, offsets = kb.concat_sets(sets)
    plan = ko.Plan(model, kernels, offsets, spec, chunk_log2=chunk_log2, engine=engine,
                   lane_entries=lane_entries)
    n = len(sets)
    ms = torch.full((max(plan.total_orders, 1),), -7, dtype=torch.int64, device=DEV)
    st = torch.zeros(8 * n, dtype=torch.int64, device=DEV)
    h = torch.zeros(max(n * n_bins, 1), dtype=torch.int64, device=DEV) if n_bins else None
    r = torch.tensor(ref, dtype=torch.int64, device=DEV) if ref is not None else None
    plan.launch(ref_makespan=r, makespans=ms, stats=st, hist=h, n_bins=n_bins)
    plan.status()
    info = plan.engine()
    plan.close()
    return ms.cpu().numpy()[:plan.total_orders], st.cpu().numpy(), (h.cpu().numpy() if h is not None else None), info


def both(model, sets, spec, **kw):
    """Both engines on the same batch; asserts equality and returns the lane run."""
    w = run(model, sets, spec, ko.ENGINE_WAVE, **kw)
    lanes = run(model, sets, spec, ko.ENGINE_LANES, **kw)
    assert w[3][0] == ko.ENGINE_WAVE and lanes[3][0] == ko.ENGINE_LANES
    assert np.array_equal(lanes[0], w[0]), np.flatnonzero(lanes[0] != w[0])[:10]
    assert np.array_equal(lanes[1], w[1])
    if w[2] is not None:
        assert np.array_equal(lanes[2], w[2])
    return lanes


def test_tiny_workload_all_orders_against_oracle():
    w = synth.WORKLOADS[0]
    ks = synth.draw_set(0, 0)
    say("tiny n=6, 16-CU model, all orders, both engines")
    want = oracle.makespans_all(w.model.as_dict(), ks)
    ms, st, h, info = both(w.model, [ks], ko.OrderSpec.all(), ref=[int(want[100])], n_bins=64)
    assert np.array_equal(ms, want)


def test_n10_rank_window_against_oracle():
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    N = math.factorial(10)
    lo, cnt = N // 2 - 9000, 20000
    say(f"n=10 rank window [{lo}, {lo + cnt}), both engines")
    ms, st, _, info = both(w.model, [ks], ko.OrderSpec.rank_range([[lo, lo + cnt]]), n_bins=16)
    rng = np.random.default_rng(10)
    pick = np.sort(rng.choice(cnt, 200, replace=False))
    want = oracle.makespans_ranks(w.model.as_dict(), ks, [lo + int(i) for i in pick])
    assert np.array_equal(ms[pick], want)
    assert info[3] == 0, "no work item should be re-run whole at full capacity"


def test_batch_sets_all_orders():
    w = synth.WORKLOADS[2]
    sets = [synth.draw_set(2, s) for s in range(96)]
    say(f"batch: {len(sets)} sets (n = 4..9), all orders, both engines")
    refs = [2_000_000 + 10_000 * s for s in range(len(sets))]
    ms, st, h, info = both(w.model, sets, ko.OrderSpec.all(), ref=refs, n_bins=32)
    off = np.concatenate([[0], np.cumsum([math.factorial(len(k)) for k in sets])])
    for s, k in enumerate(sets):
        if len(k) <= 5:
            assert np.array_equal(ms[off[s]:off[s + 1]], oracle.makespans_all(w.model.as_dict(), k)), s


@pytest.mark.parametrize("workload,per_set,n_sets", [(3, 4096, 6), (4, 2048, 4), (15, 8192, 3)])
def test_sampled_orders_large_sets(workload, per_set, n_sets):
    w = synth.WORKLOADS[workload]
    sets = [synth.draw_set(workload, s) for s in range(n_sets)]
    n = len(sets[0])
    say(f"{w.name}: {n_sets} sets x {per_set} sampled orders (n={n}), both engines")
    ms, st, _, info = both(w.model, sets, ko.OrderSpec.sampled([per_set] * n_sets, 11))
    N = math.factorial(n)
    for s in range(n_sets):
        idx = list(range(0, per_set, per_set // 16))
        want = oracle.makespans_ranks(w.model.as_dict(), sets[s], [sampled_rank(11, s, i, N) for i in idx])
        assert np.array_equal(ms[s * per_set + np.array(idx)], want), s


def test_explicit_orders():
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    rng = np.random.default_rng(5)
    orders = np.array([rng.permutation(10) for _ in range(3000)], dtype=np.uint8)
    say("explicit: 3000 orders of the n=10 set, both engines")
    flat = torch.from_numpy(orders.ravel().copy()).to(DEV)
    ms, st, _, _ = both(w.model, [ks], ko.OrderSpec.explicit(flat, [len(orders)]))
    want = oracle.makespans_orders(w.model.as_dict(), ks, orders[:100])
    assert np.array_equal(ms[:100], want)


@pytest.mark.parametrize("n_cu", [1, 5, 16, 64, 100, 255, 256])
def test_random_models(n_cu):
    """Random small models and sets: both engines and the oracle, all orders."""
    rng = np.random.default_rng(4000 + n_cu)
    for trial in range(3):
        model = synth.GpuModel(n_cu=n_cu, wave_size=int(rng.choice([32, 64])),
                               wave_cu=int(rng.integers(4, 65)), blk_cu=int(rng.integers(1, 33)),
                               reg_cu=int(rng.choice([32768, 65536, 131072])),
                               lds_cu=int(rng.choice([49152, 65536, 163840])),
                               rb_milli=int(rng.integers(1000, 12000)))
        n = int(rng.integers(1, 7))
        ks = synth.draw_kernels(rng, n, 1, 3 * n_cu)
        ks["waves_blk"] = np.minimum(ks["waves_blk"], model.wave_cu)
        ks["regs_thr"] = np.minimum(ks["regs_thr"], model.reg_cu // (ks["waves_blk"] * model.wave_size))
        ks["lds_blk"] = np.minimum(ks["lds_blk"], model.lds_cu)
        say(f"random model n_cu={n_cu} blk_cu={model.blk_cu} n={n}")
        ms, st, _, _ = both(model, [ks], ko.OrderSpec.all())
        assert np.array_equal(ms, oracle.makespans_all(model.as_dict(), ks)), (trial, ks)


def test_tiny_resource_models():
    """Very small limits: 1..8 blocks per CU and many releases per order."""
    rng = np.random.default_rng(78)
    for trial in range(12):
        model = synth.GpuModel(n_cu=int(rng.integers(1, 9)), wave_size=int(rng.integers(1, 5)),
                               wave_cu=int(rng.integers(2, 9)), blk_cu=int(rng.integers(1, 5)),
                               reg_cu=int(rng.integers(16, 200)), lds_cu=int(rng.integers(8, 100)),
                               rb_milli=1000)
        n = int(rng.integers(1, 6))
        ks = synth.random_tiny_set(rng, n, model, tblk_hi=9, inst_hi=30)
        say(f"tiny model trial {trial}: n_cu={model.n_cu} n={n}")
        ms, _, _, _ = both(model, [ks], ko.OrderSpec.all())
        assert np.array_equal(ms, oracle.makespans_all(model.as_dict(), ks)), (trial, model, ks)


@pytest.mark.parametrize("entries", [1, 2, 5])
def test_overflowing_orders_are_spilled_to_the_wave_engine(entries):
    """With 1..5 group entries per lane most orders overflow: they are recorded,
    evaluated one wavefront each and folded into the statistics; every output
    is unchanged."""
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    lo, cnt = 123_456, 6000
    say(f"lane entries={entries}: n=10 window of {cnt} orders")
    spec = ko.OrderSpec.rank_range([[lo, lo + cnt]])
    wave = run(w.model, [ks], spec, ko.ENGINE_WAVE, ref=[2_600_000], n_bins=8, chunk_log2=8)
    lanes = run(w.model, [ks], spec, ko.ENGINE_LANES, ref=[2_600_000], n_bins=8, chunk_log2=8,
                lane_entries=entries)
    assert lanes[3][1] == entries
    assert lanes[3][2] > 0, "expected spilled orders"
    assert np.array_equal(lanes[0], wave[0])
    assert np.array_equal(lanes[1], wave[1])
    assert np.array_equal(lanes[2], wave[2])


@pytest.mark.parametrize("mode", ["range", "sampled", "explicit"])
def test_full_spill_list_hands_whole_items_over(mode):
    """More spilled orders than the record list holds (65,536): the rest of
    those orders' work items are re-run whole, records of such items are
    ignored, and every output is unchanged, in each order mode."""
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    cnt = 80_000
    say(f"one entry per lane, {cnt} orders ({mode}): spill list overflows")
    if mode == "range":
        spec = ko.OrderSpec.rank_range([[777, 777 + cnt]])
    elif mode == "sampled":
        spec = ko.OrderSpec.sampled([cnt], 5)
    else:
        rng = np.random.default_rng(9)
        orders = np.array([rng.permutation(10) for _ in range(cnt)], dtype=np.uint8)
        spec = ko.OrderSpec.explicit(torch.from_numpy(orders.ravel().copy()).to(DEV), [cnt])
    wave = run(w.model, [ks], spec, ko.ENGINE_WAVE, ref=[2_600_000], n_bins=8, chunk_log2=9)
    lanes = run(w.model, [ks], spec, ko.ENGINE_LANES, ref=[2_600_000], n_bins=8, chunk_log2=9,
                lane_entries=1)
    assert lanes[3][2] > 65_536 and lanes[3][3] > 0, lanes[3]
    assert np.array_equal(lanes[0], wave[0])
    assert np.array_equal(lanes[1], wave[1])
    assert np.array_equal(lanes[2], wave[2])


def test_spilled_orders_across_sets_fold_into_their_own_set():
    """A batch of sets with few entries per lane: spilled orders of different
    sets must reach their own set's statistics."""
    w = synth.WORKLOADS[2]
    sets = [synth.draw_set(2, s) for s in range(24)]
    say("24 batch sets, 3 entries per lane")
    refs = [2_000_000 + 15_000 * s for s in range(len(sets))]
    wave = run(w.model, sets, ko.OrderSpec.all(), ko.ENGINE_WAVE, ref=refs, n_bins=16)
    lanes = run(w.model, sets, ko.OrderSpec.all(), ko.ENGINE_LANES, ref=refs, n_bins=16, lane_entries=3)
    assert lanes[3][2] > 0
    assert np.array_equal(lanes[0], wave[0])
    assert np.array_equal(lanes[1], wave[1])
    assert np.array_equal(lanes[2], wave[2])


def test_engine_choice():
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    kernels, offsets = kb.concat_sets([ks])
    say("engine choice: auto, and lanes refused for n=20")
    p = ko.Plan(w.model, kernels, offsets, ko.OrderSpec.sampled([8192], 1))
    assert p.engine()[:2] == (ko.ENGINE_LANES, 32)
    p.close()
    # too few orders to fill the lanes: one wavefront per order
    p = ko.Plan(w.model, kernels, offsets, ko.OrderSpec.sampled([8191], 1))
    assert p.engine()[0] == ko.ENGINE_WAVE
    p.close()
    big = synth.draw_kernels(np.random.default_rng(3), 20, 64, 512)
    k20, o20 = kb.concat_sets([big])
    p = ko.Plan(w.model, k20, o20, ko.OrderSpec.sampled([64], 1))
    assert p.engine()[0] == ko.ENGINE_WAVE
    p.close()
    with pytest.raises(Exception):
        ko.Plan(w.model, k20, o20, ko.OrderSpec.sampled([64], 1), engine=ko.ENGINE_LANES)
