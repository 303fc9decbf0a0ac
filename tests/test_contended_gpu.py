"""GPU parity of the memory-contention model (Section 4: the blocks that run
together share the chip's memory throughput; ko_gpu_model.mem_blocks > 0).

Every makespan the library computes under contention is compared element by
element with the oracle's event-driven contended simulation (oracle/
ko_oracle.c), which is pinned on the CPU by a hand trace, closed forms, a
cycle-by-cycle formulation and the no-contention limit.
"""

import itertools
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import sampling

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")

DEV = "cuda:0"


def say(*a):
    print("[contended-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def with_b(model, b):
    d = model if isinstance(model, dict) else model.as_dict()
    return dict(d, mem_blocks=int(b))


def gpu_batch(gpu, kernels, offsets, spec, total, ref=None):
    n_sets = len(offsets) - 1
    ms = torch.full((max(total, 1),), -7, dtype=torch.int64, device=DEV)
    st = torch.zeros(8 * n_sets, dtype=torch.int64, device=DEV)
    ko.ko_simulate_batch(gpu, kernels, offsets, spec, ref_makespan=ref, makespans=ms, stats=st)
    ko.ko_sync()
    return ms[:total].cpu().numpy(), ko.stats_records(st)


def gpu_all(gpu, ks):
    n = len(ks)
    return gpu_batch(gpu, ks, [0, n], ko.OrderSpec.all(), math.factorial(n))


def plan_run(gpu, kernels, offsets, spec, total, engine, lane_entries=0):
    """Makespans and the engine report of a plan with a forced engine."""
    plan = ko.Plan(gpu, kernels, offsets, spec, engine=engine, lane_entries=lane_entries)
    ms = torch.full((max(total, 1),), -7, dtype=torch.int64, device=DEV)
    st = torch.zeros(8 * (len(offsets) - 1), dtype=torch.int64, device=DEV)
    plan.launch(makespans=ms, stats=st)
    plan.status()
    rep = plan.engine()
    plan.close()
    return ms[:total].cpu().numpy(), ko.stats_records(st), rep


def test_e5_hand_trace_on_the_gpu(golden):
    g = golden("e5_contention.json")
    gpu = with_b(g["gpu"], g["mem_blocks"])
    ms, st = gpu_all(gpu, g["kernels"])
    # ALL enumerates lexicographic ranks, the golden file lists the orders in that order
    assert g["orders"] == [list(p) for p in itertools.permutations(range(3))]
    assert ms.tolist() == g["makespans"]
    ms0, _ = gpu_all(with_b(g["gpu"], 0), g["kernels"])
    assert ms0.tolist() == g["makespans_without_contention"]


@pytest.mark.parametrize("b", [1, 3, 16, 1 << 24])
def test_all_720_orders_small_model(b):
    ks = synth.draw_set(0, 0)
    gpu = with_b(synth.SMALL_MODEL, b)
    say("n=6 all orders, mem_blocks", b)
    ms, st = gpu_all(gpu, ks)
    want = oracle.contended_makespans(synth.SMALL_MODEL.as_dict(), ks, b, first=0, count=720)
    np.testing.assert_array_equal(ms, want)
    assert st[0]["min_makespan"] == want.min() and st[0]["max_makespan"] == want.max()
    assert st[0]["argmin"] == int(np.argmin(want)) and st[0]["argmax"] == int(np.argmax(want))
    if b == 1 << 24:
        # the chip never runs out of memory throughput: the first model's makespans
        np.testing.assert_array_equal(ms, oracle.makespans_all(synth.SMALL_MODEL.as_dict(), ks))


@pytest.mark.parametrize("b", [64, 256, 1024])
def test_n10_mi355x_rank_window_and_samples(b):
    ks = synth.draw_set(1, 0)
    base = synth.MI355X_MODEL.as_dict()
    gpu = with_b(base, b)
    lo, cnt = 1_814_000, 700
    say("n=10 rank window", lo, cnt, "mem_blocks", b)
    ms, st = gpu_batch(gpu, ks, [0, 10], ko.OrderSpec.rank_range([[lo, lo + cnt]]), cnt)
    want = oracle.contended_makespans(base, ks, b, first=lo, count=cnt)
    np.testing.assert_array_equal(ms, want)
    # sampled orders (the SAMPLED counter stream) and the percentile against them
    seed, ns = 4242, 600
    ranks = [sampling.sampled_rank(seed, 0, i, math.factorial(10)) for i in range(ns)]
    orders = np.array([oracle.unrank(10, r) for r in ranks], dtype=np.int32)
    want = oracle.contended_makespans(base, ks, b, orders)
    say("n=10 sampled", ns, "mem_blocks", b)
    ms, st = gpu_batch(gpu, ks, [0, 10], ko.OrderSpec.sampled([ns], seed), ns)
    np.testing.assert_array_equal(ms, want)
    h = ko.ko_heuristic_order(gpu, ks)
    mh = int(oracle.contended_makespans(base, ks, b, np.array([h], dtype=np.int32))[0])
    r = ko.ko_rank_percentile(gpu, ks, h, n_samples=ns, seed=seed)
    assert r["makespan"] == mh
    assert (r["n_less"], r["n_equal"], r["n_greater"]) == (
        int((want < mh).sum()), int((want == mh).sum()), int((want > mh).sum()))


def test_batch_of_uneven_sets_explicit_orders():
    kernels, offsets = synth.draw_sets(2, 0, 24)
    base = synth.MI355X_MODEL.as_dict()
    rng = np.random.default_rng(7)
    per, rows, want = [], [], []
    for s in range(24):
        n = int(offsets[s + 1] - offsets[s])
        ks = kernels[offsets[s]:offsets[s + 1]]
        o = np.array([rng.permutation(n) for _ in range(40)], dtype=np.int32)
        per.append(40)
        rows.append(o.astype(np.uint8).ravel())
        want.append(oracle.contended_makespans(base, ks, 128, o))
    spec = ko.OrderSpec.explicit(torch.tensor(np.concatenate(rows), device=DEV), np.array(per, dtype=np.int64))
    say("24 sets explicit, mem_blocks 128")
    ms, st = gpu_batch(with_b(base, 128), kernels, offsets, spec, sum(per))
    np.testing.assert_array_equal(ms, np.concatenate(want))


@pytest.mark.parametrize("seed", range(6))
def test_random_models_and_sets(seed):
    rng = np.random.default_rng(1000 + seed)
    n_cu = int(rng.choice([1, 2, 5, 64, 65, 130, 256]))
    model = synth.GpuModel(n_cu=n_cu, wave_size=int(rng.choice([32, 64])), wave_cu=int(rng.integers(4, 65)),
                           blk_cu=int(rng.integers(1, 17)), reg_cu=65536, lds_cu=65536,
                           rb_milli=int(rng.integers(500, 20000)))
    n = int(rng.integers(1, 8))
    ks = synth.random_tiny_set(rng, n, model, tblk_hi=int(rng.integers(1, 4 * n_cu + 2)), inst_hi=60)
    b = int(rng.choice([1, 2, 7, 40, 300]))
    say("random model", model, "n", n, "mem_blocks", b)
    ms, _ = gpu_all(with_b(model, b), ks)
    want = oracle.contended_makespans(model.as_dict(), ks, b, first=0, count=math.factorial(n))
    np.testing.assert_array_equal(ms, want)


def test_plans_graphs_and_noalloc_agree():
    ks = synth.draw_set(0, 3)
    gpu = with_b(synth.SMALL_MODEL, 2)
    want = oracle.contended_makespans(synth.SMALL_MODEL.as_dict(), ks, 2, first=0, count=720)
    plan = ko.Plan(gpu, ks, [0, len(ks)], ko.OrderSpec.all())
    ms = torch.full((720,), -7, dtype=torch.int64, device=DEV)
    plan.launch(makespans=ms)
    plan.status()
    np.testing.assert_array_equal(ms.cpu().numpy(), want)
    ms2 = torch.full((720,), -7, dtype=torch.int64, device=DEV)
    ko.ko_simulate_batch_noalloc(gpu, ks, [0, len(ks)], ko.OrderSpec.all(), makespans=ms2)
    np.testing.assert_array_equal(ms2.cpu().numpy(), want)
    for engine in (ko.ENGINE_WAVE, ko.ENGINE_LANES):
        ms3, _, rep = plan_run(gpu, ks, [0, len(ks)], ko.OrderSpec.all(), 720, engine)
        assert rep[0] == engine
        np.testing.assert_array_equal(ms3, want)


@pytest.mark.parametrize("b", [1, 3, 16, 1 << 24])
@pytest.mark.parametrize("entries", [0, 2])
def test_lane_engine_all_720_orders(b, entries):
    """The lane engine under contention, forced (the batch is below the size
    at which the library picks it by itself), with the class's entry
    capacity and with 2 entries per lane, which spills most orders to the
    wave engine's contended routine."""
    ks = synth.draw_set(0, 0)
    gpu = with_b(synth.SMALL_MODEL, b)
    say("lanes n=6 all orders, mem_blocks", b, "entries", entries)
    ms, st, rep = plan_run(gpu, ks, [0, 6], ko.OrderSpec.all(), 720, ko.ENGINE_LANES, lane_entries=entries)
    want = oracle.contended_makespans(synth.SMALL_MODEL.as_dict(), ks, b, first=0, count=720)
    np.testing.assert_array_equal(ms, want)
    assert st[0]["min_makespan"] == want.min() and st[0]["argmin"] == int(np.argmin(want))
    assert st[0]["max_makespan"] == want.max() and st[0]["argmax"] == int(np.argmax(want))
    if entries:
        assert rep[2] > 0  # orders went through the spill path


@pytest.mark.parametrize("b", [64, 256])
def test_lane_engine_n10_window_and_samples(b):
    ks = synth.draw_set(1, 0)
    base = synth.MI355X_MODEL.as_dict()
    gpu = with_b(base, b)
    lo, cnt = 2_400_000, 4096
    say("lanes n=10 rank window, mem_blocks", b)
    ms, _, rep = plan_run(gpu, ks, [0, 10], ko.OrderSpec.rank_range([[lo, lo + cnt]]), cnt, ko.ENGINE_LANES)
    assert rep[0] == ko.ENGINE_LANES
    np.testing.assert_array_equal(ms, oracle.contended_makespans(base, ks, b, first=lo, count=cnt))
    seed, ns = 77, 2048
    ranks = [sampling.sampled_rank(seed, 0, i, math.factorial(10)) for i in range(ns)]
    orders = np.array([oracle.unrank(10, r) for r in ranks], dtype=np.int32)
    ms, _, _ = plan_run(gpu, ks, [0, 10], ko.OrderSpec.sampled([ns], seed), ns, ko.ENGINE_LANES)
    np.testing.assert_array_equal(ms, oracle.contended_makespans(base, ks, b, orders))


def test_lane_engine_uneven_batch_and_random_models():
    """Sets of n = 4..9 under contention on the lane engine, explicit orders,
    against the oracle; then small random models (CU counts 1..256)."""
    kernels, offsets = synth.draw_sets(2, 0, 24)
    base = synth.MI355X_MODEL.as_dict()
    rng = np.random.default_rng(17)
    per, rows, want = [], [], []
    for s in range(24):
        n = int(offsets[s + 1] - offsets[s])
        ks = kernels[offsets[s]:offsets[s + 1]]
        o = np.array([rng.permutation(n) for _ in range(64)], dtype=np.int32)
        per.append(64)
        rows.append(o.astype(np.uint8).ravel())
        want.append(oracle.contended_makespans(base, ks, 96, o))
    spec = ko.OrderSpec.explicit(torch.tensor(np.concatenate(rows), device=DEV), np.array(per, dtype=np.int64))
    say("lanes 24 sets explicit, mem_blocks 96")
    ms, _, rep = plan_run(with_b(base, 96), kernels, offsets, spec, sum(per), ko.ENGINE_LANES)
    assert rep[0] == ko.ENGINE_LANES
    np.testing.assert_array_equal(ms, np.concatenate(want))
    for seed in range(4):
        r = np.random.default_rng(2000 + seed)
        n_cu = int(r.choice([1, 2, 5, 64, 130, 256]))
        model = synth.GpuModel(n_cu=n_cu, wave_size=64, wave_cu=int(r.integers(4, 65)),
                               blk_cu=int(r.integers(1, 17)), reg_cu=65536, lds_cu=65536,
                               rb_milli=int(r.integers(500, 20000)))
        n = int(r.integers(2, 8))
        ks = synth.random_tiny_set(r, n, model, tblk_hi=int(r.integers(1, 4 * n_cu + 2)), inst_hi=60)
        b = int(r.choice([1, 2, 7, 40]))
        say("lanes random model", n_cu, "n", n, "mem_blocks", b)
        ms, _, _ = plan_run(with_b(model, b), ks, [0, n], ko.OrderSpec.all(), math.factorial(n), ko.ENGINE_LANES)
        np.testing.assert_array_equal(ms, oracle.contended_makespans(model.as_dict(), ks, b, first=0,
                                                                     count=math.factorial(n)))


def test_engines_agree_on_all_n10_orders():
    """All 3,628,800 orders of the n=10 set at mem_blocks 256: the lane engine's
    contended makespans equal the wave engine's element by element (each is
    compared with the oracle on windows and samples above), with the same
    extremes and counts."""
    ks = synth.draw_set(1, 0)
    gpu = with_b(synth.MI355X_MODEL, 256)
    N = math.factorial(10)
    say("n=10 all orders, both engines, mem_blocks 256")
    lanes, st_l, rep_l = plan_run(gpu, ks, [0, 10], ko.OrderSpec.all(), N, ko.ENGINE_LANES)
    wave, st_w, rep_w = plan_run(gpu, ks, [0, 10], ko.OrderSpec.all(), N, ko.ENGINE_WAVE)
    assert rep_l[0] == ko.ENGINE_LANES and rep_w[0] == ko.ENGINE_WAVE
    np.testing.assert_array_equal(lanes, wave)
    assert st_l == st_w
