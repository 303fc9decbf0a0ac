"""Round-synchronous execution rounds (Section 2) on the GPU: ko_simulate_rounds
against the oracle's block-by-block simulation, element by element."""

import itertools
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _gpu_rounds(gpu, ks, orders):
    o = torch.from_numpy(np.ascontiguousarray(orders, dtype=np.uint8)).cuda()
    m = ko.ko_simulate_rounds(gpu, ks, o)
    torch.cuda.synchronize()
    return m.cpu().numpy()


def _check(gpu, ks, orders, label):
    print(f"rounds parity: {label} n={len(ks)} orders={len(orders)}", flush=True)
    sys.stdout.flush()
    want = oracle.rounds_makespans(gpu, ks, orders)
    got = _gpu_rounds(gpu, ks, orders)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (label, bad[:5].tolist(), got[bad[:5]].tolist(), want[bad[:5]].tolist())


def test_rounds_hand_trace(golden):
    g = golden("e4_rounds.json")
    got = _gpu_rounds(g["gpu"], g["kernels"], g["orders"])
    assert got.tolist() == g["rounds_makespans"]


@pytest.mark.parametrize("n_cu", [1, 3, 16, 64, 65, 100, 130, 200, 256])
def test_rounds_all_orders_small_sets(n_cu):
    # every order of random sets; CU counts cover 1..4 slots per lane and
    # ragged last slots
    model = synth.GpuModel(n_cu=n_cu, wave_size=64, wave_cu=32, blk_cu=8,
                           reg_cu=131072, lds_cu=163840, rb_milli=10000)
    rng = np.random.default_rng(1000 + n_cu)
    for rep in range(3):
        n = int(rng.integers(3, 7))
        ks = synth.random_tiny_set(rng, n, model, tblk_hi=max(4, 3 * n_cu), inst_hi=5000)
        orders = np.array(list(itertools.permutations(range(n))), dtype=np.int32)
        _check(model.as_dict(), ks, orders, f"n_cu={n_cu} rep={rep}")


@pytest.mark.parametrize("model_name", ["SMALL_MODEL", "GTX580_MODEL"])
def test_rounds_all_orders_seven_kernels(model_name):
    model = getattr(synth, model_name)
    rng = np.random.default_rng(77)
    ks = synth.random_tiny_set(rng, 7, model, tblk_hi=200, inst_hi=900)
    orders = np.array(list(itertools.permutations(range(7))), dtype=np.int32)
    _check(model.as_dict(), ks, orders, model_name)


def test_rounds_n10_workload_sampled():
    # the n=10 set of the all-orders workload on the MI355X-shaped model,
    # 20,000 seeded orders
    wl = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    rng = np.random.default_rng(2015)
    orders = np.array([rng.permutation(10) for _ in range(20000)], dtype=np.int32)
    _check(wl.model.as_dict(), ks, orders, wl.name)


def test_rounds_largest_sets():
    # n = 20, the largest set the ABI takes, and n = 16 search-workload sets
    model = synth.MI355X_MODEL
    rng = np.random.default_rng(20)
    ks = synth.draw_kernels(rng, 20, 64, 8192)
    orders = np.array([rng.permutation(20) for _ in range(500)], dtype=np.int32)
    _check(model.as_dict(), ks, orders, "n=20")
    for s in range(4):
        ks = synth.draw_set(4, s)
        orders = np.array([rng.permutation(16) for _ in range(500)], dtype=np.int32)
        _check(model.as_dict(), ks, orders, f"n=16 set {s}")


def test_rounds_paper_sets():
    from synth import paper_sets
    for name, ks in paper_sets.EXPERIMENTS.items():
        n = len(ks)
        orders = np.array(list(itertools.permutations(range(n))), dtype=np.int32)
        _check(paper_sets.MODEL.as_dict(), ks, orders, name)


def test_rounds_bad_index_and_empty():
    model = synth.SMALL_MODEL
    ks = synth.random_tiny_set(np.random.default_rng(4), 4, model)
    # rows 1, 3 and 4 are not permutations: an index past n, a repeated
    # index at the end, a repeated index at the front
    orders = np.array([[0, 1, 2, 3], [0, 1, 9, 3], [3, 2, 1, 0], [0, 1, 2, 2], [1, 1, 2, 3]],
                      dtype=np.uint8)
    got = _gpu_rounds(model.as_dict(), ks, orders)
    want = oracle.rounds_makespans(model.as_dict(), ks, orders[[0, 2]].astype(np.int32))
    assert got.tolist() == [int(want[0]), -1, int(want[1]), -1, -1]
    with pytest.raises(ValueError):
        oracle.rounds_makespans(model.as_dict(), ks, orders[[3]].astype(np.int32))
    empty = torch.empty((0, 4), dtype=torch.uint8, device="cuda")
    assert ko.ko_simulate_rounds(model.as_dict(), ks, empty).numel() == 0


def test_rounds_in_paper_report():
    # the report's round-model columns against the oracle over all orders
    from paper_1511_07983_amd import paper_report
    from synth import paper_sets
    rows = paper_report.report(out=lambda *a, **k: None)
    assert [r["experiment"] for r in rows] == list(paper_sets.EXPERIMENTS)
    for row in rows:
        ks = paper_sets.EXPERIMENTS[row["experiment"]]
        orders = np.array(list(itertools.permutations(range(len(ks)))), dtype=np.int32)
        want = oracle.rounds_makespans(paper_sets.MODEL.as_dict(), ks, orders)
        h = int(oracle.rounds_makespans(paper_sets.MODEL.as_dict(), ks, [row["algorithm_order"]])[0])
        r = row["rounds"]
        assert (r["best_cycles"], r["worst_cycles"], r["algorithm_cycles"]) == \
            (int(want.min()), int(want.max()), h), row["experiment"]
        assert r["percentile_inclusive"] == round(100.0 * float((want >= h).mean()), 2)


def test_rounds_rank_mode():
    # orders unranked on the device from lexicographic ranks: all 5040 orders of
    # a 7-kernel set, and a window of ranks inside the n=10 set
    model = synth.GTX580_MODEL
    ks = synth.random_tiny_set(np.random.default_rng(88), 7, model, tblk_hi=200, inst_hi=900)
    got = ko.ko_simulate_rounds(model.as_dict(), ks, None, count=5040).cpu().numpy()
    orders = np.array([oracle.unrank(7, r) for r in range(5040)], dtype=np.int32)
    want = oracle.rounds_makespans(model.as_dict(), ks, orders)
    assert np.array_equal(got, want)
    ks10 = synth.draw_set(1, 0)
    first = 1_234_567
    got = ko.ko_simulate_rounds(synth.MI355X_MODEL.as_dict(), ks10, None, first=first, count=5000).cpu().numpy()
    orders = np.array([oracle.unrank(10, first + r) for r in range(5000)], dtype=np.int32)
    want = oracle.rounds_makespans(synth.MI355X_MODEL.as_dict(), ks10, orders)
    assert np.array_equal(got, want)
    last = ko.ko_simulate_rounds(synth.MI355X_MODEL.as_dict(), ks10, None, first=3628799, count=1).cpu().numpy()
    assert last.tolist() == oracle.rounds_makespans(synth.MI355X_MODEL.as_dict(), ks10,
                                                    [list(range(9, -1, -1))]).tolist()


def test_rounds_large_grids_and_long_blocks():
    # many rounds per kernel, and makespans far above 2^32 cycles (int64
    # accumulation), near the host's limit on total block time
    model = synth.MI355X_MODEL
    ks = np.zeros(3, dtype=synth.KERNEL_DTYPE)
    ks["n_tblk"] = [20000, 7000, 13001]
    ks["n_inst"] = [1 << 30, 3 << 28, 123456789]
    ks["lds_blk"] = [0, 40000, 1000]
    ks["waves_blk"] = [16, 4, 1]
    ks["regs_thr"] = [32, 128, 8]
    ks["r_milli"] = [model.rb_milli, 2 * model.rb_milli, model.rb_milli // 3]
    orders = np.array(list(itertools.permutations(range(3))), dtype=np.int32)
    want = oracle.rounds_makespans(model.as_dict(), ks, orders)
    assert want.max() > (1 << 32)
    _check(model.as_dict(), ks, orders, "large")
    got = ko.ko_simulate_rounds(model.as_dict(), ks, None, count=6).cpu().numpy()
    assert np.array_equal(got, want)


def test_rounds_one_block_per_cu():
    # every block takes a whole CU: rounds are windows of n_CU blocks
    model = synth.GpuModel(n_cu=70, wave_size=64, wave_cu=32, blk_cu=1,
                           reg_cu=131072, lds_cu=163840, rb_milli=10000)
    rng = np.random.default_rng(71)
    ks = synth.random_tiny_set(rng, 6, model, tblk_hi=150, inst_hi=4000)
    orders = np.array(list(itertools.permutations(range(6))), dtype=np.int32)
    _check(model.as_dict(), ks, orders, "blk_cu=1")


def test_rounds_report_statistics_on_device():
    # the report's best, worst and percentile (device statistics over the
    # device's makespans) against the oracle on the same sampled orders
    from oracle.sampling import sampled_rank
    from paper_1511_07983_amd import rounds
    rec = rounds.report(n_orders=20000, reps=1, out=lambda *a, **k: None)
    ks = synth.draw_set(1, 0)
    gpu = synth.MI355X_MODEL.as_dict()
    orders = np.array([oracle.unrank(10, sampled_rank(rounds.SEED, 0, i, math.factorial(10)))
                       for i in range(20000)], dtype=np.int32)
    want = oracle.rounds_makespans(gpu, ks, orders)
    h = int(oracle.rounds_makespans(gpu, ks, [rec["heuristic_order"]])[0])
    assert (rec["best"], rec["worst"], rec["heuristic_makespan"]) == (int(want.min()), int(want.max()), h)
    assert rec["heuristic_percentile"] == round(100.0 * float((want >= h).sum()) / 20000, 2)
