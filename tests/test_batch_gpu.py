"""GPU tests of batched evaluation: plans, HIP graph replay, the autotuner,
and the per-set percentiles of the 4096-set workload (n = 4..9).

Plans must reproduce ko_simulate_batch bit for bit under every launch
configuration; every graph replay must reproduce the eager launch (replays
are interleaved with other device work and synchronisations); percentiles are
checked against the oracle on sampled sets and by exact count identities on
all sets.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle.heuristic import heuristic_order as oracle_heuristic
from oracle import stats as ostats

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")
kb = pytest.importorskip("paper_1511_07983_amd.batch")

DEV = "cuda:0"
MODEL = synth.MI355X_MODEL


def say(*a):
    print("[batch-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def batch_sets(count, first=0):
    return [synth.draw_set(2, first + s) for s in range(count)]


def run_immediate(kernels, offsets, spec, n_sets, total, ref=None, n_bins=0):
    ms = torch.full((max(total, 1),), -7, dtype=torch.int64, device=DEV)
    st = torch.zeros(8 * n_sets, dtype=torch.int64, device=DEV)
    h = torch.zeros(max(n_sets * n_bins, 1), dtype=torch.int64, device=DEV) if n_bins else None
    ko.ko_simulate_batch(MODEL, kernels, offsets, spec, ref_makespan=ref, makespans=ms, stats=st, hist=h,
                         n_bins=n_bins)
    ko.ko_sync()
    return ms, st, h


@pytest.mark.parametrize("chunk_log2,wg", [(0, 0), (4, 1), (10, 16), (6, 3)])
def test_plan_matches_immediate_path(chunk_log2, wg):
    sets = batch_sets(64)
    kernels, offsets = kb.concat_sets(sets)
    spec = ko.OrderSpec.all()
    plan = ko.Plan(MODEL, kernels, offsets, spec, chunk_log2=chunk_log2, wg_per_cu=wg)
    say(f"plan chunk=2^{chunk_log2} wg={wg}: {plan.total_orders} orders, {plan.work_items} items")
    ref = torch.from_numpy(np.arange(64, dtype=np.int64) * 50000 + 2_000_000).to(DEV)
    ms0, st0, h0 = run_immediate(kernels, offsets, spec, 64, plan.total_orders, ref=ref, n_bins=32)
    ms = torch.full_like(ms0, -5)
    st = torch.zeros_like(st0)
    h = torch.zeros_like(h0)
    plan.launch(ref_makespan=ref, makespans=ms, stats=st, hist=h, n_bins=32)
    plan.status()
    assert torch.equal(ms, ms0) and torch.equal(st, st0) and torch.equal(h, h0)
    # the smallest sets against the oracle directly
    off = np.concatenate([[0], np.cumsum([math.factorial(len(k)) for k in sets])])
    msh = ms.cpu().numpy()
    for s, k in enumerate(sets):
        if len(k) <= 5:
            assert np.array_equal(msh[off[s]:off[s + 1]], oracle.makespans_all(MODEL.as_dict(), k)), s


def test_plan_modes():
    sets = batch_sets(12, 100)
    kernels, offsets = kb.concat_sets(sets)
    lohi = [[math.factorial(len(k)) // 3, min(math.factorial(len(k)), math.factorial(len(k)) // 3 + 50)]
            for k in sets]
    for spec in (ko.OrderSpec.rank_range(lohi), ko.OrderSpec.sampled([97] * 12, 5)):
        plan = ko.Plan(MODEL, kernels, offsets, spec, chunk_log2=4)
        ms0, st0, _ = run_immediate(kernels, offsets, spec, 12, plan.total_orders)
        ms = torch.empty_like(ms0)
        st = torch.empty_like(st0)
        plan.launch(makespans=ms, stats=st)
        plan.status()
        assert torch.equal(ms, ms0) and torch.equal(st, st0)
    # explicit orders, and a malformed one reported by the plan's status
    flat = torch.from_numpy(np.concatenate([np.random.default_rng(s * 7 + r).permutation(len(k))
                                            for s, k in enumerate(sets) for r in range(3)]).astype(np.uint8)).to(DEV)
    plan = ko.Plan(MODEL, kernels, offsets, ko.OrderSpec.explicit(flat, [3] * 12))
    ms = torch.empty(36, dtype=torch.int64, device=DEV)
    plan.launch(makespans=ms)
    plan.status()
    host = flat.cpu().numpy()
    pos = 0
    for s, k in enumerate(sets):
        n = len(k)
        want = oracle.makespans_orders(MODEL.as_dict(), k, host[pos:pos + 3 * n].reshape(3, n).astype(np.int32))
        assert np.array_equal(ms.cpu().numpy()[3 * s:3 * s + 3], want)
        pos += 3 * n
    bad = flat.clone()
    bad[1] = bad[0]
    plan_bad = ko.Plan(MODEL, kernels, offsets, ko.OrderSpec.explicit(bad, [3] * 12))
    plan_bad.launch(makespans=ms)
    with pytest.raises(ko.KoError) as e:
        plan_bad.status()
    assert e.value.code == ko.KO_EHIP
    plan.launch(makespans=ms)
    plan.status()


def test_graph_replays_match_eager_launch():
    sets = batch_sets(200, 300)
    kernels, offsets = kb.concat_sets(sets)
    plan = ko.Plan(MODEL, kernels, offsets, ko.OrderSpec.all())
    T = plan.total_orders
    ref = torch.full((200,), 3_000_000, dtype=torch.int64, device=DEV)
    ms0 = torch.empty(T, dtype=torch.int64, device=DEV)
    st0 = torch.empty(1600, dtype=torch.int64, device=DEV)
    h0 = torch.empty(200 * 64, dtype=torch.int64, device=DEV)
    plan.launch(ref_makespan=ref, makespans=ms0, stats=st0, hist=h0, n_bins=64)
    plan.status()
    ms = torch.empty_like(ms0)
    st = torch.empty_like(st0)
    h = torch.empty_like(h0)
    stream = torch.cuda.Stream()
    say(f"graph over {T} orders of 200 sets")
    graph = plan.capture(stream=stream, ref_makespan=ref, makespans=ms, stats=st, hist=h, n_bins=64)
    other = batch_sets(5, 900)
    k2, o2 = kb.concat_sets(other)
    for replay in range(4):
        ms.fill_(-1)
        st.fill_(-1)
        h.fill_(-1)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        plan.status(stream)
        assert torch.equal(ms, ms0), replay
        assert torch.equal(st, st0), replay
        assert torch.equal(h, h0), replay
        # eager work of the program between replays
        run_immediate(k2, o2, ko.OrderSpec.rank_range([[0, 20]] * 5), 5, 100)
        _ = (ms0[:1000] * 2).sum().item()
    graph.close()


def test_autotuner_configs_agree_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("KO_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    sets = batch_sets(256, 1000)
    kernels, offsets = kb.concat_sets(sets)
    cfg, rows = kb.autotune(MODEL, kernels, offsets, ko.OrderSpec.all(), reps=2, chunks=(6, 8), wgs=(4, 8),
                            log=lambda r: say("tune", r))
    # both engines (the CU-state layouts) are swept, and every candidate agreed
    assert len(rows) == 8 and {r["engine"] for r in rows} == {ko.ENGINE_WAVE, ko.ENGINE_LANES}
    assert cfg["chunk_log2"] in (6, 8) and cfg["wg_per_cu"] in (4, 8)
    assert cfg["engine"] in (ko.ENGINE_WAVE, ko.ENGINE_LANES)
    again, rows2 = kb.autotune(MODEL, kernels, offsets, ko.OrderSpec.all())
    assert again == cfg and rows2 == []
    # under memory contention both engines apply and agree bit for bit
    cont = dict(MODEL.as_dict(), mem_blocks=64)
    monkeypatch.setenv("KO_AUTOTUNE_CACHE", str(tmp_path / "tune2.json"))
    cfg2, rows2 = kb.autotune(cont, kernels, offsets, ko.OrderSpec.all(), reps=1, chunks=(8,), wgs=(8,))
    assert [r["engine"] for r in rows2] == [ko.ENGINE_WAVE, ko.ENGINE_LANES]


def test_percentiles_of_the_4096_set_workload():
    """All 4096 sets (n = 4..9, 2.8e8 orders) in two plan launches: Algorithm
    1's order of each set, its exact makespan and its percentile."""
    sets = batch_sets(4096)
    say("4096-set percentiles")
    res = kb.percentiles(MODEL, sets)
    N = np.array([math.factorial(len(k)) for k in sets])
    assert np.array_equal(res["n_orders"], N)
    assert np.array_equal(res["n_less"] + res["n_equal"] + res["n_greater"], N)
    assert np.all(res["n_equal"] >= 1)  # the order itself
    assert np.all(res["best"] <= res["makespan"]) and np.all(res["makespan"] <= res["worst"])
    rng = np.random.default_rng(4096)
    gpu = MODEL.as_dict()
    for s in rng.choice(4096, 40, replace=False):
        k = sets[s]
        assert res["order"][s] == oracle_heuristic(gpu, k)[0]
        assert res["makespan"][s] == oracle.makespan(gpu, k, res["order"][s])
    small = [s for s in range(4096) if len(sets[s]) <= 6][:30]
    for s in small:
        m = oracle.makespans_all(gpu, sets[s])
        c = ostats.set_stats(m, ref=int(res["makespan"][s]))
        assert (res["n_less"][s], res["n_equal"][s], res["n_greater"][s]) == (c["n_less"], c["n_equal"],
                                                                                c["n_greater"])
        assert (res["best"][s], res["worst"][s]) == (m.min(), m.max())
    pct = res["pct_inclusive"]
    say(f"percentile of Algorithm 1's order: median {np.median(pct):.1f}, mean {pct.mean():.1f}, "
        f">= 90th in {np.mean(pct >= 90):.1%} of sets")
