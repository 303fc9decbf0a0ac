"""GPU tests of the surrogate-guided search (training data, training,
scoring, top-k, exact re-simulation, beam search) on the n=8 workload.

Exact quantities (sampled makespans, quantile thresholds, hit counts,
re-simulated makespans) are checked bit for bit against the oracle.  The
learned part is checked by what it gains: the trained network must reach an
order in the exact top 1% with fewer exact simulations than uniform random
sampling needs on average (N / hits, exact for sampling with replacement).
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
nn = pytest.importorskip("paper_1511_07983_amd.nn")
sg = pytest.importorskip("paper_1511_07983_amd.surrogate")

DEV = "cuda:0"
MODEL = synth.MI355X_MODEL


def set_list(workload, first, count):
    return [synth.draw_set(workload, first + s) for s in range(count)]


def say(*a):
    print("[surrogate-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def trained():
    """A network trained on 128 sets x 2048 exact samples (n=8), rank-quantile targets."""
    train_sets = set_list(5, 0, 128)
    table = sg.SetTable.build(MODEL, train_sets)
    say("exact training samples: 128 sets x 2048")
    data = sg.exact_samples(table, 2048, seed=11)
    data = sg.mask_suffixes(data, 0.25, seed=12)
    rng = np.random.default_rng(13)
    from oracle import mlp
    init = {name: (np.zeros(shape) if name.startswith("b") else
                   rng.normal(0.0, 1.0 / math.sqrt(shape[-1]), size=shape))
            for name, shape in mlp.SHAPES}
    sur = nn.Surrogate(mlp.flatten(init).astype(np.float32))
    say("training 1500 steps")
    log = sg.train(sur, table, data, steps=1500, batch=2048, lr=2e-3, warmup=100, seed=14, log_every=250)
    say("loss log", log)
    # mean squared error of the best constant prediction per set: the variance
    # of the (rank-quantile) targets around each set's own mean
    t = data.t_values.cpu().numpy().reshape(128, 2048).astype(np.float64) / 2048.0
    within = float(np.mean((t - t.mean(axis=1, keepdims=True)) ** 2))
    say(f"within-set target variance {within:.5f}, total {float(t.var()):.5f}")
    return sur, log, within


def test_exact_samples_match_oracle():
    sets = set_list(5, 0, 3)
    table = sg.SetTable.build(MODEL, sets)
    data = sg.exact_samples(table, 300, seed=5)
    ms = data.makespans.cpu().numpy()
    pos = data.pos.cpu().numpy()
    assert np.array_equal(data.set_of.cpu().numpy(), np.repeat(np.arange(3), 300))
    N = math.factorial(8)
    for s, ks in enumerate(sets):
        ranks = [sampled_rank(5, s, i, N) for i in range(300)]
        want = oracle.makespans_ranks(MODEL.as_dict(), ks, ranks)
        assert np.array_equal(ms[s * 300:(s + 1) * 300], want)
        for i in (0, 1, 150, 299):
            order = oracle.unrank(8, ranks[i])
            assert [int(pos[s * 300 + i][k]) for k in order] == list(range(8))
    assert table.lb_host.tolist() == [nn.lower_bound(MODEL, k) for k in sets]


def test_within_set_ranks_and_quantile_targets():
    sets = set_list(5, 0, 3)
    table = sg.SetTable.build(MODEL, sets)
    data = sg.exact_samples(table, 1000, seed=7)
    ms = data.makespans.cpu().numpy().reshape(3, 1000)
    ranks = data.t_values.cpu().numpy().reshape(3, 1000)
    for s in range(3):
        order = np.lexsort((np.arange(1000), ms[s]))
        want = np.empty(1000, dtype=np.int64)
        want[order] = np.arange(1000)
        assert np.array_equal(ranks[s], want)
    sur = nn.Surrogate(np.zeros(nn.num_params(), dtype=np.float32))
    t = sur.targets(data.t_values, data.t_center, data.t_scale, data.set_of).cpu().numpy()
    assert np.array_equal(t, (ranks.ravel() / np.float32(1000.0)).astype(np.float32))
    # a power-of-two set size, the largest allowed, and ties
    v = torch.from_numpy(np.random.default_rng(1).integers(0, 50, size=2 * 8192).astype(np.int64)).to(DEV)
    r = nn.within_set_ranks(v, 2, 8192).cpu().numpy().reshape(2, 8192)
    vh = v.cpu().numpy().reshape(2, 8192)
    for s in range(2):
        order = np.lexsort((np.arange(8192), vh[s]))
        assert np.array_equal(np.argsort(r[s]), order)


def test_targets_and_row_map():
    sets = set_list(5, 0, 2)
    table = sg.SetTable.build(MODEL, sets)
    data = sg.exact_samples(table, 100, seed=6, target="lb")
    sur = nn.Surrogate(np.zeros(nn.num_params(), dtype=np.float32))
    rows = torch.tensor([5, 150, 0, 199, 101], dtype=torch.int64, device=DEV)
    t = sur.targets(data.makespans, data.best, table.lb, data.set_of, rows=rows).cpu().numpy()
    ms = data.makespans.cpu().numpy()
    best = [int(ms[:100].min()), int(ms[100:].min())]
    assert data.best.cpu().numpy().tolist() == best
    want = np.array([(ms[r] - best[r // 100]) / table.lb_host[r // 100] for r in rows.cpu().numpy()],
                    dtype=np.float32)
    assert np.array_equal(t, want)
    x = sur.tokens(table.feat, data.pos, data.set_of, rows=rows).cpu().numpy().view(np.uint16)
    pos = data.pos.cpu().numpy()
    for b, r in enumerate(rows.cpu().numpy()):
        onehot = x[b, :, nn.N_FEAT:nn.N_FEAT + nn.N_POS]
        assert np.array_equal(np.argmax(onehot, axis=1), pos[r])


def test_top_quantile_matches_oracle():
    ks = synth.draw_set(15, 0)
    q = sg.top_quantile(MODEL, ks, 0.01)
    want = np.sort(oracle.makespans_all(MODEL.as_dict(), ks))
    k = math.ceil(0.01 * len(want))
    assert (q.n_orders, q.k, q.makespan) == (len(want), k, int(want[k - 1]))
    assert q.hits == int((want <= want[k - 1]).sum())
    assert (q.best, q.worst) == (int(want[0]), int(want[-1]))


def test_training_reduces_loss(trained):
    """The trained network beats the best per-set constant (the within-set
    variance of the targets), which knows each set's mean exactly."""
    _, log, within = trained
    assert log[-1][1] < log[0][1], log
    assert log[-1][1] < within, (log[-1], within)


def test_scoring_reaches_top1pct_with_fewer_simulations_than_random(trained):
    """The gain of the learned scorer over the method without it (uniform
    sampling), at equal terms: exact simulations to the first exact top-1%
    order, on 8 held-out sets."""
    sur, _, _ = trained
    held = set_list(15, 0, 8)
    table = sg.SetTable.build(MODEL, held)
    ratios = []
    for s, ks in enumerate(held):
        q = sg.top_quantile(MODEL, ks, 0.01)
        res = sg.score_and_rerank(sur, table, s, n_score=1 << 16, top_k=256, seed=1000 + s)
        # the re-simulated makespans are exact
        want = oracle.makespans_orders(MODEL.as_dict(), ks, res.orders[:16].astype(np.int32))
        assert np.array_equal(res.exact[:16], want)
        sims = sg.sims_to_first_hit(res.exact, q.makespan, q.random_expected)
        ratios.append(q.random_expected / sims)
        mae = sg.mae_cycles(res, q, "quantile", float(table.lb_host[s]))
        say(f"set {s}: random needs {q.random_expected:.1f}, scorer {sims:.0f}; "
            f"MAE {mae:.0f} cycles ({mae / q.best:.3%} of best); "
            f"recall@1% {np.mean(res.exact <= q.makespan):.3f}")
    gmean = float(np.exp(np.mean(np.log(ratios))))
    say(f"speedup to first top-1% order: geometric mean {gmean:.2f}x, per set {np.round(ratios, 2)}")
    print(f"[surrogate-gpu] speedup to first top-1% order: geometric mean {gmean:.2f}x, "
          f"per set {np.round(ratios, 2)}", flush=True)
    # this small fixture (128 training sets, 1500 steps, fixed seeds) is far
    # below the reported recipes; it must still beat uniform sampling clearly
    # and on most sets
    assert gmean > 2.0
    assert sum(r > 1.0 for r in ratios) >= 6


def test_beam_step_kernels_match_oracle(trained):
    """Each device step of the beam search against oracle/beam.py: the
    candidates' positions and (parent, kernel) pairs, the per-prefix cap with
    and without Gumbel noise, and the gathered prefixes."""
    from oracle import beam as obeam
    sur, _, _ = trained
    rng = np.random.default_rng(5)
    for n in (1, 5, 12, 16):
        for d in sorted({0, n // 2, n - 1}):
            W = 1 if d == 0 else 37
            pre = np.array([rng.permutation(n)[:d] for _ in range(W)], dtype=np.uint8).reshape(W, d)
            pos, cand = nn.beam_expand(torch.from_numpy(pre).to(DEV), n)
            wpos, wpar, wker = obeam.expand(pre.astype(np.int64), n)
            assert np.array_equal(pos.cpu().numpy(), wpos), (n, d)
            c = cand.cpu().numpy()
            assert np.array_equal(c >> 8, wpar) and np.array_equal(c & 255, wker), (n, d)
            m = n - d
            sc = rng.integers(0, 9, W * m).astype(np.float32)      # ties
            for cap in (0, 1, 2, 5):
                got = nn.beam_cap(torch.from_numpy(sc).to(DEV), W, m, cap).cpu().numpy()
                assert np.array_equal(got, obeam.cap(sc, m, cap)), (n, d, cap)
            scn = rng.normal(size=W * m).astype(np.float32)
            got = nn.beam_cap(torch.from_numpy(scn).to(DEV), W, m, 0, 0.5, 77).cpu().numpy()
            want = obeam.cap(scn, m, 0, 0.5, 77)
            assert np.allclose(got, want, rtol=0, atol=1e-5), (n, d)
            idx = rng.choice(W * m, size=min(W * m, 20), replace=False)
            out = nn.beam_gather(torch.from_numpy(pre).to(DEV), cand, torch.from_numpy(idx).to(DEV))
            assert np.array_equal(out.cpu().numpy(), obeam.gather(pre, wpar, wker, idx)), (n, d)


def test_beam_search_finds_complete_orders(trained):
    sur, _, _ = trained
    held = set_list(15, 0, 4)
    table = sg.SetTable.build(MODEL, held)
    for s, ks in enumerate(held):
        res = sg.beam_search(sur, table, s, width=32, max_children=2, temperature=0.2 * s, seed=s)
        assert res.orders.shape == (32, 8)
        assert all(sorted(o.tolist()) == list(range(8)) for o in res.orders)
        assert len({o.tobytes() for o in res.orders}) == 32
        assert np.all(np.diff(res.predicted) >= 0)  # ranked by the final (noise-free) score
        want = oracle.makespans_orders(MODEL.as_dict(), ks, res.orders.astype(np.int32))
        assert np.array_equal(res.exact, want)
        q = sg.top_quantile(MODEL, ks, 0.01)
        say(f"beam set {s}: best {res.exact.min()} vs top-1% threshold {q.makespan} "
            f"(best possible {q.best}); hits {int((res.exact <= q.makespan).sum())}/32")
