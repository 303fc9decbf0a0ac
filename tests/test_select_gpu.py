"""GPU parity of libko's order writer and selection calls.

ko_sample_orders must produce, bit for bit, the orders the oracle derives from
the same counter-based ranks (and the orders SAMPLED mode evaluates);
ko_topk_f32 must return exactly the k smallest values with their indices,
ordered by (value, index) as numpy's stable sort orders them; and
ko_kth_smallest_i64 must equal np.partition's k-th element.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import stats as ostats
from oracle.sampling import sampled_rank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")

DEV = "cuda:0"


def say(*a):
    print("[select-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def oracle_orders(n, set_index, seed, indices):
    N = math.factorial(n)
    return np.array([oracle.unrank(n, sampled_rank(seed, set_index, int(i), N)) for i in indices],
                    dtype=np.uint8).reshape(len(indices), n)


@pytest.mark.parametrize("n,set_index,first,count", [(1, 0, 0, 5), (6, 3, 17, 1000), (12, 0, 0, 2049),
                                                      (16, 7, (1 << 40) - 300, 300), (20, 2, 5, 777)])
def test_sample_orders_match_oracle(n, set_index, first, count):
    seed = 0x5EED + n
    say(f"sample orders n={n} set={set_index} first={first} count={count}")
    orders = torch.empty(count * n, dtype=torch.uint8, device=DEV)
    pos = torch.empty(count * n, dtype=torch.uint8, device=DEV)
    ko.ko_sample_orders(n, set_index, seed, count, first=first, orders=orders, positions=pos)
    got = orders.cpu().numpy().reshape(count, n)
    want = oracle_orders(n, set_index, seed, range(first, first + count))
    assert np.array_equal(got, want)
    inv = np.empty_like(want)
    for b in range(count):
        inv[b, want[b]] = np.arange(n)
    assert np.array_equal(pos.cpu().numpy().reshape(count, n), inv)


def test_sample_orders_by_index_list():
    n, seed = 9, 77
    idx = np.array([5, 0, 123456789, (1 << 40) - 1, 5, 42], dtype=np.int64)
    say("sample orders by index list")
    orders = torch.empty(len(idx) * n, dtype=torch.uint8, device=DEV)
    ko.ko_sample_orders(n, 1, seed, len(idx), indices=torch.from_numpy(idx).to(DEV), orders=orders)
    assert np.array_equal(orders.cpu().numpy().reshape(-1, n), oracle_orders(n, 1, seed, idx))


def test_sampled_mode_evaluates_the_written_orders():
    """SAMPLED-mode makespans equal EXPLICIT-mode makespans of the orders
    ko_sample_orders writes, and the oracle's."""
    w = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    n, count, seed = len(ks), 3000, 99
    say("sampled vs explicit on the n=10 set")
    ms_s = torch.empty(count, dtype=torch.int64, device=DEV)
    ko.ko_simulate_batch(w.model, ks, [0, n], ko.OrderSpec.sampled([count], seed), makespans=ms_s)
    orders = torch.empty(count * n, dtype=torch.uint8, device=DEV)
    ko.ko_sample_orders(n, 0, seed, count, orders=orders)
    ms_e = torch.empty(count, dtype=torch.int64, device=DEV)
    ko.ko_simulate_batch(w.model, ks, [0, n], ko.OrderSpec.explicit(orders, [count]), makespans=ms_e)
    ko.ko_sync()
    a, b = ms_s.cpu().numpy(), ms_e.cpu().numpy()
    assert np.array_equal(a, b)
    sub = np.arange(0, count, 37)
    want = oracle.makespans_orders(w.model.as_dict(), ks,
                                   orders.cpu().numpy().reshape(count, n)[sub].astype(np.int32))
    assert np.array_equal(a[sub], want)


def reference_topk(y, k):
    # by value, then index; numpy treats -0.0 and +0.0 as equal, the library
    # orders -0.0 first, hence the middle key
    keys = np.where(np.signbit(y) & (y == 0), -1, 0)
    order = np.lexsort((np.arange(len(y)), keys, y))
    return order[:k]


@pytest.mark.parametrize("count,k", [(1, 1), (300, 300), (1000, 7), (1_000_003, 1), (1_000_003, 100),
                                     (4_000_037, 16384)])
def test_topk_matches_sorting(count, k):
    rng = np.random.default_rng(count + k)
    y = rng.normal(size=count).astype(np.float32)
    y[rng.integers(0, count, count // 10 + 1)] = np.float32(0.25)  # ties
    y[: min(count, 3)] = np.array([0.0, -0.0, -1e30], dtype=np.float32)[: min(count, 3)]
    say(f"topk count={count} k={k}")
    idx, val = ko.ko_topk_f32(torch.from_numpy(y).to(DEV), k)
    want = reference_topk(y, k)
    got = idx.cpu().numpy()
    assert np.array_equal(got, want)
    assert np.array_equal(val.cpu().numpy().view(np.uint32), y[want].view(np.uint32))


def test_topk_rejects_massive_ties():
    y = torch.zeros(100000, dtype=torch.float32, device=DEV)
    with pytest.raises(ko.KoError) as e:
        ko.ko_topk_f32(y, 10)
    assert e.value.code == ko.KO_ERANGE


@pytest.mark.parametrize("count", [1, 255, 100_001, 3_000_000])
def test_kth_smallest_i64(count):
    rng = np.random.default_rng(count)
    v = rng.integers(-(1 << 62), 1 << 62, size=count, dtype=np.int64)
    v[rng.integers(0, count, count // 3 + 1)] = 12345  # ties
    t = torch.from_numpy(v).to(DEV)
    say(f"kth smallest count={count}")
    for k in sorted({1, count, (count + 1) // 2, max(1, count // 100)}):
        want = int(np.partition(v, k - 1)[k - 1])
        assert ko.ko_kth_smallest_i64(t, k) == want, k
        assert ko.ko_kth_smallest_i64(t, k, with_count=True) == (want, int((v <= want).sum())), k


@pytest.mark.parametrize("count,span", [(1, 0), (4096, 0), (4097, 300), (65_537, 1 << 20),
                                        (1_000_003, 1 << 40), (300_001, None)])
def test_sort_i64_matches_stable_argsort(count, span):
    """The device radix sort against numpy's stable argsort: values and
    positions element by element, on ragged tile counts, all-equal arrays (no
    digit pass), ties, negative values and the full int64 range (8 passes)."""
    rng = np.random.default_rng(count)
    if span is None:
        v = rng.integers(-(1 << 63), (1 << 63) - 1, size=count, dtype=np.int64, endpoint=True)
        v[:2] = [-(1 << 63), (1 << 63) - 1]
    else:
        v = -5_000 + rng.integers(0, span + 1, size=count, dtype=np.int64)
    if count > 10:
        v[rng.integers(0, count, count // 4)] = v[0]  # ties
    t = torch.from_numpy(v).to(DEV)
    say(f"sort count={count} span={span}")
    s, i = ko.ko_sort_i64(t)
    want_i = np.argsort(v, kind="stable")
    assert np.array_equal(i.cpu().numpy(), want_i)
    assert np.array_equal(s.cpu().numpy(), v[want_i])
    # in place, values only
    ko.ko_sort_i64(t, sorted_out=t, want_index=False)
    assert np.array_equal(t.cpu().numpy(), v[want_i])


def test_median_gain_on_device_matches_oracle():
    rng = np.random.default_rng(3)
    for n in (1, 2, 7, 720, 40_320):
        m = rng.integers(1000, 1300, n)
        t_alg = int(rng.integers(900, 1100))
        got = ko.median_gain(torch.from_numpy(m).to(DEV), t_alg)
        assert got == ostats.median_gain(m, t_alg), n


@pytest.mark.parametrize("count", [0, 1, 255, 256, 257, 70_001, 3_628_800])
def test_stats_i64_matches_oracle(count):
    """Device statistics of an int64 array against the oracle's set_stats:
    extremes with the smallest index on ties, counts against a reference,
    on ragged sizes, heavy ties and negative values."""
    rng = np.random.default_rng(count + 11)
    v = rng.integers(-50, 400, size=count, dtype=np.int64)
    if count > 10:
        v[rng.integers(0, count, count // 3)] = 7   # ties at a middle value
        v[count - 1] = v.min()                      # a tie of the minimum at the end
    t = torch.from_numpy(v).to(DEV)
    ref = torch.tensor([7], dtype=torch.int64, device=DEV)
    say(f"stats count={count}")
    rec = ko.stats_records(ko.ko_stats_i64(t, ref=ref))[0]
    assert rec["n_orders"] == count
    if count == 0:
        assert rec["min_makespan"] == np.iinfo(np.int64).max and rec["max_makespan"] == np.iinfo(np.int64).min
        assert rec["argmin"] == 0 and rec["argmax"] == 0
        return
    want = ostats.set_stats(v, ref=7)
    assert (rec["min_makespan"], rec["max_makespan"]) == (want["min"], want["max"])
    assert (rec["argmin"], rec["argmax"]) == (want["argmin"], want["argmax"])
    assert (rec["n_less"], rec["n_equal"], rec["n_greater"]) == (want["n_less"], want["n_equal"], want["n_greater"])
    # without a reference the counts are zero
    rec = ko.stats_records(ko.ko_stats_i64(t))[0]
    assert (rec["n_less"], rec["n_equal"], rec["n_greater"]) == (0, 0, 0)
