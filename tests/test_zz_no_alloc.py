"""GPU test of ko_simulate_batch_noalloc, the entry point that allocates
nothing: its outputs must equal ko_simulate_batch's bit for bit on two calls
in a row (the second on a smaller batch, so stale contents of the shared
static scratch would show), and a batch too large for the scratch must be
refused before any device work.
"""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")

DEV = "cuda:0"


def say(*a):
    print("[noalloc-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def run(entry, model, kernels, offsets, spec, ref=None, n_bins=0):
    n_sets = len(offsets) - 1
    _, total = ko.ko_count_orders(offsets, spec)
    ms = torch.full((max(total, 1),), -7, dtype=torch.int64, device=DEV)
    st = torch.full((8 * n_sets,), -7, dtype=torch.int64, device=DEV)
    h = torch.full((max(n_sets * n_bins, 1),), -7, dtype=torch.int64, device=DEV) if n_bins else None
    entry(model, kernels, offsets, spec, ref_makespan=ref, makespans=ms, stats=st, hist=h, n_bins=n_bins)
    ko.ko_sync()
    return (ms[:total].cpu().numpy(), st.cpu().numpy(), None if h is None else h.cpu().numpy())


def check_same(model, kernels, offsets, spec, ref=None, n_bins=0, label=""):
    say(label, "sets", len(offsets) - 1, "kernels", len(kernels))
    want = run(ko.ko_simulate_batch, model, kernels, offsets, spec, ref, n_bins)
    got = run(ko.ko_simulate_batch_noalloc, model, kernels, offsets, spec, ref, n_bins)
    assert len(want[0]) > 0
    np.testing.assert_array_equal(got[0], want[0])
    np.testing.assert_array_equal(got[1], want[1])
    if n_bins:
        np.testing.assert_array_equal(got[2], want[2])


def test_noalloc_matches_batch_on_two_calls_second_smaller():
    # first call: all 10! orders of the n = 10 set on the MI355X model (lane
    # engine), with a reference makespan and a histogram
    k1 = synth.draw_set(1, 0)
    off1 = np.array([0, len(k1)], dtype=np.int32)
    ref1 = torch.tensor([int(2_000_000)], dtype=torch.int64, device=DEV)
    check_same(synth.MI355X_MODEL, k1, off1, ko.OrderSpec.all(), ref=ref1, n_bins=512, label="n=10 all")
    # second call, smaller: the 720 orders of the n = 6 set on the 16-CU model
    # (wave engine), with a different reference and fewer bins
    k0 = synth.draw_set(0, 0)
    off0 = np.array([0, len(k0)], dtype=np.int32)
    ref0 = torch.tensor([int(300_000)], dtype=torch.int64, device=DEV)
    check_same(synth.SMALL_MODEL, k0, off0, ko.OrderSpec.all(), ref=ref0, n_bins=32, label="n=6 all")


def test_noalloc_many_sets_sampled_and_explicit():
    kernels, offsets = synth.draw_sets(2, 0, 300)
    per = np.full(300, 3000, dtype=np.int64)
    ref = torch.arange(300, dtype=torch.int64, device=DEV) * 5000 + 1_500_000
    check_same(synth.MI355X_MODEL, kernels, offsets, ko.OrderSpec.sampled(per, seed=99), ref=ref, n_bins=64,
               label="300 sets sampled")
    # then a smaller explicit batch: 3 sets, their reversed and identity orders
    kernels, offsets = synth.draw_sets(2, 7, 3)
    rows = []
    for s in range(3):
        n = int(offsets[s + 1] - offsets[s])
        rows += [list(range(n)), list(range(n))[::-1]]
    orders = torch.tensor(np.concatenate([np.asarray(r, dtype=np.uint8) for r in rows]), device=DEV)
    spec = ko.OrderSpec.explicit(orders, np.full(3, 2, dtype=np.int64))
    check_same(synth.MI355X_MODEL, kernels, offsets, spec, label="3 sets explicit")


def test_noalloc_full_batch_workload_chunks_fit():
    # all 4096 sets of the batch workload: the chunk grows so the items fit
    kernels, offsets = synth.draw_sets(2)
    check_same(synth.MI355X_MODEL, kernels, offsets, ko.OrderSpec.all(), label="4096 sets all")


def test_noalloc_rejects_a_batch_larger_than_the_scratch():
    # 200,000 one-kernel sets: their records alone exceed 16 MiB
    k = synth.draw_set(0, 0)[:1]
    kernels = np.repeat(k, 200_000)
    offsets = np.arange(200_001, dtype=np.int32)
    spec = ko.OrderSpec.all()
    with pytest.raises(ko.KoError) as e:
        ko.ko_simulate_batch_noalloc(synth.SMALL_MODEL, kernels, offsets, spec)
    assert e.value.code == ko.KO_ERANGE
    assert "static scratch" in str(e.value)
    # the entry point still works afterwards
    k0 = synth.draw_set(0, 1)
    check_same(synth.SMALL_MODEL, k0, np.array([0, len(k0)], dtype=np.int32), ko.OrderSpec.all(),
               label="after refusal")
