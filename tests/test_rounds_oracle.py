"""Pins of the oracle's round-synchronous model (Section 2's execution rounds).

Each check compares the block-by-block simulation with something it does not
compute itself: a hand trace, a closed form for one kernel, a closed form for
one block per CU, or an order-independence fact stated in Sections 2 and 3.
"""

import itertools
import math

import numpy as np
import pytest

import oracle
import synth


def _orders(n):
    return np.array(list(itertools.permutations(range(n))), dtype=np.int32)


def test_rounds_hand_trace(golden):
    g = golden("e4_rounds.json")
    _, dur = oracle.derive(g["gpu"], g["kernels"])
    assert dur.tolist() == g["durations"]
    got = oracle.rounds_makespans(g["gpu"], g["kernels"], g["orders"])
    assert got.tolist() == g["rounds_makespans"]
    # the event model releases blocks one by one and differs on this order
    assert oracle.makespan(g["gpu"], g["kernels"], g["orders"][0]) == g["event_model_makespan_ABC"]


def _cap(gpu, k):
    """Blocks of kernel k that fit one empty CU (Table 1 limits)."""
    regs = int(k["regs_thr"]) * int(k["waves_blk"]) * gpu.wave_size
    c = min(gpu.blk_cu, gpu.reg_cu // regs, gpu.wave_cu // int(k["waves_blk"]))
    if int(k["lds_blk"]) > 0:
        c = min(c, gpu.lds_cu // int(k["lds_blk"]))
    return c


@pytest.mark.parametrize("model", [synth.SMALL_MODEL, synth.GTX580_MODEL, synth.MI355X_MODEL])
def test_rounds_single_kernel_closed_form(model):
    # one kernel: every round fills every CU to the same count, so there are
    # ceil(blocks / (CUs x blocks per CU)) rounds of one block duration each
    rng = np.random.default_rng(7)
    for _ in range(40):
        ks = synth.random_tiny_set(rng, 1, model, tblk_hi=3000, inst_hi=500)
        _, dur = oracle.derive(model.as_dict(), ks)
        per_round = model.n_cu * _cap(model, ks[0])
        want = math.ceil(int(ks["n_tblk"][0]) / per_round) * int(dur[0])
        assert oracle.rounds_makespans(model.as_dict(), ks, [[0]]).tolist() == [want]


def test_rounds_one_block_per_cu_is_windows():
    # with one block slot per CU a round is exactly the next n_cu blocks of the
    # kernel-major stream, so the makespan is a sum of window maxima
    model = synth.GpuModel(n_cu=3, wave_size=32, wave_cu=64, blk_cu=1,
                           reg_cu=65536, lds_cu=65536, rb_milli=8000)
    rng = np.random.default_rng(11)
    for _ in range(12):
        n = int(rng.integers(2, 6))
        ks = synth.random_tiny_set(rng, n, model, tblk_hi=5, inst_hi=40)
        _, dur = oracle.derive(model.as_dict(), ks)
        orders = _orders(n)
        got = oracle.rounds_makespans(model.as_dict(), ks, orders)
        for o, m in zip(orders, got):
            stream = [int(dur[k]) for k in o for _ in range(int(ks["n_tblk"][k]))]
            want = sum(max(stream[i:i + model.n_cu]) for i in range(0, len(stream), model.n_cu))
            assert m == want


def test_rounds_few_blocks_one_round():
    # Section 2: with no more blocks than SMs no SM is shared and the order
    # has no effect; everything runs in one round as long as the longest block
    model = synth.SMALL_MODEL
    rng = np.random.default_rng(3)
    for _ in range(10):
        n = int(rng.integers(2, 6))
        ks = synth.random_tiny_set(rng, n, model, tblk_hi=model.n_cu // n, inst_hi=90)
        assert int(ks["n_tblk"].sum()) <= model.n_cu
        _, dur = oracle.derive(model.as_dict(), ks)
        got = oracle.rounds_makespans(model.as_dict(), ks, _orders(n))
        assert set(got.tolist()) == {int(dur.max())}


def test_rounds_identical_kernels_order_free():
    # Section 3: kernels that differ only in their block counts give the same
    # rounds in every order
    model = synth.SMALL_MODEL
    rng = np.random.default_rng(5)
    for _ in range(6):
        base = synth.random_tiny_set(rng, 1, model, tblk_hi=1, inst_hi=50)
        n = 5
        ks = np.repeat(base, n)
        ks["n_tblk"] = rng.integers(1, 60, size=n)
        got = oracle.rounds_makespans(model.as_dict(), ks, _orders(n))
        assert len(set(got.tolist())) == 1


def test_rounds_rejects_bad_orders():
    ks = synth.random_tiny_set(np.random.default_rng(1), 3, synth.SMALL_MODEL)
    with pytest.raises(ValueError):
        oracle.rounds_makespans(synth.SMALL_MODEL.as_dict(), ks, [[0, 0, 1]])


def test_rounds_one_block_per_cu_equal_durations_order_free():
    # Section 3: when every block takes a whole CU the order does not matter;
    # in this model that holds for equal block durations: every round but the
    # last is full, so the makespan is ceil(blocks / CUs) block durations
    model = synth.GpuModel(n_cu=4, wave_size=32, wave_cu=64, blk_cu=1,
                           reg_cu=65536, lds_cu=65536, rb_milli=8000)
    rng = np.random.default_rng(13)
    for _ in range(8):
        n = int(rng.integers(2, 6))
        ks = synth.random_tiny_set(rng, n, model, tblk_hi=9, equal_d=True)
        _, dur = oracle.derive(model.as_dict(), ks)
        assert len(set(dur.tolist())) == 1
        got = oracle.rounds_makespans(model.as_dict(), ks, _orders(n))
        want = math.ceil(int(ks["n_tblk"].sum()) / model.n_cu) * int(dur[0])
        assert set(got.tolist()) == {want}
