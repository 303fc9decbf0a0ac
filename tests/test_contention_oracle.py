"""Pins of the oracle's memory-contention model (Section 4: resident blocks
share the chip's memory throughput).  Nothing here touches the GPU or the
library: the event-driven oracle is checked against a hand trace, closed
forms, a cycle-by-cycle formulation, a roofline bound and the first model."""

import itertools

import numpy as np
import pytest

import oracle
from oracle.tick import tick_contended_makespan


def test_e5_hand_trace(golden):
    g = golden("e5_contention.json")
    orders = np.array(g["orders"], dtype=np.int32)
    got = oracle.contended_makespans(g["gpu"], g["kernels"], g["mem_blocks"], orders)
    assert got.tolist() == g["makespans"]
    base = oracle.makespans_orders(g["gpu"], g["kernels"], orders)
    assert base.tolist() == g["makespans_without_contention"]
    _, dur = oracle.derive(g["gpu"], g["kernels"])
    assert dur.tolist() == g["durations"]


def test_memory_bound_blocks_sharing_one_block_of_bandwidth():
    """Closed form: m memory-bound blocks of duration d, all resident from
    t = 0 on m CUs with B = 1, each get 1/m of the bandwidth, so all end
    together at m * d (m a power of two, so the rate 65536/m is exact); with
    B = m there is no slowdown and the makespan is d."""
    for m in (1, 2, 4, 8, 16):
        gpu = dict(n_cu=m, wave_size=64, wave_cu=4, blk_cu=1, reg_cu=65536, lds_cu=65536, rb_milli=10000)
        ks = [dict(n_tblk=m, n_inst=700, lds_blk=0, waves_blk=1, regs_thr=32, r_milli=2500)]
        d = 700 * 10000 // 2500
        assert oracle.contended_makespans(gpu, ks, 1, [[0]]).tolist() == [m * d]
        assert oracle.contended_makespans(gpu, ks, m, [[0]]).tolist() == [d]


def test_compute_bound_blocks_use_their_share():
    """Closed form: 8 resident compute-bound blocks with R = 4 R_B use a
    quarter of a block's bandwidth each (share 256): with B = 1 they need two
    blocks' worth, so every one runs at half speed and the makespan is 2 d;
    with B = 2 exactly the bandwidth there is, so d."""
    gpu = dict(n_cu=8, wave_size=64, wave_cu=4, blk_cu=1, reg_cu=65536, lds_cu=65536, rb_milli=2000)
    ks = [dict(n_tblk=8, n_inst=1000, lds_blk=0, waves_blk=1, regs_thr=32, r_milli=8000)]
    assert oracle.contended_makespans(gpu, ks, 1, [[0]]).tolist() == [2000]
    assert oracle.contended_makespans(gpu, ks, 2, [[0]]).tolist() == [1000]


def _random_case(rng, n_max=4):
    n = int(rng.integers(1, n_max + 1))
    gpu = dict(n_cu=int(rng.integers(1, 4)), wave_size=32, wave_cu=8, blk_cu=int(rng.integers(1, 5)),
               reg_cu=65536, lds_cu=65536, rb_milli=int(rng.integers(500, 5000)))
    ks = [dict(n_tblk=int(rng.integers(1, 7)), n_inst=int(rng.integers(1, 30)),
               lds_blk=int(rng.integers(0, 3)) * 16384, waves_blk=int(rng.integers(1, 4)), regs_thr=16,
               r_milli=int(rng.integers(100, 20000))) for _ in range(n)]
    return gpu, ks


@pytest.mark.parametrize("seed", range(12))
def test_cycle_by_cycle_formulation_agrees(seed):
    """Brute force: every order of a tiny random set, the event-driven oracle
    against the model advanced one cycle at a time."""
    rng = np.random.default_rng(1000 + seed)
    gpu, ks = _random_case(rng)
    B = int(rng.integers(1, 4))
    orders = np.array(list(itertools.permutations(range(len(ks)))), dtype=np.int32)
    got = oracle.contended_makespans(gpu, ks, B, orders)
    want = [tick_contended_makespan(gpu, ks, list(o), B) for o in orders]
    assert got.tolist() == want


@pytest.mark.parametrize("seed", range(12))
def test_enough_bandwidth_gives_the_first_model(seed):
    """When B covers every block the chip can hold, nothing slows down: the
    makespans equal the first model's for every order."""
    rng = np.random.default_rng(2000 + seed)
    gpu, ks = _random_case(rng, 5)
    B = gpu["n_cu"] * gpu["blk_cu"]
    orders = np.array(list(itertools.permutations(range(len(ks)))), dtype=np.int32)
    assert oracle.contended_makespans(gpu, ks, B, orders).tolist() == \
        oracle.makespans_orders(gpu, ks, orders).tolist()


@pytest.mark.parametrize("seed", range(8))
def test_memory_roofline_bound(seed):
    """The memory system delivers at most B blocks' worth per cycle, so the
    makespan is at least the memory work sum_blocks share * d / (1024 * B);
    and never below the first model's makespan (slowdown only stretches)."""
    rng = np.random.default_rng(3000 + seed)
    gpu, ks = _random_case(rng, 5)
    B = int(rng.integers(1, 3))
    _, dur = oracle.derive(gpu, ks)
    rb = gpu["rb_milli"]
    work = sum(k["n_tblk"] * -(-1024 * min(k["r_milli"], rb) // k["r_milli"]) * int(d) for k, d in zip(ks, dur))
    orders = np.array(list(itertools.permutations(range(len(ks)))), dtype=np.int32)
    ms = oracle.contended_makespans(gpu, ks, B, orders)
    assert (ms * 1024 * B >= work).all()
    assert (ms >= oracle.makespans_orders(gpu, ks, orders)).all()


def test_order_free_when_every_block_is_resident_at_once():
    """Section 3's case: when all blocks of the set are placed at t = 0 the
    resident set, hence the makespan, is the same for every order."""
    gpu = dict(n_cu=4, wave_size=64, wave_cu=32, blk_cu=8, reg_cu=131072, lds_cu=163840, rb_milli=10000)
    rng = np.random.default_rng(7)
    ks = [dict(n_tblk=int(rng.integers(1, 5)), n_inst=int(rng.integers(100, 5000)), lds_blk=0, waves_blk=1,
               regs_thr=16, r_milli=int(rng.integers(500, 50000))) for _ in range(5)]
    orders = np.array(list(itertools.permutations(range(5))), dtype=np.int32)
    ms = oracle.contended_makespans(gpu, ks, 2, orders)
    assert len(set(ms.tolist())) == 1


def test_ranks_and_explicit_orders_agree():
    rng = np.random.default_rng(11)
    gpu, ks = _random_case(rng, 4)
    n = len(ks)
    orders = np.array([oracle.unrank(n, r) for r in range(int(np.prod(range(1, n + 1))))], dtype=np.int32)
    a = oracle.contended_makespans(gpu, ks, 1, orders)
    b = oracle.contended_makespans(gpu, ks, 1, None, first=0, count=len(orders))
    assert a.tolist() == b.tolist()


def test_rejects_bad_input():
    gpu, ks = _random_case(np.random.default_rng(0), 3)
    with pytest.raises(ValueError):
        oracle.contended_makespans(gpu, ks, 0, [list(range(len(ks)))])
    with pytest.raises(ValueError):
        oracle.contended_makespans(gpu, ks, 1, [[0] * len(ks)] if len(ks) > 1 else [[1]])
