"""Host-side checks of libko that need no GPU: exported symbols, the
launch-order heuristic (host code) against the oracle, order counting, and the
argument validation that precedes any device work."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle.heuristic import heuristic_order as oracle_heuristic

ko = pytest.importorskip("paper_1511_07983_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ko.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(ko_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert "ko_simulate_batch" in names and "ko_heuristic_order" in names
    lib = ctypes.CDLL(ko.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ko.EXPORTED)


def test_heuristic_hand_examples(golden):
    e1 = golden("e1_two_cu.json")
    for flags in range(4):
        assert ko.ko_heuristic_order(e1["gpu"], e1["kernels"], flags) == e1["heuristic_order_all_flags"]
    e2 = golden("e2_heuristic.json")
    modes = {"per_sm_share_insert_unit": 0, "per_block_insert_unit": 1,
             "per_sm_share_full_sort": 2, "per_block_full_sort": 3}
    for name, flags in modes.items():
        order, rounds = ko.ko_heuristic_order(e2["gpu"], e2["kernels"], flags, with_rounds=True)
        assert order == e2["orders"][name]["order"]
        assert rounds == e2["orders"][name]["rounds"]


@pytest.mark.parametrize("workload", [0, 1, 2, 3, 4])
def test_heuristic_matches_oracle(workload):
    """The C++ heuristic and the Python oracle agree exactly (same binary64
    arithmetic, same tie rules) on every flag combination."""
    model = synth.WORKLOADS[workload].model
    for s in range(300 if workload != 4 else 120):
        ks = synth.draw_set(workload, s)
        for flags in range(4):
            a = ko.ko_heuristic_order(model, ks, flags, with_rounds=True)
            b = oracle_heuristic(model.as_dict(), ks, flags)
            assert (list(a[0]), list(a[1])) == (list(b[0]), list(b[1])), (s, flags)


def test_heuristic_matches_oracle_random_models():
    rng = np.random.default_rng(3)
    for trial in range(400):
        model = synth.GpuModel(n_cu=int(rng.integers(1, 64)), wave_size=int(rng.choice([32, 64])),
                               wave_cu=int(rng.integers(8, 65)), blk_cu=int(rng.integers(1, 33)),
                               reg_cu=int(rng.integers(16384, 262144)),
                               lds_cu=int(rng.integers(49152, 200000)),
                               rb_milli=int(rng.integers(500, 20000)))
        n = int(rng.integers(1, 21))
        ks = synth.draw_kernels(rng, n, 1, 500)
        ks["waves_blk"] = np.minimum(ks["waves_blk"], model.wave_cu)
        ks["regs_thr"] = np.minimum(ks["regs_thr"], model.reg_cu // (ks["waves_blk"] * model.wave_size))
        for flags in range(4):
            a = ko.ko_heuristic_order(model, ks, flags, with_rounds=True)
            b = oracle_heuristic(model.as_dict(), ks, flags)
            assert (list(a[0]), list(a[1])) == (list(b[0]), list(b[1]))


def test_count_orders():
    per, total = ko.ko_count_orders([0, 6, 16, 20], ko.OrderSpec.all())
    assert per.tolist() == [720, 3628800, 24] and total == 720 + 3628800 + 24
    per, total = ko.ko_count_orders([0, 3, 5], ko.OrderSpec.rank_range([[1, 4], [0, 2]]))
    assert per.tolist() == [3, 2]
    per, total = ko.ko_count_orders([0, 3, 5], ko.OrderSpec.sampled([7, 0], seed=1))
    assert per.tolist() == [7, 0] and total == 7
    with pytest.raises(ko.KoError) as e:
        ko.ko_count_orders([0] + [20 * (i + 1) for i in range(8)], ko.OrderSpec.all())
    assert e.value.code == ko.KO_ERANGE
    with pytest.raises(ko.KoError) as e:
        ko.ko_count_orders([0, 3], ko.OrderSpec.rank_range([[2, 7]]))
    assert e.value.code == ko.KO_EINVAL


def test_count_orders_sampled_counter_limits():
    """A sample's counter is set * 2^40 + index: at most 2^40 samples per set
    and 2^24 sets, else the streams of two samples would coincide."""
    per, total = ko.ko_count_orders([0, 3], ko.OrderSpec.sampled([1 << 40], seed=1))
    assert total == 1 << 40
    with pytest.raises(ko.KoError) as e:
        ko.ko_count_orders([0, 3], ko.OrderSpec.sampled([(1 << 40) + 1], seed=1))
    assert e.value.code == ko.KO_ERANGE
    n_sets = (1 << 24) + 1
    off = np.arange(n_sets + 1, dtype=np.int32)
    with pytest.raises(ko.KoError) as e:
        ko.ko_count_orders(off, ko.OrderSpec.sampled(np.ones(n_sets, dtype=np.int64), seed=1))
    assert e.value.code == ko.KO_ERANGE
    # the same batch of all orders is not limited by the counter
    per, total = ko.ko_count_orders(off, ko.OrderSpec.all())
    assert total == n_sets


def _call_simulate(gpu, ks, off, spec, n_bins=0, want_hist=False, want_stats=False):
    """Invoke the raw ABI with dummy non-null device pointers where a buffer is
    'given': every case here must be rejected before any device access."""
    lib = ko.library_handle()
    g = ko.gpu_model(gpu)
    k = ko.kernel_array(ks)
    o = np.ascontiguousarray(off, dtype=np.int32)
    sp = spec.c_struct()
    dummy = ctypes.c_void_p(0x1000)
    rc = lib.ko_simulate_batch(ctypes.byref(g), k.ctypes.data if len(k) else None,
                               o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(o) - 1,
                               ctypes.byref(sp), None, dummy if want_hist else None,
                               dummy if want_stats else None, dummy if want_hist else None,
                               n_bins, None)
    return rc


def test_simulate_rejects_bad_arguments_before_device_work():
    gpu = synth.MI355X_MODEL.as_dict()
    ks = synth.draw_set(0, 0)
    good = [0, len(ks)]
    assert _call_simulate(dict(gpu, n_cu=0), ks, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    assert _call_simulate(dict(gpu, n_cu=257), ks, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    assert _call_simulate(dict(gpu, blk_cu=256), ks, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    assert _call_simulate(dict(gpu, lds_cu=1 << 24), ks, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    big = ks.copy()
    big["lds_blk"][0] = gpu["lds_cu"] + 1  # one block larger than an empty CU
    assert _call_simulate(gpu, big, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    zero = ks.copy()
    zero["n_tblk"][1] = 0
    assert _call_simulate(gpu, zero, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    assert _call_simulate(gpu, ks, [0, 0, len(ks)], ko.OrderSpec.all()) == ko.KO_EINVAL
    k21 = np.concatenate([ks] * 4)[:21]
    assert _call_simulate(gpu, k21, [0, 21], ko.OrderSpec.all()) == ko.KO_EINVAL
    assert _call_simulate(gpu, ks, good, ko.OrderSpec.rank_range([[5, 4]])) == ko.KO_EINVAL
    assert _call_simulate(gpu, ks, good, ko.OrderSpec.sampled([-1], 0)) == ko.KO_EINVAL
    assert _call_simulate(gpu, ks, good, ko.OrderSpec(7)) == ko.KO_EINVAL
    # a histogram needs stats and a bin count in range
    assert _call_simulate(gpu, ks, good, ko.OrderSpec.all(), n_bins=16, want_hist=True) == ko.KO_EINVAL
    assert _call_simulate(gpu, ks, good, ko.OrderSpec.all(), n_bins=0, want_hist=True,
                          want_stats=True) == ko.KO_EINVAL
    # a duration above 2^31-1 cycles
    slow = ks.copy()
    slow["n_inst"][0] = 1 << 40
    assert _call_simulate(gpu, slow, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    assert "duration" in ko.ko_last_error()


def test_memory_contention_parameter_checks():
    """mem_blocks (Section 4's shared memory throughput) is 0 or 1 .. 2^24;
    Algorithm 1 does not read it, the round-synchronous model refuses it."""
    gpu = synth.MI355X_MODEL.as_dict()
    ks = synth.draw_set(0, 0)
    good = [0, len(ks)]
    assert _call_simulate(dict(gpu, mem_blocks=-1), ks, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    assert _call_simulate(dict(gpu, mem_blocks=(1 << 24) + 1), ks, good, ko.OrderSpec.all()) == ko.KO_EINVAL
    assert "mem_blocks" in ko.ko_last_error()
    for b in (1, 77, 1 << 24):
        assert ko.ko_heuristic_order(dict(gpu, mem_blocks=b), ks, with_rounds=True) == \
            ko.ko_heuristic_order(gpu, ks, with_rounds=True)
    lib = ko.library_handle()
    g = ko.gpu_model(dict(gpu, mem_blocks=4))
    k = ko.kernel_array(ks)
    dummy = ctypes.c_void_p(0x1000)
    rc = lib.ko_simulate_rounds(ctypes.byref(g), k.ctypes.data, len(k), None, 0, 10, dummy, None)
    assert rc == ko.KO_EINVAL and "mem_blocks" in ko.ko_last_error()


def test_rank_percentile_and_heuristic_reject_bad_arguments():
    gpu = synth.SMALL_MODEL.as_dict()
    ks = synth.draw_set(0, 0)
    with pytest.raises(ko.KoError) as e:
        ko.ko_rank_percentile(gpu, ks, [0, 1, 2, 3, 4, 4], stream=0)
    assert e.value.code == ko.KO_EINVAL
    with pytest.raises(ko.KoError) as e:
        ko.ko_heuristic_order(gpu, ks, flags=8)
    assert e.value.code == ko.KO_EINVAL
    with pytest.raises(ko.KoError):
        ko.ko_heuristic_order(gpu, [], 0)


def test_float_quotient_rule_is_exact():
    """The device computes floor(fr/u) as trunc(float(fr) * inv) minus one
    when (q * u > fr), with inv = 1/u rounded to float and raised by 3 ulps,
    clamped to the free block slots (<= 255).  Exhaustive over small u and
    near every multiple for large u, emulated in IEEE float32."""
    f32 = np.float32
    inf = f32(np.inf)
    for u in list(range(1, 600)) + [1000, 4095, 4096, 8192, 12288, 20480, 32768, 49152,
                                   131071, 131072, 163840, (1 << 24) - 1]:
        inv = f32(1.0 / u)
        for _ in range(3):
            inv = np.nextafter(inv, inf)
        cap = (1 << 24) - 1
        mults = np.arange(0, min(cap // u, 300) + 1, dtype=np.int64) * u
        fr = np.unique(np.clip(np.concatenate([mults - 1, mults, mults + 1, mults + u // 2]), 0, cap))
        if u < 64:
            fr = np.unique(np.concatenate([fr, np.arange(0, 20000, dtype=np.int64)]))
        fr = np.concatenate([fr, np.array([cap, cap - 1, cap - u], dtype=np.int64)])
        fr = fr[fr >= 0]
        q = (fr.astype(f32) * inv).astype(np.float32)
        q = np.trunc(q).astype(np.int64)
        for clamp in (255, 32, 1):
            qc = np.minimum(q, clamp)
            qc = qc - (qc * u > fr)
            assert np.array_equal(qc, np.minimum(fr // u, clamp)), (u, clamp)


def test_sampling_and_selection_reject_bad_arguments_before_device_work():
    lib = ko.library_handle()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    assert lib.ko_sample_orders(0, 0, 1, 0, None, 4, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_sample_orders(21, 0, 1, 0, None, 4, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_sample_orders(5, -1, 1, 0, None, 4, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_sample_orders(5, 1 << 24, 1, 0, None, 4, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_sample_orders(5, 0, 1, 0, None, 4, None, None, None) == ko.KO_EINVAL
    assert lib.ko_sample_orders(5, 0, 1, (1 << 40) - 3, None, 4, fake, None, None) == ko.KO_ERANGE
    assert lib.ko_sample_orders(5, 0, 1, 0, None, (1 << 40) + 1, fake, None, None) == ko.KO_ERANGE
    assert lib.ko_sample_orders(5, 0, 1, 0, None, 0, fake, None, None) == ko.KO_OK
    g = ko.gpu_model(synth.SMALL_MODEL)
    ks = ko.kernel_array(synth.random_tiny_set(np.random.default_rng(0), 4, synth.SMALL_MODEL))
    kp = ks.ctypes.data
    rounds = lib.ko_simulate_rounds
    assert rounds(ctypes.byref(g), kp, 0, fake, 0, 4, fake, None) == ko.KO_EINVAL
    assert rounds(ctypes.byref(g), kp, 21, fake, 0, 4, fake, None) == ko.KO_EINVAL
    assert rounds(ctypes.byref(g), kp, 4, fake, 0, 4, None, None) == ko.KO_EINVAL
    assert rounds(ctypes.byref(g), kp, 4, fake, 1, 4, fake, None) == ko.KO_EINVAL
    assert rounds(ctypes.byref(g), kp, 4, fake, 0, (1 << 40) + 1, fake, None) == ko.KO_ERANGE
    assert rounds(ctypes.byref(g), kp, 4, None, 20, 5, fake, None) == ko.KO_ERANGE
    assert rounds(ctypes.byref(g), kp, 4, None, 25, 0, fake, None) == ko.KO_ERANGE
    assert rounds(None, kp, 4, fake, 0, 4, fake, None) == ko.KO_EINVAL
    assert rounds(ctypes.byref(g), kp, 4, None, 24, 0, None, None) == ko.KO_OK
    assert lib.ko_topk_f32(None, 10, 1, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_topk_f32(fake, 10, 0, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_topk_f32(fake, 10, 11, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_topk_f32(fake, 0, 1, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_topk_f32(fake, 1 << 32, 5, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_topk_f32(fake, 100000, 16385, fake, None, None) == ko.KO_EINVAL
    assert lib.ko_topk_f32(fake, 10, 1, None, None, None) == ko.KO_EINVAL
    out = ctypes.c_int64()
    assert lib.ko_kth_smallest_i64(fake, 10, 0, ctypes.byref(out), None, None) == ko.KO_EINVAL
    assert lib.ko_kth_smallest_i64(fake, 10, 11, ctypes.byref(out), None, None) == ko.KO_EINVAL
    assert lib.ko_kth_smallest_i64(None, 10, 1, ctypes.byref(out), None, None) == ko.KO_EINVAL
    assert lib.ko_kth_smallest_i64(fake, 10, 1, None, None, None) == ko.KO_EINVAL


def test_plan_and_graph_reject_bad_arguments_before_device_work():
    lib = ko.library_handle()
    gpu = ko.gpu_model(dict(synth.MI355X_MODEL.as_dict(), n_cu=0))
    ks = ko.kernel_array(synth.draw_set(0, 0))
    off = np.array([0, len(ks)], dtype=np.int32)
    spec = ko.OrderSpec.all().c_struct()
    out = ctypes.c_void_p()
    cfg = ko.KoLaunchConfig(0, 0)
    assert lib.ko_plan_create(ctypes.byref(gpu), ks.ctypes.data, off.ctypes.data_as(ko._i32p), 1,
                              ctypes.byref(spec), ctypes.byref(cfg), ctypes.byref(out)) == ko.KO_EINVAL
    good = ko.gpu_model(synth.MI355X_MODEL)
    for bad in (ko.KoLaunchConfig(21, 0), ko.KoLaunchConfig(-1, 0), ko.KoLaunchConfig(0, 65),
                ko.KoLaunchConfig(0, 0, 3, 0), ko.KoLaunchConfig(0, 0, -1, 0), ko.KoLaunchConfig(0, 0, 2, 65),
                ko.KoLaunchConfig(0, 0, 2, -1)):
        assert lib.ko_plan_create(ctypes.byref(good), ks.ctypes.data, off.ctypes.data_as(ko._i32p), 1,
                                  ctypes.byref(spec), ctypes.byref(bad), ctypes.byref(out)) == ko.KO_EINVAL
    assert lib.ko_plan_create(ctypes.byref(good), ks.ctypes.data, off.ctypes.data_as(ko._i32p), 1,
                              ctypes.byref(spec), None, None) == ko.KO_EINVAL
    assert lib.ko_plan_info(None, None, None, None, None) == ko.KO_EINVAL
    assert lib.ko_plan_launch(None, None, None, None, None, 0, None) == ko.KO_EINVAL
    assert lib.ko_plan_status(None, None) == ko.KO_EINVAL
    assert lib.ko_plan_engine(None, None, None, None, None, None) == ko.KO_EINVAL
    assert lib.ko_graph_capture(None, None, None, None, None, 0, None, ctypes.byref(out)) == ko.KO_EINVAL
    assert lib.ko_graph_launch(None, None) == ko.KO_EINVAL
    assert lib.ko_plan_destroy(None) == ko.KO_OK
    assert lib.ko_graph_destroy(None) == ko.KO_OK
