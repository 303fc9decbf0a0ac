"""Host-side checks of the hardware-validation helpers (no GPU)."""

import ctypes

import numpy as np
import pytest

ko = pytest.importorskip("paper_1511_07983_amd")


def test_spearman_matches_scipy():
    stats = pytest.importorskip("scipy.stats")
    from paper_1511_07983_amd.hw import spearman
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.integers(0, 6, size=9).astype(float)  # with ties
        b = a * 0.5 + rng.normal(size=9)
        assert spearman(a, b) == pytest.approx(stats.spearmanr(a, b).statistic, abs=1e-12)
    assert spearman([1, 2, 3], [10, 20, 30]) == pytest.approx(1.0)
    assert spearman([1, 2, 3], [3, 2, 1]) == pytest.approx(-1.0)


def test_hw_timing_rejects_bad_arguments_before_device_work():
    lib = ko.library_handle()
    k = ko.kernel_array(np.zeros(2, dtype=ko.KERNEL_DTYPE))
    out = (ctypes.c_double * 4)()
    order = np.array([0, 1], dtype=np.int32)
    # n_tblk = 0 is not launchable
    assert lib.ko_hw_time_orders(k.ctypes.data, 2, order.ctypes.data_as(ko._i32p), 1, 1, 1, out) == ko.KO_EINVAL
    good = k.copy()
    good["n_tblk"] = 4
    good["waves_blk"] = 2
    good["r_milli"] = 1000
    good["n_inst"] = 100
    bad_order = np.array([1, 1], dtype=np.int32)
    assert lib.ko_hw_time_orders(good.ctypes.data, 2, bad_order.ctypes.data_as(ko._i32p), 1, 1, 1,
                                 out) == ko.KO_EINVAL
    assert lib.ko_hw_time_orders(good.ctypes.data, 2, order.ctypes.data_as(ko._i32p), 1, 0, 1,
                                 out) == ko.KO_EINVAL
    assert lib.ko_hw_vgprs(16, None) == ko.KO_EINVAL
