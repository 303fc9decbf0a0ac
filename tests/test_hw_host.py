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


def test_calibration_recovers_a_linear_map():
    """The cycles-to-milliseconds fit of the hardware validation: exact data
    give back the slope, the offset and R^2 = 1; noise lowers R^2."""
    from paper_1511_07983_amd import hw
    rng = np.random.default_rng(3)
    rows = []
    for s in range(4):
        cyc = rng.integers(10_000_000, 90_000_000, 8)
        ms = 0.4e-6 * cyc + 0.25          # 0.4 ns per cycle at full scale, 0.25 ms offset
        rows.append({"simulated_cycles": cyc.tolist(), "measured_ms": ms.tolist(), "scale": 256})
    fit = hw.calibrate(rows)
    assert abs(fit["ns_per_model_cycle"] - 0.4) < 1e-9 and abs(fit["offset_ms"] - 0.25) < 1e-9
    assert abs(fit["r2"] - 1.0) < 1e-12 and fit["points"] == 32
    for r in rows:
        r["measured_ms"] = (np.array(r["measured_ms"]) + rng.normal(0, 2.0, 8)).tolist()
    assert hw.calibrate(rows)["r2"] < 0.999
