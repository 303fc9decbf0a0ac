"""Host-side checks of the surrogate library (no GPU): exports, features and
the lower bound against the oracle."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from oracle import features as ofeat
from oracle import mlp

ko = pytest.importorskip("paper_1511_07983_amd")
nn = pytest.importorskip("paper_1511_07983_amd.nn")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    text = open(os.path.join(ROOT, "include", "ko_nn.h")).read()
    names = sorted(set(re.findall(r"^(?:int|size_t|const char \*)\s*(ko_nn_\w+)\s*\(", text, re.M)))
    lib = ctypes.CDLL(nn.LIB_NN_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(nn.EXPORTED)


def test_parameter_count_matches_oracle():
    assert nn.num_params() == mlp.n_params() == 140289


@pytest.mark.parametrize("workload", [0, 1, 2, 3, 4])
def test_features_match_oracle(workload):
    model = synth.WORKLOADS[workload].model
    for s in range(40):
        ks = synth.draw_set(workload, s)
        got = nn.features(model, ks)
        want = np.array(ofeat.features(model.as_dict(), ks), dtype=np.float64)
        assert got.shape == want.shape
        assert np.allclose(got, want.astype(np.float32), rtol=2e-7, atol=1e-7)


@pytest.mark.parametrize("workload", [0, 1, 2, 4])
def test_lower_bound_matches_oracle_and_bounds_makespans(workload):
    model = synth.WORKLOADS[workload].model
    for s in range(30):
        ks = synth.draw_set(workload, s)
        lb = nn.lower_bound(model, ks)
        assert lb == ofeat.lower_bound(model.as_dict(), ks)
    # every order's makespan respects the bound (small sets, all orders)
    ks = synth.draw_set(0, 0)
    ms = oracle.makespans_all(synth.WORKLOADS[0].model.as_dict(), ks, threads=2)
    assert ms.min() >= nn.lower_bound(synth.WORKLOADS[0].model, ks)


def test_rejects_bad_arguments():
    with pytest.raises(ko.KoError):
        nn.features(dict(synth.MI355X_MODEL.as_dict(), n_cu=0), synth.draw_set(1, 0))
