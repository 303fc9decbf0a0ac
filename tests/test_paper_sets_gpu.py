"""Paper-shaped workloads on the GPU: every order of each Table 2 experiment,
Algorithm 1's order and its percentile, against the oracle bit for bit."""

import sys

import numpy as np
import pytest

import oracle
from oracle.heuristic import heuristic_order as oracle_heuristic
from synth import paper_sets

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ko = pytest.importorskip("paper_1511_07983_amd")
kb = pytest.importorskip("paper_1511_07983_amd.batch")


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def test_all_experiments_against_oracle():
    names = list(paper_sets.EXPERIMENTS)
    sets = [paper_sets.EXPERIMENTS[k] for k in names]
    print("[paper-sets] all orders of", names, file=sys.stderr, flush=True)
    res = kb.percentiles(paper_sets.MODEL, sets, want_makespans=True)
    ms = res["makespans"].cpu().numpy()
    g = paper_sets.MODEL.as_dict()
    off = 0
    for i, ks in enumerate(sets):
        want = oracle.makespans_all(g, ks)
        got = ms[off:off + len(want)]
        off += len(want)
        assert np.array_equal(got, want), names[i]
        order = oracle_heuristic(g, ks)[0]
        assert list(res["order"][i]) == list(order), names[i]
        ref = oracle.makespan(g, ks, order)
        assert res["makespan"][i] == ref
        assert res["n_less"][i] == int((want < ref).sum()) and res["n_equal"][i] == int((want == ref).sum())
        assert res["best"][i] == want.min() and res["worst"][i] == want.max()
