"""Host logic of the surrogate's beam search: the capped selection keeps the
best-scored candidates (ties by index) with at most `cap` per parent, exactly
as a greedy scan in score order would."""

import numpy as np
import pytest

pytest.importorskip("torch")
from paper_1511_07983_amd.surrogate import _capped_best  # noqa: E402


def test_capped_selection_matches_greedy_scan():
    rng = np.random.default_rng(0)
    for trial in range(300):
        n = int(rng.integers(1, 300))
        sc = rng.integers(0, 20, n).astype(np.float32)   # many ties
        par = rng.integers(0, int(rng.integers(1, 40)), n)
        keep = int(rng.integers(1, n + 1))
        cap = int(rng.integers(1, 6))
        want, cnt = [], {}
        for i in sorted(range(n), key=lambda i: (sc[i], i)):
            if cnt.get(par[i], 0) < cap:
                want.append(i)
                cnt[par[i]] = cnt.get(par[i], 0) + 1
            if len(want) == keep:
                break
        assert list(_capped_best(sc, par, keep, cap)) == want, trial


def test_large_cap_is_plain_top_k():
    rng = np.random.default_rng(1)
    sc = rng.normal(size=500).astype(np.float32)
    par = rng.integers(0, 7, 500)
    got = _capped_best(sc, par, 64, 10_000)
    assert list(got) == list(np.lexsort((np.arange(500), sc))[:64])
