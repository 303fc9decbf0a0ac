"""The beam step's selection rule, on the CPU: applying the per-prefix cap
(oracle/beam.py: only the `cap` best children of each prefix keep a finite
score) and then taking the `keep` lowest scores by (score, index) is the same
as a greedy scan of all candidates in score order that skips a candidate once
its prefix has `cap` children chosen.  The device runs the first form
(ko_nn_beam_cap, then ko_topk_f32); the GPU tests compare it with the oracle."""

import math

import numpy as np

from oracle import beam


def _select(ruled, keep):
    finite = [i for i in range(len(ruled)) if math.isfinite(ruled[i])]
    return sorted(finite, key=lambda i: (ruled[i], i))[:keep]


def test_cap_then_top_k_equals_greedy_scan():
    rng = np.random.default_rng(0)
    for trial in range(300):
        W = int(rng.integers(1, 40))
        m = int(rng.integers(1, 17))
        sc = rng.integers(0, 20, W * m).astype(np.float32)   # many ties
        par = np.repeat(np.arange(W), m)
        cap = int(rng.integers(1, 6))
        keep = int(rng.integers(1, W * min(cap, m) + 1))
        want, cnt = [], {}
        for i in sorted(range(W * m), key=lambda i: (sc[i], i)):
            if cnt.get(par[i], 0) < cap:
                want.append(i)
                cnt[par[i]] = cnt.get(par[i], 0) + 1
            if len(want) == keep:
                break
        assert _select(beam.cap(sc, m, cap), keep) == want, trial


def test_no_cap_is_plain_top_k():
    rng = np.random.default_rng(1)
    sc = rng.normal(size=7 * 12).astype(np.float32)
    got = _select(beam.cap(sc, 12, 0), 64)
    assert got == list(np.lexsort((np.arange(len(sc)), sc))[:64])
