"""Oracle: the bookkeeping of one beam-search step over launch orders.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A prefix is the list of kernels at launch positions 0..d-1.  One step:
  * expand: every prefix w grows by each of its n - d unused kernels, in
    increasing kernel index; candidate c = w (n - d) + t holds the position of
    every kernel (the prefix's position, d for the new kernel, 16 for a kernel
    not placed yet) and the pair (w, new kernel);
  * diversity rules on the candidates' scores: optionally a Gumbel variate
    times a temperature is added (u from SplitMix64 at counter (seed, c):
    u = (top 24 bits + 1/2) / 2^24, G = -log(-log u)); optionally only the
    `cap` lowest scores among one prefix's children are kept (ties by
    candidate order), the rest become +inf;
  * gather: the kept candidates' prefixes, each followed by its new kernel.
The selection of the best candidates is a plain sort by (score, index).
"""

from __future__ import annotations

import math

import numpy as np

from .sampling import splitmix64_at

UNPLACED = 16


def expand(prefix, n: int):
    """prefix: int array [W, d].  Returns (pos [W (n-d), n] uint8, parent [C], kernel [C])."""
    prefix = np.asarray(prefix, dtype=np.int64)
    W, d = prefix.shape
    pos, parent, kernel = [], [], []
    for w in range(W):
        unused = [k for k in range(n) if k not in set(prefix[w].tolist())]
        for k in unused:
            p = [UNPLACED] * n
            for j, kk in enumerate(prefix[w]):
                p[kk] = j
            p[k] = d
            pos.append(p)
            parent.append(w)
            kernel.append(k)
    return np.array(pos, dtype=np.uint8).reshape(-1, n), np.array(parent), np.array(kernel)


def gumbel(seed: int, c: int) -> float:
    """The Gumbel variate of candidate c, in float32 steps as the device takes them."""
    x = splitmix64_at(seed, c)
    u = np.float32((x >> 40) + 0.5) * np.float32(1.0 / 16777216.0)
    return float(-np.log(-np.log(np.float32(u), dtype=np.float32), dtype=np.float32))


def cap(scores, m: int, cap_children: int, temperature: float = 0.0, seed: int = 0) -> np.ndarray:
    """scores: [W * m] float32.  Returns the ruled scores (float32)."""
    v = np.array(scores, dtype=np.float32).reshape(-1, m)
    W = v.shape[0]
    if temperature > 0.0:
        for w in range(W):
            for t in range(m):
                g = np.float32(temperature) * np.float32(gumbel(seed, w * m + t))
                v[w, t] = np.float32(v[w, t] + g)
    if 0 < cap_children < m:
        out = v.copy()
        for w in range(W):
            order = sorted(range(m), key=lambda t: (v[w, t], t))
            for t in order[cap_children:]:
                out[w, t] = np.float32(math.inf)
        v = out
    return v.ravel()


def gather(prefix, parent, kernel, idx) -> np.ndarray:
    prefix = np.asarray(prefix, dtype=np.int64)
    rows = [list(prefix[parent[c]]) + [int(kernel[c])] for c in idx]
    return np.array(rows, dtype=np.uint8)
