"""Surrogate-guided search for good launch orders on one GPU.

The exact simulator (libko) prices one launch order per wavefront; a learned
scorer (libko_nn) prices an order with two 256x256 BF16 MFMA layers after a
gather-sum, so it can rank orders by the hundred million.  Every order the
scorer proposes is re-simulated exactly, so reported makespans, quantiles and
hit counts are exact integers; the scorer only decides which orders are
simulated.

Steps (each one a call into the two libraries; this module only sequences
them and owns the host-side bookkeeping):

  training data   sampled orders of many sets, their exact makespans
                  (ko_simulate_batch, SAMPLED) and positions (ko_sample_orders);
  training        shuffled minibatches -> tokens and targets (by default the
                  rank quantile of a sample among its set's samples, from a
                  device sort per set; or makespan minus the set's best sampled
                  makespan over the set's area lower bound) -> forward/backward
                  -> Adam,
                  all in libko_nn; with `mask_suffix` some samples hide a
                  random suffix of their order ("unplaced"), which teaches the
                  scorer partial orders for beam search;
  scoring         the set's layer-1 table, then scores of sampled orders from
                  positions, in batches; top-k (ko_topk_f32); the top-k orders
                  regenerated from their sample numbers and re-simulated
                  exactly;
  beam search     partial orders grown one position at a time, the best
                  `width` kept by score; the complete orders are re-simulated;
  quantile        the exact makespan of the best 1% from a full enumeration
                  (ko_kth_smallest_i64) and how many orders reach it.

The figure of merit is the number of exact simulations needed to reach an
order in the exact top 1%: uniform random sampling needs N / hits on average
(geometric, with replacement); the scorer needs the 1-based position of the
first hit in its ranked list.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import (OrderSpec, kernel_array, ko_kth_smallest_i64, ko_sample_orders, ko_simulate_batch, ko_sync,
               ko_topk_f32)
from . import nn


def _torch():
    import torch
    return torch


@dataclass
class SetTable:
    """Kernel sets of one size n on one GPU model, with device-side features
    [S, n, 8] and area lower bounds [S]."""
    model: object
    sets: list
    n: int
    feat: object
    lb: object
    lb_host: np.ndarray
    kernels: np.ndarray
    offsets: np.ndarray

    @classmethod
    def build(cls, model, sets, device="cuda:0"):
        torch = _torch()
        n = len(sets[0])
        if any(len(k) != n for k in sets):
            raise ValueError("all sets of a SetTable must have the same size")
        feats = np.stack([nn.features(model, k) for k in sets]).astype(np.float32)
        lbs = np.array([nn.lower_bound(model, k) for k in sets], dtype=np.int64)
        return cls(model=model, sets=list(sets), n=n, feat=torch.from_numpy(feats).to(device),
                   lb=torch.from_numpy(lbs).to(device), lb_host=lbs,
                   kernels=np.concatenate([kernel_array(k) for k in sets]),
                   offsets=(np.arange(len(sets) + 1) * n).astype(np.int32))


@dataclass
class Samples:
    """Set-major sample tables: row r = set r // per_set, sample r % per_set."""
    per_set: int
    seed: int
    makespans: object   # int64 [R]
    pos: object         # uint8 [R, n]
    set_of: object      # int32 [R]
    best: object        # int64 [S]: each set's best sampled makespan
    target: str = "quantile"
    t_values: object = None   # int64 [R]; targets are (t_values - t_center[s]) / t_scale[s]
    t_center: object = None   # int64 [S]
    t_scale: object = None    # int64 [S]

    @property
    def count(self) -> int:
        return int(self.makespans.shape[0])


def exact_samples(table: SetTable, per_set: int, seed: int, device="cuda:0", target: str = "quantile") -> Samples:
    """`per_set` sampled orders of every set with their exact makespans and
    training targets: "quantile" = rank among the set's samples / per_set,
    "lb" = (makespan - best sampled) / area lower bound."""
    torch = _torch()
    S, n = len(table.sets), table.n
    R = S * per_set
    ms = torch.empty(R, dtype=torch.int64, device=device)
    st = torch.empty(8 * S, dtype=torch.int64, device=device)
    ko_simulate_batch(table.model, table.kernels, table.offsets, OrderSpec.sampled([per_set] * S, seed),
                      makespans=ms, stats=st)
    pos = torch.empty((R, n), dtype=torch.uint8, device=device)
    flat = pos.view(-1)
    for s in range(S):
        ko_sample_orders(n, s, seed, per_set, positions=flat[s * per_set * n:(s + 1) * per_set * n])
    set_of = torch.from_numpy(np.repeat(np.arange(S, dtype=np.int32), per_set)).to(device)
    ko_sync()
    best = st.view(S, 8)[:, 0].contiguous()  # min_makespan is the first field of a stats record
    if target == "quantile":
        values = nn.within_set_ranks(ms, S, per_set)
        center = torch.zeros(S, dtype=torch.int64, device=device)
        scale = torch.full((S,), per_set, dtype=torch.int64, device=device)
    elif target == "lb":
        values, center, scale = ms, best, table.lb
    else:
        raise ValueError(f"unknown target {target!r}")
    return Samples(per_set=per_set, seed=seed, makespans=ms, pos=pos, set_of=set_of, best=best, target=target,
                   t_values=values, t_center=center, t_scale=scale)


def mask_suffixes(samples: Samples, frac: float, seed: int) -> Samples:
    """A copy of the samples where a fraction `frac` of the rows keep only a
    random prefix of their order (the other kernels' positions become
    "unplaced"); targets stay the full order's exact makespan."""
    torch = _torch()
    pos = samples.pos.cpu().numpy().copy()
    R, n = pos.shape
    rng = np.random.default_rng(seed)
    rows = np.flatnonzero(rng.random(R) < frac)
    keep = rng.integers(0, n, size=len(rows))  # positions < keep stay placed
    sub = pos[rows]
    sub[sub >= keep[:, None]] = nn.UNPLACED
    pos[rows] = sub
    return Samples(per_set=samples.per_set, seed=samples.seed, makespans=samples.makespans,
                   pos=torch.from_numpy(pos).to(samples.pos.device), set_of=samples.set_of,
                   best=samples.best, target=samples.target, t_values=samples.t_values,
                   t_center=samples.t_center, t_scale=samples.t_scale)


def train(sur: "nn.Surrogate", table: SetTable, data: Samples, *, steps: int, batch: int = 4096,
          lr: float = 2e-3, warmup: int = 100, seed: int = 0, log_every: int = 100):
    """Adam on shuffled minibatches; returns [(step, loss)] at log points.
    Learning rate: linear warm-up, then cosine decay to 5% of `lr`.

    A step is one replay of a captured HIP graph (ko_nn_step_capture): the
    minibatch is picked from the pass's permutation, and forward, backward and
    Adam run with the step counter and rate kept on the device; the host only
    writes each pass's permutation between replays."""
    torch = _torch()
    dev = data.makespans.device
    R = data.count
    if batch > R:
        batch = R
    rng = np.random.default_rng(seed)
    per_epoch = R // batch
    perm = torch.empty(per_epoch * batch, dtype=torch.int64, device=dev)
    sch = nn.sched(lr=lr, warmup=warmup, total=steps, lr_final=0.05, per_epoch=per_epoch, device=dev)
    stream = torch.cuda.Stream(device=dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    graph = sur.capture_step(table.feat, data.pos, data.set_of, data.t_values, data.t_center, data.t_scale, perm,
                             sch, batch, stream=stream)
    log = []
    with torch.cuda.stream(stream):
        for step in range(1, steps + 1):
            if (step - 1) % per_epoch == 0:
                perm.copy_(torch.from_numpy(rng.permutation(R)[:per_epoch * batch].astype(np.int64)))
            graph.launch(stream)
            if step == 1 or step % log_every == 0 or step == steps:
                log.append((step, float(graph.loss.cpu()[0])))
    torch.cuda.current_stream(dev).wait_stream(stream)
    stream.synchronize()
    graph.close()
    return log


class Ensemble:
    """Several scorers trained alike from different initial weights and
    minibatch orders; an order's score is their mean, computed in the scoring
    kernel (ko_nn_score_split_acc: the first member writes score / m, each
    other adds its score / m, in member order).  Exposes the scorer calls the
    searches use (split_table, score_split)."""

    def __init__(self, members):
        self.members = list(members)

    def split_table(self, feat):
        return [m.split_table(feat) for m in self.members]

    def score_split(self, split, pos, y=None, stream=None):
        scale = 1.0 / len(self.members)
        for k, (m, t) in enumerate(zip(self.members, split)):
            y = m.score_split(t, pos, y=y, scale=scale, accumulate=k > 0, stream=stream)
        return y


def train_members(table: SetTable, data: Samples, members: int, *, seed: int, steps: int, batch: int, lr: float,
                  log_every: int):
    """`members` scorers on the same samples: member k starts from the weights
    of seed + 1000 k and draws its minibatches with seed + 1 + 1000 k.
    Returns (the ensemble, the first member's loss log)."""
    models, first_log = [], None
    for k in range(members):
        sur = nn.Surrogate(_init_params(seed + 1000 * k))
        log = train(sur, table, data, steps=steps, batch=batch, lr=lr, warmup=min(200, steps // 10),
                    seed=seed + 1 + 1000 * k, log_every=log_every)
        first_log = first_log or log
        models.append(sur)
    return Ensemble(models), first_log


def predict(sur: "nn.Surrogate", table: SetTable, set_index: int, pos):
    """Scores of one set's orders given as positions [B, n] (device), float64
    host: lower is better.  With rank-quantile training a score estimates the
    order's quantile among the set's orders; with "lb" training it is cycles
    above the set's best over its lower bound."""
    split = sur.split_table(table.feat[set_index])
    return sur.score_split(split, pos).cpu().numpy().astype(np.float64)


def mae_cycles(res: "SearchResult", q: Quantile, target: str, lb: float) -> float:
    """MAE in cycles of the re-simulated candidates.  Quantile scores are
    mapped to cycles through the set's exact makespan distribution; "lb"
    scores are cycles above the best over the lower bound, put on the
    absolute scale by one per-set offset."""
    if target == "quantile":
        return float(np.mean(np.abs(q.cycles_at(res.predicted) - res.exact)))
    return calibrated_mae(res.predicted * lb, res.exact)


def calibrated_mae(predicted_rel: np.ndarray, exact: np.ndarray) -> float:
    """Mean absolute error in cycles after one per-set offset (the median of
    exact - predicted) restores the set's unknown best makespan."""
    off = float(np.median(exact.astype(np.float64) - predicted_rel))
    return float(np.mean(np.abs(predicted_rel + off - exact)))


@dataclass
class Quantile:
    n_orders: int
    k: int
    makespan: int      # the k-th smallest exact makespan
    hits: int          # orders with makespan <= it
    best: int
    worst: int
    hist: np.ndarray = None   # exact makespan histogram over [best, worst] (equal-width bins)

    @property
    def random_expected(self) -> float:
        """Mean exact simulations of uniform sampling (with replacement) to the first hit."""
        return self.n_orders / self.hits

    def cycles_at(self, quantile) -> np.ndarray:
        """The makespan at the given quantile(s) of all orders, read from the
        exact histogram with linear interpolation inside a bin."""
        q = np.clip(np.asarray(quantile, dtype=np.float64), 0.0, 1.0)
        cdf = np.concatenate([[0.0], np.cumsum(self.hist) / self.n_orders])
        edges = self.best + (self.worst - self.best + 1) * np.arange(len(self.hist) + 1) / len(self.hist)
        return np.interp(q, cdf, edges)


def top_quantile(model, kernels, frac: float = 0.01, device="cuda:0") -> Quantile:
    """Exact best-`frac` threshold of one set by full enumeration on the GPU."""
    torch = _torch()
    n = len(kernels)
    N = math.factorial(n)
    ms = torch.empty(N, dtype=torch.int64, device=device)
    st = torch.empty(8, dtype=torch.int64, device=device)
    h = torch.empty(1024, dtype=torch.int64, device=device)
    ko_simulate_batch(model, kernels, [0, n], OrderSpec.all(), makespans=ms, stats=st, hist=h, n_bins=1024)
    k = max(1, math.ceil(frac * N))
    q, hits = ko_kth_smallest_i64(ms, k, with_count=True)
    from . import stats_records
    rec = stats_records(st)[0]
    out = Quantile(n_orders=N, k=k, makespan=q, hits=hits, best=int(rec["min_makespan"]),
                   worst=int(rec["max_makespan"]), hist=h.cpu().numpy().astype(np.float64))
    del ms
    return out


@dataclass
class SearchResult:
    sample_index: np.ndarray   # sample numbers of the ranked orders (SAMPLED-mode counters)
    orders: np.ndarray         # [K, n] uint8, best predicted first
    predicted: np.ndarray      # network scores, best first (see predict)
    exact: np.ndarray          # int64 cycles, exact re-simulation
    n_scored: int


def score_and_rerank(sur: "nn.Surrogate", table: SetTable, set_index: int, *, n_score: int, top_k: int,
                     seed: int, batch: int = 1 << 18, device="cuda:0") -> SearchResult:
    """Score `n_score` sampled orders, keep the `top_k` best predicted, re-simulate them exactly."""
    torch = _torch()
    n = table.n
    split = sur.split_table(table.feat[set_index])
    scores = torch.empty(n_score, dtype=torch.float32, device=device)
    pos = torch.empty(min(batch, n_score) * n, dtype=torch.uint8, device=device)
    for b0 in range(0, n_score, batch):
        c = min(batch, n_score - b0)
        ko_sample_orders(n, set_index, seed, c, first=b0, positions=pos[:c * n])
        sur.score_split(split, pos[:c * n].view(c, n), y=scores[b0:b0 + c])
    idx, val = ko_topk_f32(scores, top_k)
    orders = torch.empty(top_k * n, dtype=torch.uint8, device=device)
    ko_sample_orders(n, set_index, seed, top_k, indices=idx, orders=orders)
    ms = torch.empty(top_k, dtype=torch.int64, device=device)
    kern = table.sets[set_index]
    ko_simulate_batch(table.model, kern, [0, n], OrderSpec.explicit(orders, [top_k]), makespans=ms)
    ko_sync()
    lb = float(table.lb_host[set_index])
    return SearchResult(sample_index=idx.cpu().numpy(), orders=orders.cpu().numpy().reshape(top_k, n),
                        predicted=val.cpu().numpy().astype(np.float64),
                        exact=ms.cpu().numpy(), n_scored=n_score)


def beam_search(sur: "nn.Surrogate", table: SetTable, set_index: int, *, width: int = 256,
                max_children: int = 0, temperature: float = 0.0, seed: int = 0, device="cuda:0") -> SearchResult:
    """Grow orders position by position on the device, keeping the `width`
    best-scored prefixes (kernels not yet placed are "unplaced").  Each step
    expands every kept prefix by each unused kernel (ko_nn_beam_expand),
    scores the partial orders (ko_nn_score_split), applies the diversity rules
    (ko_nn_beam_cap: at most `max_children` children of one prefix survive,
    and with temperature > 0 Gumbel noise perturbs the scores, seeded per
    step), keeps the best (ko_topk_f32) and gathers their prefixes
    (ko_nn_beam_gather).  The last step scores the complete orders without
    noise; they are ranked by that score and re-simulated exactly."""
    torch = _torch()
    n = table.n
    split = sur.split_table(table.feat[set_index])
    prefix = torch.empty((1, 0), dtype=torch.uint8, device=device)
    n_scored = 0
    val = None
    for d in range(n):
        W, m = prefix.shape[0], n - d
        pos, cand = nn.beam_expand(prefix, n)
        scores = sur.score_split(split, pos)
        n_scored += W * m
        last = d == n - 1
        if not last and (max_children > 0 or temperature > 0):
            nn.beam_cap(scores, W, m, max_children, temperature, seed + d)
        finite = W * (min(max_children, m) if max_children > 0 and not last else m)
        idx, val = ko_topk_f32(scores, min(width, finite))
        prefix = nn.beam_gather(prefix, cand, idx)
    K = prefix.shape[0]
    orders = prefix.reshape(-1).contiguous()
    ms = torch.empty(K, dtype=torch.int64, device=device)
    ko_simulate_batch(table.model, table.sets[set_index], [0, n], OrderSpec.explicit(orders, [K]),
                      makespans=ms)
    ko_sync()
    return SearchResult(sample_index=np.full(K, -1), orders=prefix.cpu().numpy(),
                        predicted=val.cpu().numpy().astype(np.float64), exact=ms.cpu().numpy(),
                        n_scored=n_scored)


def sims_to_first_hit(exact_ranked: np.ndarray, threshold: int, random_expected: float) -> float:
    """Exact simulations the ranked list needs to reach makespan <= threshold;
    after an exhausted list the search continues with random sampling."""
    hit = np.flatnonzero(exact_ranked <= threshold)
    if len(hit):
        return float(hit[0] + 1)
    return float(len(exact_ranked)) + random_expected


# ------------------------------------------------------------------ report

def _init_params(seed: int) -> np.ndarray:
    """He-style initial weights (zero biases) in the flat parameter order."""
    rng = np.random.default_rng(seed)
    shapes = ((256, 32), (256,), (256, 256), (256,), (256, 256), (256,), (256,), (1,))
    parts = []
    for i, shape in enumerate(shapes):
        if len(shape) == 1 and i != 6:
            parts.append(np.zeros(shape))
        else:
            parts.append(rng.normal(0.0, 1.0 / math.sqrt(shape[-1]), size=shape))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def report(*, train_workload: int = 3, heldout_workload: int = 13, train_sets: int = 8192,
           per_set: int = 512, heldout: int = 32, n_score: int = 1 << 18, top_k: int = 10_000,
           steps: int = 65536, batch: int = 4096, lr: float = 1e-3, seed: int = 2015, target: str = "quantile",
           members: int = 4, quantiles: dict | None = None, out=print):
    """Train `members` scorers on exact samples (an Ensemble), then per
    held-out set: exact top-1% threshold by full enumeration, scoring of
    `n_score` sampled orders, exact re-simulation of the `top_k` best (the
    default 2^18 lies in the range 2^14..2^19 over which the first-hit ratio
    of validation sets, disjoint from the held-out ones, stays flat; scoring
    10^8 orders reaches further into the scores' extremes, where they are
    least reliable, and does worse).  Prints
    one JSON line per held-out set and a summary.  `quantiles` (held-out set
    index -> Quantile), when given, keeps the thresholds of earlier calls on
    the same held-out sets and is filled in."""
    import json
    import time

    import synth

    torch = _torch()
    t0 = time.perf_counter()
    tr_sets = [synth.draw_set(train_workload, s) for s in range(train_sets)]
    table = SetTable.build(synth.WORKLOADS[train_workload].model, tr_sets)
    data = exact_samples(table, per_set, seed=seed, target=target)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    sur, log = train_members(table, data, members, seed=seed + 1, steps=steps, batch=batch, lr=lr,
                             log_every=max(1, steps // 8))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    out(json.dumps({"phase": "train", "target": target, "samples": data.count, "sets": train_sets, "n": table.n,
                    "members": members, "data_s": round(t_data, 3), "train_s": round(t_train, 3), "steps": steps,
                    "batch": batch, "loss": log}), flush=True)
    del data
    model = synth.WORKLOADS[heldout_workload].model
    held = [synth.draw_set(heldout_workload, s) for s in range(heldout)]
    htab = SetTable.build(model, held)
    rows = []
    for s, ks in enumerate(held):
        t0 = time.perf_counter()
        if quantiles is not None and s in quantiles:
            q = quantiles[s]
        else:
            q = top_quantile(model, ks, 0.01)
            if quantiles is not None:
                quantiles[s] = q
        torch.cuda.synchronize()
        t_enum = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = score_and_rerank(sur, htab, s, n_score=n_score, top_k=top_k, seed=seed + 100 + s)
        t_score = time.perf_counter() - t0
        sims = sims_to_first_hit(res.exact, q.makespan, q.random_expected)
        row = {"phase": "heldout", "set": s, "n_orders": q.n_orders, "top1pct_makespan": q.makespan,
               "hits": q.hits, "best": q.best, "worst": q.worst,
               "random_sims_expected": q.random_expected, "surrogate_sims": sims,
               "speedup": q.random_expected / sims,
               "recall_at_1pct": float(np.mean(res.exact <= q.makespan)),
               "mae_cycles": mae_cycles(res, q, target, float(htab.lb_host[s])),
               "best_of_topk": int(res.exact.min()), "enum_s": round(t_enum, 3),
               "score_rerank_s": round(t_score, 3), "n_score": n_score, "top_k": top_k}
        rows.append(row)
        out(json.dumps(row), flush=True)
    sp = np.array([r["speedup"] for r in rows])
    out(json.dumps({"phase": "summary", "heldout_sets": heldout,
                    "speedup_geomean": float(np.exp(np.mean(np.log(sp)))),
                    "speedup_min": float(sp.min()), "speedup_max": float(sp.max()),
                    "recall_at_1pct_mean": float(np.mean([r["recall_at_1pct"] for r in rows])),
                    "mae_cycles_mean": float(np.mean([r["mae_cycles"] for r in rows])),
                    "target": target}), flush=True)
    return rows


def _search_row(exact_ranked: np.ndarray, exact: np.ndarray, threshold, random_expected):
    """(best makespan, top-1% hits, exact simulations to the first hit)."""
    return (int(exact.min()), int((exact <= threshold).sum()),
            sims_to_first_hit(exact_ranked, int(threshold), float(random_expected)))


def report_beam(*, train_workload: int = 14, eval_workload: int = 4, train_sets: int = 8192, per_set: int = 512,
                eval_sets: int = 1024, width: int = 256, q_samples: int = 4096, steps: int = 32768,
                batch: int = 4096, lr: float = 1e-3, mask_frac: float = 0.25, seed: int = 2016,
                max_children: int = 2, temperature: float = 0.0, n_score: int = 1 << 20, members: int = 4,
                eval_first: int = 0, sur=None, out=print):
    """Surrogate-guided search on n=16 sets against uniform sampling at the
    same exact budget (`width` exact simulations per set): beam search (width
    `width`, at most `max_children` children per prefix per step, optional
    Gumbel noise) and sample-then-score (score `n_score` uniformly sampled
    orders, re-simulate the best `width`).  The top-1% threshold of each set is
    the ceil(q_samples/100)-th smallest of `q_samples` exact random orders (n!
    is out of reach at n=16); uniform sampling needs q_samples / (samples at or
    below it) simulations on average to reach it.  A search needs the 1-based
    position of its first hit in its predicted order (its budget plus uniform
    sampling's expectation if it has none).  `sur`, when given, is a trained
    scorer used as is (no training).  The evaluation sets are draws
    eval_first .. eval_first + eval_sets - 1 of the workload.  Prints one JSON
    summary line."""
    import json
    import time

    import synth

    torch = _torch()
    if sur is None:
        t0 = time.perf_counter()
        tr = [synth.draw_set(train_workload, s) for s in range(train_sets)]
        table = SetTable.build(synth.WORKLOADS[train_workload].model, tr)
        data = mask_suffixes(exact_samples(table, per_set, seed=seed, target="quantile"), mask_frac, seed + 1)
        sur, log = train_members(table, data, members, seed=seed + 2, steps=steps, batch=batch, lr=lr,
                                 log_every=max(1, steps // 8))
        torch.cuda.synchronize()
        out(json.dumps({"phase": "train", "sets": train_sets, "n": table.n, "samples": data.count,
                        "mask_frac": mask_frac, "members": members, "train_s": round(time.perf_counter() - t0, 2),
                        "loss": log}), flush=True)
        del data
    model = synth.WORKLOADS[eval_workload].model
    ev = [synth.draw_set(eval_workload, eval_first + s) for s in range(eval_sets)]
    etab = SetTable.build(model, ev)
    S = len(ev)
    # exact random samples of every set in one batch: q_samples for the
    # threshold, then `width` more as the random-search budget
    t0 = time.perf_counter()
    qms = torch.empty(S * q_samples, dtype=torch.int64, device="cuda:0")
    ko_simulate_batch(model, etab.kernels, etab.offsets, OrderSpec.sampled([q_samples] * S, seed + 10),
                      makespans=qms)
    rms = torch.empty(S * width, dtype=torch.int64, device="cuda:0")
    ko_simulate_batch(model, etab.kernels, etab.offsets, OrderSpec.sampled([width] * S, seed + 11),
                      makespans=rms)
    ko_sync()
    k = max(1, math.ceil(q_samples / 100))
    thr, rexp = np.zeros(S, dtype=np.int64), np.zeros(S)
    for s in range(S):
        thr[s], hits = ko_kth_smallest_i64(qms[s * q_samples:(s + 1) * q_samples], k, with_count=True)
        rexp[s] = q_samples / hits
    rnd = rms.cpu().numpy().reshape(S, width)
    t_exact = time.perf_counter() - t0
    rows = {"beam": [], "sample_then_score": [], "merged": []}
    times = {}
    found = {"beam": [], "sample_then_score": []}
    for name in ("beam", "sample_then_score"):
        t0 = time.perf_counter()
        for s in range(S):
            if name == "beam":
                res = beam_search(sur, etab, s, width=width, max_children=max_children, temperature=temperature,
                                  seed=seed + 20 + s)
            else:
                res = score_and_rerank(sur, etab, s, n_score=n_score, top_k=width, seed=seed + 30)
            found[name].append(res)
            rows[name].append(_search_row(res.exact, res.exact, thr[s], rexp[s]))
        times[name] = round(time.perf_counter() - t0, 2)
    # both searches' complete orders ranked together by the same scorer; the
    # best `width` distinct ones are the merged search's exact budget
    for s in range(S):
        b, r = found["beam"][s], found["sample_then_score"][s]
        orders = np.concatenate([b.orders, r.orders])
        pred = np.concatenate([b.predicted, r.predicted])
        exact = np.concatenate([b.exact, r.exact])
        _, first = np.unique(orders, axis=0, return_index=True)
        keep = first[np.lexsort((first, pred[first]))][:width]
        rows["merged"].append(_search_row(exact[keep], exact[keep], thr[s], rexp[s]))
    times["merged"] = times["beam"] + times["sample_then_score"]
    rnd_best = rnd.min(axis=1)
    rnd_hits = (rnd <= thr[:, None]).sum(axis=1)
    summary = {"phase": "search_vs_random", "eval_sets": S, "n": etab.n, "exact_budget_per_set": width,
               "q_samples": q_samples, "random_sims_expected_mean": float(rexp.mean()),
               "sets_random_found_top1pct": float(np.mean(rnd_hits > 0)),
               "random_hits_top1pct_mean": float(rnd_hits.mean()), "exact_sampling_s": round(t_exact, 2)}
    for name, r in rows.items():
        a = np.array(r, dtype=np.float64)
        speed = rexp / a[:, 2]
        summary[name] = {"sets_found_top1pct": float(np.mean(a[:, 1] > 0)),
                         "hits_top1pct_mean": float(a[:, 1].mean()),
                         "best_better_than_random_frac": float(np.mean(a[:, 0] < rnd_best)),
                         "best_ratio_over_random_mean": float(np.mean(a[:, 0] / rnd_best)),
                         "sims_to_top1pct_mean": float(a[:, 2].mean()),
                         "speedup_geomean": float(np.exp(np.mean(np.log(speed)))),
                         "speedup_median": float(np.median(speed)),
                         "sets_at_least_10x": float(np.mean(speed >= 10.0)),
                         "search_s": times[name]}
    summary["beam"].update({"width": width, "max_children": max_children, "temperature": temperature})
    summary["sample_then_score"].update({"n_score": n_score})
    summary["merged"].update({"of": "beam and sample_then_score, ranked together by score"})
    out(json.dumps(summary), flush=True)
    return summary


if __name__ == "__main__":
    import argparse
    import os
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="surrogate-guided search report (one GPU)")
    ap.add_argument("--train-sets", type=int, default=8192)
    ap.add_argument("--per-set", type=int, default=512)
    ap.add_argument("--heldout", type=int, default=32)
    ap.add_argument("--n-score", type=int, default=1 << 18)
    ap.add_argument("--top-k", type=int, default=10_000)
    ap.add_argument("--steps", type=int, default=65536)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--target", default="quantile", choices=("quantile", "lb"))
    ap.add_argument("--train-workload", type=int, default=3)
    ap.add_argument("--heldout-workload", type=int, default=13)
    ap.add_argument("--beam", action="store_true", help="n=16 beam search vs random sampling instead")
    ap.add_argument("--eval-sets", type=int, default=1024)
    ap.add_argument("--width", type=int, default=256)
    ap.add_argument("--max-children", type=int, default=2,
                    help="beam: at most this many children of one prefix per step (0 = no cap)")
    ap.add_argument("--temperature", type=float, default=0.0, help="beam: Gumbel noise on each step's scores")
    ap.add_argument("--beam-n-score", type=int, default=1 << 20,
                    help="--beam: orders scored per set by sample-then-score")
    ap.add_argument("--members", type=int, default=4, help="scorers trained and averaged (an ensemble)")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if a.beam:
        report_beam(train_sets=a.train_sets, per_set=a.per_set, eval_sets=a.eval_sets, width=a.width,
                    steps=a.steps, batch=a.batch, lr=a.lr, max_children=a.max_children,
                    temperature=a.temperature, n_score=a.beam_n_score, members=a.members)
        raise SystemExit(0)
    report(train_workload=a.train_workload, heldout_workload=a.heldout_workload, train_sets=a.train_sets,
           per_set=a.per_set, heldout=a.heldout, n_score=a.n_score, top_k=a.top_k, steps=a.steps,
           batch=a.batch, lr=a.lr, target=a.target, members=a.members)
