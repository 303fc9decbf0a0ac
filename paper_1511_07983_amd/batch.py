"""Many kernel sets at once: plans, graph replay, an autotuner, percentiles.

A batch of thousands of kernel sets of uneven size (n = 4..9, so 24 to 362,880
orders each) runs as one persistent launch fed by a device work queue of
(set, chunk of ranks) items (ko_plan_*).  The launch configuration (the
engine, i.e. how CU state is laid out: one wavefront per order with lanes
owning CUs, or one lane per order with CU states as runs; orders per work
item; persistent workgroups per CU) is picked by `autotune`, which times each
candidate with HIP events on the caller's stream, checks that every candidate
produces identical makespans, and caches its choice in a JSON file keyed by
the device, the model and the batch's shape.

`percentiles` is the batch form of Table 3's "percentile rank": Algorithm 1's
order of every set (host), its exact makespan (one EXPLICIT plan launch for
all sets), then the counts of all orders below, equal to and above it (one
ALL plan launch with per-set references).
"""

from __future__ import annotations

import hashlib
import json
import math
import os
import time

import numpy as np

from . import (ENGINE_LANES, ENGINE_WAVE, KO_EINVAL, KoError, OrderSpec, Plan, gpu_model, kernel_array,
               ko_heuristic_order, stats_records)

# candidate orders per work item (log2) and persistent workgroups per CU, per engine
SWEEP = {ENGINE_WAVE: ((5, 6, 8, 10), (4, 8, 16)),   # 32 .. 1024 orders, one wavefront each
         ENGINE_LANES: ((6, 7, 8), (4, 8, 16))}      # 1 .. 4 orders per lane
CHUNKS = SWEEP[ENGINE_WAVE][0]
WG_PER_CU = SWEEP[ENGINE_WAVE][1]


def _cache_path():
    return os.environ.get("KO_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1511_07983_amd", "autotune.json"))


def batch_key(gpu, kernels, set_offsets, spec: OrderSpec) -> str:
    """Device name, model, mode and the histogram of set sizes (the shape the
    launch configuration depends on), hashed."""
    import torch
    g = gpu_model(gpu)
    sizes = np.diff(np.asarray(set_offsets, dtype=np.int64))
    hist = np.bincount(sizes, minlength=21)
    text = json.dumps({"device": torch.cuda.get_device_name(), "model": [g.n_cu, g.wave_size, g.wave_cu, g.blk_cu,
                                                                          g.reg_cu, g.lds_cu, g.rb_milli,
                                                                          g.mem_blocks],
                       "mode": spec.mode, "sizes": hist.tolist()}, sort_keys=True)
    return hashlib.sha256(text.encode()).hexdigest()[:24]


def _time_plan(plan: Plan, reps: int, out) -> float:
    import torch
    plan.launch(makespans=out)  # warm-up (and first-touch of the output)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.launch(makespans=out)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    plan.status()
    return float(np.median(times))


def _candidates(engines, chunks, wgs):
    for e in engines:
        c_list = chunks if chunks is not None else SWEEP[e][0]
        w_list = wgs if wgs is not None else SWEEP[e][1]
        for c in c_list:
            for w in w_list:
                yield e, c, w


def autotune(gpu, kernels, set_offsets, spec: OrderSpec, *, reps: int = 3, use_cache: bool = True,
             engines=(ENGINE_WAVE, ENGINE_LANES), chunks=None, wgs=None, log=None):
    """Best (engine, chunk_log2, wg_per_cu) for this batch; every candidate must
    give the same makespans bit for bit.  An engine that does not apply to the
    batch (the lane engine past 16 kernels or 256 CUs) is left
    out.  `chunks`/`wgs` override the per-engine candidate lists.  Returns
    (config dict, sweep rows)."""
    import torch
    key = batch_key(gpu, kernels, set_offsets, spec)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key], []
    ref = None
    rows = []
    total = None
    for e, c, w in _candidates(engines, chunks, wgs):
        try:
            plan = Plan(gpu, kernels, set_offsets, spec, chunk_log2=c, wg_per_cu=w, engine=e)
        except KoError as exc:
            if exc.code == KO_EINVAL and e == ENGINE_LANES:
                continue  # the lane engine does not take this batch
            raise
        total = plan.total_orders
        out = torch.empty(max(total, 1), dtype=torch.int64, device="cuda:0")
        ms = _time_plan(plan, reps, out)
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError(f"configuration engine={e} chunk=2^{c} wg={w} changed the makespans")
        rows.append({"engine": e, "chunk_log2": c, "wg_per_cu": w, "ms": ms, "work_items": plan.work_items})
        if log:
            log(rows[-1])
        plan.close()
    best = min(rows, key=lambda r: r["ms"])
    cfg = {"engine": best["engine"], "chunk_log2": best["chunk_log2"], "wg_per_cu": best["wg_per_cu"],
           "ms": best["ms"], "orders": int(total), "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache[key] = cfg
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return cfg, rows


def concat_sets(sets):
    kernels = np.concatenate([kernel_array(k) for k in sets])
    offsets = np.zeros(len(sets) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(k) for k in sets])
    return kernels, offsets


def percentiles(gpu, sets, *, config=None, n_bins: int = 0, want_makespans: bool = False):
    """Algorithm 1's order of every set and its exact percentile among all of
    the set's orders.  Returns a dict of per-set arrays (and, if asked, the
    concatenated makespans of all orders and per-set histograms)."""
    import torch
    dev = "cuda:0"
    kernels, offsets = concat_sets(sets)
    S = len(sets)
    orders = [ko_heuristic_order(gpu, k) for k in sets]
    flat = torch.from_numpy(np.concatenate([np.asarray(o, dtype=np.uint8) for o in orders])).to(dev)
    ref = torch.empty(S, dtype=torch.int64, device=dev)
    cfg = config or {}
    p1 = Plan(gpu, kernels, offsets, OrderSpec.explicit(flat, [1] * S))
    p1.launch(makespans=ref)
    p1.status()
    p2 = Plan(gpu, kernels, offsets, OrderSpec.all(), chunk_log2=cfg.get("chunk_log2", 0),
              wg_per_cu=cfg.get("wg_per_cu", 0), engine=cfg.get("engine", 0))
    st = torch.empty(8 * S, dtype=torch.int64, device=dev)
    ms = torch.empty(max(p2.total_orders, 1), dtype=torch.int64, device=dev) if (want_makespans or n_bins) else None
    hist = torch.empty(S * n_bins, dtype=torch.int64, device=dev) if n_bins else None
    p2.launch(ref_makespan=ref, makespans=ms, stats=st, hist=hist, n_bins=n_bins)
    p2.status()
    rec = stats_records(st)
    n_less = rec["n_less"].astype(np.int64)
    n_eq = rec["n_equal"].astype(np.int64)
    n_tot = rec["n_orders"].astype(np.int64)
    out = {"order": orders, "makespan": ref.cpu().numpy(), "n_less": n_less, "n_equal": n_eq,
           "n_greater": rec["n_greater"].astype(np.int64), "n_orders": n_tot,
           "pct_inclusive": 100.0 * (n_tot - n_less) / n_tot,
           "best": rec["min_makespan"], "worst": rec["max_makespan"]}
    if ms is not None:
        out["makespans"] = ms
    if hist is not None:
        out["hist"] = hist.cpu().numpy().view(np.uint64).reshape(S, n_bins)
    p1.close()
    p2.close()
    return out


def report(*, workload: int = 2, sets: int = 4096, tune_sets: int = 512, reps: int = 5, tune: bool = True,
           out=print):
    """Exact evaluations per second over every order of a batch of kernel sets:
    autotune on a subset (or take the library's defaults), then replay a
    captured graph of the whole batch."""
    import torch

    import synth
    w = synth.WORKLOADS[workload]
    all_sets = [synth.draw_set(workload, s) for s in range(sets)]
    if tune:
        k_t, o_t = concat_sets(all_sets[:tune_sets])
        cfg, rows = autotune(w.model, k_t, o_t, OrderSpec.all(), reps=2, use_cache=False)
    else:
        cfg, rows = {"engine": 0, "chunk_log2": 0, "wg_per_cu": 0}, []
    kernels, offsets = concat_sets(all_sets)
    plan = Plan(w.model, kernels, offsets, OrderSpec.all(), chunk_log2=cfg["chunk_log2"],
                wg_per_cu=cfg["wg_per_cu"], engine=cfg.get("engine", 0))
    st = torch.empty(8 * sets, dtype=torch.int64, device="cuda:0")
    ms = torch.empty(plan.total_orders, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.Stream()
    graph = plan.capture(stream=stream, makespans=ms, stats=st)
    graph.launch(stream)
    stream.synchronize()
    plan.status(stream)
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        graph.launch(stream)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    plan.status(stream)
    engine, entries, spilled, handed = plan.engine(stream)
    t = float(np.median(times))
    out(json.dumps({"workload": w.name, "sets": sets, "orders": int(plan.total_orders),
                    "engine": {"engine": engine, "lane_entries": entries, "spilled_orders": spilled,
                               "items_re_run": handed},
                    "config": {"engine": cfg.get("engine", 0), "chunk_log2": cfg["chunk_log2"],
                               "wg_per_cu": cfg["wg_per_cu"]},
                    "tuning": rows, "graph_replay_s": t, "orders_per_s": plan.total_orders / t,
                    "work_items": int(plan.work_items)}), flush=True)
    graph.close()
    plan.close()


if __name__ == "__main__":
    import argparse
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="exact orders/s over every order of a batch of sets")
    ap.add_argument("--workload", type=int, default=2, help="synthetic workload (default 2: 4096 sets, n=4..9)")
    ap.add_argument("--sets", type=int, default=4096)
    ap.add_argument("--tune-sets", type=int, default=512)
    ap.add_argument("--no-tune", action="store_true", help="library defaults instead of the autotuner")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    report(workload=args.workload, sets=args.sets, tune_sets=args.tune_sets, reps=args.reps,
           tune=not args.no_tune)
