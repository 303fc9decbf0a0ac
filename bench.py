#!/usr/bin/env python3
"""Exact launch-order evaluations per second on one MI355X.

One step is the whole evaluation path over one kernel set of the n=10
workload (10 kernels, 256-CU MI355X-shaped model, 3,628,800 launch orders):

  1. derive per-block use and durations, and the launch order of Algorithm 1
     (host, inside libko);
  2. the makespan of that order (device);
  3. the makespans of all n! orders, with per-set extremes, the rank counts
     against the heuristic order's makespan (its percentile) and a 1024-bin
     histogram (device).

Inputs are synthetic and seeded (SeedSequence([20151123, 1, 0])) and resident
in HBM before timing starts.  After the timed steps, untimed legs add objects
to the same line: the round-synchronous model ("rounds") and memory contention
("contended") on the same set, all 720 orders of the n=6 set on the 16-CU model
("small"), all orders of the 4096-set batch in one captured graph ("batch";
--no-legs skips these two), the metric's second part on the n=12 workload
("surrogate": exact simulations to the first order in the exact top 1%, learned
scorer against uniform sampling, two training recipes) and on the n=16 sets
("search_n16": beam search and sample-then-score at an equal exact budget;
--no-surrogate skips both), then the CPU oracle at every core and at one
thread ("cpu_baseline").
Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# integer VALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic int32 lane-operations per order: 13 per block of the set
# (8 to test and claim a CU, 4 to release it, 1 for the finish time)
OPS_PER_BLOCK = 13

# HBM bytes per all-orders launch of the simulate kernel on the n=10 set, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs calibrated against a 256 MiB copy
# (profiles/ holds the summaries).  They hold for the kernel sources they were
# measured on (identified by hash) and for the launch's work decomposition
# (orders per work item and item count, which set the partials written); any
# change to either reports null until the counters are taken again.
TRAFFIC_SOURCES = ("paper_1511_07983_amd/csrc/ko_sim.hip", "paper_1511_07983_amd/csrc/ko_lanes.hip",
                   "paper_1511_07983_amd/csrc/ko_wave.h", "paper_1511_07983_amd/csrc/ko_orders.h",
                   "paper_1511_07983_amd/csrc/ko_device.h")
TRAFFIC_MEASURED = {"20f15ebbf50dfdea:64:56700": int((283.2 * 2 + 33825.9) * 1024)}


def measured_traffic(chunk: int, work_items: int):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC_MEASURED.get(f"{h.hexdigest()[:16]}:{chunk}:{work_items}")


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", type=int, default=1, help="synthetic workload index (default 1: n=10)")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target duration of the CPU oracle sample (0 = skip)")
    p.add_argument("--no-surrogate", action="store_true",
                   help="skip the surrogate leg (n=12: train, then exact simulations to a top-1%% order)")
    p.add_argument("--surrogate-heldout", type=int, default=32)
    p.add_argument("--no-legs", action="store_true",
                   help="skip the n=6 (16-CU) and 4096-set batch legs")
    p.add_argument("--copy-mb", type=int, default=0,
                   help="after timing, copy this many MiB device-to-device once (untimed): a "
                        "plain copy of known size that calibrates HBM byte counters in a profile")
    return p.parse_args()


def cpu_model_name() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(model, ks, seconds: float, threads: int, lo: int):
    """Orders/s of the oracle on lexicographic ranks from `lo`, about `seconds` long."""
    import oracle
    pilot = 200 * threads
    t0 = time.perf_counter()
    oracle.makespans_range(model.as_dict(), ks, lo, pilot, threads)
    dt = time.perf_counter() - t0
    count = max(pilot, int(pilot * max(seconds - dt, 0.0) / max(dt, 1e-9)))
    t0 = time.perf_counter()
    oracle.makespans_range(model.as_dict(), ks, lo + pilot, count, threads)
    dt = time.perf_counter() - t0
    return count / dt, lo + pilot, count, dt


def cpu_baseline(model, ks, seconds: float) -> dict:
    """The CPU oracle, as it stands, on bounded samples of the same orders: with
    every core this process may use, then with one thread."""
    import oracle
    threads = oracle.default_threads()
    rate, lo, count, dt = _oracle_rate(model, ks, 0.6 * seconds, threads, 0)
    rate1, lo1, count1, dt1 = _oracle_rate(model, ks, 0.4 * seconds, 1, lo + count)
    return {"value": rate, "unit": "orders/s", "cores": threads, "kind": "oracle",
            "sample": f"lexicographic ranks {lo}..{lo + count - 1} of the same set "
                      f"({count} orders, {dt:.1f} s, plain C event-driven oracle, -O2, "
                      f"{threads} threads)",
            "single_thread": {"value": rate1, "unit": "orders/s", "cores": 1,
                              "sample": f"ranks {lo1}..{lo1 + count1 - 1} ({count1} orders, {dt1:.1f} s)"},
            "cpu_model": cpu_model_name()}


def _surrogate_recipe(heldout: int, train_sets: int, per_set: int, quantiles: dict, exact_rate: float) -> dict:
    import json as _json

    from paper_1511_07983_amd import surrogate
    lines = []

    def keep(text, flush=True):
        rec = _json.loads(text)
        lines.append(rec)
        print(f"[bench] surrogate {train_sets}x{per_set} {rec.get('phase')} done", file=sys.stderr, flush=True)

    try:
        surrogate.report(heldout=heldout, train_sets=train_sets, per_set=per_set, quantiles=quantiles, out=keep)
    except Exception as exc:  # keep the throughput line even if this leg fails
        return {"error": f"{type(exc).__name__}: {exc}"}
    train = next(l for l in lines if l.get("phase") == "train")
    summary = next(l for l in lines if l.get("phase") == "summary")
    rows = [l for l in lines if l.get("phase") == "heldout"]
    score_s = float(sum(r["score_rerank_s"] for r in rows) / max(1, len(rows)))
    random_sims = float(np.mean([r["random_sims_expected"] for r in rows]))
    return {"train_sets": train["sets"], "samples_per_set": per_set, "train_samples": train["samples"],
            "speedup_geomean": summary["speedup_geomean"], "per_set": [round(r["speedup"], 3) for r in rows],
            "recall_at_1pct_mean": summary["recall_at_1pct_mean"], "mae_cycles_mean": summary["mae_cycles_mean"],
            "train_s": train["train_s"], "score_rerank_s_per_set": round(score_s, 3),
            # what the saved simulations would cost: uniform sampling's expected
            # exact simulations at the exact simulator's rate on these sets
            "random_sims_mean": round(random_sims, 1),
            "random_sims_exact_s": random_sims / exact_rate if exact_rate > 0 else None}


def surrogate_leg(heldout: int) -> dict:
    """The metric's second part on the n=12 workload (not in `value`): train the
    scorer on 2^22 exact samples, then per held-out set score 2^18 sampled
    orders, re-simulate the best 10^4 exactly and count exact simulations to the
    first order in the exact top 1% (full enumeration), against uniform
    sampling's exact expectation N / hits.  Two training recipes: 512 sets x
    8192 orders (the workload as specified) and 8192 sets x 512 orders.  The
    first hit varies widely from set to set, so the geometric mean is taken
    over 32 held-out sets."""
    import torch

    import paper_1511_07983_amd as ko
    import synth
    w = synth.WORKLOADS[13]
    quantiles = {}
    # the exact simulator's rate on n=12 orders (sampled, all held-out sets' model)
    ks = synth.draw_set(13, 0)
    ms = torch.empty(1 << 22, dtype=torch.int64, device="cuda:0")
    spec = ko.OrderSpec.sampled([1 << 22], seed=7)
    ko.ko_simulate_batch(w.model, ks, [0, len(ks)], spec, makespans=ms)
    ko.ko_sync()
    t0 = time.perf_counter()
    ko.ko_simulate_batch(w.model, ks, [0, len(ks)], spec, makespans=ms)
    ko.ko_sync()
    exact_rate = (1 << 22) / (time.perf_counter() - t0)
    del ms
    out = {"workload": w.name, "heldout_sets": heldout, "exact_orders_per_s_n12": exact_rate,
           "as_specified_512x8192": _surrogate_recipe(heldout, 512, 8192, quantiles, exact_rate),
           "wide_8192x512": _surrogate_recipe(heldout, 8192, 512, quantiles, exact_rate)}
    return out


def search_n16_leg() -> dict:
    """Surrogate-guided search on the 1024 n=16 sets (N_tblk 256..8192) at an
    equal budget of 256 exact simulations per set against uniform sampling:
    beam search (width 256, at most 2 children per prefix), sample-then-score
    (2^20 scored orders, the best 256 simulated) and both ranked together."""
    import json as _json

    from paper_1511_07983_amd import surrogate
    recs = []
    try:
        surrogate.report_beam(eval_sets=1024, out=lambda t, **kw: recs.append(_json.loads(t)))
    except Exception as exc:  # keep the throughput line even if this leg fails
        return {"error": f"{type(exc).__name__}: {exc}"}
    print("[bench] search n=16 done", file=sys.stderr, flush=True)
    train = next(r for r in recs if r.get("phase") == "train")
    res = next(r for r in recs if r.get("phase") == "search_vs_random")
    res["train_s"] = train["train_s"]
    res["train_samples"] = train["samples"]
    res.pop("phase", None)
    return res


def _event_time(fn, stream, reps: int) -> float:
    """Median seconds of fn() enqueued on `stream`, HIP events around each call."""
    import torch
    fn()
    stream.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    return float(np.median(times))


def small_leg() -> dict:
    """All 720 orders of the n=6 set on the 16-CU model: one ko_simulate_batch
    call (host preparation, upload, simulate, per-set statistics) and one
    replay of a captured graph of a prepared plan, HIP events around each."""
    import torch

    import paper_1511_07983_amd as ko
    import synth
    w = synth.WORKLOADS[0]
    ks = synth.draw_set(0, 0)
    N = math.factorial(len(ks))
    ms = torch.empty(N, dtype=torch.int64, device="cuda:0")
    st = torch.empty(8, dtype=torch.int64, device="cuda:0")
    kern = ko.kernel_array(ks)
    off = [0, len(ks)]
    spec = ko.OrderSpec.all()
    stream = torch.cuda.Stream()
    t_call = _event_time(lambda: ko.ko_simulate_batch(w.model, kern, off, spec, makespans=ms, stats=st,
                                                      stream=stream), stream, 50)
    ko.ko_sync(stream)
    plan = ko.Plan(w.model, kern, off, spec)
    graph = plan.capture(stream=stream, makespans=ms, stats=st)
    t_graph = _event_time(lambda: graph.launch(stream), stream, 50)
    plan.status(stream)
    graph.close()
    plan.close()
    ops = OPS_PER_BLOCK * int(ks["n_tblk"].sum()) * N
    print("[bench] small done", file=sys.stderr, flush=True)
    return {"workload": w.name, "orders": N, "ms_per_call": 1e3 * t_call, "ms_per_graph_replay": 1e3 * t_graph,
            "orders_per_s": N / t_graph, "achieved": ops / t_graph / 1e12,
            "frac": ops / t_graph / 1e12 / ALU_PEAK_TOPS,
            "note": "latency-bound: 720 orders, one wavefront each, on a 1,024-SIMD chip"}


def batch_leg() -> dict:
    """All orders of all 4096 sets of the batch workload (n = 4..9) in one
    captured graph of a planned launch, autotuned (engine, orders per work
    item, workgroups per CU) on 128 of the sets."""
    import json as _json

    import synth
    from paper_1511_07983_amd import batch
    recs = []
    try:
        batch.report(workload=2, sets=4096, tune_sets=128, reps=5, tune=True,
                     out=lambda t, **kw: recs.append(_json.loads(t)))
    except Exception as exc:
        return {"error": f"{type(exc).__name__}: {exc}"}
    rec = recs[-1]
    ops = 0
    for s in range(4096):
        ks = synth.draw_set(2, s)
        ops += OPS_PER_BLOCK * int(ks["n_tblk"].sum()) * math.factorial(len(ks))
    t = rec["graph_replay_s"]
    print("[bench] batch done", file=sys.stderr, flush=True)
    return {"workload": rec["workload"], "sets": rec["sets"], "orders": rec["orders"], "graph_replay_s": t,
            "orders_per_s": rec["orders_per_s"], "achieved": ops / t / 1e12, "frac": ops / t / 1e12 / ALU_PEAK_TOPS,
            "engine": rec["engine"], "config": rec["config"], "work_items": rec["work_items"]}


def contended_leg(model, kernels, off, N, ops_per_order, mem_blocks: int = 256) -> dict:
    """All orders of the same set when resident blocks share the chip's memory
    throughput (mem_blocks = one memory-bound block per CU at full speed):
    the engine the library picks (the lane engine for this set), HIP events
    around the simulate kernel and its follow-up launches."""
    import torch

    import paper_1511_07983_amd as ko
    gpu = dict(model.as_dict(), mem_blocks=mem_blocks)
    probe = ko.Plan(gpu, kernels, off, ko.OrderSpec.all())
    engine = probe.engine()[0]
    probe.close()
    n = int(off[1] - off[0])
    cls = 8 if n <= 8 else 10 if n <= 10 else 12 if n <= 12 else 16
    kernel = (f"ko::simulate_lanes_kernel<{12 if cls <= 10 else 16 if cls == 12 else 20}, {cls}, contended>"
              if engine == ko.ENGINE_LANES else "ko::simulate_kernel<4, true>")
    ms = torch.empty(N, dtype=torch.int64, device="cuda:0")
    st = torch.empty(8, dtype=torch.int64, device="cuda:0")
    spec = ko.OrderSpec.all()
    ko.ko_simulate_batch(gpu, kernels, off, spec, makespans=ms, stats=st)
    ko.ko_sync()
    ko.ko_set_kernel_timing(True)
    t = []
    for _ in range(3):
        ko.ko_simulate_batch(gpu, kernels, off, spec, makespans=ms, stats=st)
        t.append(ko.ko_last_kernel_ms() / 1e3)
    ko.ko_set_kernel_timing(False)
    ko.ko_sync()
    rec = ko.stats_records(st)[0]
    k = float(np.median(t))
    print("[bench] contended done", file=sys.stderr, flush=True)
    return {"kernel": kernel, "mem_blocks": mem_blocks, "orders": N,
            "kernel_ms": 1e3 * k, "orders_per_s": N / k, "achieved": ops_per_order * N / k / 1e12,
            "frac": ops_per_order * N / k / 1e12 / ALU_PEAK_TOPS,
            "min_makespan": int(rec["min_makespan"]), "max_makespan": int(rec["max_makespan"])}


def rounds_leg(ops_per_order: int):
    """The round-synchronous reading of the execution rounds on the same set, all
    orders unranked on the device (not in `value`): HIP-event time per launch,
    the same ALU fraction, and Algorithm 1's exact percentile under that model."""
    from paper_1511_07983_amd import rounds
    try:
        rec = rounds.report(reps=5, all_orders=True, out=lambda text: None)
    except Exception as exc:  # keep the throughput line even if this leg fails
        return {"error": f"{type(exc).__name__}: {exc}"}
    print("[bench] rounds done", file=sys.stderr, flush=True)
    achieved = ops_per_order * rec["orders"] / (rec["ms_per_launch"] / 1e3) / 1e12
    return {"kernel": "ko::rounds_kernel<4>", "orders": rec["orders"], "ms_per_launch": rec["ms_per_launch"],
            "orders_per_s": rec["orders_per_s"], "achieved": achieved, "frac": achieved / ALU_PEAK_TOPS,
            "heuristic_pct_inclusive": rec["heuristic_percentile"],
            "min_makespan": rec["best"], "max_makespan": rec["worst"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(an evaluation would shard across GPUs by rank range; this build runs on one)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1511_07983_amd as ko
    import synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.WORKLOADS[args.workload]
    ks = synth.draw_set(args.workload, 0)
    n = len(ks)
    N = math.factorial(n)
    off = [0, n]
    kernels = ko.kernel_array(ks)
    b_total = int(ks["n_tblk"].sum())

    # the kernel the all-orders leg runs (the library picks the engine by set size)
    probe = ko.Plan(w.model, kernels, off, ko.OrderSpec.all())
    engine = probe.engine()[0]
    probe_chunk, probe_items = probe.chunk, probe.work_items
    probe.close()
    if engine == ko.ENGINE_LANES:
        rc, gc = (12, 8) if n <= 8 else (12, 10) if n <= 10 else (16, 12) if n <= 12 else (20, 16)
        kernel_name = f"ko::simulate_lanes_kernel<{rc}, {gc}>"
    else:
        kernel_name = "ko::simulate_kernel<4>"

    ms = torch.empty(N, dtype=torch.int64, device=dev)
    st = torch.empty(8, dtype=torch.int64, device=dev)
    hist = torch.empty(1024, dtype=torch.int64, device=dev)
    ref = torch.empty(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    spec_all = ko.OrderSpec.all()

    def step():
        # 1. Algorithm 1's order (host), 2. its makespan, 3. all n! orders
        order = ko.ko_heuristic_order(w.model, kernels)
        order_dev = torch.tensor(order, dtype=torch.uint8).to(dev)
        ko.ko_simulate_batch(w.model, kernels, off, ko.OrderSpec.explicit(order_dev, [1]),
                             makespans=ref, stream=stream)
        ko.ko_simulate_batch(w.model, kernels, off, spec_all, ref_makespan=ref, makespans=ms,
                             stats=st, hist=hist, n_bins=1024, stream=stream)
        return order

    for _ in range(args.warmup):
        step()
    ko.ko_sync()
    # the simulate kernel of every timed all-orders call is bracketed by two
    # events on its own stream inside libko; the durations are read per step
    ko.ko_set_kernel_timing(True)
    torch.cuda.synchronize()
    kernel_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        kernel_s.append(ko.ko_last_kernel_ms() / 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ko.ko_set_kernel_timing(False)
    ko.ko_sync()
    elapsed = t1 - t0
    kernel_avg = float(np.mean(kernel_s))

    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    rec = ko.stats_records(st)[0]
    assert rec["n_orders"] == N
    assert rec["n_less"] + rec["n_equal"] + rec["n_greater"] == N
    assert int(hist.cpu().numpy().view(np.uint64).sum()) == N
    pct = 100.0 * (rec["n_greater"] + rec["n_equal"]) / N

    ops_per_order = OPS_PER_BLOCK * b_total
    achieved = ops_per_order * N / kernel_avg / 1e12
    out = {
        "metric": "exact launch-order evals/s; surrogate speedup to exact top-1% order",
        "value": N * args.steps / elapsed,
        "unit": "orders/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_kernels": n, "orders_per_step": N, "blocks_per_order": b_total,
                   "cu_model": w.model.n_cu, "seed": f"SeedSequence([20151123, {w.index}, 0])",
                   "histogram_bins": 1024},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "Top/s",
                     "frac": achieved / ALU_PEAK_TOPS, "traffic": measured_traffic(probe_chunk, probe_items),
                     "traffic_unit": "bytes per launch", "work_items": probe_items, "orders_per_item": probe_chunk,
                     "kernel": kernel_name, "kernel_ms": 1e3 * kernel_avg,
                     "ops_per_order": ops_per_order},
        "heuristic": {"order": ko.ko_heuristic_order(w.model, kernels), "pct_inclusive": pct,
                      "min_makespan": int(rec["min_makespan"]), "max_makespan": int(rec["max_makespan"])},
    }
    out["rounds"] = rounds_leg(ops_per_order)
    out["contended"] = contended_leg(w.model, kernels, off, N, ops_per_order)
    if not args.no_legs:
        out["small"] = small_leg()
        out["batch"] = batch_leg()
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(args.surrogate_heldout)
        out["search_n16"] = search_n16_leg()
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(w.model, ks, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
