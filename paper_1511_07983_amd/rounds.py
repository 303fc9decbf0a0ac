"""Round-synchronous execution rounds (Section 2) over sampled launch orders.

Times ko_simulate_rounds on the n=10 set of the all-orders workload (MI355X-shaped
model), over the same seeded sampled orders that ko_simulate_batch evaluates in
sampled mode or (--all) over all 10! orders unranked on the device, and reports
Algorithm 1's order under this model: its makespan and its percentile among the
evaluated orders (the share of them with a makespan at least as long).  The
makespans, the best and worst order and the counts behind the percentile are
computed on the device (ko_simulate_rounds, then ko_stats_i64); only the
64-byte statistics record comes back.

    python -m paper_1511_07983_amd.rounds [--orders N | --all] [--reps R]
"""

from __future__ import annotations

import argparse
import json
import sys

import numpy as np

SEED = 0x5EED0F2


def report(n_orders: int = 1 << 22, reps: int = 5, all_orders: bool = False, out=print) -> dict:
    import torch

    import synth

    from . import ko_heuristic_order, ko_sample_orders, ko_simulate_rounds, ko_stats_i64, stats_records

    wl = synth.WORKLOADS[1]
    ks = synth.draw_set(1, 0)
    n = len(ks)
    gpu = wl.model.as_dict()
    dev = torch.device("cuda", 0)
    if all_orders:
        n_orders = 1
        for i in range(2, n + 1):
            n_orders *= i
        orders = None
    else:
        orders = torch.empty((n_orders, n), dtype=torch.uint8, device=dev)
        ko_sample_orders(n, 0, SEED, n_orders, orders=orders)
    ms = torch.empty(n_orders, dtype=torch.int64, device=dev)
    ko_simulate_rounds(gpu, ks, orders, ms, count=n_orders)          # warm-up
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        ko_simulate_rounds(gpu, ks, orders, ms, count=n_orders)
    stop.record()
    torch.cuda.synchronize()
    ms_per_launch = start.elapsed_time(stop) / reps
    heur = ko_heuristic_order(gpu, ks)
    h = torch.tensor([heur], dtype=torch.uint8, device=dev)
    h_ms = ko_simulate_rounds(gpu, ks, h)
    st = stats_records(ko_stats_i64(ms, ref=h_ms))[0]
    if st["min_makespan"] < 0:
        raise RuntimeError("negative round makespan from the device")
    h_ms = int(h_ms.cpu()[0])
    rec = {
        "model": "round-synchronous execution rounds",
        "workload": wl.name,
        "n": n,
        "orders": n_orders,
        "orders_kind": "all, by lexicographic rank" if all_orders else "sampled",
        "ms_per_launch": round(ms_per_launch, 3),
        "orders_per_s": round(n_orders / (ms_per_launch / 1e3)),
        "best": int(st["min_makespan"]),
        "worst": int(st["max_makespan"]),
        "heuristic_order": heur,
        "heuristic_makespan": h_ms,
        "heuristic_percentile": round(100.0 * float(st["n_equal"] + st["n_greater"]) / n_orders, 2),
    }
    out(json.dumps(rec))
    return rec


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--orders", type=int, default=1 << 22)
    ap.add_argument("--all", action="store_true", help="all n! orders instead of sampled ones")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    report(a.orders, a.reps, a.all)
    return 0


if __name__ == "__main__":
    sys.exit(main())
