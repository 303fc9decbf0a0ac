"""Validation of the dispatch model against the GPU it models.

For each kernel set, Algorithm 1's order and seeded random orders run on the
hardware as synthetic kernels (ko_hw_time_orders: one stream per kernel, in
launch order, makespan by HIP events) and are simulated exactly with the same
kernel parameters, except that each kernel's registers per thread are the
VGPR count of the compiled kernel that stands in for it (ko_hw_vgprs).  The
agreement is measured by the Spearman rank correlation of simulated and
measured makespans across the orders of a set: the model is meant to rank
launch orders, not to predict milliseconds.  This validates the model; it is
not a parity target.

The number of hardware queues HIP spreads the streams over is fixed when HIP
initialises (GPU_MAX_HW_QUEUES), so each setting is its own process: with as
many queues as kernels, every kernel has a queue of its own and dispatches
concurrently; with one queue, kernels are dispatched strictly in launch order,
which is the discipline the model assumes.
"""

from __future__ import annotations

import json
import math

import numpy as np

from . import OrderSpec, kernel_array, ko_heuristic_order, ko_hw_time_orders, ko_hw_vgprs, ko_simulate_batch, ko_sync


def spearman(a, b) -> float:
    """Spearman's rank correlation (average ranks for ties)."""
    def ranks(x):
        x = np.asarray(x, dtype=np.float64)
        order = np.argsort(x, kind="stable")
        r = np.empty(len(x))
        r[order] = np.arange(len(x), dtype=np.float64)
        # average the ranks of ties
        for v in np.unique(x):
            idx = np.flatnonzero(x == v)
            if len(idx) > 1:
                r[idx] = r[idx].mean()
        return r
    ra, rb = ranks(a), ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = math.sqrt(float((ra * ra).sum() * (rb * rb).sum()))
    return float((ra * rb).sum() / den) if den > 0 else float("nan")


def calibrate(rows) -> dict:
    """Least-squares fit of measured milliseconds against model cycles over every
    order of every set: ms = a * cycles / scale + b, where scale divides the
    synthetic kernels' work.  Returns ns per model cycle at full scale (a / scale
    in ns), the offset b in ms and R^2.  The within-set Spearman asks whether the
    model ranks orders; this asks whether its cycles predict time across sets."""
    c = np.concatenate([np.asarray(r["simulated_cycles"], dtype=np.float64) / r["scale"] for r in rows])
    m = np.concatenate([np.asarray(r["measured_ms"], dtype=np.float64) for r in rows])
    A = np.vstack([c, np.ones_like(c)]).T
    (a, b), *_ = np.linalg.lstsq(A, m, rcond=None)
    pred = A @ np.array([a, b])
    ss = float(((m - m.mean()) ** 2).sum())
    r2 = 1.0 - float(((m - pred) ** 2).sum()) / ss if ss > 0 else float("nan")
    scales = {int(r["scale"]) for r in rows}
    per_cycle_ns = a * 1e6 / scales.pop() if len(scales) == 1 else float("nan")
    return {"ns_per_model_cycle": per_cycle_ns, "ms_per_scaled_cycle": float(a), "offset_ms": float(b),
            "r2": r2, "points": int(len(m))}


def hardware_kernels(kernels) -> np.ndarray:
    """The set as the model should see the hardware stand-ins: registers per
    thread replaced by the VGPR count of the compiled variant."""
    k = kernel_array(kernels).copy()
    k["regs_thr"] = [ko_hw_vgprs(int(r)) for r in k["regs_thr"]]
    return k


def simulate(model, kernels, orders) -> np.ndarray:
    import torch
    n = len(kernels)
    o = torch.from_numpy(np.ascontiguousarray(orders, dtype=np.uint8).ravel()).to("cuda:0")
    ms = torch.empty(len(orders), dtype=torch.int64, device="cuda:0")
    ko_simulate_batch(model, kernels, [0, n], OrderSpec.explicit(o, [len(orders)]), makespans=ms)
    ko_sync()
    return ms.cpu().numpy()


def validate_set(model, kernels, *, n_random: int, seed: int, target_ms: float = 100.0, reps: int = 2,
                 probe_scale: int = 4096, mem_blocks=()):
    hk = hardware_kernels(kernels)
    n = len(hk)
    rng = np.random.default_rng(seed)
    orders = [ko_heuristic_order(model, hk)] + [rng.permutation(n).tolist() for _ in range(n_random)]
    orders = np.array(orders, dtype=np.int32)
    probe = ko_hw_time_orders(kernels, orders[:1], probe_scale, 1)[0]
    # at least 256: bounds the largest synthetic kernel to ~0.5 TB of streaming loads
    scale = max(256, int(round(probe_scale * probe / target_ms)))
    measured = ko_hw_time_orders(kernels, orders, scale, reps)
    simulated = simulate(model, hk, orders)
    # the same orders under the memory-contention mode (Section 4's balance of
    # instructions and memory accesses across co-resident blocks), one B each
    base = model if isinstance(model, dict) else model.as_dict()
    contended = {int(b): simulate(dict(base, mem_blocks=int(b)), hk, orders) for b in mem_blocks}
    return {"orders": orders.tolist(), "scale": scale, "measured_ms": measured.tolist(),
            "simulated_cycles": simulated.tolist(), "spearman": spearman(simulated, measured),
            "spearman_contended": {b: spearman(c, measured) for b, c in contended.items()},
            "contended_cycles": {b: c.tolist() for b, c in contended.items()},
            "heuristic_rank_measured": int((measured < measured[0]).sum()),
            "heuristic_rank_simulated": int((simulated < simulated[0]).sum())}


def main(argv=None):
    import argparse
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="dispatch model vs hardware (one GPU)")
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--sets", type=int, default=8)
    ap.add_argument("--random-orders", type=int, default=7)
    ap.add_argument("--target-ms", type=float, default=100.0)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--mem-blocks", default="",
                    help="comma-separated mem_blocks values: also rank the orders under memory contention")
    a = ap.parse_args(argv)
    mem_blocks = [int(b) for b in a.mem_blocks.split(",") if b.strip()]
    queues = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    import torch
    import synth
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[a.workload]
    rows = []
    for s in range(a.sets):
        ks = synth.draw_set(a.workload, s)
        row = validate_set(w.model, ks, n_random=a.random_orders, seed=1000 + s, target_ms=a.target_ms,
                           reps=a.reps, mem_blocks=mem_blocks)
        row["set"] = s
        row["hw_queues"] = queues
        m = np.array(row["measured_ms"])
        c = np.array(row["simulated_cycles"], dtype=np.float64)
        row["spread_measured"] = float(m.max() / m.min() - 1.0)
        row["spread_simulated"] = float(c.max() / c.min() - 1.0)
        rows.append(row)
        print(json.dumps({k: row[k] for k in ("set", "hw_queues", "scale", "spearman", "spearman_contended",
                                              "spread_measured", "spread_simulated", "heuristic_rank_measured",
                                              "heuristic_rank_simulated", "measured_ms", "simulated_cycles")}),
              flush=True)
    rho = [r["spearman"] for r in rows]
    print(json.dumps({"calibration": True, "hw_queues": queues, **calibrate(rows)}), flush=True)
    contended = {b: float(np.nanmean([r["spearman_contended"][b] for r in rows])) for b in mem_blocks}
    print(json.dumps({"summary": True, "hw_queues": queues, "sets": a.sets, "orders_per_set": a.random_orders + 1,
                      "spearman_mean": float(np.nanmean(rho)), "spearman_min": float(np.nanmin(rho)),
                      "spearman_max": float(np.nanmax(rho)), "spearman_mean_contended": contended}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
