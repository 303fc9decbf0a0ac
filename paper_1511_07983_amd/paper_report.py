"""Paper-shaped workloads: the experiments of Table 2 on the GTX580 model.

Each experiment's kernels (synth/paper_sets.py, with its stated assumptions)
are evaluated exactly over all orders (6! or 8!) in one batch: the best and
worst makespan, Algorithm 1's order and its makespan, its percentile rank, the
speedup over the worst order and the deviation from the best, i.e. Table 3's
columns, in model cycles.  Table 3's own figures were measured on the paper's
kernels on a GTX580 and are printed beside them as context, not as targets.
Each row also gives the same figures under the round-synchronous reading of the
execution rounds (ko_simulate_rounds over all orders).

    python -m paper_1511_07983_amd.paper_report
"""

from __future__ import annotations

import json

# Table 3: optimal, worst and algorithm times (ms), percentile rank (%), speedup
# over worst, deviation from optimal (%), as printed in the paper
TABLE3 = {
    "EP-6-shm": (140.46, 249.15, 146.38, 91.5, 1.702, 4.21),
    "EP-6-grid": (123.39, 156.03, 123.45, 96.3, 1.264, 0.049),
    "BS-6-blk": (699.29, 1699.04, 702.29, 96.5, 2.419, 0.43),
    "EpBs-6": (100.03, 167.47, 100.20, 96.1, 1.671, 0.17),
    "EpBs-6-shm": (251.90, 311.79, 251.95, 99.4, 1.238, 0.02),
    "EpBsEsSw-8": (109.21, 597.43, 115.23, 94.8, 5.185, 5.51),
}


def report(out=print):
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import paper_sets

    import itertools

    import numpy as np
    import torch

    from . import batch, ko_simulate_rounds, ko_stats_i64, stats_records
    names = list(paper_sets.EXPERIMENTS)
    sets = [paper_sets.EXPERIMENTS[k] for k in names]
    res = batch.percentiles(paper_sets.MODEL, sets)
    rows = []
    for i, name in enumerate(names):
        best, worst, alg = int(res["best"][i]), int(res["worst"][i]), int(res["makespan"][i])
        row = {"experiment": name, "n": len(sets[i]), "orders": int(res["n_orders"][i]),
               "best_cycles": best, "worst_cycles": worst, "algorithm_cycles": alg,
               "algorithm_order": [int(x) for x in res["order"][i]],
               "percentile_inclusive": float(res["pct_inclusive"][i]),
               "speedup_over_worst": worst / alg, "deviation_from_best": (alg - best) / best,
               "table3_context": dict(zip(("optimal_ms", "worst_ms", "algorithm_ms", "percentile",
                                           "speedup", "deviation_pct"), TABLE3[name]))}
        # the same orders under the round-synchronous reading of the execution rounds
        n = len(sets[i])
        perms = np.array(list(itertools.permutations(range(n))), dtype=np.uint8)
        rms = ko_simulate_rounds(paper_sets.MODEL.as_dict(), sets[i], torch.from_numpy(perms).cuda())
        h = torch.tensor([row["algorithm_order"]], dtype=torch.uint8).cuda()
        h_ms = ko_simulate_rounds(paper_sets.MODEL.as_dict(), sets[i], h)
        st = stats_records(ko_stats_i64(rms, ref=h_ms))[0]
        row["rounds"] = {"best_cycles": int(st["min_makespan"]), "worst_cycles": int(st["max_makespan"]),
                         "algorithm_cycles": int(h_ms.cpu()[0]),
                         "percentile_inclusive": round(100.0 * float(st["n_equal"] + st["n_greater"])
                                                       / len(perms), 2)}
        rows.append(row)
        out(json.dumps(row), flush=True)
    return rows


if __name__ == "__main__":
    import torch
    torch.cuda.set_device(0)
    report()
