"""Benchmark: lambda(omega)-mapped gasket steps on one MI355X.

Default workload: a level-14 Sierpinski gasket (n = 16384, 4,782,969 cells);
one benchmark step = one uint8 B3/S23 automaton step plus one float32 heat
step (alpha = 0.2), both through the lambda kernels at their tuned tile size.
`value` = gasket cells updated per second over the timed K steps (both
rules), with the state resident in HBM.  The line also carries the roofline
of the dominant kernel, the bounding-box comparison and the CPU oracle's rate
on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload k14|k16]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
ALPHA = 0.2
# Algorithmic bytes per cell-update: one read and one write of every 64-byte
# row segment that holds a gasket member (64 B = the memory request size);
# a level-k gasket has 4^g * 3^(k-g) cells in such segments, g = log2(64/s):
#   uint8:   2 * (4/3)^6 = 11.237 B per member cell
#   float32: 8 * (4/3)^4 = 25.284 B per member cell
BYTES_PER_CELL = {0: 2.0 * (4.0 / 3.0) ** 6, 1: 8.0 * (4.0 / 3.0) ** 4}
WORKLOADS = {"k14": 14, "k16": 16}
KERNEL_SRC = ["device_tile.hpp", "device_map.hpp", "step_kernels.hip"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        with open(os.path.join(ROOT, "paper_2004_13475_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, rule_name: str):
    """Per-launch HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    committed counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"step_{rule_name}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="k14", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-bb", action="store_true", help="skip the bounding-box leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2004_13475_amd as F

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    k = WORKLOADS[args.workload]
    n = 1 << k
    cells = 3 ** k
    K, W = args.steps, args.warmup
    alpha = float(np.float32(ALPHA))

    bufs = {}
    for rule, dt in ((0, torch.uint8), (1, torch.float32)):
        b0 = torch.empty((n, n), dtype=dt, device=dev)
        b1 = torch.zeros((n, n), dtype=dt, device=dev)
        F.seed_fill(k, rule, 1, b0)
        bufs[rule] = [b0, b1]
    torch.cuda.synchronize()

    # autotune the lambda launch for each rule (records the cached tuning)
    tunings = {}
    for rule in (0, 1):
        tunings[rule] = F.autotune(k, rule, alpha, bufs[rule][0], bufs[rule][1])
        F.seed_fill(k, rule, 1, bufs[rule][0])
        bufs[rule][1].zero_()
    torch.cuda.synchronize()

    def run(rule, steps, map_=F.MAP_LAMBDA, tuning=None):
        b0, b1 = bufs[rule]
        t = tuning or tunings[rule]
        F.step_tuned(map_, k, rule, alpha, b0, b1, steps, t[0], t[1], t[2])
        if steps % 2:
            bufs[rule].reverse()

    # warm-up
    run(0, W)
    run(1, W)
    torch.cuda.synchronize()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    run(0, K)
    ev[1].record(stream)
    run(1, K)
    ev[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_ca = ev[0].elapsed_time(ev[1])
    ms_heat = ev[1].elapsed_time(ev[2])
    total_ms = ms_ca + ms_heat
    value = 2.0 * cells * K / (total_ms / 1e3)

    per_launch = {0: ms_ca / K * 1e-3, 1: ms_heat / K * 1e-3}
    dom = 1 if per_launch[1] >= per_launch[0] else 0
    rule_name = {0: "ca", 1: "heat"}
    alg_bytes = {r: BYTES_PER_CELL[r] * cells for r in (0, 1)}
    achieved = alg_bytes[dom] / per_launch[dom] / 1e9
    traffic = read_traffic(args.workload, rule_name[dom])

    # bounding box: same tile size, and its own best tile size
    bb = {}
    if not args.no_bb:
        nbb = max(10, min(K, 200))
        for rule in (0, 1):
            res = {}
            for r in range(max(2, k - 15), 7):
                tb = (r, 256 if (r >= 5 and rule == 1) or r >= 6 else 64, 0)
                run(rule, 2, F.MAP_BB, tb)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                run(rule, nbb, F.MAP_BB, tb)
                e1.record(stream)
                torch.cuda.synchronize()
                res[r] = e0.elapsed_time(e1) / nbb
            lam_ms = per_launch[rule] * 1e3
            best_r = min(res, key=res.get)
            bb[rule_name[rule]] = {
                "lambda_ms_per_step": lam_ms, "lambda_r": tunings[rule][0],
                "bb_ms_per_step_same_r": res.get(tunings[rule][0]),
                "bb_best_r": best_r, "bb_ms_per_step_best": res[best_r],
                "speedup_same_r": res.get(tunings[rule][0], float("nan")) / lam_ms,
                "speedup_best": res[best_r] / lam_ms,
            }

    cpu = None
    if not args.no_cpu:
        import fractal_inputs as fi
        import oracle
        ck = 14
        states = {0: fi.full_state(ck, 0, 1), 1: fi.full_state(ck, 1, 1, dtype=np.float64)}
        nsteps = {0: 4, 1: 2}
        tc = time.perf_counter()
        oracle.ca_run(ck, states[0], nsteps[0])
        oracle.heat_run(ck, states[1], alpha, nsteps[1])
        dtc = time.perf_counter() - tc
        cpu = {"value": 3 ** ck * (nsteps[0] + nsteps[1]) / dtc, "unit": "cells/s",
               "cores": oracle.threads(), "kind": "oracle",
               "sample": f"level-14 gasket, whole array: {nsteps[0]} automaton steps + "
                         f"{nsteps[1]} float64 heat steps ({dtc:.1f} s)"}

    line = {
        "metric": "fractal cells updated/s and HBM GB/s (% peak), lambda vs BB; "
                  "served p50/p99 latency",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": total_ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8+f32", "data": "synthetic",
        "config": {"workload": f"sierpinski-k{k}-lambda-ca-u8+heat-f32",
                   "k": k, "n": n, "cells": cells,
                   "tuning_ca": list(tunings[0]), "tuning_heat": list(tunings[1]),
                   "wall_s": wall},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"lambda_step_{rule_name[dom]}",
                     "alg_bytes_per_launch": alg_bytes[dom],
                     "avg_launch_us": per_launch[dom] * 1e6},
        "per_rule": {rule_name[r]: {"ms_per_step": per_launch[r] * 1e3,
                                    "cells_per_s": cells / per_launch[r],
                                    "alg_GBs": alg_bytes[r] / per_launch[r] / 1e9}
                     for r in (0, 1)},
        "bb": bb,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
