"""Benchmark: lambda(omega)-mapped gasket steps on one MI355X.

Default workload (the one `value` is quoted on): a level-16 Sierpinski
gasket (n = 65536, 43,046,721 cells; 4.3 GB uint8 / 17.2 GB float32 per
buffer, far beyond the caches); one benchmark step = one uint8 B3/S23
automaton step plus one float32 heat step (alpha = 0.2), both through the
lambda kernels at the library's default launch for the level (the measured
fastest; --autotune times every candidate first instead).  `value` = gasket
cells updated per second over the timed K steps (both rules), state resident
in HBM, timed with HIP events on the stream the kernels run on.

Also on the same JSON line:
  roofline      dominant kernel's algorithmic HBM GB/s vs the 8 TB/s peak;
                its launch duration is the mean (and standard error) of 10
                sub-averages, each over 4 back-to-back whole launches
  k14           level-14 gasket (cache-assisted: its member segments fit the
                256 MB last-level cache): per-rule rates and rooflines
  bb            bounding-box steps at the same tile size and at BB's best
  lambda_vs_bb_by_k  lambda vs the bounding box at levels 10, 12, 14, 16
                (each at its best launch), plus the level-10, 16 x 16-tile,
                100-step automaton in microseconds per step
  batch         256 gaskets of levels 8..14, 500 steps, one graph launch vs
                256 plain lambda_step calls
  serve         Poisson request stream (--serve SECONDS, 60 by default),
                p50/p99 latency, saturated and sequential throughput
  sw_rd         tests SW (single write) and RD (reduction), lambda vs BB
  compact       compact storage through lambda^-1 at levels 16, 18, 20
  nbb           carpet and Vicsek fractals: SW, RD, CA, lambda vs BB
  cpu_baseline  the CPU oracle on a bounded sample of the default workload

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload k16|k14]
                    [--no-cpu] [--no-bb] [--no-k14] [--no-batch] [--no-sweep]
                    [--serve SECONDS] [--copy-calibration]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
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
AUTOTUNE = False  # set by --autotune
RULE_NAME = {0: "ca", 1: "heat"}
KERNEL_SRC = ["device_tile.hpp", "device_map.hpp", "step_kernel.hpp", "step_kernels.hip",
              "device_march.hpp", "march_pick.hpp", "step_march.hip", "step_march_ca.hip",
              "step_march_heat.hip", "step_march_mid_ca.hip", "step_march_mid_heat.hip",
              "block_engine.hpp", "block_slots.inc", "block_heat.hpp", "block_heat.hip",
              "block_ca.hpp", "block_ca.hip"]


def kernel_hash() -> str:
    """Hash of the kernel sources' code: comments and whitespace are left
    out, so editing a comment does not orphan the counter summaries."""
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        with open(os.path.join(ROOT, "paper_2004_13475_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)  # block comments
        src = re.sub(r"//[^\n]*", " ", src)                # line comments
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def read_traffic(workload: str, rule_name: str):
    """Per-launch HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    committed counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"lambda_step_{rule_name}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


def read_valu_issue(kernel: str):
    """Fraction of the VALU issue ceiling a full-depth launch of `kernel`
    reached (SQ counters), from the committed summary, if it was taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", "block_k16_sq_counters.md")
    if not kernel or not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    m = re.search(rf"valu_issue_frac {re.escape(kernel)}:\s*([0-9.]+)", txt)
    if not m_hash or not m or m_hash.group(1) != kernel_hash():
        return None
    return float(m.group(1))


class Gasket:
    """A pair of state buffers per rule for one level, plus timing helpers."""

    def __init__(self, F, torch, k, seed=1):
        self.F, self.torch, self.k = F, torch, k
        self.n = 1 << k
        self.cells = 3 ** k
        self.alpha = float(__import__("numpy").float32(ALPHA))
        self.stream = torch.cuda.current_stream()
        self.bufs = {}
        for rule, dt in ((0, torch.uint8), (1, torch.float32)):
            b0 = torch.empty((self.n, self.n), dtype=dt, device="cuda")
            b1 = torch.zeros((self.n, self.n), dtype=dt, device="cuda")
            F.seed_fill(k, rule, seed, b0)
            self.bufs[rule] = [b0, b1]
        self.tunings = {}
        torch.cuda.synchronize()

    def reseed(self, rule, seed=1):
        self.F.seed_fill(self.k, rule, seed, self.bufs[rule][0])
        self.bufs[rule][1].zero_()

    def autotune(self, search=None):
        """Launch parameters per rule: the library default for the level, or
        (search, or --autotune) the autotuner's pick."""
        search = AUTOTUNE if search is None else search
        for rule in (0, 1):
            if search:
                self.tunings[rule] = self.F.autotune(self.k, rule, self.alpha, *self.bufs[rule])
                self.reseed(rule)
            else:
                self.tunings[rule] = self.F.get_tuning(self.k, rule)
        self.torch.cuda.synchronize()

    def run(self, rule, steps, map_=None, tuning=None):
        F = self.F
        t = tuning or self.tunings[rule]
        F.step_tuned(F.MAP_LAMBDA if map_ is None else map_, self.k, rule, self.alpha,
                     self.bufs[rule][0], self.bufs[rule][1], steps, t[0], t[1], t[2],
                     t[3] if len(t) > 3 else 0)
        if steps % 2:
            self.bufs[rule].reverse()

    def time(self, rule, steps, map_=None, tuning=None):
        """Seconds per launch, HIP events around `steps` back-to-back launches."""
        torch = self.torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        self.run(rule, steps, map_, tuning)
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / steps

    def free(self):
        self.bufs.clear()
        self.torch.cuda.empty_cache()


def steps_per_launch(tuning):
    """Steps one launch advances: 36, 32, 24 (block engine), 16, 8, 4 or 2
    for fused launches, else 1."""
    fl = tuning[3] if len(tuning) > 3 else 0
    for flag, T in ((32768, 36), (16384, 32), (8192, 24), (128, 16), (64, 8), (16, 4), (8, 2)):
        if fl & flag:
            return T
    return 1


def kernel_name(tuning, rule):
    """Name of the step kernel template a tuning launches."""
    fl = tuning[3] if len(tuning) > 3 else 0
    if fl & 4096:
        if tuning[0] == 7:
            return "block2_ca_kernel" if rule == 0 else "block2_heat_kernel"
        return "block_ca_kernel" if rule == 0 else "block_heat_kernel"
    return "march_kernel" if fl & 32 else "step_kernel"


def roofline(rule, cells, stats, tuning, traffic=None, kernel=""):
    """Roofline of one launch.  A launch reads and writes every member
    segment once however many steps it advances (intermediate steps stay in
    LDS or registers), so its algorithmic bytes are the per-cell figure
    times 3^k; `stats` is launch_stats()'s measured launch duration (mean
    and standard error of sub-averages) of the tuned step count."""
    spl = steps_per_launch(tuning)
    sec_per_launch = stats["mean_s"]
    alg = BYTES_PER_CELL[rule] * cells
    achieved = alg / sec_per_launch / 1e9
    rate = None if traffic is None else traffic / sec_per_launch / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_GBs": rate, "traffic_frac": None if rate is None else rate / HBM_PEAK_GBS,
            "traffic_over_alg": None if traffic is None else traffic / alg,
            "kernel": kernel,
            "steps_per_launch": spl, "alg_bytes_per_launch": alg,
            "avg_launch_us": sec_per_launch * 1e6,
            "avg_launch_us_stderr": stats["stderr_s"] * 1e6,
            "timing": f"{stats['reps']} sub-averages of {stats['launches']} back-to-back "
                      f"{spl}-step launches (HIP events on the launch stream)",
            "per_step_equivalent_GBs": alg * spl / sec_per_launch / 1e9,
            # the other limit of a deep launch: the share of the VALU issue
            # ceiling its steps use (committed SQ counters)
            "valu_issue_frac": read_valu_issue(kernel)}


def launch_stats(g, rule, map_=None, tuning=None, reps=10, pairs=2):
    """Duration of one whole launch of the tuned T-step kernel, in the
    spirit of Section 6.2's method (a mean of sub-averages of consecutive
    synchronised calls): `reps` sub-averages, each HIP events around 2 *
    `pairs` back-to-back T-step launches (runs of 2T steps, which the library
    issues as two T-step launches), after one warm-up run; mean and standard
    error of the sub-averages, independent of the benchmark's step count."""
    torch = g.torch
    t = tuning or g.tunings[rule]
    T = steps_per_launch(t)
    g.run(rule, 2 * T, map_, t)
    torch.cuda.synchronize()
    subs = [g.time(rule, 2 * T * pairs, map_, t) * T for _ in range(reps)]
    mean = sum(subs) / reps
    var = sum((x - mean) ** 2 for x in subs) / (reps - 1)
    return {"mean_s": mean, "stderr_s": math.sqrt(var / reps), "reps": reps,
            "launches": 2 * pairs}


def bb_tuning(g, rule, r, lam=None):
    """The bounding-box launch compared with lambda's: lambda's engine and
    flags at tile size r where that tile size takes them, else one step per
    launch with whole segments."""
    t = lam or g.tunings[rule]
    fl = t[3]
    if fl & g.F.FLAG_BLOCK and r not in (6, 7):
        # the block engine takes 64 x 64 and 128 x 128 tiles: the
        # march at other sizes (16 steps per launch at most)
        fl = (fl & ~g.F.FLAG_BLOCK) | g.F.FLAG_MARCH
        deep = g.F.FLAG_FUSE24 | g.F.FLAG_FUSE32 | g.F.FLAG_FUSE36
        if fl & deep:
            fl = (fl & ~deep) | g.F.FLAG_FUSE16
    if fl & g.F.FLAG_FUSE16 and rule == 1 and r < 4:
        fl = (fl & ~g.F.FLAG_FUSE16) | g.F.FLAG_FUSE8  # heat: 16 steps need 16-cell tiles
    if (1 << r) * (1 if rule == 0 else 4) < 16:
        fl = 3
    return (r, 256 if (r >= 3 or fl & 32 or fl & g.F.FLAG_BLOCK) else 64, g.F.ORDER_NATURAL, fl)


def bb_leg(g, per_launch, nsteps):
    F = g.F
    out = {}
    for rule in (0, 1):
        res = {}
        lds = {}
        for r in range(max(2, g.k - 12), 8):
            tb = bb_tuning(g, rule, r)
            g.run(rule, 2 * steps_per_launch(tb), F.MAP_BB, tb)
            res[r] = g.time(rule, nsteps, F.MAP_BB, tb)
            if tb[3] & (F.FLAG_MARCH | F.FLAG_BLOCK):
                # the LDS engine (one workgroup per block, empty blocks exit
                # at once) may suit the bounding box better
                tl = (r, 256 if r >= 3 else 64, F.ORDER_NATURAL, 19 if rule == 1 else 11)
                g.run(rule, 8, F.MAP_BB, tl)
                lds[r] = g.time(rule, nsteps, F.MAP_BB, tl)
                res[r] = min(res[r], lds[r])
        lam = per_launch[rule]
        best = min(res, key=res.get)
        same = res.get(g.tunings[rule][0])
        out[RULE_NAME[rule]] = {
            "lambda_us": lam * 1e6, "lambda_r": g.tunings[rule][0],
            "bb_us_same_r": None if same is None else same * 1e6,
            "bb_best_r": best, "bb_us_best": res[best] * 1e6,
            "speedup_same_r": None if same is None else same / lam,
            "speedup_best": res[best] / lam,
            "bb_us_by_r": {str(r): v * 1e6 for r, v in res.items()},
            "bb_lds_engine_us_by_r": {str(r): v * 1e6 for r, v in lds.items()},
        }
    return out


def sw_rd_leg(F, torch, k, reps=20):
    """Tests SW and RD of Section 6.2 at level k: each map at tile sides
    16..128, seconds per call (HIP events over `reps` calls); lambda vs BB at
    lambda's best tile size and at each map's best.  Algorithmic bytes: the
    member segments written (SW) or read (RD) once, half the step figure."""
    stream = torch.cuda.current_stream()
    out = {}
    for rule, dt in ((0, torch.uint8), (1, torch.float32)):
        n = 1 << k
        buf = torch.zeros((n, n), dtype=dt, device="cuda")
        res = {"sw": {}, "rd": {}}
        for r in range(4, 8):
            if k - r > 15:
                continue
            work = torch.empty(max(8, F.reduce_workspace(k, r)), dtype=torch.uint8, device="cuda")
            val = torch.zeros(1, dtype=torch.float64, device="cuda")
            for map_ in (F.MAP_LAMBDA, F.MAP_BB):
                for op in ("sw", "rd"):
                    def call():
                        if op == "sw":
                            F.single_write(map_, k, r, rule, 1, buf)
                        else:
                            F.reduce(map_, k, r, rule, buf, work, val)
                    call()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        call()
                    e1.record(stream)
                    torch.cuda.synchronize()
                    res[op][(r, map_)] = e0.elapsed_time(e1) * 1e-3 / reps
            del work, val
        alg = BYTES_PER_CELL[rule] / 2 * 3 ** k
        row = {}
        for op in ("sw", "rd"):
            lam = {r: t for (r, m), t in res[op].items() if m == F.MAP_LAMBDA}
            bb = {r: t for (r, m), t in res[op].items() if m == F.MAP_BB}
            rl, rbb = min(lam, key=lam.get), min(bb, key=bb.get)
            achieved = alg / lam[rl] / 1e9
            row[op] = {"lambda_r": rl, "lambda_us": lam[rl] * 1e6, "bb_r": rbb,
                       "bb_us": bb[rbb] * 1e6, "bb_us_same_r": bb[rl] * 1e6,
                       "speedup_same_r": bb[rl] / lam[rl], "speedup_best": bb[rbb] / lam[rl],
                       "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                    "alg_bytes": alg},
                       "lambda_us_by_r": {str(r): t * 1e6 for r, t in lam.items()},
                       "bb_us_by_r": {str(r): t * 1e6 for r, t in bb.items()}}
        out[RULE_NAME[rule]] = row
        del buf
        torch.cuda.empty_cache()
    return out


def compact_leg(F, torch, steps=64):
    """Compact storage (tiles kept in lambda order): per-step time and cell
    rate at levels 16, 18 and 20 with the default compact launch (the block
    engine on 64 x 64 tiles), and the state bytes against the n x n array's;
    beside it the register march on compact states (the automaton on the
    same tiles, heat on 32 x 32 tiles)."""
    stream = torch.cuda.current_stream()
    alpha = float(__import__("numpy").float32(ALPHA))
    out = {}
    march = F.FLAG_MARCH | F.FLAG_SEGMENTS
    for name, rule, r, flags in (("ca", 0, 6, 0), ("heat", 1, 6, 0),
                                 ("ca_march", 0, 6, march | F.FLAG_FUSE16 | F.FLAG_NT_STORE),
                                 ("heat_march_r5", 1, 5, 0)):
        row = {}
        for k in (16, 18, 20):
            nbytes = F.compact_bytes(k, r, rule)
            free, _ = torch.cuda.mem_get_info()
            if 2 * nbytes + (1 << 30) > free:
                row[f"k{k}"] = {"skipped": "device memory"}
                continue
            c0 = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            c1 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
            F.compact_seed_fill(k, r, rule, 1, c0)
            F.compact_step(k, r, rule, alpha, c0, c1, 32, flags)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            F.compact_step(k, r, rule, alpha, c0, c1, steps, flags)
            e1.record(stream)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / steps
            row[f"k{k}"] = {"r": r, "us_per_step": sec * 1e6, "cells_per_s": 3 ** k / sec,
                            "state_GB": nbytes / 1e9,
                            "array_state_GB": (1 << (2 * k)) * (1 if rule == 0 else 4) / 1e9}
            del c0, c1
            torch.cuda.empty_cache()
        out[name] = row
    return out


def nbb_leg(F, torch, reps=5):
    """The general NBB family: Sierpinski carpet (8, 3) at level 9 and Vicsek
    (5, 3) at level 9 (19683 x 19683), tests SW, RD and CA (one step) through
    lambda and the bounding box at tile sides 3..81; seconds per call and
    lambda's speedup at each map's best tile side."""
    import numpy as np
    stream = torch.cuda.current_stream()
    out = {}
    for name, which in (("carpet", F.NBB_CARPET), ("vicsek", F.NBB_VICSEK)):
        f = F.nbb_builtin(which)
        level = 9
        n = f.s ** level
        buf = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
        b1 = torch.zeros_like(buf)
        F.nbb_single_write(f, F.MAP_LAMBDA, level, 2, 1, buf)
        res = {"sw": {}, "rd": {}, "ca": {}}
        for r in range(1, 5):
            work = torch.empty(max(8, F.nbb_reduce_workspace(f, level, r)), dtype=torch.uint8,
                               device="cuda")
            val = torch.zeros(1, dtype=torch.int64, device="cuda")
            for map_ in (F.MAP_LAMBDA, F.MAP_BB):
                for op in ("sw", "rd", "ca"):
                    def call():
                        if op == "sw":
                            F.nbb_single_write(f, map_, level, r, 1, buf)
                        elif op == "rd":
                            F.nbb_reduce(f, map_, level, r, buf, work, val)
                        else:
                            F.nbb_ca_step(f, map_, level, r, buf, b1, 1)
                    call()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        call()
                    e1.record(stream)
                    torch.cuda.synchronize()
                    res[op][(r, map_)] = e0.elapsed_time(e1) * 1e-3 / reps
            del work, val
        row = {"k": f.k, "s": f.s, "level": level, "members": f.k ** level}
        for op, d in res.items():
            lam = {r: t for (r, m), t in d.items() if m == F.MAP_LAMBDA}
            bb = {r: t for (r, m), t in d.items() if m == F.MAP_BB}
            rl, rbb = min(lam, key=lam.get), min(bb, key=bb.get)
            row[op] = {"lambda_tile": f.s ** rl, "lambda_us": lam[rl] * 1e6,
                       "bb_tile": f.s ** rbb, "bb_us": bb[rbb] * 1e6,
                       "speedup_best": bb[rbb] / lam[rl],
                       "speedup_by_tile": {str(f.s ** r): bb[r] / lam[r] for r in lam}}
        out[name] = row
        del buf, b1
        torch.cuda.empty_cache()
    return out


def copy_ceiling(torch, nbytes=1 << 32, reps=5):
    """Device-to-device copy rate (read + write bytes per second): the
    practical ceiling for a one-step stencil, which moves copy-like traffic."""
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / sec / 1e9


def sweep_k_leg(F, torch, levels=(10, 12, 14, 16)):
    """lambda vs bounding box per level (Theorem 2: the margin grows with n),
    each at its best launch: lambda at the library's default launch for the
    level (--autotune: the autotuner's pick), the bounding box over tile
    sizes 16..128 (launch order, whole segments, fused steps where allowed).
    Seconds per step over runs of 64 (level >= 15) or 256 steps.  Level 10
    also gives the small configuration as stated (16 x 16 tiles for both
    maps, 100 automaton steps): microseconds per step."""
    out = {}
    for k in levels:
        g = Gasket(F, torch, k)
        g.autotune()
        steps = 64 if k >= 15 else 256
        row = {}
        for rule in (0, 1):
            g.run(rule, 16)
            lam = g.time(rule, steps)
            bbs = {}
            for r in range(4, min(k, 7) + 1):
                if k - r > 15:
                    continue
                tb = bb_tuning(g, rule, r)
                g.run(rule, 16, F.MAP_BB, tb)
                bbs[r] = g.time(rule, steps, F.MAP_BB, tb)
            best = min(bbs, key=bbs.get)
            row[RULE_NAME[rule]] = {"lambda_us": lam * 1e6, "lambda_tuning": list(g.tunings[rule]),
                                    "bb_us": bbs[best] * 1e6, "bb_r": best,
                                    "speedup": bbs[best] / lam,
                                    "bb_us_by_r": {str(r): v * 1e6 for r, v in bbs.items()}}
        if k == 10:
            # 16 x 16 tiles, 100 automaton steps, lambda vs BB at that tile
            lam_t = F.get_tuning(k, 0)
            tl = (4, lam_t[1], lam_t[2], lam_t[3]) if lam_t[0] == 4 else \
                (4, 256, F.ORDER_NATURAL, F.FLAG_MARCH | F.FLAG_SEGMENTS | F.FLAG_FUSE16)
            tb = bb_tuning(g, 0, 4, tl)
            res = {}
            for name, m, t in (("lambda", F.MAP_LAMBDA, tl), ("bb", F.MAP_BB, tb)):
                g.reseed(0)
                g.run(0, 16, m, t)
                g.reseed(0)
                res[name] = g.time(0, 100, m, t)
            row["ca_r4_100_steps"] = {"lambda_us_per_step": res["lambda"] * 1e6,
                                      "bb_us_per_step": res["bb"] * 1e6,
                                      "speedup": res["bb"] / res["lambda"],
                                      "lambda_tuning": list(tl), "bb_tuning": list(tb)}
        out[str(k)] = row
        g.free()
    return out


def mfma_leg(g, steps):
    """lambda computed by two ballots vs by the matrix-core product
    (Variant 1), same tile launch (the LDS engine: the matrix-core map has no
    march form), same level."""
    F = g.F
    out = {}
    for rule in (0, 1):
        t = g.tunings[rule]
        if t[3] & (F.FLAG_MARCH | F.FLAG_BLOCK):
            t = (t[0], 256 if t[0] >= 3 else 64, t[2], 11 if rule == 0 else 17)
        g.run(rule, 8, F.MAP_MFMA, t)
        mf = g.time(rule, steps, F.MAP_MFMA, t)
        g.run(rule, 8, F.MAP_LAMBDA, t)
        lb = g.time(rule, steps, F.MAP_LAMBDA, t)
        out[RULE_NAME[rule]] = {"ballot_us_per_step": lb * 1e6, "mfma_us_per_step": mf * 1e6,
                                "mfma_speedup": lb / mf}
    return out


def level_leg(F, torch, k, steps, label):
    """Per-rule rates and launch rooflines at level k with the default
    launches, plus the bounding box at lambda's tile size and at rho = 32
    (the paper's best BB block)."""
    g = Gasket(F, torch, k)
    g.autotune()
    out = {"k": k, "cells": g.cells, "steps": steps, "note": label}
    for rule in (0, 1):
        g.run(rule, 16)
        sec = g.time(rule, steps)
        rf = roofline(rule, g.cells, launch_stats(g, rule), g.tunings[rule],
                      read_traffic(f"k{k}", RULE_NAME[rule]), kernel_name(g.tunings[rule], rule))
        out[RULE_NAME[rule]] = {"tuning": list(g.tunings[rule]), "lambda_us": sec * 1e6,
                                "cells_per_s": g.cells / sec, "roofline": rf}
    for rule in (0, 1):
        r = g.tunings[rule][0]
        for rr in sorted({r, 5}):
            tb = bb_tuning(g, rule, rr)
            g.run(rule, 16, F.MAP_BB, tb)
            sec = g.time(rule, max(16, steps // 2), F.MAP_BB, tb)
            out[RULE_NAME[rule]][f"bb_r{rr}_us"] = sec * 1e6
    g.free()
    return out


def batch_leg(F, torch, count=256, steps=500, seed=2004):
    import fractal_inputs as fi
    pairs = fi.batch_instances(count, seed, 8, 14)
    alpha = float(__import__("numpy").float32(ALPHA))
    bufs = []
    for j, (k, rule) in enumerate(pairs):
        dt = torch.uint8 if rule == 0 else torch.float32
        n = 1 << k
        b0 = torch.empty((n, n), dtype=dt, device="cuda")
        b1 = torch.zeros((n, n), dtype=dt, device="cuda")
        bufs.append((k, rule, b0, b1))

    def reseed():
        for j, (k, rule, b0, b1) in enumerate(bufs):
            F.seed_fill(k, rule, 7000 + j, b0)
            b1.zero_()
        torch.cuda.synchronize()

    cells = sum(3 ** k for (k, _, _, _) in bufs) * steps
    stream = torch.cuda.current_stream()
    inst = [(k, rule, steps, alpha, b0, b1) for (k, rule, b0, b1) in bufs]

    def sums():
        return [int((b0 if steps % 2 == 0 else b1).view(torch.uint8).to(torch.int64).sum())
                for (k, rule, b0, b1) in bufs]

    def timed(fn):
        reseed()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3, time.perf_counter() - t0, sums()

    # warm the graph path once on a short run
    reseed()
    F.batch_step([(k, rule, 2, alpha, b0, b1) for (k, rule, b0, b1) in bufs])
    modes = {"per_tile": None, "persistent": (F.R_AUTO, 64, 2, F.FLAG_PERSISTENT)}
    res = {}
    for name, tun in modes.items():
        res[name] = timed(lambda: F.batch_step(inst, tuning=tun))

    def plain():
        for (k, rule, b0, b1) in bufs:
            F.lambda_step(k, F.R_AUTO, rule, alpha, b0, b1, steps)

    tp, wall_plain, sums_plain = timed(plain)
    out = {"instances": count, "steps": steps, "cell_updates": cells,
           "state_GB": sum(2 * (1 << (2 * k)) * (1 if r == 0 else 4) for (k, r, _, _) in bufs) / 1e9,
           "plain_s": tp, "plain_wall_s": wall_plain, "plain_cells_per_s": cells / tp}
    for name, (tb, wall, sm) in res.items():
        out[name] = {"s": tb, "wall_s": wall, "cells_per_s": cells / tb,
                     "speedup_vs_plain": tp / tb, "same_result": sm == sums_plain}
    del bufs
    torch.cuda.empty_cache()
    return out


def serve_leg(F, torch, seconds, rate=200.0, seed=2004, arena_gb=200.0):
    """Continuous batching: `seconds` of open-loop Poisson arrivals at `rate`
    req/s (levels 9..15, steps 10..1000, rule 50/50) through the server --
    latency = done minus scheduled arrival, p50/p99 --; the same requests
    submitted at once (saturated server: cells/s over the drain time); and
    the same requests solved one at a time with plain lambda_step calls."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    nreq = int(rate * seconds)
    gaps = rng.exponential(1.0 / rate, size=nreq)
    arrivals = np.cumsum(gaps)
    ks = rng.integers(9, 16, size=nreq)
    steps = rng.integers(10, 1001, size=nreq)
    rules = rng.integers(0, 2, size=nreq)
    nbytes = int(arena_gb * 1e9) // 256 * 256
    arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    cells = int(sum(3 ** int(k) * int(s) for k, s in zip(ks, steps)))
    alpha = float(np.float32(ALPHA))

    def run(paced):
        tickets = []
        with F.Server(arena, nbytes, max_slots=256, steps_per_iter=32) as srv:
            t0 = F.now()
            for i in range(nreq):
                target = t0 + (float(arrivals[i]) if paced else 0.0)
                while paced and F.now() < target:
                    time.sleep(min(0.0005, max(0.0, target - F.now())))
                tickets.append(srv.submit(int(ks[i]), int(rules[i]), int(steps[i]), alpha,
                                          seed=10000 + i, t_arrival=target))
            res = {}
            while len(res) < nreq:
                for t in tickets:
                    if t not in res:
                        r = srv.poll(t)
                        if r is not None:
                            res[t] = r
                time.sleep(0.002)
            t_end = F.now()
        lat = np.array([res[t][3] - res[t][1] for t in tickets])
        sums = [res[t][4] for t in tickets]
        return t_end - t0, lat, all(res[t][0] == 0 for t in tickets), sums

    drain, lat, ok, sums_paced = run(True)
    out = {"requests": nreq, "rate": rate, "arrival_s": float(arrivals[-1]),
           "drain_s": drain, "cell_updates": cells,
           "cells_per_s": cells / drain, "p50_s": float(np.percentile(lat, 50)),
           "p99_s": float(np.percentile(lat, 99)), "all_ok": ok}
    burst, _, ok_b, sums_burst = run(False)
    out.update({"saturated_drain_s": burst, "saturated_cells_per_s": cells / burst,
                "saturated_all_ok": ok_b, "same_results_paced_and_saturated": sums_paced == sums_burst})
    # the same trace solved one request at a time with plain launches
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e0.record(stream)
    for i in range(nreq):
        k, rule = int(ks[i]), int(rules[i])
        n = 1 << k
        one = n * n * (1 if rule == 0 else 4)
        b0 = arena[: one]
        b1 = arena[one: 2 * one]
        F.seed_fill(k, rule, 10000 + i, b0)
        b1.zero_()
        F.lambda_step(k, F.R_AUTO, rule, alpha, b0, b1, int(steps[i]))
    e1.record(stream)
    torch.cuda.synchronize()
    seq = e0.elapsed_time(e1) * 1e-3
    out.update({"sequential_s": seq, "sequential_wall_s": time.perf_counter() - t1,
                "sequential_cells_per_s": cells / seq,
                "saturated_vs_sequential": seq / burst})
    del arena
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_one_thread(k=12, steps=20):
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1;
    it touches no GPU): level-12 automaton steps over the whole array."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import fractal_inputs as fi, oracle; "
            "s = fi.full_state(%d, 0, 1); t = time.perf_counter(); oracle.ca_run(%d, s, %d); "
            "print(time.perf_counter() - t, oracle.threads())" % (ROOT, k, k, steps))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                             text=True, timeout=300, check=True).stdout.split()
        sec, thr = float(out[0]), int(out[1])
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None
    return {"value": 3 ** k * steps / sec, "unit": "cells/s", "threads": thr,
            "sample": f"level-{k} gasket, whole array: {steps} automaton steps ({sec:.1f} s)"}


def progress(msg: str) -> None:
    """One line per finished leg on stderr (stdout carries only the JSON)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_leg(k, alpha, bands=4, h=512, ca_steps=64, heat_steps=32, seed=2004):
    """The oracle on a bounded sample of the level-k workload: full-width
    bands of h rows at seeded offsets, ca_steps automaton steps and
    heat_steps float64 heat steps on each (the same seeded initial state as
    the GPU run); cell-updates counted over the members of each band's exact
    interior (rows farther than the step count from a cut edge)."""
    import numpy as np

    import fractal_inputs as fi
    import oracle
    n = 1 << k
    rng = np.random.Generator(np.random.PCG64(seed))
    offs = sorted(int(v) for v in rng.integers(h, n - 2 * h, size=bands))
    upd = 0
    sec = 0.0
    for y0 in offs:
        for rule, steps in ((0, ca_steps), (1, heat_steps)):
            st = fi.window_values(k, rule, 1, 0, y0, n, h)
            if rule == 1:
                st = st.astype(np.float64)
            t0 = time.perf_counter()
            if rule == 0:
                oracle.ca_run(k, st, steps, 0, y0)
            else:
                oracle.heat_run(k, st, alpha, steps, 0, y0)
            sec += time.perf_counter() - t0
            rs, cs = oracle.valid_interior(k, 0, y0, n, h, steps)
            upd += int(fi.member_mask(k, 0, y0 + rs.start, n, rs.stop - rs.start).sum()) * steps
    return {"value": upd / sec, "unit": "cells/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"level-{k} gasket: {bands} full-width bands of {h} rows at seeded "
                      f"offsets {offs}, {ca_steps} automaton steps and {heat_steps} float64 "
                      f"heat steps each; {upd} member cell-updates of the exact band "
                      f"interiors in {sec:.1f} s",
            "cpu_model": cpu_model(), "one_thread": oracle_one_thread()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="k16", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-bb", action="store_true",
                    help="skip the bounding-box, matrix-core, SW/RD and NBB legs")
    ap.add_argument("--no-k14", action="store_true", help="skip the level-14 leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-gasket batch leg")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip lambda vs bounding box at levels 10, 12, 14, 16")
    ap.add_argument("--no-compact", action="store_true", help="skip the compact-storage leg")
    ap.add_argument("--serve", type=float, default=60.0,
                    help="seconds of Poisson arrivals for the serving leg (0 = skip)")
    ap.add_argument("--autotune", action="store_true",
                    help="time every launch candidate first instead of the library defaults")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 4 GiB with a plain device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        return 2

    import torch

    import paper_2004_13475_amd as F

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 32, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    global AUTOTUNE
    AUTOTUNE = args.autotune
    K, W = args.steps, args.warmup
    g = Gasket(F, torch, WORKLOADS[args.workload])
    g.autotune()
    g.run(0, W)
    g.run(1, W)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t0 = time.perf_counter()
    ev[0].record(g.stream)
    g.run(0, K)
    ev[1].record(g.stream)
    g.run(1, K)
    ev[2].record(g.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_ca, ms_heat = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    total_ms = ms_ca + ms_heat
    value = 2.0 * g.cells * K / (total_ms / 1e3)
    per_step = {0: ms_ca / K * 1e-3, 1: ms_heat / K * 1e-3}  # seconds per step
    progress(f"timed {K} steps of each rule at level {g.k}: {total_ms:.2f} ms")
    stats = {r: launch_stats(g, r) for r in (0, 1)}
    # the dominant kernel: the rule whose launches take the larger share of
    # the timed region
    dom = 1 if per_step[1] >= per_step[0] else 0
    rfs = {r: roofline(r, g.cells, stats[r], g.tunings[r],
                       read_traffic(args.workload, RULE_NAME[r]), kernel_name(g.tunings[r], r))
           for r in (0, 1)}
    rf = dict(rfs[dom], rule=RULE_NAME[dom])

    bb = None if args.no_bb else bb_leg(g, per_step, max(16, min(K, 64)))
    mfma = None if args.no_bb else mfma_leg(g, 32)
    k, cells, tunings = g.k, g.cells, dict(g.tunings)
    g.free()
    progress("bounding box and matrix-core legs done")
    k14 = None if (args.no_k14 or k == 14) else level_leg(
        F, torch, 14, 256, "cache-assisted: the level-14 member segments (23-161 MB per step) "
        "fit the 256 MB last-level cache")
    sweep = None if args.no_sweep else sweep_k_leg(F, torch)
    progress("level-14 and per-level sweep legs done")
    batch = None if args.no_batch else batch_leg(F, torch)
    progress("batch leg done")
    serve = serve_leg(F, torch, args.serve) if args.serve > 0 else None
    progress("serving leg done")
    swrd = None if args.no_bb else {f"k{kk}": sw_rd_leg(F, torch, kk) for kk in sorted({k, 16})}
    compact = None if args.no_compact else compact_leg(F, torch)
    nbb = None if args.no_bb else nbb_leg(F, torch)
    ceiling = None if args.no_bb else copy_ceiling(torch)
    progress("SW/RD, compact, NBB and copy legs done")

    cpu = None
    if not args.no_cpu:
        import numpy as np
        cpu = cpu_leg(k, float(np.float32(ALPHA)))
        progress("oracle leg done")

    line = {
        "metric": "fractal cells updated/s and HBM GB/s (% peak), lambda vs BB; "
                  "served p50/p99 latency",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": total_ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8+f32", "data": "synthetic",
        "config": {"workload": f"sierpinski-k{k}-lambda-ca-u8+heat-f32", "k": k,
                   "n": 1 << k, "cells": cells, "tuning_ca": list(tunings[0]),
                   "tuning_heat": list(tunings[1]), "wall_s": wall},
        "roofline": rf,
        "per_rule": {RULE_NAME[r]: {"us_per_step": per_step[r] * 1e6,
                                    "cells_per_s": cells / per_step[r],
                                    "steps_per_launch": steps_per_launch(tunings[r]),
                                    "roofline": rfs[r]}
                     for r in (0, 1)},
        "bb": bb, "mfma_lambda": mfma, "k14": k14, "lambda_vs_bb_by_k": sweep,
        "batch": batch, "serve": serve, "sw_rd": swrd, "compact": compact, "nbb": nbb,
        "device_copy_GBs": ceiling,
        "cpu_baseline": cpu,
        "kernel_source_hash": kernel_hash(),
    }
    print(json.dumps(line, default=lambda o: None if isinstance(o, float) and math.isnan(o) else o))
    return 0


if __name__ == "__main__":
    sys.exit(main())
