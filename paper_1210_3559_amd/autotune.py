"""Launch-shape autotuner for the all-pairs sweeps and the cell list.

For an all-pairs workload it times every supported (ipt, waves_i, waves_j)
shape and a few work-splitting targets with whole velocity-Verlet steps
replayed from HIP graphs, and keeps the fastest; for a cell-list workload it
times the list skin (``cell_skin``: a longer list against fewer rebuilds).
Results are cached as JSON keyed by (device architecture, precision,
cluster-size bucket, cluster count bucket, and "cell" for the cell list), so
``Simulation(..., tuning="auto")`` can pick them up later.

    python -m paper_1210_3559_amd.autotune --workloads ni2243_cooling,batch256 [--cache PATH]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import scmd

SHAPES = [(1, 4, 1), (2, 4, 1), (1, 2, 2), (2, 2, 2), (1, 1, 4), (2, 1, 4), (1, 2, 4), (2, 2, 4), (1, 4, 4),
          (1, 1, 8), (2, 1, 8), (1, 2, 8), (1, 1, 16), (4, 1, 2), (4, 1, 4), (4, 2, 2)]
TARGETS = [1, 512, 2048, 8192]
ROW_WAVES = [4, 8, 16]
ROW_TARGETS = [256, 512, 1024]  # workgroups per row sweep
CELL_SKINS = [0.2, 0.3, 0.4, 0.5, 0.6]  # A; rebuilds every step at 0, LDS stage overflow from ~0.8
# measured on MI355X by `python -m paper_1210_3559_amd.autotune` and committed with the package
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")
ARCH = "gfx950"


def bucket(offsets, precision: str, cell: bool = False) -> str:
    sizes = np.diff(np.asarray(offsets))
    nmax = int(sizes.max()) if len(sizes) else 0
    key = f"{ARCH}/{precision}/nmax2^{max(0, math.ceil(math.log2(max(nmax, 1))))}/nc2^{math.ceil(math.log2(max(len(sizes), 1)))}"
    return key + "/cell" if cell else key


def _time(sim: "scmd.Simulation", steps: int) -> float:
    t0 = time.perf_counter()
    sim.step(steps)
    return (time.perf_counter() - t0) / steps


def tune(w, precision: str | None = None, budget_s: float = 0.25, shapes=SHAPES, targets=TARGETS, verbose=True,
         symmetric: bool = True, row: bool = True):
    """Time every shape/target (cell list: every skin) on workload w; returns
    (best tuning dict, table)."""
    precision = precision or w.precision
    pairs = float(np.sum(w.sizes().astype(np.float64) ** 2))
    table = []
    if w.rc > 0:
        tunings = [dict(cell_skin=s) for s in CELL_SKINS]
    else:
        tunings = [dict(cand, target_items=tgt) for cand, tgts in candidate_plans(w.sizes(), shapes, targets,
                                                                                  symmetric, row) for tgt in tgts]
    for tun in tunings:
        with scmd.Simulation.from_workload(w, precision=precision, tuning=tun) as sim:
            sim.step(32)
            dt1 = _time(sim, 32)
            steps = int(max(32, min(4096, budget_s / max(dt1, 1e-7))))
            steps = 32 * max(1, steps // 32)
            dt = _time(sim, steps)
        table.append(dict(tuning=tun, ms_per_step=1e3 * dt))
        if verbose:
            rate = (f"{w.n_atoms / dt:.4g} atom-steps/s" if w.rc > 0 else
                    f"{pairs / dt / 1e9:.1f} G ordered pairs/s")
            print(f"[tune] {w.name} {precision} {tun} {1e3 * dt:.4f} ms/step ({rate})", file=sys.stderr, flush=True)
    best = min(table, key=lambda r: r["ms_per_step"])
    return best["tuning"], table


def candidate_plans(sizes, shapes=SHAPES, targets=TARGETS, symmetric: bool = True, row: bool = True):
    """(tuning, work-splitting targets) pairs worth timing for clusters of
    these sizes: row sweeps only where every cluster fits the LDS staging
    (<= 4096 atoms) and the batch is small, one-sided shapes only for
    clusters up to 16k atoms (beyond, they evaluate every pair twice and lose
    to the symmetric sweeps by about 2x), symmetric sweeps always, with item
    targets up to 16384 for large pair counts."""
    sizes = np.asarray(sizes, dtype=np.int64)
    nmax = int(sizes.max()) if len(sizes) else 0
    pairs = float(np.sum(sizes.astype(np.float64) * (sizes - 1) / 2.0))
    out = []
    if nmax <= 16384:
        out += [(dict(ipt=ipt, waves_i=wi, waves_j=wj, pairs=1), targets) for ipt, wi, wj in shapes]
    if symmetric:
        sym_targets = sorted(set(list(targets) + ([4096, 16384] if pairs > 1e8 else [])))
        out += [(dict(ipt=ipt, pairs=2), sym_targets) for ipt in (2, 4, 8)]
    if row and nmax <= 4096 and pairs <= 1e8:
        out += [(dict(waves_j=wv, pairs=3), ROW_TARGETS) for wv in ROW_WAVES]
    return out


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(offsets, precision: str, path: str = DEFAULT_CACHE, cell: bool = False):
    """Cached tuning for this cluster layout (cell: the cell-list variant), or None."""
    entry = load_cache(path).get(bucket(offsets, precision, cell))
    return None if entry is None else dict(entry["tuning"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="ni2243_cooling")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--budget", type=float, default=0.25, help="seconds per timed configuration")
    ap.add_argument("--report", default=None, help="write the full timing table (JSON) here")
    args = ap.parse_args(argv)
    from . import inputs
    cache = load_cache(args.cache)
    report = {}
    for name in args.workloads.split(","):
        w = inputs.by_name(name)
        prec = args.precision or w.precision
        best, table = tune(w, prec, args.budget)
        key = bucket(w.offsets, prec, w.rc > 0)
        cache[key] = dict(tuning=best, ms_per_step=min(r["ms_per_step"] for r in table), workload=w.name)
        report[w.name] = dict(key=key, best=best, table=table)
        print(json.dumps(dict(workload=w.name, key=key, best=best, ms=cache[key]["ms_per_step"])), flush=True)
    with open(args.cache, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
