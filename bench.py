#!/usr/bin/env python3
"""Throughput benchmark of the Sutton-Chen cluster-MD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-forms]

One step is a whole velocity-Verlet step of every cluster of the workload
(drift, density sweep, density reduce, force sweep, force reduce + kick,
thermostat), replayed from captured HIP graphs, with the inputs resident in
HBM before the timed region starts.  The default workload is a 2243-atom
spherical fcc Ni cut (R = 18 A), +-0.05 A jitter, Maxwell-Boltzmann start at
2000 K, Berendsen cooling 2000 -> 800 K over 200k steps of 2 fs, all pairs,
FP64.  Prints one JSON line:

  value        whole-job atom-steps/s over exactly K timed steps
  roofline     the force sweep (dominant kernel; on the cell list the longer
               of the two sweeps): algorithmic FLOP per launch
               (30 FLOP per unordered pair: a step without the pair-energy
               term, like all but the last step of each 32-step graph) / its
               device time per launch,
               measured with HIP events inside the timed region, against the
               FP64 vector peak of MI355X (78.6 TFLOP/s)
  cpu_baseline the FP64 oracle on the host cores on a bounded sample of the
               same workload
  forms        the other forms measured briefly (mixed precision, batched,
               large all-pairs, cell list) with their own rooflines
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "atom-steps/s and pair-interactions/s, Ni SC MD at 1 GPU: FP64 vs mixed vs batched"
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector (256 CU x 2.4 GHz x 128 FLOP/clk/CU)
FLOP_DENSITY_PER_PAIR = 13.0  # algorithmic FLOP per unordered pair, density sweep
# algorithmic FLOP per unordered pair of the timed force sweep: 31 with the
# pair-energy term, 30 without it; the library accumulates the pair energy
# only on the last step of each run (32-step graph replays, sampled steps),
# and the sampled launch is a step without it
FLOP_FORCE_PER_PAIR = 30.0


def measured_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/traffic.json), or None when the kernel sources changed
    since the counters were taken or the workload was not measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("sha256"):
        return None
    return rec.get("dominant_bytes_per_launch", {}).get(workload)


def _pairs(sizes) -> int:
    s = np.asarray(sizes, dtype=np.int64)
    return int(np.sum(s * (s - 1) // 2))


def _workload(name: str):
    from paper_1210_3559_amd import inputs
    try:
        return inputs.by_name(name)
    except KeyError as exc:
        raise SystemExit(str(exc))


def time_gpu(w, steps: int, warmup: int, tuning=None):
    """Warm up, then time exactly `steps` steps; returns a result dict."""
    import torch

    from paper_1210_3559_amd import scmd
    sim = scmd.Simulation.from_workload(w, tuning=tuning)
    try:
        sim.step(warmup)
        scmd.scmd_set_profiling(sim.ctx, True)
        # the timed steps go in chunks so that the sampled kernel times (one
        # sample per graph replay, kept per call) cover the whole region
        # whole 32-step graphs per chunk where possible (the remainder of a
        # chunk runs eagerly), the rest of the steps in the last chunk
        chunks = max(1, min(25, steps // 256))
        per = (steps // chunks) // 32 * 32 or steps // chunks
        sizes = [per] * (chunks - 1) + [steps - per * (chunks - 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in sizes:
            sim.step(n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        f_ms, f_n = scmd.scmd_get_kernel_time(sim.ctx, scmd.SCMD_KERNEL_FORCE)
        d_ms, d_n = scmd.scmd_get_kernel_time(sim.ctx, scmd.SCMD_KERNEL_DENSITY)
        scmd.scmd_set_profiling(sim.ctx, False)
        e = sim.energy()
        # with a cutoff the algorithmic pairs are those closer than rc: one
        # histogram bin of width rc counts them (ordered) at the final positions
        pairs_rc = None
        if w.rc > 0:
            pairs_rc = sum(int(sim.rdf(k, w.rc, 1)[0][0]) for k in range(sim.nclusters)) // 2
        T = [sim.temperature(k)[0] for k in range(min(sim.nclusters, 1))]
    finally:
        sim.close()
    sizes = w.sizes()
    natoms = int(sizes.sum())
    pairs = _pairs(sizes)
    cut = w.rc > 0
    res = {
        "workload": w.name,
        "precision": w.precision,
        "n_atoms": natoms,
        "n_clusters": int(len(sizes)),
        "steps": steps,
        "seconds": dt,
        "ms_per_step": 1e3 * dt / steps,
        "atom_steps_per_s": natoms * steps / dt,
        "force_ms_per_launch": f_ms,
        "force_launches_timed": f_n,
        "density_ms_per_launch": d_ms,
        "density_launches_timed": d_n,
        "final_energy_eV": e[2],
        "final_T_K": T[0] if T else None,
    }
    if cut:
        pairs = pairs_rc
        res["pairs_within_rc"] = pairs_rc
    res["pair_interactions_per_s"] = pairs * steps / dt
    res["pairs_per_step"] = pairs
    # the roofline is that of the longer sweep (the force sweep, except on
    # the cell list, where the density sweep also finds the pairs within rc);
    # the other sweep's figures go beside it
    sweeps = []
    if f_ms > 0:
        sweeps.append(("force sweep", f_ms, FLOP_FORCE_PER_PAIR * pairs / (f_ms * 1e-3) / 1e12))
    if d_ms > 0:
        sweeps.append(("density sweep", d_ms, FLOP_DENSITY_PER_PAIR * pairs / (d_ms * 1e-3) / 1e12))
    sweeps.sort(key=lambda x: -x[1])
    if sweeps:
        name, _, ach = sweeps[0]
        res["roofline"] = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                           "frac": ach / PEAK_FP64_TFLOPS, "traffic": None, "kernel": name}
    if len(sweeps) > 1:
        name, _, ach = sweeps[1]
        res["other_sweep_roofline"] = {"kernel": name, "achieved": ach, "frac": ach / PEAK_FP64_TFLOPS}
    return res


def cpu_baseline(w, budget_s: float):
    """Time the FP64 oracle on the host cores on a bounded sample of the workload."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    th = w.thermostat[0]
    pos, vel = w.pos, w.vel
    # one untimed step builds the initial forces
    r, v, f, _ = oracle.vv_run(pos, vel, 1, dt=w.dt, thermostat=th, nthreads=threads, with_log=False)
    steps, t_used = 0, 0.0
    while t_used < budget_s:
        t0 = time.perf_counter()
        r, v, f, _ = oracle.vv_run(r, v, 1, dt=w.dt, thermostat=th, force=f, step0=1 + steps, nthreads=threads,
                                   with_log=False)
        t_used += time.perf_counter() - t0
        steps += 1
    n = len(pos)
    # single core, as the paper compares against one CPU core
    t0 = time.perf_counter()
    oracle.vv_run(r, v, 1, dt=w.dt, thermostat=th, force=f, nthreads=1, with_log=False)
    t1 = time.perf_counter() - t0
    return {
        "value": n * steps / t_used,
        "unit": "atom-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps} velocity-Verlet steps of the {w.name} workload ({n} atoms) after one untimed step",
        "single_core_atom_steps_per_s": n / t1,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="ni2243_cooling")
    ap.add_argument("--no-forms", action="store_true", help="skip the extra forms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--tuning", default=None,
                    help="JSON launch-shape override for the main workload, e.g. '{\"pairs\": 2, \"ipt\": 8}'")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device once (a plain copy kernel of known "
                         "size, to scale hardware byte counters when profiling)")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library runs every cluster on a single MI355X; "
              "multi-GPU sharding is a design note, not a code path", file=sys.stderr)
        return 2

    w = _workload(args.workload)
    print(f"[bench] {w.name}: {w.n_atoms} atoms, {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    main_res = time_gpu(w, args.steps, args.warmup, tuning=json.loads(args.tuning) if args.tuning else None)
    # the committed counters are those of force-sweep kernels
    if main_res.get("roofline") is not None and main_res["roofline"]["kernel"] == "force sweep":
        main_res["roofline"]["traffic"] = measured_traffic(args.workload)
    print(f"[bench] {main_res['atom_steps_per_s']:.4e} atom-steps/s, {main_res['ms_per_step']:.4f} ms/step",
          file=sys.stderr, flush=True)

    if args.copy_mib > 0:
        import torch
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copied {args.copy_mib} MiB ({n * 8} bytes) device to device", file=sys.stderr, flush=True)
        del src, dst

    forms = {}
    if not args.no_forms:
        plan = [("fp64_ni2243", None, None), ("mixed_ni2243", "ni2243_cooling", "mixed"),
                ("allpairs_fp64_ni48077", "ni48077_allpairs", None), ("allpairs_fp64_ni50000", "ni50000_allpairs", None),
                ("mixed_ni15000", "ni15000_mixed", None), ("fp64_ni15000", "ni15000_fp64", None),
                ("batched_fp64_256", "batch256", None), ("batched_mixed_256", "batch256_mixed", None),
                ("cell_fp64_ni48077", "ni48077_cell", None),
                ("langevin_fp64_ni2243", "ni2243_langevin", None), ("langevin_batched_fp64_256", "batch256_langevin", None)]
        for key, name, prec in plan:
            if name is None:
                forms[key] = {k: main_res[k] for k in ("atom_steps_per_s", "pair_interactions_per_s", "ms_per_step")}
                continue
            try:
                fw = _workload(name)
                if prec:
                    fw.precision = prec
                n = fw.n_atoms
                steps = max(20, min(2000, int(2e10 / max(1, _pairs(fw.sizes())))))
                print(f"[bench] form {key}: {n} atoms, {steps} steps", file=sys.stderr, flush=True)
                r = time_gpu(fw, steps, min(20, steps))
                forms[key] = {k: r[k] for k in ("atom_steps_per_s", "pair_interactions_per_s", "ms_per_step",
                                                "force_ms_per_launch", "density_ms_per_launch", "roofline",
                                                "steps", "n_atoms", "n_clusters", "pairs_within_rc") if k in r}
            except Exception as exc:  # a form that is not available is reported, not fatal
                forms[key] = {"error": str(exc)}

    cpu = None
    if not args.no_cpu:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, args.cpu_budget)

    out = {
        "metric": METRIC,
        "value": main_res["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_atoms": w.n_atoms, "n_clusters": w.n_clusters, "dt_fs": w.dt,
                   "neighbour": "cell" if w.rc > 0 else "allpairs", "precision": w.precision,
                   "pairs_per_step": main_res.get("pairs_per_step"), "parallelism": "single_gpu"},
        "pair_interactions_per_s": main_res.get("pair_interactions_per_s"),
        "roofline": main_res.get("roofline"),
        "kernel_timing": {k: main_res.get(k) for k in ("force_ms_per_launch", "force_launches_timed",
                                                       "density_ms_per_launch")},
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
