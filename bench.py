#!/usr/bin/env python3
"""Throughput benchmark of the Sutton-Chen cluster-MD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-forms]

One step is a whole velocity-Verlet step of every cluster of the workload
(drift, density sweep, density reduce, force sweep, force reduce + kick,
thermostat) with the inputs resident in HBM before the timed region starts.
The K timed steps are one library call, replayed from captured HIP graphs
(32-step graphs plus one graph of the remainder), exactly as a user's
scmd_step runs them, with profiling off.  The default workload is the largest single-GPU
all-pairs configuration: a 48,077-atom spherical fcc Ni cut (R = 50 A),
+-0.05 A jitter, Maxwell-Boltzmann start at 1900 K, Berendsen at 1900 K,
dt = 1 fs, all pairs, FP64.  Prints one JSON line:

  value        whole-job atom-steps/s over exactly K timed steps
  roofline     the dominant kernel (the force sweep; on the cell list the
               longer of the two sweeps): algorithmic FLOP per launch (30
               FLOP per unordered pair for a step without the pair-energy
               term, which is every step but the last of a run, and the
               sampled one) / its device time per launch, from HIP events
               recorded inside the replayed graphs on the context stream
               (one sampled step per replay) during a second timed call of
               K steps, against the FP64 vector peak of MI355X (78.6
               TFLOP/s)
  cpu_baseline the FP64 oracle on the host cores on a bounded sample of the
               same workload
  forms        the other forms measured briefly (mixed precision, batched,
               cell list, Langevin bath) with their own rooflines; mixed
               forms also report their force and energy error against the
               FP64 oracle at their final positions
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
# MI355X FP64 vector peak (256 CU x 2.4 GHz x 128 FLOP/clk/CU).  The mixed
# form's single-precision pair terms run as unpacked FP32 instructions (this
# build disables packed FP32), whose issue rate is the FP64 vector rate, so
# the same peak bounds both forms; the 157.3 TFLOP/s FP32 figure needs packed
# two-wide instructions.
PEAK_FP64_TFLOPS = 78.6
FLOP_DENSITY_PER_PAIR = 13.0  # algorithmic FLOP per unordered pair, density sweep
# algorithmic FLOP per unordered pair of the timed force sweep: 31 with the
# pair-energy term, 30 without it; the library accumulates the pair energy
# only on the last step of each run, and the sampled launch is a step without it
FLOP_FORCE_PER_PAIR = 30.0
MIN_KERNEL_SAMPLES = 8
ORACLE_FLAGS = "gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fno-fast-math (no host-specific ISA)"


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


def _kernel_times(sim, scmd):
    f_ms, f_n = scmd.scmd_get_kernel_time(sim.ctx, scmd.SCMD_KERNEL_FORCE)
    d_ms, d_n = scmd.scmd_get_kernel_time(sim.ctx, scmd.SCMD_KERNEL_DENSITY)
    return f_ms, f_n, d_ms, d_n


def time_gpu(w, steps: int, warmup: int, tuning=None, keep_state: bool = False):
    """Warm up, then time exactly `steps` steps in one library call; returns a
    result dict (and the final positions, forces and per-cluster potential
    energies under "state" when keep_state)."""
    import torch

    from paper_1210_3559_amd import scmd
    sim = scmd.Simulation.from_workload(w, tuning=tuning)
    try:
        # warm-up; a run of steps % 32 steps captures the graph of the
        # timed call's remainder, so the timed call only replays graphs
        sim.step(warmup)
        sim.step(steps % 32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # kernel times: the same call again with profiling events recorded
        # inside the replayed graphs (one sampled step per replay), timed on
        # its own so that the events' cost shows
        scmd.scmd_set_profiling(sim.ctx, True)
        sim.step(steps % 32)
        sim.step(32)
        scmd.scmd_set_profiling(sim.ctx, True)  # resets the averages, keeps the graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt_prof = time.perf_counter() - t0
        f_ms, f_n, d_ms, d_n = _kernel_times(sim, scmd)
        timed_samples = f_n
        if f_n < MIN_KERNEL_SAMPLES:
            # too few sampled launches in that call (one per graph replay):
            # add replays of the same graphs
            for _ in range(MIN_KERNEL_SAMPLES - f_n):
                sim.step(steps)
            f_ms, f_n, d_ms, d_n = _kernel_times(sim, scmd)
        scmd.scmd_set_profiling(sim.ctx, False)
        e = sim.energy()
        # with a cutoff the algorithmic pairs are those closer than rc: one
        # histogram bin of width rc counts them (ordered) at the final positions
        pairs_rc = None
        if w.rc > 0:
            pairs_rc = sum(int(sim.rdf(k, w.rc, 1)[0][0]) for k in range(sim.nclusters)) // 2
        T = sim.temperature(0)[0]
        state = None
        if keep_state:
            state = {"pos": sim.positions(), "forces": sim.forces(),
                     "epot": [sim.energy(k)[0] for k in range(sim.nclusters)]}
    finally:
        sim.close()
    sizes = w.sizes()
    natoms = int(sizes.sum())
    pairs = _pairs(sizes)
    res = {
        "workload": w.name,
        "precision": w.precision,
        "n_atoms": natoms,
        "n_clusters": int(len(sizes)),
        "steps": steps,
        "seconds": dt,
        "ms_per_step": 1e3 * dt / steps,
        "ms_per_step_with_profiling_events": 1e3 * dt_prof / steps,
        "atom_steps_per_s": natoms * steps / dt,
        "force_ms_per_launch": f_ms,
        "force_launches_sampled": f_n,
        "force_launches_sampled_in_profiled_call": timed_samples,
        "density_ms_per_launch": d_ms,
        "density_launches_sampled": d_n,
        "final_energy_eV": e[2],
        "final_T_K": T,
    }
    if w.rc > 0:
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
    if state is not None:
        res["state"] = state
    return res


def autotune_pick(w):
    """The autotuner's launch plan for this workload's cluster layout and
    precision (None when the table has no entry: library defaults)."""
    from paper_1210_3559_amd import autotune
    return autotune.lookup(w.offsets, w.precision, cell=w.rc > 0)


def mixed_error(w, state, nthreads: int, max_clusters: int = 4, sample: int = 64):
    """Force and energy error of a mixed-precision run against the FP64
    oracle at the run's final GPU positions: force relative norm error and
    worst per-atom error (|dF_i| / max(|F_i|, F_rms)) over a fixed sample of
    atoms, energy relative error of the cluster's potential energy.  Batches:
    the smallest, the largest and two middle clusters."""
    import oracle
    sizes = w.sizes()
    order = np.argsort(sizes, kind="stable")
    picks = sorted(set(int(order[int(q * (len(order) - 1))]) for q in np.linspace(0, 1, max_clusters)))
    out = {"clusters": [], "sample_atoms_per_cluster": sample}
    worst = [0.0, 0.0, 0.0]
    for k in picks:
        a, b = int(w.offsets[k]), int(w.offsets[k + 1])
        pos, f = state["pos"][a:b], state["forces"][a:b]
        idx = np.sort(np.random.default_rng(k).choice(b - a, min(sample, b - a), replace=False))
        f_ref, _ = oracle.forces_subset(pos, idx, nthreads=nthreads)
        frms = np.sqrt(np.mean(np.sum(f ** 2, axis=1)))
        fn = float(np.linalg.norm(f[idx] - f_ref) / np.linalg.norm(f_ref))
        fw = float(np.max(np.linalg.norm(f[idx] - f_ref, axis=1) /
                          np.maximum(np.linalg.norm(f_ref, axis=1), frms)))
        e_ref = oracle.energy(pos, nthreads=nthreads)
        ee = float(abs(state["epot"][k] - e_ref) / abs(e_ref))
        out["clusters"].append({"cluster": k, "atoms": b - a, "force_rel_norm": fn, "force_worst_atom": fw,
                                "energy_rel": ee})
        worst = [max(worst[0], fn), max(worst[1], fw), max(worst[2], ee)]
    out["force_rel_norm_max"], out["force_worst_atom_max"], out["energy_rel_max"] = worst
    return out


def cpu_baseline(w, budget_s: float):
    """Time the FP64 oracle on the host cores on a bounded sample of the
    workload: whole velocity-Verlet steps when one fits the budget, else one
    force evaluation (the pair work of a step; the step's O(N) kick and drift
    are negligible beside it), on all cores; then one core on the atoms
    nearest the centre of the largest cluster, converted through its
    pair-interaction rate (an all-pairs step costs the same per pair at any
    size)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    sizes = w.sizes()
    k = int(np.argmax(sizes))
    pos, vel = w.cluster(k)
    th = w.thermostat[k]
    n = len(pos)
    pairs_cluster = n * (n - 1) / 2
    t0 = time.perf_counter()
    f, _, _ = oracle.forces(pos, nthreads=threads)
    t_eval = time.perf_counter() - t0
    steps, t_steps = 0, 0.0
    if t_eval < budget_s / 3:
        r, v = pos, vel
        while t_steps < budget_s:
            t0 = time.perf_counter()
            r, v, f, _ = oracle.vv_run(r, v, 1, dt=w.dt, thermostat=th, force=f, step0=steps, nthreads=threads,
                                       with_log=False)
            t_steps += time.perf_counter() - t0
            steps += 1
        rate_pairs = pairs_cluster * steps / t_steps
        sample = (f"{steps} whole velocity-Verlet steps of cluster {k} ({n} atoms) of the {w.name} workload, "
                  f"{t_steps:.1f} s on {threads} threads")
    else:
        rate_pairs = pairs_cluster / t_eval
        sample = (f"one force evaluation (density and force sweeps: the pair work of one step) of cluster {k} "
                  f"({n} atoms) of the {w.name} workload, {t_eval:.1f} s on {threads} threads")
    # one core: the atoms nearest the cluster's centre, a compact sub-cluster
    # sized for a few seconds
    m = min(n, 4000)
    sub = pos[np.argsort(np.sum((pos - pos.mean(axis=0)) ** 2, axis=1), kind="stable")[:m]]
    t0 = time.perf_counter()
    oracle.forces(sub, nthreads=1)
    t1 = time.perf_counter() - t0
    rate1 = m * (m - 1) / 2 / t1
    # atom-steps/s of the whole workload at the measured pair rate
    total_pairs = _pairs(sizes)
    natoms = int(sizes.sum())
    return {
        "value": rate_pairs * natoms / total_pairs,
        "unit": "atom-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": sample + "; atom-steps/s of the whole workload = that pair rate x atoms / pairs per step",
        "pair_interactions_per_s": rate_pairs,
        "compiler": ORACLE_FLAGS,
        "single_core": {"atom_steps_per_s": rate1 * natoms / total_pairs, "pair_interactions_per_s": rate1,
                        "sample": f"one force evaluation of the {m} atoms nearest the centre of cluster {k}, "
                                  f"{t1:.2f} s on 1 thread"},
    }


FORMS = [("c2_fp64_ni2243", "ni2243_cooling", None), ("c2_mixed_ni2243", "ni2243_cooling", "mixed"),
         ("c3_allpairs_fp64_ni48077", "ni48077_allpairs", None), ("allpairs_fp64_ni50000", "ni50000_allpairs", None),
         ("c4_mixed_ni15000", "ni15000_mixed", None), ("c4_fp64_ni15000", "ni15000_fp64", None),
         ("c5_batched_fp64_256", "batch256", None), ("c5_batched_mixed_256", "batch256_mixed", None),
         ("c3_cell_fp64_ni48077", "ni48077_cell", None),
         ("langevin_fp64_ni2243", "ni2243_langevin", None), ("langevin_batched_fp64_256", "batch256_langevin", None)]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", default="ni48077_allpairs")
    ap.add_argument("--no-forms", action="store_true", help="skip the extra forms")
    ap.add_argument("--forms", default=None, help="comma-separated subset of the extra forms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-error", action="store_true", help="skip the mixed forms' oracle error")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
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

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    w = _workload(args.workload)
    print(f"[bench] {w.name}: {w.n_atoms} atoms, {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    tuning = json.loads(args.tuning) if args.tuning else None
    main_res = time_gpu(w, args.steps, args.warmup, tuning=tuning, keep_state=w.precision == "mixed")
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
        wanted = set(args.forms.split(",")) if args.forms else None
        for key, name, prec in FORMS:
            if wanted is not None and key not in wanted:
                continue
            if name == args.workload and prec is None:
                forms[key] = {k: main_res[k] for k in ("atom_steps_per_s", "pair_interactions_per_s", "ms_per_step")}
                forms[key]["headline"] = True
                continue
            try:
                fw = _workload(name)
                if prec:
                    fw.precision = prec
                steps = max(32, min(2000, int(2e10 / max(1, _pairs(fw.sizes())))))
                if fw.rc > 0:
                    steps = 640  # a cell list rebuilds every few steps: average over many
                print(f"[bench] form {key}: {fw.n_atoms} atoms, {steps} steps", file=sys.stderr, flush=True)
                # batches run the launch plan and the cell list the skin that
                # the autotuner measured for them (paper_1210_3559_amd/tuning_cache.json)
                tun = "auto" if fw.n_clusters > 1 or fw.rc > 0 else None
                r = time_gpu(fw, steps, min(64, steps), tuning=tun,
                             keep_state=fw.precision == "mixed" and not args.no_error)
                if tun:
                    r["tuning"] = autotune_pick(fw)
                forms[key] = {k: r[k] for k in ("atom_steps_per_s", "pair_interactions_per_s", "ms_per_step",
                                                "force_ms_per_launch", "density_ms_per_launch", "roofline",
                                                "steps", "n_atoms", "n_clusters", "pairs_within_rc", "tuning")
                              if k in r}
                if "state" in r:
                    print(f"[bench] form {key}: error against the FP64 oracle", file=sys.stderr, flush=True)
                    forms[key]["error_vs_fp64_oracle"] = mixed_error(fw, r["state"], threads)
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
        "kernel_timing": {k: main_res.get(k) for k in (
            "force_ms_per_launch", "force_launches_sampled", "force_launches_sampled_in_profiled_call",
            "density_ms_per_launch", "ms_per_step_with_profiling_events")},
        "cpu_baseline": cpu,
        "forms": forms,
    }
    if "state" in main_res and not args.no_error:
        out["error_vs_fp64_oracle"] = mixed_error(w, main_res["state"], threads)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
