"""Solidification kinetics of overcooled nickel clusters (the paper's Sec. 3,
"Solidification process" and "Kinetics of the solidification phase
transition"): molten Ni2057 clusters are held in a Langevin bath below the
melting point until they crystallise; the lifetime of the overcooled liquid
is the time at which the total energy starts to drop abruptly, the escape
rate is kappa = 1/<t> (Eq. (rate2)), and its temperature dependence is fitted
with ln(kappa * 1 ps) = a - b / (k_B T (T - T0)^2) (Eq. (rate3)).

    python -m paper_1210_3559_amd.kinetics --T 780 [--replicas 15]
        [--max-ps 4000] [--T-melt 1400 --melt-ps 100] [--out file.json]
    python -m paper_1210_3559_amd.kinetics --fit 780.json 800.json ...

Replicas are independent clusters of one batch (own initial velocities and
bath seeds): they are melted together at T_melt, quenched to T, and stepped
until every one has crystallised or the time limit is reached (runs without
a transition are censored at the limit).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, scmd

K_B = 8.617333262145179e-05  # eV/K
A2_PER_PS_TO_CM2_PER_S = 1e-4  # 1 A^2/ps = 1e-16 cm^2 / 1e-12 s


def rdf_g(counts, n_ref: int, dr: float, rho_bar: float = 4.0 / 3.52 ** 3):
    """g(r) = rho(r) / rho_bar (Sec. 3, Eq. (Rdist)) at the bin centres from a
    pair-distance histogram: counts / (n_ref rho_bar V_shell), V_shell the
    volume of the bin's spherical shell; rho_bar defaults to the number
    density of fcc nickel, 4 / a^3."""
    c = np.asarray(counts, dtype=np.float64)
    b = np.arange(len(c), dtype=np.float64)
    shell = 4.0 * np.pi / 3.0 * ((b + 1.0) ** 3 - b ** 3) * dr ** 3
    r = (b + 0.5) * dr
    return r, c / (max(int(n_ref), 1) * rho_bar * shell)


def running_mean(x, w: int) -> np.ndarray:
    """Centred running mean over w samples (shorter at the ends)."""
    x = np.asarray(x, dtype=np.float64)
    if len(x) == 0 or w <= 1:
        return x.copy()
    c = np.concatenate([[0.0], np.cumsum(x)])
    h = w // 2
    lo = np.clip(np.arange(len(x)) - h, 0, len(x))
    hi = np.clip(np.arange(len(x)) + h + 1, 0, len(x))
    return (c[hi] - c[lo]) / (hi - lo)


def transition_time(t, e, drop: float, settle: float = 10.0, ref: float = 40.0, smooth: int = 5):
    """Time at which the energy per atom e(t) starts its abrupt drop by about
    `drop` (eV/atom), or None if it never falls that far.

    The liquid level is the median of the smoothed trace over [settle, settle
    + ref] after the start; the drop is found where the smoothed trace first
    falls below level - drop/2, and its start is the last earlier time at
    which the trace was still above level - drop/5.
    """
    t = np.asarray(t, dtype=np.float64)
    s = running_mean(e, smooth)
    win = (t >= t[0] + settle) & (t <= t[0] + settle + ref)
    if not win.any():
        return None
    level = float(np.median(s[win]))
    below = np.nonzero((s < level - 0.5 * drop) & (t >= t[0] + settle))[0]
    if len(below) == 0:
        return None
    k = int(below[0])
    above = np.nonzero(s[:k] >= level - 0.2 * drop)[0]
    return float(t[above[-1]] if len(above) else t[0])


def escape_rate(lifetimes, censored_at=()):
    """(kappa = 1/<t> over the observed lifetimes, as Eq. (rate2); the
    maximum-likelihood rate of an exponential law with censored runs,
    events / (sum of lifetimes + sum of censoring times))."""
    t = np.asarray(lifetimes, dtype=np.float64)
    c = np.asarray(censored_at, dtype=np.float64)
    k_mean = 1.0 / t.mean() if len(t) else float("nan")
    tot = t.sum() + c.sum()
    k_mle = len(t) / tot if tot > 0 else float("nan")
    return k_mean, k_mle


def fit_rate3(T, kappa_per_ps, T0=None, p0=(1.2, 3.0e4, 1030.0), events=None, with_errors: bool = False):
    """Least-squares fit of ln(kappa * 1 ps) = a - b / (k_B T (T - T0)^2)
    (kappa in 1/ps, b in eV K^2); returns (a, b, T0).  With T0 given only a
    and b are fitted (three temperatures far below T0 do not determine it).
    events: the number of observed transitions behind each rate; the fit is
    then weighted by the rate's statistical error, sigma(ln kappa) =
    1/sqrt(events) for an exponential lifetime.  with_errors: also return the
    standard errors of the fitted parameters (from the fit's covariance;
    absolute when weighted)."""
    from scipy.optimize import curve_fit
    T = np.asarray(T, dtype=np.float64)
    y = np.log(np.asarray(kappa_per_ps, dtype=np.float64))
    sig = None if events is None else 1.0 / np.sqrt(np.asarray(events, dtype=np.float64))
    kw = dict(maxfev=20000, sigma=sig, absolute_sigma=sig is not None)
    if T0 is not None:
        def f2(x, a, b):
            return a - b / (K_B * x * (x - T0) ** 2)

        p, cov = curve_fit(f2, T, y, p0=p0[:2], **kw)
        res = (float(p[0]), float(p[1]), float(T0))
        err = (float(np.sqrt(cov[0, 0])), float(np.sqrt(cov[1, 1])), 0.0)
    else:
        def f(x, a, b, t0):
            return a - b / (K_B * x * (x - t0) ** 2)

        p, cov = curve_fit(f, T, y, p0=p0, **kw)
        res = tuple(float(v) for v in p)
        err = tuple(float(np.sqrt(cov[i, i])) for i in range(3))
    return (res, err) if with_errors else res


def structure_series(sim, cluster: int, nframes: int, frame_ps: float, rdf_counts, rdf_nref,
                     window_ps: float = 1000.0, stride_ps: float = 500.0, radius: float = 10.0, segments: int = 10,
                     dr: float = 0.4):
    """D(t) and g(r) of one trajectory as the paper computes them: at window
    centres every stride_ps, D from the window's frames held in the cluster's
    device frame store (10 segments, central atoms within `radius`; computed
    by the library), g(r) of the central atoms (per-frame histograms summed
    over the window)."""
    nwin = max(1, int(round(window_ps / frame_ps)))
    out = []
    centre = window_ps / 2.0
    while (centre + window_ps / 2.0) / frame_ps <= nframes + 1e-9:
        a = int(round((centre - window_ps / 2.0) / frame_ps))
        b = min(nframes, a + nwin)
        d, nc = sim.diffusion(cluster, a, b - a, frame_ps, radius, segments)
        cnt = np.sum(rdf_counts[a:b], axis=0)
        nref = int(np.sum(rdf_nref[a:b]))
        r, g = rdf_g(cnt, nref, dr)
        out.append({"t_ps": centre, "D_cm2_per_s": d * A2_PER_PS_TO_CM2_PER_S, "central_atoms": nc,
                    "rdf_r": [float(x) for x in r], "rdf_g": [float(x) for x in g], "rdf_refs": nref})
        centre += stride_ps
    return out


def run(T: float, replicas: int = 15, max_ps: float = 4000.0, T_melt: float = 1400.0, melt_ps: float = 100.0,
        gamma: float = 10.0, seed: int = 820, dt: float = 1.0, sample_ps: float = 1.0, chunk_ps: float = 100.0,
        drop: float = 0.03, track: int = 0, frame_ps: float = 10.0, rdf_select: float = 3.0, rdf_dr: float = 0.4,
        rdf_bins: int = 40, min_ps: float = 0.0, log=sys.stderr) -> dict:
    """Melt `replicas` Mackay Ni2057 clusters at T_melt, quench them to T and
    step until all have crystallised or max_ps has passed.  The first
    `track` replicas also keep a frame every frame_ps (for D(t)) and the
    pair-distance histogram of their central atoms (for g(r))."""
    w = inputs.ni2057_cycle(replicas, seed=seed, T_low=T_melt, gamma=gamma, dt=dt)
    n = int(w.sizes()[0])
    every = max(1, int(round(sample_ps * 1000.0 / dt)))
    chunk = max(every, int(round(chunk_ps * 1000.0 / dt)) // every * every)
    melt_steps = int(round(melt_ps * 1000.0 / dt)) // every * every
    max_steps = int(round(max_ps * 1000.0 / dt))
    cap = (max_steps + melt_steps) // every + 8
    t0 = time.perf_counter()
    with scmd.Simulation(w.offsets, w.pos, w.vel, dt=dt, thermostats=w.thermostat) as sim:
        sim.set_sampling(every, capacity=cap)
        sim.step(melt_steps)
        for k in range(replicas):
            sim.set_thermostat(k, dict(w.thermostat[k], T_start=T, T_end=T, ramp_steps=0))
        done, found = 0, [None] * replicas
        fstep = max(every, int(round(frame_ps * 1000.0 / dt)) // every * every) if track > 0 else chunk
        for k in range(track):
            sim.set_frames(k, max_steps // fstep + 1)
        nframes = 0
        hists = [[] for _ in range(track)]
        nrefs = [[] for _ in range(track)]
        while done < max_steps:
            c = min(chunk, max_steps - done)
            left = c
            while left > 0:
                f = min(fstep, left)
                sim.step(f)
                left -= f
                if track > 0 and f == fstep:
                    sim.record_frame()
                    nframes += 1
                    for k in range(track):
                        h, nr = sim.rdf(k, rdf_dr, rdf_bins, rdf_select)
                        hists[k].append(h)
                        nrefs[k].append(nr)
            done += c
            for k in range(replicas):
                if found[k] is None:
                    s, _ = sim.samples(k, cap)
                    iso = s[s[:, 0] > melt_steps]
                    tk = (iso[:, 0] - melt_steps) * dt * 1e-3  # ps since the quench
                    found[k] = transition_time(tk, (iso[:, 1] + iso[:, 2]) / n, drop)
            nf = sum(x is not None for x in found)
            print(f"[kinetics] T={T:.0f} K: {done * dt * 1e-3:.0f} ps, {nf}/{replicas} crystallised, "
                  f"{time.perf_counter() - t0:.1f} s", file=log, flush=True)
            if nf == replicas and done * dt * 1e-3 >= min_ps:
                break
        traces = []
        for k in range(replicas):
            s, _ = sim.samples(k, cap)
            iso = s[s[:, 0] > melt_steps]
            traces.append(((iso[:, 0] - melt_steps) * dt * 1e-3, (iso[:, 1] + iso[:, 2]) / n, iso[:, 3]))
        series = [structure_series(sim, k, nframes, frame_ps, hists[k], nrefs[k], dr=rdf_dr) for k in range(track)
                  if nframes * frame_ps >= 1000.0]
    wall = time.perf_counter() - t0
    run_ps = done * dt * 1e-3
    life = [x for x in found if x is not None]
    cens = [run_ps] * (replicas - len(life))
    k_mean, k_mle = escape_rate(life, cens)
    # latent heat: liquid level before the drop minus the solid level at the end
    lat = []
    for (tk, ek, _), x in zip(traces, found):
        if x is not None and tk[-1] - x > 60.0:
            liq = np.median(ek[(tk >= 10.0) & (tk <= max(20.0, x - 5.0))])
            sol = np.median(ek[tk >= tk[-1] - 30.0])
            lat.append(float(liq - sol) * n)
    return {
        "T_K": T, "replicas": replicas, "seed": seed, "atoms_per_cluster": n, "gamma_per_ps": gamma, "dt_fs": dt,
        "tracked": series,
        "melt": {"T_K": T_melt, "ps": melt_steps * dt * 1e-3}, "max_ps": max_ps, "run_ps": run_ps,
        "lifetimes_ps": [x for x in found], "n_crystallised": len(life), "mean_lifetime_ps": (
            float(np.mean(life)) if life else None),
        "kappa_per_ps": k_mean, "kappa_mle_per_ps": k_mle, "latent_heat_eV": (float(np.mean(lat)) if lat else None),
        "seconds": wall, "us_per_step": 1e6 * wall / (done + melt_steps),
        "traces": [{"t_ps": [float(v) for v in tk[::10]], "e_per_atom": [float(v) for v in ek[::10]]}
                   for tk, ek, _ in traces],
    }


def _shared_replicas(r1, r2) -> bool:
    """Whether two results repeat a replica: replica k of a run with base seed
    s takes its velocities from s + 1 + k and its bath from s + k, so two runs
    of one protocol share a replica exactly when their seeds differ by less
    than the replica count of the run with the lower seed."""
    keys = ("T_K", "gamma_per_ps", "dt_fs", "melt")
    if "seed" not in r1 or "seed" not in r2 or any(r1.get(k) != r2.get(k) for k in keys):
        return False
    d = int(r2["seed"]) - int(r1["seed"])
    return -int(r2["replicas"]) < d < int(r1["replicas"])


def pooled_rates(results):
    """Per temperature, the escape rate of all runs of the given results
    (dicts as returned by run()) pooled: (T, kappa MLE, kappa 1/<t>, events),
    sorted by T.  The MLE counts runs that had not crystallised at their time
    limit (censored); 1/<t> uses the observed lifetimes only.  Raises
    ValueError for two results that repeat a replica (seeds too close)."""
    for i, r1 in enumerate(results):
        for r2 in results[i + 1:]:
            if _shared_replicas(r1, r2):
                raise ValueError(f"runs at {r1['T_K']} K with seeds {r1['seed']} and {r2['seed']} repeat replicas: "
                                 f"seeds of one protocol need to be at least the replica count apart")
    by_T = {}
    for r in results:
        d = by_T.setdefault(float(r["T_K"]), ([], []))
        for x in r["lifetimes_ps"]:
            (d[0] if x is not None else d[1]).append(float(x) if x is not None else float(r["run_ps"]))
    out = []
    for T in sorted(by_T):
        life, cens = by_T[T]
        k_mean, k_mle = escape_rate(life, cens)
        out.append((T, k_mle, k_mean, len(life)))
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--fit", nargs="+", default=None, metavar="RESULT_JSON",
                    help="fit Eq. (rate3) to the pooled rates of these --out files instead of running")
    ap.add_argument("--T", type=float, default=None, help="bath temperature, K")
    ap.add_argument("--replicas", type=int, default=15)
    ap.add_argument("--max-ps", type=float, default=4000.0)
    ap.add_argument("--seed", type=int, default=820,
                    help="replica k takes its velocities from seed + 1 + k and its bath from seed + k: "
                         "independent runs need seeds at least --replicas + 1 apart")
    ap.add_argument("--track", type=int, default=0, help="replicas whose D(t) and g(r) are recorded")
    ap.add_argument("--min-ps", type=float, default=0.0, help="run at least this long")
    ap.add_argument("--T-melt", type=float, default=1400.0, help="bath temperature of the melt, K")
    ap.add_argument("--melt-ps", type=float, default=100.0, help="length of the melt, ps")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.fit:
        results = []
        for path in args.fit:
            with open(path) as f:
                results.append(json.load(f))
        rates = pooled_rates(results)
        T, k, _, ev = zip(*rates)
        (a, b, t0), err = fit_rate3(T, k, events=ev, with_errors=True)
        print(json.dumps({"rates": [dict(T_K=t, kappa_mle_per_ps=km, kappa_mean_per_ps=kn, events=e)
                                    for t, km, kn, e in rates],
                          "fit": dict(a=a, b_eV_K2=b, T0_K=t0, a_err=err[0], b_err=err[1], T0_err=err[2])}))
        return 0
    if args.T is None:
        ap.error("--T is required unless --fit is given")
    res = run(args.T, args.replicas, args.max_ps, T_melt=args.T_melt, melt_ps=args.melt_ps, seed=args.seed,
              track=args.track, min_ps=args.min_ps)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    brief = {k: v for k, v in res.items() if k not in ("traces", "tracked")}
    brief["D_cm2_per_s"] = [[(round(x["t_ps"]), x["D_cm2_per_s"]) for x in s] for s in res["tracked"]]
    print(json.dumps(brief))
    return 0


if __name__ == "__main__":
    sys.exit(main())
