"""Seeded synthetic inputs for Ni-cluster molecular dynamics.

This module only builds geometries, velocities and run recipes.  It holds
none of the Sutton-Chen arithmetic (no density, force, energy, integrator or
thermostat), so that the test oracle and the HIP library can both take their
inputs from it without sharing any of the method's code.

Structures follow the paper's workloads (arXiv:1210.3559):
  * icosahedral starting geometry of the heating runs (Sec. 3, "MD
    simulations of Ni2047 clusters"): Mackay icosahedra, magic sizes
    1 + sum_k (10 k^2 + 2) = 13, 55, 147, 309, ..., 2057;
  * molten starting structures of the solidification runs (Sec. 3.1): here a
    spherical fcc cut with random jitter and hot Maxwell-Boltzmann velocities;
  * ensembles of independent runs (Sec. 3.1, up to 15 trajectories per
    temperature): here batches of clusters of log-uniform sizes.

Random numbers come from numpy's PCG64 (``numpy.random.default_rng(seed)``).
Units: Angstrom, fs, K, atomic mass unit u.
"""
from __future__ import annotations

import itertools
import math
import re
from dataclasses import dataclass, field

import numpy as np

# Unit constants for drawing velocities in Angstrom/fs.
# 1 u*A^2/fs^2 = 103.64269652680505 eV (CODATA 2018 e and u); k_B in eV/K.
_EV_PER_U_A2_FS2 = 103.64269652680505
_KB_EV = 8.617333262145179e-05

NI_LATTICE_A = 3.52  # fcc lattice constant of the Sutton-Chen Ni set, Angstrom
NI_MASS_U = 58.6934  # standard atomic weight of Ni


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------
def _icosahedron_unit():
    """Vertices (unit circumradius) and triangular faces of a regular icosahedron."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * phi))
            v.append((s1, s2 * phi, 0.0))
            v.append((s2 * phi, 0.0, s1))
    v = np.array(v) / math.sqrt(1.0 + phi * phi)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=-1)
    edge = np.min(d[d > 1e-9])
    adj = np.abs(d - edge) < 1e-9
    faces = [f for f in itertools.combinations(range(12), 3)
             if adj[f[0], f[1]] and adj[f[1], f[2]] and adj[f[0], f[2]]]
    assert len(faces) == 20
    return v, faces


def mackay_icosahedron(shells: int, spacing: float = 2.49) -> np.ndarray:
    """Mackay icosahedron with ``shells`` closed shells around a central atom.

    Shell k holds the barycentric lattice points of the 20 triangular faces of
    an icosahedron whose 12 vertices sit at radius ``k * spacing``:
    12 vertices, 30 (k-1) edge points, 10 (k-1)(k-2) face points, i.e.
    10 k^2 + 2 atoms.  ``spacing`` is the centre-to-first-shell distance.
    Atoms are ordered by shell, then lexicographically, so the result is
    deterministic.
    """
    if shells < 0:
        raise ValueError("shells must be >= 0")
    verts, faces = _icosahedron_unit()
    pts = [np.zeros((1, 3))]
    for k in range(1, shells + 1):
        shell = {}
        for (ia, ib, ic) in faces:
            A, B, C = verts[ia] * k, verts[ib] * k, verts[ic] * k
            for i in range(k + 1):
                for j in range(k + 1 - i):
                    l = k - i - j
                    p = (i * A + j * B + l * C) / k * spacing
                    key = tuple(np.round(p, 9))
                    shell[key] = p
        arr = np.array(sorted(shell.values(), key=lambda q: (round(q[0], 9), round(q[1], 9), round(q[2], 9))))
        assert len(arr) == 10 * k * k + 2
        pts.append(arr)
    return np.ascontiguousarray(np.concatenate(pts, axis=0))


def mackay_size(shells: int) -> int:
    return 1 + sum(10 * k * k + 2 for k in range(1, shells + 1))


def _fcc_block(a: float, radius: float) -> np.ndarray:
    """All fcc sites (conventional cube edge a, origin on a site) with |r| <= radius + a."""
    m = int(math.ceil((radius + a) / (0.5 * a))) + 1
    r = np.arange(-m, m + 1)
    i, j, k = np.meshgrid(r, r, r, indexing="ij")
    keep = ((i + j + k) % 2) == 0
    p = np.stack([i[keep], j[keep], k[keep]], axis=1).astype(np.float64) * (0.5 * a)
    return p


def _ordered(p: np.ndarray) -> np.ndarray:
    """Sort by (|r|^2, x, y, z): breaks ties between sites of one shell deterministically."""
    r2 = np.round(np.einsum("ij,ij->i", p, p), 9)
    order = np.lexsort((np.round(p[:, 2], 9), np.round(p[:, 1], 9), np.round(p[:, 0], 9), r2))
    return p[order]


def fcc_sphere(radius: float, a: float = NI_LATTICE_A) -> np.ndarray:
    """Spherical cut of a perfect fcc lattice centred on a site: |r|^2 <= R^2 + 1e-9."""
    p = _fcc_block(a, radius)
    keep = np.einsum("ij,ij->i", p, p) <= radius * radius + 1e-9
    return np.ascontiguousarray(_ordered(p[keep]))


def fcc_exact(n: int, a: float = NI_LATTICE_A) -> np.ndarray:
    """The n fcc sites nearest to a lattice site, ties broken by (x, y, z)."""
    if n < 0:
        raise ValueError("n must be >= 0")
    if n == 0:
        return np.zeros((0, 3))
    # 4 sites per a^3; pad the radius by two lattice constants.
    radius = (3.0 * n / (4.0 * math.pi * 4.0 / a ** 3)) ** (1.0 / 3.0) + 2.0 * a
    p = _ordered(_fcc_block(a, radius))
    assert len(p) >= n
    return np.ascontiguousarray(p[:n])


def jitter(pos: np.ndarray, amplitude: float, rng: np.random.Generator) -> np.ndarray:
    """Independent uniform displacement in [-amplitude, amplitude] per component."""
    return np.ascontiguousarray(pos + rng.uniform(-amplitude, amplitude, size=pos.shape))


# --------------------------------------------------------------------------
# Velocities
# --------------------------------------------------------------------------
def maxwell_boltzmann(pos: np.ndarray, temperature: float, rng: np.random.Generator,
                      mass_u: float = NI_MASS_U) -> np.ndarray:
    """Gaussian velocities (A/fs) with per-component variance k_B T / m, then the
    centre-of-mass velocity and the angular momentum about the centre of mass
    removed (a free cluster at rest).  No rescaling to an exact temperature:
    the draw is a sample of the Maxwell-Boltzmann distribution at ``temperature``."""
    n = len(pos)
    if n == 0:
        return np.zeros((0, 3))
    sigma = math.sqrt(_KB_EV * temperature / (mass_u * _EV_PER_U_A2_FS2))
    v = rng.normal(0.0, sigma, size=(n, 3))
    v -= v.mean(axis=0)
    if n >= 3:
        r = pos - pos.mean(axis=0)
        L = np.cross(r, v).sum(axis=0)
        inertia = np.einsum("ij,ij->", r, r) * np.eye(3) - r.T @ r
        omega = np.linalg.lstsq(inertia, L, rcond=None)[0]
        v -= np.cross(omega, r)
        v -= v.mean(axis=0)
    elif n == 2:
        # a dimer can only vibrate: keep the component along the bond
        b = pos[1] - pos[0]
        b = b / np.linalg.norm(b)
        v = np.outer(v @ b, b)
        v -= v.mean(axis=0)
    else:
        v[:] = 0.0
    return np.ascontiguousarray(v)


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------
@dataclass
class Workload:
    """One run recipe: concatenated clusters (CSR offsets), velocities and the
    integrator/thermostat settings to run them with."""
    name: str
    pos: np.ndarray                 # (sum N, 3) float64
    vel: np.ndarray                 # (sum N, 3) float64
    offsets: np.ndarray             # (n_clusters + 1,) int64
    dt: float                       # fs
    steps: int                      # steps of the full run
    # per cluster: None, dict(T_start, T_end, ramp_steps, tau) for Berendsen,
    # or dict(kind="langevin", T_start, T_end, ramp_steps, gamma, seed)
    thermostat: list = field(default_factory=list)
    rc: float = 0.0                 # cutoff radius for the cell-list variant (0 = all pairs)
    precision: str = "fp64"

    @property
    def n_clusters(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_atoms(self) -> int:
        return int(self.offsets[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def cluster(self, k: int):
        a, b = int(self.offsets[k]), int(self.offsets[k + 1])
        return self.pos[a:b], self.vel[a:b]


def _single(name, pos, vel, dt, steps, thermostat=None, **kw) -> Workload:
    return Workload(name, np.ascontiguousarray(pos), np.ascontiguousarray(vel),
                    np.array([0, len(pos)], dtype=np.int64), dt, steps, [thermostat], **kw)


def c1_icosahedron(seed: int = 147) -> Workload:
    """Ni147 Mackay icosahedron (3 shells, 2.49 A radial spacing), MB 1200 K, NVE, 1 fs, 1000 steps."""
    rng = np.random.default_rng(seed)
    pos = mackay_icosahedron(3, 2.49)
    return _single("ni147_icosahedron_nve", pos, maxwell_boltzmann(pos, 1200.0, rng), 1.0, 1000)


def c2_cooling(seed: int = 2057) -> Workload:
    """fcc sphere R = 18 A (2243 atoms), +-0.05 A jitter, MB 2000 K, Berendsen
    (tau 100 fs) linear cooling 2000 -> 800 K over 200k steps of 2 fs."""
    rng = np.random.default_rng(seed)
    pos = jitter(fcc_sphere(18.0), 0.05, rng)
    vel = maxwell_boltzmann(pos, 2000.0, np.random.default_rng(seed + 1))
    th = dict(T_start=2000.0, T_end=800.0, ramp_steps=200_000, tau=100.0)
    return _single("ni2243_fcc_r18_berendsen_cooling", pos, vel, 2.0, 200_000, th)


def c3_large(seed: int = 4780, cutoff: bool = False) -> Workload:
    """fcc sphere R = 50 A (48,077 atoms), jitter, MB 1900 K, Berendsen at 1900 K, 1 fs, 10k steps;
    all pairs, or the cell-list variant with rc = 2.5 a = 8.8 A (shifted)."""
    rng = np.random.default_rng(seed)
    pos = jitter(fcc_sphere(50.0), 0.05, rng)
    vel = maxwell_boltzmann(pos, 1900.0, np.random.default_rng(seed + 1))
    th = dict(T_start=1900.0, T_end=1900.0, ramp_steps=0, tau=100.0)
    name = "ni48077_fcc_r50_nvt" + ("_cell_rc8.8" if cutoff else "_allpairs")
    return _single(name, pos, vel, 1.0, 10_000, th, rc=(2.5 * NI_LATTICE_A if cutoff else 0.0))


def c4_mixed(seed: int = 15000) -> Workload:
    """15,000-atom exact fcc cut, jitter, MB 1500 K, NVE, 1 fs, 20k steps (mixed-precision form)."""
    rng = np.random.default_rng(seed)
    pos = jitter(fcc_exact(15_000), 0.05, rng)
    vel = maxwell_boltzmann(pos, 1500.0, np.random.default_rng(seed + 1))
    return _single("ni15000_fcc_nve_mixed", pos, vel, 1.0, 20_000, None, precision="mixed")


def batch_sizes(n_clusters: int, seed: int, n_min: int = 147, n_max: int = 6000) -> np.ndarray:
    """Log-uniform cluster sizes floor(exp(U(ln n_min, ln (n_max + 1))))."""
    rng = np.random.default_rng(seed)
    s = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max + 1), size=n_clusters))).astype(np.int64)
    return np.clip(s, n_min, n_max)


def c5_batch(seed: int = 355900, n_clusters: int = 256, n_min: int = 147, n_max: int = 6000,
             T_start: float = 2000.0, T_end: float = 800.0, dt: float = 1.0, steps: int = 2000) -> Workload:
    """Batch of independent cooling runs: exact fcc cuts of log-uniform size,
    jitter, MB at T_start, Berendsen (tau 100 fs) cooling at a rate drawn
    uniformly from [1e11, 1e13] K/s down to T_end."""
    sizes = batch_sizes(n_clusters, seed, n_min, n_max)
    rates = np.random.default_rng(seed + 1).uniform(1e11, 1e13, size=n_clusters)  # K/s
    pos, vel, th = [], [], []
    for k, n in enumerate(sizes):
        rng = np.random.default_rng(seed + 2 + k)
        p = jitter(fcc_exact(int(n)), 0.05, rng)
        pos.append(p)
        vel.append(maxwell_boltzmann(p, T_start, rng))
        ramp_fs = (T_start - T_end) / (rates[k] * 1e-15)
        th.append(dict(T_start=T_start, T_end=T_end, ramp_steps=int(round(ramp_fs / dt)), tau=100.0))
    offsets = np.zeros(n_clusters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return Workload(f"batch{n_clusters}_ni{n_min}-{n_max}_cooling", np.ascontiguousarray(np.concatenate(pos)),
                    np.ascontiguousarray(np.concatenate(vel)), offsets, dt, steps, th)


def in_langevin_bath(w: Workload, gamma: float = 10.0, seed: int = 1) -> Workload:
    """The same clusters and temperature programme in a Langevin bath of
    damping gamma (1/ps; the paper uses 10), cluster k keyed by seed + k."""
    th = []
    for k, t in enumerate(w.thermostat):
        if t is None:
            th.append(None)
        else:
            th.append(dict(kind="langevin", T_start=t["T_start"], T_end=t["T_end"],
                           ramp_steps=t.get("ramp_steps", 0), gamma=gamma, seed=seed + k))
    name = w.name.replace("berendsen", "langevin") if "berendsen" in w.name else w.name + "_langevin"
    return Workload(name, w.pos, w.vel, w.offsets, w.dt, w.steps, th, w.rc, w.precision)


def heating_cooling_legs(T_low: float = 400.0, T_high: float = 1400.0, rate_K_per_ps: float = 1.0,
                         dt: float = 1.0):
    """Temperature programme of a heating-cooling cycle at a constant rate:
    [(T_start, T_end, steps)] for the heating and the cooling leg."""
    steps = int(round(abs(T_high - T_low) / rate_K_per_ps * 1000.0 / dt))
    return [(T_low, T_high, steps), (T_high, T_low, steps)]


def ni2057_cycle(replicas: int = 1, seed: int = 2057, T_low: float = 400.0, gamma: float = 10.0,
                 dt: float = 1.0) -> Workload:
    """Mackay Ni2057 icosahedron (8 shells, 2.49 A) with Maxwell-Boltzmann
    velocities at T_low, in a Langevin bath at T_low; `replicas` independent
    copies (own velocities and bath seeds) form a batch.  The cycle's legs
    come from heating_cooling_legs."""
    base = mackay_icosahedron(8, 2.49)
    pos, vel, th = [], [], []
    for k in range(replicas):
        pos.append(base)
        vel.append(maxwell_boltzmann(base, T_low, np.random.default_rng(seed + 1 + k)))
        th.append(dict(kind="langevin", T_start=T_low, T_end=T_low, ramp_steps=0, gamma=gamma, seed=seed + k))
    offsets = np.arange(replicas + 1, dtype=np.int64) * len(base)
    return Workload(f"ni2057_icosahedron_cycle_x{replicas}", np.ascontiguousarray(np.concatenate(pos)),
                    np.ascontiguousarray(np.concatenate(vel)), offsets, dt, 0, th)


def concat(workloads) -> Workload:
    """Concatenate single- or multi-cluster workloads into one batch (same dt)."""
    pos = np.concatenate([w.pos for w in workloads])
    vel = np.concatenate([w.vel for w in workloads])
    sizes = np.concatenate([w.sizes() for w in workloads])
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    th = sum((list(w.thermostat) for w in workloads), [])
    return Workload("+".join(w.name for w in workloads), np.ascontiguousarray(pos), np.ascontiguousarray(vel),
                    offsets, workloads[0].dt, max(w.steps for w in workloads), th)


def by_name(name: str) -> Workload:
    """Named workloads of the benchmark and the autotuner."""
    if name == "ni2243_cooling":
        return c2_cooling()
    if name == "ni147_nve":
        return c1_icosahedron()
    if name == "ni48077_allpairs":
        return c3_large()
    if name == "ni48077_cell":
        return c3_large(cutoff=True)
    if name == "ni15000_mixed":
        return c4_mixed()
    if name == "ni15000_fp64":
        w = c4_mixed()
        w.precision = "fp64"
        w.name = "ni15000_fcc_nve_fp64"
        return w
    if name == "batch256":
        return c5_batch()
    if name == "batch256_mixed":
        w = c5_batch()
        w.precision = "mixed"
        w.name += "_mixed"
        return w
    if name == "ni2243_langevin":
        return in_langevin_bath(c2_cooling(), seed=2057)
    if name == "batch256_langevin":
        return in_langevin_bath(c5_batch(), seed=355900)
    m = re.fullmatch(r"ni2057_cycle(?:_x(\d+))?", name)
    if m:
        w = ni2057_cycle(int(m.group(1) or 1))
        lo, hi, n = heating_cooling_legs()[0]
        w.thermostat = [dict(t, T_start=lo, T_end=hi, ramp_steps=n) for t in w.thermostat]
        w.steps = n
        return w
    m = re.fullmatch(r"fcc(\d+)_nve", name)
    if m:
        n = int(m.group(1))
        pos = jitter(fcc_exact(n), 0.05, np.random.default_rng(n))
        return _single(name, pos, maxwell_boltzmann(pos, 1200.0, np.random.default_rng(n + 1)), 1.0, 1000)
    if name == "ni50000_allpairs":
        pos = jitter(fcc_exact(50000), 0.05, np.random.default_rng(50000))
        vel = maxwell_boltzmann(pos, 1900.0, np.random.default_rng(50001))
        th = dict(T_start=1900.0, T_end=1900.0, ramp_steps=0, tau=100.0)
        return _single("ni50000_fcc_nvt_allpairs", pos, vel, 1.0, 10_000, th)
    raise KeyError(f"unknown workload {name}")
