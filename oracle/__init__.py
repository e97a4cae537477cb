"""Sutton-Chen FP64 CPU oracle (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
the two share no code: the C source here is a plain double loop over ordered
pairs written from the paper's definitions (Yakubovich et al.,
arXiv:1210.3559, Sec. 2.1 Eqs. (SC) and (rho); Sec. 2 "Computational
approach" for the two-sweep structure and the Verlet step).

Every function is pinned by tests that do not call back into the oracle's
own formula: the dimer and equilateral-trimer closed forms, the perfect-fcc
lattice sums, finite differences of the energy, the net force and torque
invariants, Mackay-icosahedron symmetry, NVE energy drift, time
reversibility and Berendsen relaxation; the Langevin bath by the published
Philox4x32-10 known-answer blocks, the normal law of its deviates, the
reduction to velocity-Verlet at zero damping, the closed-form decay of a free
atom in a bath at 0 K and the equipartition temperature of free atoms and of
a cluster; the pair-distance histogram by the fcc neighbour-shell
multiplicities, the pair count and the dimer and trimer.  Nothing in this
package is "parity unpinned".

Arrays are numpy float64 of shape (n, 3) for positions, velocities and
forces.  Units: Angstrom, fs, eV, u, K.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsc_oracle.so")

# Parameter set of Sutton and Chen for nickel, as quoted in Sec. 2.1 of the
# paper (text after Eq. (rho)).
NI_PARAMS = dict(eps=1.5707e-2, a=3.52, c=39.432, n=9, m=6, rc=0.0)
# Standard atomic weight of nickel (IUPAC); the paper gives no mass.
NI_MASS_U = 58.6934

NVE = 0
BERENDSEN = 1
LANGEVIN = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: IEEE double, no fast-math, no FMA
    contraction, no host-specific ISA (the library travels to other hosts)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("a", ctypes.c_double), ("c", ctypes.c_double),
                ("n", ctypes.c_int), ("m", ctypes.c_int), ("rc", ctypes.c_double)]


class _Thermo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("T_start", ctypes.c_double), ("T_end", ctypes.c_double),
                ("ramp_steps", ctypes.c_int64), ("tau", ctypes.c_double), ("gamma", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("ramp_origin", ctypes.c_int64)]


_lib = None


def _configure(lib):
    i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    pp = ctypes.POINTER(_Params)
    lib.sco_density.argtypes = [i64, vp, pp, vp, ctypes.c_int]
    lib.sco_density.restype = None
    lib.sco_forces.argtypes = [i64, vp, pp, vp, vp, vp, ctypes.c_int]
    lib.sco_forces.restype = None
    lib.sco_forces_subset.argtypes = [i64, vp, pp, vp, i64, vp, vp, ctypes.c_int]
    lib.sco_forces_subset.restype = None
    lib.sco_energy.argtypes = [i64, vp, pp, vp, ctypes.c_int]
    lib.sco_energy.restype = dbl
    lib.sco_ndof.argtypes = [i64]
    lib.sco_ndof.restype = i64
    lib.sco_ndof_kind.argtypes = [i64, ctypes.c_int]
    lib.sco_ndof_kind.restype = i64
    lib.sco_temperature_dof.argtypes = [i64, vp, dbl, i64]
    lib.sco_temperature_dof.restype = dbl
    lib.sco_philox4x32_10.argtypes = [vp, vp, vp]
    lib.sco_philox4x32_10.restype = None
    lib.sco_gauss3.argtypes = [ctypes.c_uint64, i64, i64, vp]
    lib.sco_gauss3.restype = None
    lib.sco_rdf.argtypes = [i64, vp, dbl, dbl, ctypes.c_int, vp, ctypes.POINTER(i64)]
    lib.sco_rdf.restype = ctypes.c_int
    lib.sco_kinetic.argtypes = [i64, vp, dbl]
    lib.sco_kinetic.restype = dbl
    lib.sco_temperature.argtypes = [i64, vp, dbl]
    lib.sco_temperature.restype = dbl
    lib.sco_target_temperature.argtypes = [ctypes.POINTER(_Thermo), i64]
    lib.sco_target_temperature.restype = dbl
    lib.sco_berendsen_lambda.argtypes = [dbl, dbl, dbl, dbl]
    lib.sco_berendsen_lambda.restype = dbl
    lib.sco_vv_run.argtypes = [i64, vp, vp, vp, ctypes.c_int, pp, dbl, dbl, i64,
                               ctypes.POINTER(_Thermo), i64, vp, ctypes.c_int]
    lib.sco_vv_run.restype = ctypes.c_int
    lib.sco_ke_conversion.restype = dbl
    lib.sco_kb.restype = dbl
    lib.sco_max_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _params(p=None) -> _Params:
    q = dict(NI_PARAMS)
    if p:
        q.update(p)
    if not (int(q["n"]) > int(q["m"]) > 0):
        raise ValueError("Sutton-Chen exponents need n > m > 0")
    return _Params(float(q["eps"]), float(q["a"]), float(q["c"]), int(q["n"]), int(q["m"]), float(q["rc"]))


def _pos(x) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("expected an (n, 3) array")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().sco_max_threads())


def ke_conversion() -> float:
    """eV per u*A^2/fs^2."""
    return float(_load().sco_ke_conversion())


def kb() -> float:
    """Boltzmann constant, eV/K."""
    return float(_load().sco_kb())


def density(pos, params=None, nthreads: int = 1) -> np.ndarray:
    """Eq. (rho): rho_i for every atom (shifted at rc when params['rc'] > 0)."""
    r = _pos(pos)
    out = np.zeros(len(r))
    p = _params(params)
    _load().sco_density(len(r), _ptr(r), ctypes.byref(p), _ptr(out), nthreads)
    return out


def forces(pos, params=None, nthreads: int = 1):
    """Return (F (n,3), rho (n,), site energies (n,)) at the given positions."""
    r = _pos(pos)
    n = len(r)
    f = np.zeros((n, 3))
    rho = np.zeros(n)
    site = np.zeros(n)
    p = _params(params)
    _load().sco_forces(n, _ptr(r), ctypes.byref(p), _ptr(f), _ptr(rho), _ptr(site), nthreads)
    return f, rho, site


def forces_subset(pos, idx, params=None, nthreads: int = 1):
    """Forces of the listed atoms only (k x 3) and the full density (n,)."""
    r = _pos(pos)
    ix = np.ascontiguousarray(idx, dtype=np.int64)
    if ix.size and (ix.min() < 0 or ix.max() >= len(r)):
        raise ValueError("atom index out of range")
    f = np.zeros((len(ix), 3))
    rho = np.zeros(len(r))
    p = _params(params)
    _load().sco_forces_subset(len(r), _ptr(r), ctypes.byref(p), _ptr(ix), len(ix), _ptr(f), _ptr(rho), nthreads)
    return f, rho


def energy(pos, params=None, nthreads: int = 1) -> float:
    """Eq. (SC): total potential energy, eV."""
    r = _pos(pos)
    p = _params(params)
    return float(_load().sco_energy(len(r), _ptr(r), ctypes.byref(p), None, nthreads))


def site_energies(pos, params=None, nthreads: int = 1) -> np.ndarray:
    r = _pos(pos)
    out = np.zeros(len(r))
    p = _params(params)
    _load().sco_energy(len(r), _ptr(r), ctypes.byref(p), _ptr(out), nthreads)
    return out


def ndof(n: int, kind: int = NVE) -> int:
    """Thermal degrees of freedom: 3N - 6 for a free cluster (1 for a dimer),
    3N under the Langevin bath."""
    return int(_load().sco_ndof_kind(n, kind))


def philox4x32_10(ctr, key) -> tuple:
    """Philox4x32-10 block of a 4-word counter under a 2-word key."""
    c = np.ascontiguousarray([int(x) & 0xFFFFFFFF for x in ctr], dtype=np.uint32)
    k = np.ascontiguousarray([int(x) & 0xFFFFFFFF for x in key], dtype=np.uint32)
    if c.size != 4 or k.size != 2:
        raise ValueError("counter has 4 words, key 2")
    out = np.zeros(4, dtype=np.uint32)
    _load().sco_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(x) for x in out)


def gauss3(seed: int, step: int, atom: int) -> np.ndarray:
    """The three standard normal deviates of the Langevin noise of one atom
    at one step (numbered from 1)."""
    out = np.zeros(3)
    _load().sco_gauss3(int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), int(atom), _ptr(out))
    return out


def kinetic(vel, mass_u: float = NI_MASS_U) -> float:
    v = _pos(vel)
    return float(_load().sco_kinetic(len(v), _ptr(v), mass_u))


def temperature(vel, mass_u: float = NI_MASS_U, kind: int = NVE) -> float:
    v = _pos(vel)
    lib = _load()
    return float(lib.sco_temperature_dof(len(v), _ptr(v), mass_u, lib.sco_ndof_kind(len(v), kind)))


def target_temperature(T_start, T_end, ramp_steps, k, ramp_origin: int = 0) -> float:
    t = _Thermo(BERENDSEN, T_start, T_end, ramp_steps, 1.0, 0.0, 0, int(ramp_origin))
    return float(_load().sco_target_temperature(ctypes.byref(t), k))


def berendsen_lambda(T, T_target, dt, tau) -> float:
    return float(_load().sco_berendsen_lambda(T, T_target, dt, tau))


def vv_run(pos, vel, nsteps, dt=1.0, params=None, mass_u=NI_MASS_U, thermostat=None, step0=0,
           force=None, nthreads: int = 1, with_log: bool = True):
    """Velocity-Verlet trajectory, optionally thermostatted.

    thermostat: None (NVE), dict(T_start, T_end, ramp_steps, tau) for
    Berendsen, or dict(kind="langevin", T_start, T_end, ramp_steps, gamma
    (1/ps), seed) for the Langevin bath (BAOAB; the steps of the trajectory
    are numbered step0 + 1, step0 + 2, ... for the noise and the ramp).
    Either may carry ramp_origin, the step count at which its ramp starts.
    Returns (pos, vel, force, log) with log[k] = (E_pot, E_kin, T, T_target)
    of the state after step k.
    """
    r = _pos(pos).copy()
    v = _pos(vel).copy()
    n = len(r)
    f = np.zeros((n, 3)) if force is None else _pos(force).copy()
    th = None
    if thermostat is not None:
        if thermostat.get("kind", "berendsen") == "langevin":
            th = _Thermo(LANGEVIN, float(thermostat["T_start"]), float(thermostat["T_end"]),
                         int(thermostat.get("ramp_steps", 0)), 0.0, float(thermostat["gamma"]),
                         int(thermostat.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF,
                         int(thermostat.get("ramp_origin", 0)))
        else:
            th = _Thermo(BERENDSEN, float(thermostat["T_start"]), float(thermostat["T_end"]),
                         int(thermostat.get("ramp_steps", 0)), float(thermostat["tau"]), 0.0, 0,
                         int(thermostat.get("ramp_origin", 0)))
    log = np.zeros((max(nsteps, 0), 4))
    p = _params(params)
    rc = _load().sco_vv_run(n, _ptr(r), _ptr(v), _ptr(f), 0 if force is None else 1, ctypes.byref(p),
                            float(mass_u), float(dt), int(nsteps), ctypes.byref(th) if th else None,
                            int(step0), _ptr(log) if (nsteps > 0 and with_log) else None, nthreads)
    if rc != 0:
        raise ValueError("invalid trajectory arguments")
    return r, v, f, log


def rdf_counts(pos, dr: float, nbins: int, r_select: float = 0.0):
    """(counts (nbins,) uint64, n_ref): pair-distance histogram of the atoms
    within r_select of the centre of mass (all atoms when r_select <= 0)
    against every other atom; bin = floor(|r_i - r_j| / dr)."""
    r = _pos(pos)
    counts = np.zeros(int(nbins), dtype=np.uint64)
    nref = ctypes.c_int64(0)
    rc = _load().sco_rdf(len(r), _ptr(r), float(r_select), float(dr), int(nbins), _ptr(counts), ctypes.byref(nref))
    if rc != 0:
        raise ValueError("invalid histogram arguments")
    return counts, int(nref.value)


def load_variant(lib_path: str):
    """Bind the same API to another build of the oracle source (used by the
    tests that plant a mistake in a copy of the oracle and check that the
    pins catch it).  Returns a namespace with the module's functions."""
    import types
    lib = _configure(ctypes.CDLL(lib_path))
    ns = types.SimpleNamespace(NI_PARAMS=NI_PARAMS, NI_MASS_U=NI_MASS_U)
    g = globals()
    for name in ("max_threads", "ke_conversion", "kb", "density", "forces", "forces_subset", "energy", "site_energies", "ndof",
                 "kinetic", "temperature", "target_temperature", "berendsen_lambda", "vv_run", "philox4x32_10",
                 "gauss3", "rdf_counts"):
        fn = g[name]
        def bound(*a, _fn=fn, **k):
            global _lib
            saved = _lib
            _lib = lib
            try:
                return _fn(*a, **k)
            finally:
                _lib = saved
        setattr(ns, name, bound)
    return ns
