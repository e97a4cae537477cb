"""ctypes binding of ``libscmd.so`` (declared in ``include/scmd.h``).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Functions keep the C names; a non-zero status raises
:class:`ScmdError` carrying the code and the library's message.  If the
library has not been built this module raises at first use (there is no CPU
fallback): build it with ``python -m paper_1210_3559_amd.build``.

PyTorch is optional and used only for streams and device buffers
(``scmd_create(stream=torch.cuda.current_stream())`` and
``scmd_get_forces_device`` into a CUDA tensor).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libscmd.so")

SCMD_OK = 0
SCMD_EINVAL = -1
SCMD_ENOMEM = -2
SCMD_EDEVICE = -3
SCMD_ENONFINITE = -4
SCMD_ESTATE = -5
SCMD_EBOX = -6
SCMD_EUNSUPPORTED = -7

SCMD_FP64 = 0
SCMD_MIXED = 1
SCMD_ALLPAIRS = 0
SCMD_CELLLIST = 1
SCMD_NVE = 0
SCMD_BERENDSEN = 1
SCMD_LANGEVIN = 2
SCMD_KERNEL_DENSITY = 0
SCMD_KERNEL_FORCE = 1

# Every symbol include/scmd.h declares.
EXPORTS = (
    "scmd_abi_version", "scmd_status_string", "scmd_create", "scmd_destroy", "scmd_init_clusters",
    "scmd_set_potential", "scmd_set_integrator", "scmd_set_thermostat", "scmd_set_langevin", "scmd_set_tuning",
    "scmd_set_cell_skin", "scmd_get_cell_rebuilds",
    "scmd_compute",
    "scmd_step", "scmd_step_async", "scmd_synchronize", "scmd_get_step", "scmd_get_energy",
    "scmd_get_temperature", "scmd_get_positions", "scmd_get_velocities", "scmd_get_forces", "scmd_get_density",
    "scmd_get_forces_device", "scmd_get_state", "scmd_set_state", "scmd_set_profiling", "scmd_get_kernel_time",
    "scmd_set_sampling", "scmd_get_samples", "scmd_rdf", "scmd_rdf_noalloc", "scmd_set_frames", "scmd_record_frame",
    "scmd_get_frame_count", "scmd_diffusion", "scmd_last_error",
)


class ScmdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"scmd status {status}: {message}")
        self.status = status
        self.message = message


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("a", ctypes.c_double), ("c", ctypes.c_double),
                ("n", ctypes.c_int), ("m", ctypes.c_int), ("rc", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("ipt", ctypes.c_int), ("waves_i", ctypes.c_int), ("waves_j", ctypes.c_int),
                ("target_items", ctypes.c_int), ("pairs", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1210_3559_amd.build`")
    # PyTorch-ROCm ships its own HIP runtime (same soname).  Loading torch
    # first makes the library bind to that instance, so one process never
    # holds two HIP runtimes and torch streams/pointers are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "scmd_abi_version": (i32, []),
        "scmd_status_string": (ctypes.c_char_p, [i32]),
        "scmd_create": (i32, [ctypes.POINTER(vp), i32, vp]),
        "scmd_destroy": (i32, [vp]),
        "scmd_init_clusters": (i32, [vp, i32, dp, dp, dp, dbl]),
        "scmd_set_potential": (i32, [vp, ctypes.POINTER(_Params)]),
        "scmd_set_integrator": (i32, [vp, dbl, i32, i32]),
        "scmd_set_thermostat": (i32, [vp, i32, i32, dbl, dbl, i64, dbl]),
        "scmd_set_langevin": (i32, [vp, i32, dbl, dbl, i64, dbl, ctypes.c_uint64]),
        "scmd_set_tuning": (i32, [vp, ctypes.POINTER(_Tuning)]),
        "scmd_set_cell_skin": (i32, [vp, dbl]),
        "scmd_get_cell_rebuilds": (i32, [vp, ctypes.POINTER(i64)]),
        "scmd_compute": (i32, [vp]),
        "scmd_step": (i32, [vp, i64]),
        "scmd_step_async": (i32, [vp, i64]),
        "scmd_synchronize": (i32, [vp]),
        "scmd_get_step": (i32, [vp, ctypes.POINTER(i64)]),
        "scmd_get_energy": (i32, [vp, i32, dp]),
        "scmd_get_temperature": (i32, [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "scmd_get_positions": (i32, [vp, dp]),
        "scmd_get_velocities": (i32, [vp, dp]),
        "scmd_get_forces": (i32, [vp, dp]),
        "scmd_get_density": (i32, [vp, dp]),
        "scmd_get_forces_device": (i32, [vp, vp]),
        "scmd_rdf": (i32, [vp, i32, dbl, dbl, i32, vp, ctypes.POINTER(i64)]),
        "scmd_rdf_noalloc": (i32, [vp, i32, dbl, dbl, i32, vp, vp]),
        "scmd_set_frames": (i32, [vp, i32, i32]),
        "scmd_record_frame": (i32, [vp]),
        "scmd_get_frame_count": (i32, [vp, i32, ctypes.POINTER(i64)]),
        "scmd_diffusion": (i32, [vp, i32, i64, i32, dbl, dbl, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "scmd_get_state": (i32, [vp, vp, ctypes.POINTER(ctypes.c_size_t)]),
        "scmd_set_state": (i32, [vp, vp, ctypes.c_size_t]),
        "scmd_set_profiling": (i32, [vp, i32]),
        "scmd_get_kernel_time": (i32, [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "scmd_set_sampling": (i32, [vp, i64, i32]),
        "scmd_get_samples": (i32, [vp, i32, dp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
        "scmd_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(ctx, status: int):
    if status != SCMD_OK:
        msg = load().scmd_last_error(ctx)
        raise ScmdError(status, msg.decode() if msg else "")
    return status


def _f64(a, shape_tail=(3,)) -> np.ndarray:
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if shape_tail and (arr.ndim != 2 or arr.shape[1] != shape_tail[0]):
        raise ValueError("expected an (n, 3) float64 array")
    return arr


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------
def scmd_abi_version() -> int:
    return load().scmd_abi_version()


def scmd_status_string(status: int) -> str:
    return load().scmd_status_string(status).decode()


def scmd_create(device: int = 0, stream=None):
    """Create a context.  stream: None, a torch.cuda.Stream, or a raw hipStream_t integer."""
    handle = ctypes.c_void_p()
    raw = None
    if stream is not None:
        raw = int(getattr(stream, "cuda_stream", stream)) or None
    _check(None, load().scmd_create(ctypes.byref(handle), device, raw))
    return handle


def scmd_destroy(ctx) -> None:
    load().scmd_destroy(ctx)


def scmd_init_clusters(ctx, offsets, pos, vel=None, mass_u: float = 58.6934) -> None:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    p = _f64(pos)
    v = None if vel is None else _f64(vel)
    if len(off) < 2 or off[-1] != len(p) or (v is not None and len(v) != len(p)):
        raise ValueError("offsets must end at the atom count and vel must match pos")
    _check(ctx, load().scmd_init_clusters(ctx, len(off) - 1, _ptr(off), _ptr(p), None if v is None else _ptr(v),
                                          float(mass_u)))


def scmd_set_potential(ctx, eps=1.5707e-2, a=3.52, c=39.432, n=9, m=6, rc=0.0) -> None:
    prm = _Params(float(eps), float(a), float(c), int(n), int(m), float(rc))
    _check(ctx, load().scmd_set_potential(ctx, ctypes.byref(prm)))


def scmd_set_integrator(ctx, dt_fs: float, precision: int = SCMD_FP64, neighbour: int = SCMD_ALLPAIRS) -> None:
    _check(ctx, load().scmd_set_integrator(ctx, float(dt_fs), int(precision), int(neighbour)))


def scmd_set_thermostat(ctx, cluster: int, kind: int, T_start_K: float = 0.0, T_end_K: float = 0.0,
                        ramp_steps: int = 0, tau_fs: float = 100.0) -> None:
    _check(ctx, load().scmd_set_thermostat(ctx, int(cluster), int(kind), float(T_start_K), float(T_end_K),
                                           int(ramp_steps), float(tau_fs)))


def scmd_set_langevin(ctx, cluster: int, T_start_K: float, T_end_K: float, ramp_steps: int = 0,
                      gamma_per_ps: float = 10.0, seed: int = 0) -> None:
    _check(ctx, load().scmd_set_langevin(ctx, int(cluster), float(T_start_K), float(T_end_K), int(ramp_steps),
                                         float(gamma_per_ps), int(seed) & 0xFFFFFFFFFFFFFFFF))


def scmd_set_tuning(ctx, ipt: int = 0, waves_i: int = 0, waves_j: int = 0, target_items: int = 0,
                    pairs: int = 0) -> None:
    t = _Tuning(int(ipt), int(waves_i), int(waves_j), int(target_items), int(pairs))
    _check(ctx, load().scmd_set_tuning(ctx, ctypes.byref(t)))


def scmd_set_cell_skin(ctx, skin_A: float) -> None:
    _check(ctx, load().scmd_set_cell_skin(ctx, float(skin_A)))


def scmd_get_cell_rebuilds(ctx) -> int:
    n = ctypes.c_int64()
    _check(ctx, load().scmd_get_cell_rebuilds(ctx, ctypes.byref(n)))
    return n.value


def scmd_compute(ctx) -> None:
    _check(ctx, load().scmd_compute(ctx))


def scmd_step(ctx, nsteps: int) -> None:
    _check(ctx, load().scmd_step(ctx, int(nsteps)))


def scmd_step_async(ctx, nsteps: int) -> None:
    _check(ctx, load().scmd_step_async(ctx, int(nsteps)))


def scmd_synchronize(ctx) -> None:
    _check(ctx, load().scmd_synchronize(ctx))


def scmd_get_step(ctx) -> int:
    s = ctypes.c_int64()
    _check(ctx, load().scmd_get_step(ctx, ctypes.byref(s)))
    return s.value


def scmd_get_energy(ctx, cluster: int = -1):
    out = np.zeros(3)
    _check(ctx, load().scmd_get_energy(ctx, int(cluster), _ptr(out)))
    return float(out[0]), float(out[1]), float(out[2])


def scmd_get_temperature(ctx, cluster: int = 0):
    t = ctypes.c_double()
    d = ctypes.c_int64()
    _check(ctx, load().scmd_get_temperature(ctx, int(cluster), ctypes.byref(t), ctypes.byref(d)))
    return t.value, d.value


def scmd_set_sampling(ctx, every: int, capacity: int = 1024) -> None:
    _check(ctx, load().scmd_set_sampling(ctx, int(every), int(capacity)))


def scmd_get_samples(ctx, cluster: int = 0, max_samples: int = 1 << 20):
    """(samples, recorded): samples is an (n, 5) array of step, E_pot, E_kin,
    T, T_target, oldest first; recorded counts every sample taken."""
    out = np.zeros((max(int(max_samples), 1), 5))
    n = ctypes.c_int()
    rec = ctypes.c_int64()
    _check(ctx, load().scmd_get_samples(ctx, int(cluster), _ptr(out), int(max_samples), ctypes.byref(n),
                                        ctypes.byref(rec)))
    return out[: n.value].copy(), rec.value


def _get3(fn, ctx, natoms):
    out = np.zeros((natoms, 3))
    _check(ctx, fn(ctx, _ptr(out)))
    return out


def scmd_get_positions(ctx, natoms: int) -> np.ndarray:
    return _get3(load().scmd_get_positions, ctx, natoms)


def scmd_get_velocities(ctx, natoms: int) -> np.ndarray:
    return _get3(load().scmd_get_velocities, ctx, natoms)


def scmd_get_forces(ctx, natoms: int) -> np.ndarray:
    return _get3(load().scmd_get_forces, ctx, natoms)


def scmd_get_density(ctx, natoms: int) -> np.ndarray:
    out = np.zeros(natoms)
    _check(ctx, load().scmd_get_density(ctx, _ptr(out)))
    return out


def scmd_get_forces_device(ctx, out_tensor) -> None:
    """Write forces into a contiguous float64 CUDA tensor of shape (n, 3) on the context stream."""
    if not out_tensor.is_contiguous() or str(out_tensor.dtype) != "torch.float64":
        raise ValueError("need a contiguous float64 tensor")
    _check(ctx, load().scmd_get_forces_device(ctx, ctypes.c_void_p(out_tensor.data_ptr())))


def scmd_rdf(ctx, cluster: int, dr: float, nbins: int, r_select: float = 0.0, counts=None, n_ref: int = 0):
    """(counts uint64 (nbins,), n_ref): the pair-distance histogram of the
    cluster's current positions, added to `counts` / `n_ref` when given (a
    contiguous uint64 `counts` is updated in place and returned)."""
    out = np.zeros(int(nbins), dtype=np.uint64) if counts is None else np.ascontiguousarray(counts, dtype=np.uint64)
    if out.shape != (int(nbins),):
        raise ValueError("counts must have nbins entries")
    nr = ctypes.c_int64(int(n_ref))
    _check(ctx, load().scmd_rdf(ctx, int(cluster), float(r_select), float(dr), int(nbins),
                                out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nr)))
    return out, int(nr.value)


def scmd_rdf_noalloc(ctx, cluster: int, dr: float, nbins: int, dev_counts, dev_n_ref, r_select: float = 0.0) -> None:
    """Add the pair-distance histogram to device memory without allocating
    or waiting: dev_counts is a contiguous 64-bit CUDA tensor of nbins
    entries, dev_n_ref one of at least 1 entry (or raw device addresses)."""
    def addr(x, need):
        if hasattr(x, "data_ptr"):
            if not x.is_cuda or not x.is_contiguous() or x.element_size() != 8 or x.numel() < need:
                raise ValueError(f"need a contiguous 64-bit CUDA tensor of at least {need} entries")
            return ctypes.c_void_p(x.data_ptr())
        return ctypes.c_void_p(int(x))
    _check(ctx, load().scmd_rdf_noalloc(ctx, int(cluster), float(r_select), float(dr), int(nbins),
                                        addr(dev_counts, int(nbins)), addr(dev_n_ref, 1)))


def scmd_set_frames(ctx, cluster: int, capacity: int) -> None:
    _check(ctx, load().scmd_set_frames(ctx, int(cluster), int(capacity)))


def scmd_record_frame(ctx) -> None:
    _check(ctx, load().scmd_record_frame(ctx))


def scmd_get_frame_count(ctx, cluster: int) -> int:
    n = ctypes.c_int64()
    _check(ctx, load().scmd_get_frame_count(ctx, int(cluster), ctypes.byref(n)))
    return n.value


def scmd_diffusion(ctx, cluster: int, first: int, nframes: int, frame_dt_ps: float, radius: float = 10.0,
                   segments: int = 10):
    """(D in A^2/ps, number of central atoms) from stored frames."""
    d = ctypes.c_double()
    nc = ctypes.c_int64()
    _check(ctx, load().scmd_diffusion(ctx, int(cluster), int(first), int(nframes), float(frame_dt_ps),
                                      float(radius), int(segments), ctypes.byref(d), ctypes.byref(nc)))
    return d.value, nc.value


def scmd_get_state(ctx) -> bytes:
    n = ctypes.c_size_t(0)
    _check(ctx, load().scmd_get_state(ctx, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(ctx, load().scmd_get_state(ctx, buf, ctypes.byref(n)))
    return buf.raw[: n.value]


def scmd_set_state(ctx, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(ctx, load().scmd_set_state(ctx, buf, len(blob)))


def scmd_set_profiling(ctx, enable: bool) -> None:
    _check(ctx, load().scmd_set_profiling(ctx, 1 if enable else 0))


def scmd_get_kernel_time(ctx, kernel: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(ctx, load().scmd_get_kernel_time(ctx, int(kernel), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def scmd_last_error(ctx=None) -> str:
    msg = load().scmd_last_error(ctx)
    return msg.decode() if msg else ""


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------
PRECISIONS = {"fp64": SCMD_FP64, "mixed": SCMD_MIXED}


class Simulation:
    """One context holding a batch of clusters (see inputs.Workload)."""

    def __init__(self, offsets, pos, vel=None, dt: float = 1.0, precision: str = "fp64", rc: float = 0.0,
                 params: dict | None = None, mass_u: float = 58.6934, device: int = 0, stream=None,
                 thermostats=None, tuning: dict | None = None):
        self.ctx = scmd_create(device, stream)
        self.natoms = int(np.asarray(offsets)[-1])
        self.nclusters = len(offsets) - 1
        try:
            scmd_init_clusters(self.ctx, offsets, pos, vel, mass_u)
            p = dict(eps=1.5707e-2, a=3.52, c=39.432, n=9, m=6, rc=rc)
            if params:
                p.update(params)
            scmd_set_potential(self.ctx, **p)
            scmd_set_integrator(self.ctx, dt, PRECISIONS[precision],
                                SCMD_CELLLIST if p["rc"] > 0 else SCMD_ALLPAIRS)
            if tuning == "auto":
                from . import autotune
                tuning = autotune.lookup(offsets, precision, cell=p["rc"] > 0)
            if tuning:
                tuning = dict(tuning)
                if "cell_skin" in tuning:
                    scmd_set_cell_skin(self.ctx, tuning.pop("cell_skin"))
                if tuning:
                    scmd_set_tuning(self.ctx, **tuning)
            for k, th in enumerate(thermostats or []):
                if th is not None:
                    self.set_thermostat(k, th)
        except Exception:
            scmd_destroy(self.ctx)
            self.ctx = None
            raise

    @classmethod
    def from_workload(cls, w, precision: str | None = None, **kw):
        return cls(w.offsets, w.pos, w.vel, dt=w.dt, precision=precision or w.precision, rc=w.rc,
                   thermostats=w.thermostat, **kw)

    def close(self):
        if self.ctx is not None:
            scmd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def compute(self):
        scmd_compute(self.ctx)

    def step(self, n: int):
        scmd_step(self.ctx, n)

    def positions(self):
        return scmd_get_positions(self.ctx, self.natoms)

    def velocities(self):
        return scmd_get_velocities(self.ctx, self.natoms)

    def forces(self):
        return scmd_get_forces(self.ctx, self.natoms)

    def density(self):
        return scmd_get_density(self.ctx, self.natoms)

    def energy(self, cluster: int = -1):
        return scmd_get_energy(self.ctx, cluster)

    def temperature(self, cluster: int = 0):
        return scmd_get_temperature(self.ctx, cluster)

    def set_thermostat(self, cluster: int, th: dict | None):
        """th: None (NVE), dict(T_start, T_end, ramp_steps, tau) for Berendsen,
        or dict(kind="langevin", T_start, T_end, ramp_steps, gamma, seed)."""
        if th is None:
            scmd_set_thermostat(self.ctx, cluster, SCMD_NVE)
        elif th.get("kind", "berendsen") == "langevin":
            scmd_set_langevin(self.ctx, cluster, th["T_start"], th["T_end"], th.get("ramp_steps", 0),
                              th.get("gamma", 10.0), th.get("seed", 0))
        else:
            scmd_set_thermostat(self.ctx, cluster, SCMD_BERENDSEN, th["T_start"], th["T_end"],
                                th.get("ramp_steps", 0), th["tau"])

    def set_cell_skin(self, skin_A: float):
        scmd_set_cell_skin(self.ctx, skin_A)

    def cell_rebuilds(self) -> int:
        return scmd_get_cell_rebuilds(self.ctx)

    def set_sampling(self, every: int, capacity: int = 1024):
        scmd_set_sampling(self.ctx, every, capacity)

    def samples(self, cluster: int = 0, max_samples: int = 1 << 20):
        return scmd_get_samples(self.ctx, cluster, max_samples)

    def rdf(self, cluster: int, dr: float, nbins: int, r_select: float = 0.0, counts=None, n_ref: int = 0):
        return scmd_rdf(self.ctx, cluster, dr, nbins, r_select, counts, n_ref)

    def set_frames(self, cluster: int, capacity: int):
        scmd_set_frames(self.ctx, cluster, capacity)

    def record_frame(self):
        scmd_record_frame(self.ctx)

    def frame_count(self, cluster: int) -> int:
        return scmd_get_frame_count(self.ctx, cluster)

    def diffusion(self, cluster: int, first: int, nframes: int, frame_dt_ps: float, radius: float = 10.0,
                  segments: int = 10):
        return scmd_diffusion(self.ctx, cluster, first, nframes, frame_dt_ps, radius, segments)
