"""Self-diffusion coefficient of the central atoms of a cluster (the paper's
Sec. 3, "Diffusion coefficient as a fingerprint of solidification phase
transition", Eq. (diffusion): D = <dr^2> / (2 z dt), z = 3).

Frames (positions of one cluster at equal time intervals) are first
superimposed on a reference frame by the translation and rotation that
minimise the RMS displacement (Kabsch's construction), which removes the
cluster's overall motion; the window of frames is split into segments, and D
is the mean squared displacement of the atoms within `radius` of the centre
of mass (in the reference frame) from the first to the last frame of each
segment, divided by 6 times its duration, averaged over atoms and segments.

This is host-side analysis of frames read from the device (a few O(N)
passes and a 3x3 SVD per frame).
"""
from __future__ import annotations

import numpy as np

A2_PER_PS_TO_CM2_PER_S = 1e-4  # 1 A^2/ps = 1e-16 cm^2 / 1e-12 s


def kabsch(p: np.ndarray, q: np.ndarray):
    """Rotation R and translation t with R p_i + t closest to q_i in the least
    squares sense (proper rotation, det R = +1)."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    pc, qc = p.mean(axis=0), q.mean(axis=0)
    h = (p - pc).T @ (q - qc)
    u, _, vt = np.linalg.svd(h)
    d = np.sign(np.linalg.det(vt.T @ u.T))
    r = vt.T @ np.diag([1.0, 1.0, d]) @ u.T
    return r, qc - r @ pc


def superpose(frames, ref: np.ndarray) -> np.ndarray:
    """Every frame moved rigidly onto ref (array of shape (F, N, 3))."""
    out = []
    for f in frames:
        r, t = kabsch(f, ref)
        out.append(np.asarray(f, dtype=np.float64) @ r.T + t)
    return np.stack(out)


def diffusion_coefficient(frames, dt_ps: float, radius: float = 10.0, segments: int = 10):
    """D in A^2/ps from F frames dt_ps apart (see the module comment); returns
    (D, number of central atoms)."""
    fr = np.asarray(frames, dtype=np.float64)
    if fr.ndim != 3 or fr.shape[0] < 2 * segments or fr.shape[2] != 3:
        raise ValueError("need (F, N, 3) frames with F >= 2 * segments")
    al = superpose(fr, fr[0])
    c = al[0].mean(axis=0)
    central = np.nonzero(np.sqrt(((al[0] - c) ** 2).sum(axis=1)) < radius)[0]
    if len(central) == 0:
        raise ValueError("no atom within radius of the centre of mass")
    seg = fr.shape[0] // segments
    ds = []
    for s in range(segments):
        a, b = s * seg, (s + 1) * seg - 1
        msd = ((al[b, central] - al[a, central]) ** 2).sum(axis=1).mean()
        ds.append(msd / (6.0 * (b - a) * dt_ps))
    return float(np.mean(ds)), int(len(central))
