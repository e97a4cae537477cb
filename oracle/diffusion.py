"""Self-diffusion coefficient of the central atoms of a cluster: plain NumPy
oracle (test infrastructure; only tests/ and bench.py's CPU-baseline leg use
this package).

Definition (Yakubovich et al., arXiv:1210.3559, Sec. 3, "Diffusion
coefficient as a fingerprint of solidification phase transition",
Eq. (diffusion)): D = <dr^2> / (2 z dt) with z = 3.  The paper's procedure,
step by step:

1. every recorded structure of the window is translated and rotated as a
   whole so that the root-mean-square displacement of its atoms from a
   reference structure is smallest (here: the first frame of the window is
   the reference; the optimal rotation is Kabsch's, from the singular value
   decomposition of the 3x3 cross-covariance, restricted to proper
   rotations);
2. the window is split into `segments` (the paper: 10) equal parts;
3. for the atoms within `radius` (the paper: 10 A) of the centre of mass,
   dr^2 is the squared displacement between the first and the last frame of
   a segment and dt the time between those two frames;
4. D is the average over those atoms and the segments.

Readings (the paper does not say): the centre of mass and the central atoms
are those of the reference frame; with F frames and S segments each segment
holds floor(F / S) consecutive frames (trailing frames unused), so its
dt is (floor(F / S) - 1) frame intervals.

Pinned in tests/test_oracle_diffusion.py by closed forms: a known rigid
motion is recovered, a mirror image never yields a reflection, a rigidly
tumbling and drifting crystal has D = 0, independent Gaussian steps of
variance s^2 per component and frame give D = s^2 / (2 dt_frame), and only
the central atoms count.
"""
from __future__ import annotations

import numpy as np


def optimal_rigid_motion(moving, reference):
    """Proper rotation R and translation t minimising sum |R p_i + t - q_i|^2
    (p: moving, q: reference, both (N, 3))."""
    p = np.asarray(moving, dtype=np.float64)
    q = np.asarray(reference, dtype=np.float64)
    pc = p.mean(axis=0)
    qc = q.mean(axis=0)
    h = (p - pc).T @ (q - qc)          # cross-covariance sum p'_a q'_b
    u, _, vt = np.linalg.svd(h)
    v = vt.T
    d = 1.0 if np.linalg.det(v @ u.T) >= 0.0 else -1.0
    rot = v @ np.diag([1.0, 1.0, d]) @ u.T
    return rot, qc - rot @ pc


def diffusion(frames, dt_ps: float, radius: float = 10.0, segments: int = 10):
    """(D in A^2/ps, number of central atoms) from frames (F, N, 3) taken
    dt_ps apart, following the steps in the module comment."""
    fr = np.asarray(frames, dtype=np.float64)
    if fr.ndim != 3 or fr.shape[2] != 3:
        raise ValueError("frames must have shape (F, N, 3)")
    nf = fr.shape[0]
    seg = nf // segments if segments > 0 else 0
    if seg < 2:
        raise ValueError("need at least two frames per segment")
    ref = fr[0]
    # step 1: every frame superimposed on the reference
    moved = np.empty_like(fr)
    for k in range(nf):
        rot, t = optimal_rigid_motion(fr[k], ref)
        moved[k] = fr[k] @ rot.T + t
    # central atoms of the reference frame
    com = ref.mean(axis=0)
    central = np.nonzero(np.linalg.norm(ref - com, axis=1) < radius)[0]
    if len(central) == 0:
        raise ValueError("no atom within radius of the centre of mass")
    # steps 2-4
    d = []
    for s in range(segments):
        first, last = s * seg, (s + 1) * seg - 1
        dr2 = np.sum((moved[last, central] - moved[first, central]) ** 2, axis=1)
        d.append(np.mean(dr2) / (2.0 * 3.0 * (last - first) * dt_ps))
    return float(np.mean(d)), int(len(central))
