"""Host analysis of the self-diffusion coefficient (Sec. 3, Eq. (diffusion)),
pinned by cases with a closed-form answer: Kabsch superposition recovers a
known rigid motion (and never returns a reflection), a rigidly tumbling and
drifting crystal has D = 0, and independent Gaussian steps of variance s^2
per component per frame give D = s^2 / (2 dt)."""
import numpy as np
import pytest

from paper_1210_3559_amd import diffusion, inputs


def _rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_kabsch_recovers_a_rigid_motion():
    rng = np.random.default_rng(1)
    p = inputs.jitter(inputs.fcc_exact(300), 0.2, rng)
    r0, t0 = _rot(rng), np.array([3.0, -7.5, 0.25])
    q = p @ r0.T + t0
    r, t = diffusion.kabsch(p, q)
    np.testing.assert_allclose(r, r0, atol=1e-12)
    np.testing.assert_allclose(t, t0, atol=1e-11)
    assert np.linalg.det(r) == pytest.approx(1.0)


def test_kabsch_never_reflects():
    rng = np.random.default_rng(2)
    p = rng.normal(size=(50, 3))
    q = p * np.array([1.0, 1.0, -1.0])  # a mirror image
    r, _ = diffusion.kabsch(p, q)
    assert np.linalg.det(r) == pytest.approx(1.0)


def test_rigid_motion_has_no_diffusion():
    rng = np.random.default_rng(3)
    p = inputs.jitter(inputs.fcc_exact(500), 0.05, rng)
    frames = [p @ _rot(rng).T + rng.normal(size=3) * 10 for _ in range(40)]
    d, nc = diffusion.diffusion_coefficient(frames, 10.0, radius=8.0, segments=10)
    assert nc > 20
    assert abs(d) < 1e-20


def test_random_walk_gives_its_diffusion_coefficient():
    rng = np.random.default_rng(4)
    n, nf, s, dt = 3000, 200, 0.3, 10.0
    p0 = rng.uniform(-30, 30, size=(n, 3))
    steps = rng.normal(0, s, size=(nf, n, 3))
    steps[0] = 0.0
    frames = p0 + np.cumsum(steps, axis=0)
    d, nc = diffusion.diffusion_coefficient(frames, dt, radius=1e9, segments=10)
    assert nc == n
    assert d == pytest.approx(s * s / (2.0 * dt), rel=0.03)
    # and in the paper's units
    assert d * diffusion.A2_PER_PS_TO_CM2_PER_S == pytest.approx(s * s / (2.0 * dt) * 1e-4, rel=0.03)
