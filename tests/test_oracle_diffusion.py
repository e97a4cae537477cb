"""Pins of the oracle's diffusion coefficient (Sec. 3, Eq. (diffusion)) by
closed forms and invariants; none of them re-types the oracle's formula."""
import numpy as np
import pytest

from oracle import diffusion as odiff
from paper_1210_3559_amd import inputs


def _rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_optimal_motion_recovers_a_rigid_motion():
    rng = np.random.default_rng(1)
    p = inputs.jitter(inputs.fcc_exact(300), 0.2, rng)
    r0, t0 = _rot(rng), np.array([3.0, -7.5, 0.25])
    q = p @ r0.T + t0
    r, t = odiff.optimal_rigid_motion(p, q)
    np.testing.assert_allclose(r, r0, atol=1e-12)
    np.testing.assert_allclose(t, t0, atol=1e-11)


def test_optimal_motion_is_never_a_reflection():
    rng = np.random.default_rng(2)
    p = rng.normal(size=(50, 3))
    q = p * np.array([1.0, 1.0, -1.0])  # a mirror image
    r, _ = odiff.optimal_rigid_motion(p, q)
    assert np.linalg.det(r) == pytest.approx(1.0)
    np.testing.assert_allclose(r @ r.T, np.eye(3), atol=1e-12)


def test_optimal_motion_beats_nearby_motions():
    # the least-squares optimum: small perturbations of R (kept proper) and t
    # never lower the residual
    rng = np.random.default_rng(5)
    p = rng.normal(size=(80, 3)) * 5
    q = p @ _rot(rng).T + rng.normal(size=(80, 3)) * 0.3 + 2.0
    r, t = odiff.optimal_rigid_motion(p, q)
    best = np.sum((p @ r.T + t - q) ** 2)
    for _ in range(50):
        w = rng.normal(size=3) * 1e-3
        k = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        dr = np.linalg.qr(np.eye(3) + k)[0]
        dr = dr @ np.diag(np.sign(np.diag(np.linalg.qr(np.eye(3) + k)[1])))
        alt = np.sum((p @ (dr @ r).T + t + rng.normal(size=3) * 1e-3 - q) ** 2)
        assert alt >= best - 1e-9


def test_rigid_tumbling_crystal_has_no_diffusion():
    rng = np.random.default_rng(3)
    p = inputs.jitter(inputs.fcc_exact(500), 0.05, rng)
    frames = [p @ _rot(rng).T + rng.normal(size=3) * 10 for _ in range(40)]
    d, nc = odiff.diffusion(frames, 10.0, radius=8.0, segments=10)
    assert nc > 20
    assert abs(d) < 1e-20


def test_random_walk_gives_its_diffusion_coefficient():
    # independent Gaussian steps of variance s^2 per component and frame:
    # <dr^2> = 3 s^2 per frame interval, D = s^2 / (2 dt)
    rng = np.random.default_rng(4)
    n, nf, s, dt = 3000, 200, 0.3, 10.0
    p0 = rng.uniform(-30, 30, size=(n, 3))
    steps = rng.normal(0, s, size=(nf, n, 3))
    steps[0] = 0.0
    frames = p0 + np.cumsum(steps, axis=0)
    d, nc = odiff.diffusion(frames, dt, radius=1e9, segments=10)
    assert nc == n
    assert d == pytest.approx(s * s / (2.0 * dt), rel=0.03)


def test_only_central_atoms_count():
    # a rigid core inside a shell of walkers: within the core radius D = 0;
    # with the shell included D > 0
    rng = np.random.default_rng(6)
    core = inputs.fcc_exact(200)
    shell = rng.normal(size=(300, 3))
    shell = 25.0 * shell / np.linalg.norm(shell, axis=1, keepdims=True)
    nf = 40
    frames = []
    walk = np.zeros_like(shell)
    for _ in range(nf):
        frames.append(np.concatenate([core, shell + walk]))
        # walkers move tangentially and in balanced pairs, so the centre of
        # mass and the best superposition stay those of the core
        step = rng.normal(size=(150, 3)) * 0.2
        walk = walk + np.concatenate([step, -step])
    d_core, nc = odiff.diffusion(frames, 1.0, radius=8.0, segments=4)
    assert nc == int(np.sum(np.linalg.norm(core - np.concatenate([core, shell]).mean(0), axis=1) < 8.0))
    d_all, _ = odiff.diffusion(frames, 1.0, radius=1e9, segments=4)
    assert d_all > 1e3 * max(abs(d_core), 1e-12)


def test_segment_time_and_dimension():
    # uniform drift of the central atoms relative to a fixed frame is not
    # removed when it is not rigid: two atoms moving apart at speed u each
    # along x (and a heavy fixed body that pins the superposition)
    body = inputs.fcc_exact(400) * 1.0
    nf, u, dt = 30, 0.01, 2.0
    frames = []
    for k in range(nf):
        a = np.array([[0.0, 0.0, 0.0]]) + [u * k, 0, 0]
        b = np.array([[0.0, 0.0, 0.0]]) - [u * k, 0, 0]
        frames.append(np.concatenate([body + [100.0, 0, 0], a, b]))
    frames = np.array(frames)
    # radius selects the two movers only (centre of mass is near the body,
    # so select by a large radius excluding nothing, then compare with the
    # closed form for the whole set)
    d, nc = odiff.diffusion(frames, dt, radius=1e9, segments=3)
    # per segment (10 frames, 9 intervals): each mover moves 9u along x; the
    # body is rigid; superposition on the body leaves the movers' motion
    # (up to the tiny pull they exert on the least-squares fit)
    seg = nf // 3
    expect = 2 * (u * (seg - 1)) ** 2 / (len(frames[0]) * 6.0 * (seg - 1) * dt)
    assert d == pytest.approx(expect, rel=2e-2)
