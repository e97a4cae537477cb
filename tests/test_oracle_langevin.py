"""Pins of the oracle's Langevin bath (the paper's thermostat, Sec. 2
"Computational approach": damping constant 10 1/ps), integrated with BAOAB.

What fixes each expected value:
  * the noise generator: the published Philox4x32-10 known-answer blocks
    (tests/golden/philox4x32_10_kat.json) and, for the Box-Muller deviates,
    the normal law (moments, Kolmogorov-Smirnov against scipy's normal CDF)
    and the polar structure that tells which word feeds which deviate;
  * the B and A parts: zero damping reduces BAOAB to velocity-Verlet, which
    the NVE pins already fix;
  * the O part: a free atom in a bath at 0 K decays as exp(-gamma t) and
    travels (dt/2) v0 (1 + c1)(1 - c1^s)/(1 - c1) (geometric series);
  * the noise amplitude and the 3N degrees of freedom: free atoms reach the
    bath temperature exactly (the Ornstein-Uhlenbeck stationary variance is
    k_B T/m for any dt), and a nickel cluster reaches it up to the O(dt^2)
    bias of BAOAB's kinetic temperature.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_1210_3559_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")))
GAMMA = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reference_values.json")))[
    "paper_md_settings"]["langevin_damping_per_ps"]

# CODATA 2018 / SI 2019 constants: k_B/e in eV/K and u*A^2/fs^2 in eV.
KB = 1.380649e-23 / 1.602176634e-19
KE = 1.66053906660e-27 * 1e-20 / 1e-30 / 1.602176634e-19
MASS = 58.6934


def _langevin(T, gamma=GAMMA, seed=7, ramp=0, T_start=None):
    return dict(kind="langevin", T_start=T if T_start is None else T_start, T_end=T, ramp_steps=ramp,
                gamma=gamma, seed=seed)


def _free_atoms(k, spacing=4000.0):
    g = np.arange(k) * spacing
    return np.array([[x, y, z] for x in g for y in g for z in g], dtype=np.float64)


def test_philox_known_answers(oracle_mod):
    for v in GOLDEN["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert oracle_mod.philox4x32_10(ctr, key) == tuple(int(x, 16) for x in v["out"])


def test_noise_is_standard_normal(oracle_mod):
    # 40,000 atoms x 3 deviates at one step, and one atom over 20,000 steps
    a = np.array([oracle_mod.gauss3(11, 5, i) for i in range(40000)])
    b = np.array([oracle_mod.gauss3(11, s, 3) for s in range(1, 20001)])
    for x in (a.ravel(), b.ravel(), a[:, 2]):
        n = len(x)
        assert abs(x.mean()) < 5.0 / math.sqrt(n)
        assert abs(x.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
        assert abs(stats.skew(x)) < 5.0 * math.sqrt(6.0 / n)
        assert abs(stats.kurtosis(x)) < 5.0 * math.sqrt(24.0 / n)
        assert stats.kstest(x, "norm").pvalue > 1e-4
    # the three components are uncorrelated, and so are neighbouring atoms
    c = np.corrcoef(a.T)
    assert np.max(np.abs(c - np.eye(3))) < 5.0 / math.sqrt(len(a))
    assert abs(np.corrcoef(a[:-1, 0], a[1:, 0])[0, 1]) < 5.0 / math.sqrt(len(a))
    # other seeds and steps give other numbers
    assert not np.array_equal(oracle_mod.gauss3(11, 5, 0), oracle_mod.gauss3(12, 5, 0))
    assert not np.array_equal(oracle_mod.gauss3(11, 5, 0), oracle_mod.gauss3(11, 6, 0))
    assert not np.array_equal(oracle_mod.gauss3(11, 1 << 32, 0), oracle_mod.gauss3(11, 0, 0))


def test_noise_box_muller_structure(oracle_mod):
    # (x, y) come from words 0 and 1 of the block with key (seed lo, seed hi)
    # and counter (atom, 0, step lo, step hi): x^2 + y^2 = -2 ln u0 and the
    # polar angle is 2 pi u1; z = sqrt(-2 ln u2) cos(2 pi u3)
    for seed, step, atom in [(0, 1, 0), (2 ** 40 + 3, 7, 12345), (99, 2 ** 33 + 5, 2)]:
        w = oracle_mod.philox4x32_10([atom, 0, step & 0xFFFFFFFF, step >> 32], [seed & 0xFFFFFFFF, seed >> 32])
        u = [(x + 0.5) / 2.0 ** 32 for x in w]
        g = oracle_mod.gauss3(seed, step, atom)
        assert g[0] ** 2 + g[1] ** 2 == pytest.approx(-2.0 * math.log(u[0]), rel=1e-13)
        ang = math.atan2(g[1], g[0]) % (2.0 * math.pi)
        assert ang == pytest.approx(2.0 * math.pi * u[1], rel=1e-12, abs=1e-12)
        rz = math.sqrt(-2.0 * math.log(u[2]))
        assert abs(g[2]) <= rz * (1 + 1e-15)
        assert math.acos(g[2] / rz) == pytest.approx(min(2 * math.pi * u[3], 2 * math.pi * (1 - u[3])), abs=1e-7)


def test_zero_damping_is_velocity_verlet(oracle_mod):
    st = inputs.c1_icosahedron()
    r0, v0 = st.pos, st.vel
    rn, vn, _, ln = oracle_mod.vv_run(r0, v0, 40, dt=1.0, nthreads=4)
    rl, vl, _, ll = oracle_mod.vv_run(r0, v0, 40, dt=1.0, thermostat=_langevin(900.0, gamma=0.0), nthreads=4)
    np.testing.assert_allclose(rl, rn, rtol=0, atol=1e-10)
    np.testing.assert_allclose(vl, vn, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ll[:, 0], ln[:, 0], rtol=1e-12)
    # T counts 3N degrees of freedom under the bath, 3N - 6 without it
    n = len(r0)
    np.testing.assert_allclose(ll[:, 2], ln[:, 2] * (3 * n - 6) / (3 * n), rtol=1e-9)
    np.testing.assert_allclose(ll[:, 3], 900.0)


@pytest.mark.parametrize("dt", [1.0, 2.5])
def test_free_atom_decays_in_a_cold_bath(oracle_mod, dt):
    # one atom: no forces; at T = 0 the O step is v <- c1 v exactly
    r0 = np.array([[1.0, -2.0, 0.5]])
    v0 = np.array([[0.012, -0.004, 0.007]])
    s = 300
    r, v, f, log = oracle_mod.vv_run(r0, v0, s, dt=dt, thermostat=_langevin(0.0))
    assert not f.any()
    c1 = math.exp(-GAMMA * 1e-3 * dt)
    np.testing.assert_allclose(v, v0 * c1 ** s, rtol=1e-12)
    travel = 0.5 * dt * (1.0 + c1) * (1.0 - c1 ** s) / (1.0 - c1)
    np.testing.assert_allclose(r, r0 + travel * v0, rtol=1e-12)
    np.testing.assert_allclose(log[:, 1], 0.5 * MASS * KE * (v0 ** 2).sum() * c1 ** (2 * np.arange(1, s + 1)),
                               rtol=1e-11)


def test_free_atoms_reach_bath_temperature(oracle_mod):
    # 8 atoms 4000 A apart (forces below 1e-12 eV/A): the velocity of each
    # component is an Ornstein-Uhlenbeck chain whose stationary variance is
    # k_B T/m for any time step, so <E_kin> = (3N/2) k_B T and <T> = T
    pos = _free_atoms(2)
    f, _, _ = oracle_mod.forces(pos)
    assert np.abs(f).max() < 1e-12
    T = 700.0
    nsteps = 120000
    _, v, _, log = oracle_mod.vv_run(pos, np.zeros_like(pos), nsteps, dt=2.0, thermostat=_langevin(T, seed=3))
    tail = log[2000:]
    n = len(pos)
    # correlation time of v^2 is 1/(2 gamma) = 50 fs = 25 steps
    neff = len(tail) / 50.0
    sd = math.sqrt(2.0 / (3 * n)) / math.sqrt(neff)
    assert tail[:, 1].mean() == pytest.approx(1.5 * n * KB * T, rel=5 * sd)
    assert tail[:, 2].mean() == pytest.approx(T, rel=5 * sd)
    np.testing.assert_allclose(tail[:, 3], T)


def test_noise_follows_the_step_count(oracle_mod):
    # a trajectory split in two calls (step0) is the same trajectory
    st = inputs.c1_icosahedron()
    th = _langevin(800.0, seed=21, ramp=50, T_start=1200.0)
    r1, v1, f1, l1 = oracle_mod.vv_run(st.pos, st.vel, 30, thermostat=th, nthreads=4)
    ra, va, fa, la = oracle_mod.vv_run(st.pos, st.vel, 12, thermostat=th, nthreads=4)
    rb, vb, fb, lb = oracle_mod.vv_run(ra, va, 18, thermostat=th, step0=12, force=fa, nthreads=4)
    assert np.array_equal(r1, rb) and np.array_equal(v1, vb)
    assert np.array_equal(l1, np.concatenate([la, lb]))
    # the ramp of the bath temperature is indexed like the Berendsen target
    # (the step being completed, counted from 1)
    _, _, _, lber = oracle_mod.vv_run(st.pos, st.vel, 30, nthreads=4,
                                      thermostat=dict(T_start=1200.0, T_end=800.0, ramp_steps=50, tau=100.0))
    np.testing.assert_array_equal(l1[:, 3], lber[:, 3])
    # and a different seed gives a different trajectory
    r2, _, _, _ = oracle_mod.vv_run(st.pos, st.vel, 30, thermostat=dict(th, seed=22), nthreads=4)
    assert np.abs(r2 - r1).max() > 1e-6


def test_cluster_reaches_bath_temperature(oracle_mod):
    # Mackay Ni147 started cold in a 600 K bath: after 10 damping times the
    # mean kinetic temperature is the bath's (BAOAB's kinetic bias at 1 fs
    # is ~(gamma dt)^2 / 12 and far below the statistical error here)
    st = inputs.c1_icosahedron()
    T = 600.0
    _, _, _, log = oracle_mod.vv_run(st.pos, np.zeros_like(st.vel), 8000, dt=1.0,
                                     thermostat=_langevin(T, seed=5), nthreads=8)
    tail = log[1000:, 2]
    n = len(st.pos)
    # block means over 200 fs give the error of the mean
    blocks = tail[: len(tail) // 200 * 200].reshape(-1, 200).mean(axis=1)
    sem = blocks.std(ddof=1) / math.sqrt(len(blocks))
    assert sem < 0.02 * T
    assert tail.mean() == pytest.approx(T, abs=max(4 * sem, 0.01 * T))
    # and equipartition in the fluctuations: std(T)/T = sqrt(2/(3N)) for
    # independent Maxwell-Boltzmann velocities
    assert tail.std() / T == pytest.approx(math.sqrt(2.0 / (3 * n)), rel=0.25)
