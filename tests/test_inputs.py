"""Input generators: structure sizes, symmetry and momentum of the seeded workloads."""
import json
import os

import numpy as np
import pytest

from paper_1210_3559_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reference_values.json")))


def test_mackay_magic_numbers():
    sizes = [len(inputs.mackay_icosahedron(k)) for k in range(0, 6)]
    assert sizes == GOLDEN["mackay_magic_numbers"]["values"][:6]
    assert inputs.mackay_size(8) == 2057


def test_mackay_geometry():
    p = inputs.mackay_icosahedron(3, 2.49)
    d = np.linalg.norm(p[:, None] - p[None], axis=-1)
    np.fill_diagonal(d, np.inf)
    assert d.min() == pytest.approx(2.49, rel=1e-12)
    assert np.abs(p.mean(axis=0)).max() < 1e-12
    # 12 neighbours of the centre on the first shell
    assert np.sum(np.isclose(d[0], 2.49)) == 12


def test_fcc_sphere_counts():
    # origin on a site: shell counts of fcc 1, 12, 6, 24, 12, ...
    assert len(inputs.fcc_sphere(3.52 / np.sqrt(2) + 1e-6)) == 13
    assert len(inputs.fcc_sphere(3.52 + 1e-6)) == 19
    assert len(inputs.fcc_sphere(18.0)) == 2243
    assert len(inputs.fcc_sphere(50.0)) == 48077


def test_fcc_exact_is_prefix_of_ordered_sites():
    p = inputs.fcc_exact(15000)
    assert p.shape == (15000, 3)
    r2 = np.einsum("ij,ij->i", p, p)
    assert np.all(np.diff(np.round(r2, 9)) >= 0)
    assert len(np.unique(np.round(p, 9), axis=0)) == 15000
    q = inputs.fcc_exact(15001)
    np.testing.assert_array_equal(q[:15000], p)


def test_maxwell_boltzmann_momentum_free():
    p = inputs.jitter(inputs.fcc_exact(500), 0.05, np.random.default_rng(1))
    v = inputs.maxwell_boltzmann(p, 1200.0, np.random.default_rng(2))
    assert np.abs(v.sum(axis=0)).max() < 1e-13
    L = np.cross(p - p.mean(axis=0), v).sum(axis=0)
    assert np.abs(L).max() < 1e-11


def test_seeded_workloads_are_deterministic():
    a, b = inputs.c2_cooling(), inputs.c2_cooling()
    np.testing.assert_array_equal(a.pos, b.pos)
    np.testing.assert_array_equal(a.vel, b.vel)
    assert a.n_atoms == 2243 and a.dt == 2.0
    assert a.thermostat[0] == dict(T_start=2000.0, T_end=800.0, ramp_steps=200000, tau=100.0)
    assert np.abs(a.pos - inputs.fcc_sphere(18.0)).max() <= 0.05


def test_batch_sizes_log_uniform():
    s = inputs.batch_sizes(256, 355900)
    assert s.min() >= 147 and s.max() <= 6000
    # log-uniform: the median sits near the geometric mean of the range
    assert 0.6 < np.median(s) / np.sqrt(147 * 6000) < 1.5
