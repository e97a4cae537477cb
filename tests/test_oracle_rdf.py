"""Pins of the oracle's pair-distance histogram (the radial distribution
function of Sec. 3, Eq. (Rdist)) against facts fixed outside its code: the
fcc neighbour-shell multiplicities (12, 6, 24, 12, 24, 8, 48, 6, 36, 24 at
distances a sqrt(k/2), k = 1..10; standard crystallography tables), the
total pair count, the dimer and equilateral trimer, the Mackay shells and
invariance under rigid motions and relabelling."""
import math

import numpy as np
import pytest

from paper_1210_3559_amd import inputs

A = 3.52
FCC_SHELLS = [12, 6, 24, 12, 24, 8, 48, 6, 36, 24]


def test_fcc_central_atom_shells(oracle_mod):
    pos = inputs.fcc_sphere(14.0)
    dr = 0.05
    counts, nref = oracle_mod.rdf_counts(pos, dr, 400, r_select=0.5)
    assert nref == 1
    for k, m in enumerate(FCC_SHELLS, start=1):
        b = int(math.floor(A * math.sqrt(k / 2.0) / dr))
        assert counts[b] == m, (k, counts[b - 1:b + 2])
    # nothing between the shells
    shells = {int(math.floor(A * math.sqrt(k / 2.0) / dr)) for k in range(1, 11)}
    r10 = A * math.sqrt(10 / 2.0)
    for b in range(int(r10 / dr)):
        if b not in shells:
            assert counts[b] == 0, b


def test_total_count_is_every_ordered_pair(oracle_mod):
    pos = inputs.jitter(inputs.fcc_exact(300), 0.1, np.random.default_rng(3))
    counts, nref = oracle_mod.rdf_counts(pos, 0.3, 200)  # 60 A covers the cluster
    assert nref == 300
    assert int(counts.sum()) == 300 * 299
    # a selection keeps its atoms' pairs only
    counts, nref = oracle_mod.rdf_counts(pos, 0.3, 200, r_select=6.0)
    assert 0 < nref < 300 and int(counts.sum()) == nref * 299


def test_dimer_and_trimer(oracle_mod):
    r = 2.6183
    counts, nref = oracle_mod.rdf_counts(np.array([[0.0, 0, 0], [r, 0, 0]]), 0.1, 50)
    assert nref == 2 and counts[int(r / 0.1)] == 2 and counts.sum() == 2
    s = 2.49
    tri = np.array([[0.0, 0, 0], [s, 0, 0], [0.5 * s, 0.5 * math.sqrt(3.0) * s, 0]])
    counts, nref = oracle_mod.rdf_counts(tri, 0.2, 50)
    assert nref == 3 and counts[int(s / 0.2)] == 6 and counts.sum() == 6


def test_mackay_selection(oracle_mod):
    pos = inputs.mackay_icosahedron(3, 2.49)
    _, n0 = oracle_mod.rdf_counts(pos, 0.1, 100, r_select=1.0)
    _, n1 = oracle_mod.rdf_counts(pos, 0.1, 100, r_select=2.6)
    _, n2 = oracle_mod.rdf_counts(pos, 0.1, 100, r_select=5.1)
    assert (n0, n1, n2) == (1, 13, 55)
    counts, _ = oracle_mod.rdf_counts(pos, 0.01, 400, r_select=1.0)
    assert counts[int(2.49 / 0.01)] == 12  # the central atom's first shell


def test_invariant_under_rigid_motion_and_relabelling(oracle_mod):
    rng = np.random.default_rng(8)
    pos = inputs.jitter(inputs.fcc_exact(200), 0.2, rng)
    base, nref = oracle_mod.rdf_counts(pos, 0.37, 60, r_select=7.0)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    moved = pos[rng.permutation(len(pos))] @ q.T + np.array([13.1, -4.2, 7.7])
    other, nref2 = oracle_mod.rdf_counts(moved, 0.37, 60, r_select=7.0)
    assert nref2 == nref
    # a pair may move across a bin edge by rounding: allow that and no more
    assert np.abs(other.astype(np.int64) - base.astype(np.int64)).sum() <= 4
