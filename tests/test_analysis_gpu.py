"""GPU parity of the on-device pair-distance histogram (radial distribution
function, Sec. 3 Eq. (Rdist)) against the oracle, bit for bit: the bin of a
pair is floor(sqrt(dx*dx + dy*dy + dz*dz) / dr) in IEEE double on both
sides, and counts are integers.  Perfect lattices put many distances exactly
on bin edges (2.49 A / 0.01 A), which only agree when both sides round every
operation correctly.  Reference selection (within r_select of the centre of
mass) is checked to be away from ties before comparing."""
import numpy as np
import pytest

import oracle
from paper_1210_3559_amd import inputs
from paper_1210_3559_amd import scmd

pytestmark = pytest.mark.gpu


def _no_selection_tie(pos, r_select, margin=1e-9):
    if r_select <= 0 or len(pos) == 0:
        return True
    c = pos.mean(axis=0)
    d = np.sqrt(((pos - c) ** 2).sum(axis=1))
    return np.all(np.abs(d - r_select) > margin)


def _check(sim, k, pos, dr, nbins, r_select):
    assert _no_selection_tie(pos, r_select)
    got, nr = sim.rdf(k, dr, nbins, r_select)
    ref, nref = oracle.rdf_counts(pos, dr, nbins, r_select)
    assert nr == nref
    np.testing.assert_array_equal(got, ref)
    return got, nr


CASES = [
    ("fcc_jitter", 1, 0.1, 64, 0.0), ("fcc_jitter", 2, 0.1, 64, 0.0), ("fcc_jitter", 3, 0.1, 64, 0.0),
    ("fcc_jitter", 64, 0.1, 200, 0.0), ("fcc_jitter", 257, 0.37, 100, 5.5), ("fcc_jitter", 1000, 0.4, 120, 3.0),
    ("fcc_jitter", 2243, 0.05, 1200, 0.0), ("fcc_sphere", 12.0, 0.05, 500, 0.5), ("fcc_sphere", 12.0, 0.01, 2500, 7.9),
    ("mackay", 3, 0.01, 1200, 0.0), ("mackay", 8, 0.4, 100, 3.0), ("mackay", 8, 0.01, 4000, 11.0),
]


@pytest.mark.parametrize("kind,size,dr,nbins,r_select", CASES)
def test_rdf_counts_match_oracle_exactly(kind, size, dr, nbins, r_select):
    if kind == "fcc_jitter":
        pos = inputs.jitter(inputs.fcc_exact(size), 0.07, np.random.default_rng(size))
    elif kind == "fcc_sphere":
        pos = inputs.fcc_sphere(size)
    else:
        pos = inputs.mackay_icosahedron(size, 2.49)
    print(f"[rdf] {kind} {size} dr={dr} nbins={nbins} r_select={r_select}", flush=True)
    with scmd.Simulation(np.array([0, len(pos)]), pos, None) as sim:
        got, nr = _check(sim, 0, pos, dr, nbins, r_select)
        # a second call adds to the first (in place: a uint64 array passed in
        # is the one returned)
        acc = got.copy()
        again, nr2 = sim.rdf(0, dr, nbins, r_select, counts=acc, n_ref=nr)
        assert again is acc
        np.testing.assert_array_equal(again, 2 * got)
        assert nr2 == 2 * nr


def test_rdf_of_each_batch_cluster_after_steps():
    # positions after fused row steps (batch) are the ones analysed
    sizes = [147, 0, 530, 2057]
    rng = np.random.default_rng(12)
    parts = [inputs.jitter(inputs.fcc_exact(n), 0.05, rng) for n in sizes]
    vels = [inputs.maxwell_boltzmann(p, 900.0, rng) if len(p) else np.zeros((0, 3)) for p in parts]
    off = np.concatenate([[0], np.cumsum(sizes)])
    print("[rdf] batch after 37 steps", flush=True)
    with scmd.Simulation(off, np.concatenate(parts), np.concatenate(vels), dt=1.0) as sim:
        sim.step(37)
        pos = sim.positions()
        for k in range(len(sizes)):
            p = pos[off[k]:off[k + 1]]
            _check(sim, k, p, 0.2, 150, 0.0 if k != 3 else 9.0)


def test_rdf_argument_errors():
    pos = inputs.fcc_exact(20)
    with scmd.Simulation(np.array([0, 20]), pos, None) as sim:
        for args in [(1, 0.1, 10), (-1, 0.1, 10), (0, 0.0, 10), (0, -0.1, 10), (0, np.inf, 10), (0, 0.1, 0),
                     (0, 0.1, 40000)]:
            with pytest.raises(scmd.ScmdError) as e:
                sim.rdf(*args)
            assert e.value.status == scmd.SCMD_EINVAL
        with pytest.raises(scmd.ScmdError):
            sim.rdf(0, 0.1, 10, r_select=np.nan)
