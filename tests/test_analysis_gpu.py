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


# ---------------------------------------------------------------------------
# Diffusion coefficient (Sec. 3, Eq. (diffusion)) from the device frame store
# against the oracle's SVD-based superposition on the same frames.  The two
# sides find the optimal rotation by different methods (quaternion
# eigenvector on the device, singular value decomposition in the oracle) and
# sum in different orders, so D agrees to rounding (1e-9 relative); the
# number of central atoms is exact once no atom sits within 1e-9 A of the
# radius sphere.
# ---------------------------------------------------------------------------
def _central_tie_free(ref, radius, margin=1e-9):
    d = np.sqrt(((ref - ref.mean(axis=0)) ** 2).sum(axis=1))
    return np.all(np.abs(d - radius) > margin)


def _trajectory_frames(sim, k, off, nframes, every):
    frames = []
    for _ in range(nframes):
        sim.step(every)
        sim.record_frame()
        frames.append(sim.positions()[off[k]:off[k + 1]].copy())
    return np.stack(frames)


@pytest.mark.parametrize("first,nframes,segments,radius", [(0, 60, 10, 8.0), (7, 45, 4, 6.5), (0, 60, 1, 1e6),
                                                            (30, 30, 15, 9.0)])
def test_diffusion_matches_oracle_on_a_hot_cluster(first, nframes, segments, radius):
    from oracle import diffusion as odiff
    rng = np.random.default_rng(601)
    pos = inputs.jitter(inputs.fcc_exact(600), 0.05, rng)
    vel = inputs.maxwell_boltzmann(pos, 2200.0, rng)
    print(f"[diffusion] Ni600 at 2200 K, window first={first} n={nframes} segments={segments}", flush=True)
    with scmd.Simulation(np.array([0, 600]), pos, vel, dt=2.0) as sim:
        sim.set_frames(0, 64)
        frames = _trajectory_frames(sim, 0, [0, 600], 60, 10)
        assert sim.frame_count(0) == 60
        win = frames[first:first + nframes]
        assert _central_tie_free(win[0], radius)
        d, nc = sim.diffusion(0, first, nframes, 0.02, radius, segments)
    d_ref, nc_ref = odiff.diffusion(win, 0.02, radius=radius, segments=segments)
    assert nc == nc_ref
    assert d > 0.0
    assert d == pytest.approx(d_ref, rel=1e-9)


def test_diffusion_of_a_batch_cluster_with_a_wrapped_store():
    from oracle import diffusion as odiff
    sizes = [147, 1000, 0, 320]
    rng = np.random.default_rng(602)
    parts = [inputs.jitter(inputs.fcc_exact(n), 0.05, rng) for n in sizes]
    vels = [inputs.maxwell_boltzmann(p, 1900.0, rng) if len(p) else np.zeros((0, 3)) for p in parts]
    off = np.concatenate([[0], np.cumsum(sizes)])
    print("[diffusion] batch, stores on clusters 1 and 3, 50 frames in rings of 24 and 50", flush=True)
    with scmd.Simulation(off, np.concatenate(parts), np.concatenate(vels), dt=1.0) as sim:
        sim.set_frames(1, 24)
        sim.set_frames(3, 50)
        f1, f3 = [], []
        for _ in range(50):
            sim.step(8)
            sim.record_frame()
            p = sim.positions()
            f1.append(p[off[1]:off[2]].copy())
            f3.append(p[off[3]:off[4]].copy())
        assert sim.frame_count(1) == 50 and sim.frame_count(3) == 50
        # only the last 24 frames of cluster 1 are still held
        with pytest.raises(scmd.ScmdError) as e:
            sim.diffusion(1, 25, 24, 0.008, 7.0, 4)
        assert e.value.status == scmd.SCMD_EINVAL
        got1 = sim.diffusion(1, 26, 24, 0.008, 7.0, 4)
        got3 = sim.diffusion(3, 0, 50, 0.008, 5.0, 5)
        for args in [(0, 0, 10, 0.01, 5.0, 2), (3, 0, 51, 0.01, 5.0, 5), (3, 0, 9, 0.01, 5.0, 5),
                     (3, 0, 50, 0.0, 5.0, 5), (3, 0, 50, 0.01, -1.0, 5), (3, 0, 50, 0.01, 5.0, 0),
                     (3, -1, 20, 0.01, 5.0, 5), (3, 0, 50, 0.01, 1e-3, 5)]:
            with pytest.raises(scmd.ScmdError) as e:
                sim.diffusion(*args)
            assert e.value.status == scmd.SCMD_EINVAL
        sim.set_frames(3, 0)
        with pytest.raises(scmd.ScmdError):
            sim.frame_count(3)
    w1, w3 = np.stack(f1[26:50]), np.stack(f3)
    assert _central_tie_free(w1[0], 7.0) and _central_tie_free(w3[0], 5.0)
    ref1 = odiff.diffusion(w1, 0.008, radius=7.0, segments=4)
    ref3 = odiff.diffusion(w3, 0.008, radius=5.0, segments=5)
    assert got1[1] == ref1[1] and got3[1] == ref3[1]
    assert got1[0] == pytest.approx(ref1[0], rel=1e-9)
    assert got3[0] == pytest.approx(ref3[0], rel=1e-9)
