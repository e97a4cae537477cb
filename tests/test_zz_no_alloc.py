"""scmd_rdf_noalloc (the allocation-free pair-distance histogram for callers
under graph capture or in serving loops) against scmd_rdf, the entry point it
varies, through the C ABI: the same counts and reference-atom count, bit for
bit, on two calls in a row, the second on a smaller cluster.  The histogram
itself is pinned to the oracle by the analysis parity tests."""
import ctypes

import numpy as np
import pytest

from paper_1210_3559_amd import inputs
from paper_1210_3559_amd import scmd

pytestmark = pytest.mark.gpu


def _noalloc(lib, ctx, cluster, r_select, dr, nbins):
    import torch
    counts = torch.zeros(nbins, dtype=torch.int64, device="cuda")
    nref = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    st = lib.scmd_rdf_noalloc(ctx, cluster, r_select, dr, nbins, ctypes.c_void_p(counts.data_ptr()),
                              ctypes.c_void_p(nref.data_ptr()))
    assert st == scmd.SCMD_OK, scmd.scmd_last_error(ctx)
    assert lib.scmd_synchronize(ctx) == scmd.SCMD_OK
    return counts.cpu().numpy().view(np.uint64), int(nref.cpu().item())


def _allocating(lib, ctx, cluster, r_select, dr, nbins):
    counts = np.zeros(nbins, dtype=np.uint64)
    nref = ctypes.c_int64(0)
    st = lib.scmd_rdf(ctx, cluster, r_select, dr, nbins, counts.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nref))
    assert st == scmd.SCMD_OK, scmd.scmd_last_error(ctx)
    return counts, nref.value


def test_noalloc_histogram_matches_scmd_rdf_twice():
    lib = scmd.load()
    rng = np.random.default_rng(77)
    sizes = [2243, 0, 530]
    parts = [inputs.jitter(inputs.fcc_exact(n), 0.05, rng) for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)])
    print("[noalloc] batch 2243 + 0 + 530 atoms: cluster 0, then the smaller cluster 2", flush=True)
    with scmd.Simulation(off, np.concatenate(parts), None, dt=1.0) as sim:
        sim.step(3)
        for cluster, r_select, dr, nbins in ((0, 9.0, 0.05, 900), (2, 0.0, 0.1, 200)):
            got, nr = _noalloc(lib, sim.ctx, cluster, r_select, dr, nbins)
            ref, nref = _allocating(lib, sim.ctx, cluster, r_select, dr, nbins)
            assert nr == nref and nr > 0
            np.testing.assert_array_equal(got, ref)
        # results add to what the caller's buffers hold
        import torch
        counts = torch.zeros(200, dtype=torch.int64, device="cuda")
        nref = torch.zeros(1, dtype=torch.int64, device="cuda")
        for _ in range(2):
            scmd.scmd_rdf_noalloc(sim.ctx, 2, 0.1, 200, counts, nref)
        scmd.scmd_synchronize(sim.ctx)
        ref, nr1 = _allocating(lib, sim.ctx, 2, 0.0, 0.1, 200)
        np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), 2 * ref)
        assert int(nref.cpu().item()) == 2 * nr1


def test_noalloc_rejects_bad_arguments():
    import torch
    lib = scmd.load()
    pos = inputs.fcc_exact(20)
    counts = torch.zeros(16, dtype=torch.int64, device="cuda")
    nref = torch.zeros(1, dtype=torch.int64, device="cuda")
    with scmd.Simulation(np.array([0, 20]), pos, None) as sim:
        cp, npp = ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(nref.data_ptr())
        for args in [(1, 0.0, 0.1, 16, cp, npp), (0, 0.0, 0.0, 16, cp, npp), (0, 0.0, 0.1, 0, cp, npp),
                     (0, 0.0, 0.1, 40000, cp, npp), (0, float("nan"), 0.1, 16, cp, npp),
                     (0, 0.0, 0.1, 16, None, npp), (0, 0.0, 0.1, 16, cp, None)]:
            assert lib.scmd_rdf_noalloc(sim.ctx, *args) == scmd.SCMD_EINVAL
        with pytest.raises(ValueError):
            scmd.scmd_rdf_noalloc(sim.ctx, 0, 0.1, 32, counts, nref)  # tensor shorter than nbins
