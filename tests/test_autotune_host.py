"""Autotuner host logic (no GPU): cache keys and lookups."""
import json

import numpy as np

from paper_1210_3559_amd import autotune


def test_bucket_groups_by_size_and_count():
    a = autotune.bucket(np.array([0, 2243]), "fp64")
    b = autotune.bucket(np.array([0, 3000]), "fp64")
    c = autotune.bucket(np.array([0, 5000]), "fp64")
    assert a == b != c
    assert autotune.bucket(np.array([0, 2243]), "mixed") != a
    batch = autotune.bucket(np.concatenate([[0], np.cumsum(np.full(256, 100))]), "fp64")
    assert batch.endswith("nc2^8")


def test_lookup_reads_cache(tmp_path):
    path = tmp_path / "cache.json"
    key = autotune.bucket(np.array([0, 2243]), "fp64")
    path.write_text(json.dumps({key: {"tuning": {"ipt": 1, "waves_i": 1, "waves_j": 8, "target_items": 2048,
                                                 "pairs": 1}, "ms_per_step": 0.03}}))
    t = autotune.lookup(np.array([0, 2100]), "fp64", str(path))
    assert t == {"ipt": 1, "waves_i": 1, "waves_j": 8, "target_items": 2048, "pairs": 1}
    assert autotune.lookup(np.array([0, 20000]), "fp64", str(path)) is None
    assert autotune.lookup(np.array([0, 20]), "fp64", str(tmp_path / "missing.json")) is None


def test_candidate_shapes_are_supported_by_the_header():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "scmd.h")).read()
    listed = set(re.findall(r"\((\d),(\d),(\d+)\)", hdr))
    for s in autotune.SHAPES:
        assert tuple(str(x) for x in s) in listed, s


def test_candidates_follow_cluster_sizes():
    small = autotune.candidate_plans([2243])
    assert any(c["pairs"] == 3 for c, _ in small) and any(c["pairs"] == 1 for c, _ in small)
    large = autotune.candidate_plans([48077])
    assert all(c["pairs"] == 2 for c, _ in large)
    assert any(16384 in t for c, t in large)
    batch = autotune.candidate_plans(np.full(256, 1750))
    assert not any(c["pairs"] == 3 for c, _ in batch)


def test_committed_table_covers_the_benchmark_workloads():
    import os
    from paper_1210_3559_amd import inputs
    assert os.path.exists(autotune.DEFAULT_CACHE)
    table = autotune.load_cache()
    for name in ("ni2243_cooling", "ni15000_fp64", "ni15000_mixed", "ni48077_allpairs", "batch256", "batch256_mixed"):
        w = inputs.by_name(name)
        t = autotune.lookup(w.offsets, w.precision)
        assert t is not None, name
        assert t["pairs"] in (1, 2, 3)
        if t["pairs"] == 2:
            assert t["ipt"] in (2, 4, 8)
        if t["pairs"] == 1:
            assert (t["ipt"], t["waves_i"], t["waves_j"]) in autotune.SHAPES
    assert all("ms_per_step" in e and "workload" in e for e in table.values())
    w = inputs.by_name("ni48077_cell")
    t = autotune.lookup(w.offsets, w.precision, cell=True)
    assert t is not None and set(t) == {"cell_skin"} and t["cell_skin"] in autotune.CELL_SKINS


def test_cell_list_layouts_have_their_own_key_and_skin_entries(tmp_path):
    import json
    off = np.array([0, 48077])
    assert autotune.bucket(off, "fp64", cell=True) != autotune.bucket(off, "fp64")
    assert autotune.bucket(off, "fp64", cell=True).endswith("/cell")
    path = tmp_path / "t.json"
    path.write_text(json.dumps({autotune.bucket(off, "fp64", cell=True):
                                dict(tuning=dict(cell_skin=0.5), ms_per_step=0.1, workload="x")}))
    assert autotune.lookup(off, "fp64", str(path), cell=True) == {"cell_skin": 0.5}
    assert autotune.lookup(off, "fp64", str(path)) is None
    assert all(0.0 < s < 0.8 for s in autotune.CELL_SKINS)
