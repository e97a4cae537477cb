"""The heating-cooling and kinetics drivers run end to end on the GPU (short
programmes): the sampled series have the expected length and bath targets,
and the structure analysis of a tracked replica is finite and in range."""
import math

import numpy as np
import pytest

from paper_1210_3559_amd import hysteresis, kinetics

pytestmark = pytest.mark.gpu


def test_heating_cooling_cycle_runs():
    # 400 -> 1400 -> 400 K at 250 K/ps: 4000 steps per leg, a sample every 100
    print("[drivers] fast heating-cooling cycle", flush=True)
    res = hysteresis.run(replicas=2, rate=250.0, sample_every=100, chunk=1000)
    assert res["steps"] == 8000 and res["replicas"] == 2
    for c in res["clusters"]:
        s = np.array(c["samples"])
        assert len(s) == 80
        np.testing.assert_array_equal(s[:, 0], np.arange(100, 8001, 100))
        # the bath target climbs to 1400 K and comes back
        assert s[39, 1] == pytest.approx(1400.0) and s[-1, 1] == pytest.approx(400.0)
        assert np.all(np.isfinite(s[:, 2:]))
        assert math.isfinite(c["T_melt_K"]) and math.isfinite(c["T_freeze_K"])


def test_kinetics_run_with_tracking():
    print("[drivers] short isothermal run with a tracked replica", flush=True)
    res = kinetics.run(750.0, replicas=2, max_ps=60.0, melt_ps=20.0, chunk_ps=20.0, track=1, frame_ps=2.0,
                       min_ps=60.0)
    assert res["run_ps"] == pytest.approx(60.0)
    assert len(res["traces"]) == 2
    for tr in res["traces"]:
        assert len(tr["t_ps"]) == 6 and np.all(np.isfinite(tr["e_per_atom"]))
    # 30 frames of 2 ps: no full 1 ns window, so no structure series yet
    assert res["tracked"] == []
    k_mean, k_mle = res["kappa_per_ps"], res["kappa_mle_per_ps"]
    assert (math.isnan(k_mean) or k_mean > 0) and (math.isnan(k_mle) or k_mle >= 0)
