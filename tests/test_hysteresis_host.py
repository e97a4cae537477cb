"""Host logic of the heating-cooling driver: the programme's leg lengths
and the transition-temperature estimator on curves with a known answer."""
import numpy as np
import pytest

from paper_1210_3559_amd import hysteresis, inputs


def test_legs_follow_the_rate():
    legs = inputs.heating_cooling_legs(400.0, 1400.0, 1.0, 1.0)
    # 1000 K at 1 K/ps = 1000 ps = 1e6 steps of 1 fs, each way
    assert legs == [(400.0, 1400.0, 1_000_000), (1400.0, 400.0, 1_000_000)]
    assert inputs.heating_cooling_legs(400.0, 1400.0, 5.0, 2.0)[0][2] == 100_000


@pytest.mark.parametrize("t_jump", [731.0, 1150.0, 1298.0])
def test_transition_at_the_energy_jump(t_jump):
    rng = np.random.default_rng(1)
    T = np.linspace(400.0, 1400.0, 2001)
    e = -4.3 + 2.6e-4 * (T - 400.0) + 0.06 * (T > t_jump) + rng.normal(0, 2e-4, T.size)
    assert abs(hysteresis.transition_temperature(T, e) - t_jump) <= 20.0
    # the cooling leg visits the same temperatures in the other order
    assert abs(hysteresis.transition_temperature(T[::-1], e[::-1]) - t_jump) <= 20.0


def test_ni2057_cycle_workload():
    w = inputs.ni2057_cycle(3)
    assert list(w.sizes()) == [2057] * 3
    assert [t["seed"] for t in w.thermostat] == [2057, 2058, 2059]
    assert not np.array_equal(w.vel[:2057], w.vel[2057:4114])
    np.testing.assert_array_equal(w.pos[:2057], w.pos[2057:4114])
