"""GPU parity of the Langevin bath (the paper's thermostat, Sec. 2
"Computational approach"; BAOAB splitting, Philox4x32-10 / Box-Muller noise
keyed by seed, step and atom) against the oracle's trajectories.

Both sides draw the same noise from the same definition, so the
trajectories agree up to the rounding of the force sums and of the noise's
log/cos/sin (a few ulp per step): over the 60-120 steps here positions agree
to 1e-9 A and velocities to 1e-10 A/fs, as for the deterministic thermostat.
The mixed-precision form is held to its force tolerance carried through the
steps (1e-6 A, 1e-7 A/fs).  Runs are split into calls of uneven length so
that graph-replayed, eager and first-of-run steps all occur.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1210_3559_amd import inputs
from paper_1210_3559_amd import scmd

pytestmark = pytest.mark.gpu

NT = min(16, os.cpu_count() or 1)
GAMMA = 10.0  # 1/ps, the paper's damping constant


def _bath(T_end, seed, T_start=None, ramp=0, gamma=GAMMA):
    return dict(kind="langevin", T_start=T_end if T_start is None else T_start, T_end=T_end, ramp_steps=ramp,
                gamma=gamma, seed=seed)


def _run(w_off, pos, vel, dt, baths, chunks, precision="fp64", tuning=None, rc=0.0):
    with scmd.Simulation(w_off, pos, vel, dt=dt, precision=precision, thermostats=baths, tuning=tuning,
                         rc=rc) as sim:
        for c in chunks:
            sim.step(c)
        out = dict(r=sim.positions(), v=sim.velocities(), f=sim.forces(),
                   e=[sim.energy(k) for k in range(len(w_off) - 1)],
                   T=[sim.temperature(k) for k in range(len(w_off) - 1)])
    return out


PATHS = {
    "row_fused": (None, "fp64", 0.0),
    "mixed_symmetric": (dict(pairs=2, ipt=4), "mixed", 0.0),
    "symmetric": (dict(pairs=2, ipt=4), "fp64", 0.0),
    "one_sided": (dict(pairs=1, ipt=1, waves_i=1, waves_j=4), "fp64", 0.0),
    "row_waves4": (dict(pairs=3, waves_j=4), "fp64", 0.0),
    "cell_list": (None, "fp64", 8.8),
    "mixed_row": (None, "mixed", 0.0),
}


@pytest.mark.parametrize("path", sorted(PATHS))
def test_langevin_trajectory_parity(path):
    tuning, precision, rc = PATHS[path]
    w = inputs.c2_cooling()
    th = _bath(900.0, seed=2024, T_start=1500.0, ramp=50)
    nsteps = 77
    print(f"[langevin] Ni2243 {path} {nsteps} steps", flush=True)
    params = dict(rc=rc) if rc > 0 else None
    r_ref, v_ref, f_ref, log = oracle.vv_run(w.pos, w.vel, nsteps, dt=1.0, thermostat=th, params=params,
                                             nthreads=NT)
    g = _run(w.offsets, w.pos, w.vel, 1.0, [th], (5, 32, 40), precision, tuning, rc)
    rt, vt = (1e-9, 1e-10) if precision == "fp64" else (1e-6, 1e-7)
    assert np.abs(g["r"] - r_ref).max() < rt
    assert np.abs(g["v"] - v_ref).max() < vt
    et = 1e-10 if precision == "fp64" else 1e-6
    ep, ek, _ = g["e"][0]
    assert ep == pytest.approx(log[-1, 0], rel=et)
    assert ek == pytest.approx(log[-1, 1], rel=100 * et)
    T, ndof = g["T"][0]
    assert ndof == 3 * 2243
    assert T == pytest.approx(log[-1, 2], rel=100 * et)


def test_langevin_batch_parity_mixed_kinds():
    # three baths with their own seeds and an NVE cluster in one batch
    rng = np.random.default_rng(5)
    sizes = [147, 0, 530, 61, 1000]
    clusters = [inputs.jitter(inputs.fcc_exact(n), 0.05, rng) for n in sizes]
    vels = [inputs.maxwell_boltzmann(p, 1100.0, rng) if len(p) else np.zeros((0, 3)) for p in clusters]
    ths = [_bath(700.0, 1), _bath(700.0, 1), None, _bath(1200.0, 99, T_start=400.0, ramp=30), _bath(300.0, 7)]
    off = np.concatenate([[0], np.cumsum(sizes)])
    print("[langevin] batch of 5 with an NVE member", flush=True)
    g = _run(off, np.concatenate(clusters), np.concatenate(vels), 1.0, ths, (33, 31))
    for k, n in enumerate(sizes):
        if n == 0:
            continue
        r_ref, v_ref, _, log = oracle.vv_run(clusters[k], vels[k], 64, dt=1.0, thermostat=ths[k], nthreads=NT)
        a, b = off[k], off[k + 1]
        assert np.abs(g["r"][a:b] - r_ref).max() < 1e-9, k
        assert np.abs(g["v"][a:b] - v_ref).max() < 1e-10, k
        assert g["e"][k][0] == pytest.approx(log[-1, 0], rel=1e-10)
        T, ndof = g["T"][k]
        assert ndof == (3 * n if ths[k] else 3 * n - 6)
        assert T == pytest.approx(log[-1, 2], rel=1e-8)


@pytest.mark.parametrize("tuning", [None, dict(pairs=2, ipt=4)])
def test_switch_from_berendsen_to_langevin(tuning):
    # the Berendsen factor of the last rescaling step is still pending when
    # the bath takes over; the first bath drift must apply it
    w = inputs.c1_icosahedron()
    ber = dict(T_start=1200.0, T_end=600.0, ramp_steps=40, tau=50.0)
    th = _bath(500.0, seed=3)
    r1, v1, f1, _ = oracle.vv_run(w.pos, w.vel, 30, dt=1.0, thermostat=ber, nthreads=NT)
    r2, v2, _, log = oracle.vv_run(r1, v1, 45, dt=1.0, thermostat=th, step0=30, force=f1, nthreads=NT)
    print(f"[langevin] Berendsen -> Langevin switch tuning={tuning}", flush=True)
    with scmd.Simulation(w.offsets, w.pos, w.vel, dt=1.0, thermostats=[ber], tuning=tuning) as sim:
        sim.step(30)
        sim.set_thermostat(0, th)
        sim.step(13)
        sim.step(32)
        r, v = sim.positions(), sim.velocities()
        T, ndof = sim.temperature(0)
    assert ndof == 3 * 147
    assert np.abs(r - r2).max() < 1e-9
    assert np.abs(v - v2).max() < 1e-10
    assert T == pytest.approx(log[-1, 2], rel=1e-8)


def test_langevin_is_deterministic_and_seeded():
    w = inputs.c2_cooling()
    outs = []
    for seed in (11, 11, 12):
        print(f"[langevin] determinism seed={seed}", flush=True)
        outs.append(_run(w.offsets, w.pos, w.vel, 1.0, [_bath(800.0, seed)], (40,)))
    np.testing.assert_array_equal(outs[0]["r"], outs[1]["r"])
    np.testing.assert_array_equal(outs[0]["v"], outs[1]["v"])
    assert np.abs(outs[0]["r"] - outs[2]["r"]).max() > 1e-6


def test_langevin_checkpoint_resume_is_bitwise():
    w = inputs.c2_cooling()
    print("[langevin] checkpoint resume", flush=True)
    with scmd.Simulation(w.offsets, w.pos, w.vel, dt=1.0, thermostats=[_bath(900.0, 5, 1400.0, 100)]) as sim:
        sim.step(40)
        blob = scmd.scmd_get_state(sim.ctx)
        sim.step(50)
        ra, va, ea = sim.positions(), sim.velocities(), sim.energy()
    # a fresh context restored from the blob (thermostat settings included)
    with scmd.Simulation(w.offsets, w.pos, w.vel, dt=1.0) as sim:
        scmd.scmd_set_state(sim.ctx, blob)
        assert scmd.scmd_get_step(sim.ctx) == 40
        sim.step(50)
        np.testing.assert_array_equal(sim.positions(), ra)
        np.testing.assert_array_equal(sim.velocities(), va)
        assert sim.energy() == ea


def test_langevin_samples_report_bath_target():
    w = inputs.c1_icosahedron()
    th = _bath(300.0, seed=8, T_start=900.0, ramp=60)
    _, _, _, log = oracle.vv_run(w.pos, w.vel, 90, dt=1.0, thermostat=th, nthreads=NT)
    print("[langevin] sampling", flush=True)
    with scmd.Simulation(w.offsets, w.pos, w.vel, dt=1.0, thermostats=[th]) as sim:
        sim.set_sampling(15, capacity=16)
        sim.step(50)
        sim.step(40)
        smp, recorded = sim.samples(0)
    assert recorded == 6
    for row in smp:
        k = int(row[0])
        np.testing.assert_allclose(row[1:4], log[k - 1, :3], rtol=1e-9)
        assert row[4] == log[k - 1, 3]


@pytest.mark.parametrize("path", ["row_fused", "symmetric"])
def test_langevin_cluster_reaches_bath_temperature(path):
    # Ni2243 started cold in a 1000 K bath: after ~10 damping times the mean
    # kinetic temperature over 20 ps is the bath's within its statistical
    # error (std(T)/T = sqrt(2/3N) = 1.7 % per step, correlation ~0.1 ps)
    tuning = PATHS[path][0]
    w = inputs.c2_cooling()
    print(f"[langevin] equipartition {path}", flush=True)
    with scmd.Simulation(w.offsets, w.pos, np.zeros_like(w.vel), dt=1.0, thermostats=[_bath(1000.0, 17)],
                         tuning=tuning) as sim:
        sim.step(3000)
        sim.set_sampling(10, capacity=4096)
        sim.step(20000)
        smp, recorded = sim.samples(0)
    assert recorded == 2000
    T = smp[:, 3]
    blocks = T.reshape(-1, 20).mean(axis=1)
    sem = blocks.std(ddof=1) / np.sqrt(len(blocks))
    print(f"[langevin] <T> = {T.mean():.2f} K +- {sem:.2f}", flush=True)
    assert sem < 5.0
    assert abs(T.mean() - 1000.0) < max(4.0 * sem, 5.0)
    assert T.std() / 1000.0 == pytest.approx(np.sqrt(2.0 / (3 * 2243)), rel=0.3)


def test_langevin_argument_errors():
    ctx = scmd.scmd_create(0)
    try:
        with pytest.raises(scmd.ScmdError) as e:
            scmd.scmd_set_langevin(ctx, 0, 300.0, 300.0)
        assert e.value.status == scmd.SCMD_ESTATE
        scmd.scmd_init_clusters(ctx, np.array([0, 20]), inputs.fcc_exact(20), None, 58.6934)
        for args in [(0, -1.0, 300.0, 0, 10.0), (0, 300.0, np.inf, 0, 10.0), (0, 300.0, 300.0, 0, -0.5),
                     (0, 300.0, 300.0, 0, np.nan), (1, 300.0, 300.0, 0, 10.0), (-2, 300.0, 300.0, 0, 10.0)]:
            with pytest.raises(scmd.ScmdError) as e:
                scmd.scmd_set_langevin(ctx, *args, seed=1)
            assert e.value.status == scmd.SCMD_EINVAL
        with pytest.raises(scmd.ScmdError) as e:
            scmd.scmd_set_thermostat(ctx, 0, scmd.SCMD_LANGEVIN, 300, 300, 0, 100)
        assert e.value.status == scmd.SCMD_EINVAL
        scmd.scmd_set_langevin(ctx, -1, 300.0, 300.0, 0, 0.0, seed=2 ** 64 - 1)
    finally:
        scmd.scmd_destroy(ctx)


@pytest.mark.parametrize("kind", ["langevin", "berendsen"])
def test_two_leg_temperature_programme(kind):
    # heating then cooling: the second leg's ramp starts at the step count
    # where it is set (ramp_origin), as a programme of legs needs
    w = inputs.c1_icosahedron()
    if kind == "langevin":
        leg1 = _bath(900.0, seed=4, T_start=500.0, ramp=30)
        leg2 = _bath(300.0, seed=4, T_start=900.0, ramp=40)
    else:
        leg1 = dict(T_start=500.0, T_end=900.0, ramp_steps=30, tau=40.0)
        leg2 = dict(T_start=900.0, T_end=300.0, ramp_steps=40, tau=40.0)
    r1, v1, f1, l1 = oracle.vv_run(w.pos, w.vel, 37, dt=1.0, thermostat=leg1, nthreads=NT)
    r2, v2, _, l2 = oracle.vv_run(r1, v1, 50, dt=1.0, thermostat=dict(leg2, ramp_origin=37), step0=37, force=f1,
                                  nthreads=NT)
    assert l2[0, 3] < 900.0 and l2[39, 3] == 300.0 and l1[29, 3] == 900.0
    print(f"[langevin] two-leg programme {kind}", flush=True)
    with scmd.Simulation(w.offsets, w.pos, w.vel, dt=1.0, thermostats=[leg1]) as sim:
        sim.set_sampling(1, capacity=128)
        sim.step(37)
        sim.set_thermostat(0, leg2)
        sim.step(18)
        sim.step(32)
        r, v = sim.positions(), sim.velocities()
        smp, recorded = sim.samples(0)
    assert recorded == 87
    np.testing.assert_array_equal(smp[:, 4], np.concatenate([l1[:, 3], l2[:, 3]]))
    assert np.abs(r - r2).max() < 1e-9
    assert np.abs(v - v2).max() < 1e-10


@pytest.mark.parametrize("tuning", [None, dict(pairs=1, ipt=1, waves_i=1, waves_j=4)])
def test_langevin_with_generic_exponents(tuning):
    # (n, m) = (12, 6): the generic-exponent kernels carry the same bath code
    params = dict(n=12, m=6)
    w = inputs.c1_icosahedron()
    th = _bath(700.0, seed=12, T_start=1000.0, ramp=30)
    print(f"[langevin] generic exponents tuning={tuning}", flush=True)
    r_ref, v_ref, _, log = oracle.vv_run(w.pos, w.vel, 45, dt=1.0, thermostat=th, params=params, nthreads=NT)
    with scmd.Simulation(w.offsets, w.pos, w.vel, dt=1.0, thermostats=[th], tuning=tuning, params=params) as sim:
        sim.step(13)
        sim.step(32)
        r, v = sim.positions(), sim.velocities()
        ep = sim.energy(0)[0]
    assert np.abs(r - r_ref).max() < 1e-9
    assert np.abs(v - v_ref).max() < 1e-10
    assert ep == pytest.approx(log[-1, 0], rel=1e-10)
