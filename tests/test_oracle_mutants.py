"""The pins are sharp: plant plausible mistakes in a copy of the oracle source
(a dropped factor, a swapped index, a wrong sign or exponent, a wrong
integrator or thermostat constant), build the copy on the CPU and check that
at least one pin of ``test_oracle_pins`` fails for every mutant."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_langevin as lpins
import test_oracle_pins as pins
import test_oracle_rdf as rpins
from paper_1210_3559_amd import inputs

SRC = os.path.join(os.path.dirname(oracle.__file__), "sc_oracle.c")

MUTANTS = {
    "psi_index": ("(psi[i] + psi[j])", "(psi[i] + psi[i])"),
    "pair_half_dropped": ("0.5 * pair_sum", "pair_sum"),
    "embedding_half_dropped": ("0.5 * p->c * (double)p->m", "p->c * (double)p->m"),
    "dy_transposed": ("pos[3 * i + 1] - pos[3 * j + 1]", "pos[3 * j + 1] - pos[3 * i + 1]"),
    "inverse_r_not_squared": ("/ (r * r)", "/ r"),
    "repulsive_exponent": ("double an = pow(p->a / r, (double)p->n);", "double an = pow(p->a / r, (double)p->m);"),
    "embedding_sign": ("- p->c * sqrt(rho[i])", "+ p->c * sqrt(rho[i])"),
    "full_kick": ("double h = 0.5 * dt /", "double h = dt /"),
    "ndof": ("return 3 * n - 6;", "return 3 * n;"),
    "berendsen_ratio": ("(T_target / T - 1.0)", "(T / T_target - 1.0)"),
    "shift_sign": ("if (p->rc > 0.0) v -= pow(", "if (p->rc > 0.0) v += pow("),
    "ke_half": ("return 0.5 * mass_u * s *", "return mass_u * s *"),
    "langevin_gamma_units": ("exp(-thermo->gamma * 1e-3 * dt)", "exp(-thermo->gamma * dt)"),
    "langevin_c2_variance": ("sqrt((1.0 - c1 * c1) * SCO_KB", "sqrt((1.0 - c1) * SCO_KB"),
    "langevin_half_drifts_doubled": ("pos[i] += 0.5 * dt * vel[i];", "pos[i] += dt * vel[i];"),
    "langevin_ndof": ("if (kind == SCO_LANGEVIN) return 3 * n;", "if (kind == SCO_LANGEVIN) return 3 * n - 6;"),
    "langevin_ramp_index": ("Tt = sco_target_temperature(thermo, s);", "Tt = sco_target_temperature(thermo, s - 1);"),
    "philox_key_increment": ("k1 += SCO_PHILOX_W1;", "k1 += SCO_PHILOX_W0;"),
    "philox_word_order": ("const uint32_t n1 = (uint32_t)p1;", "const uint32_t n1 = (uint32_t)p0;"),
    "box_muller_pair": ("out[1] = ra * sin(two_pi * u[1]);", "out[1] = ra * cos(two_pi * u[1]);"),
    "noise_ignores_step": ("(uint32_t)atom, 0u, (uint32_t)st,", "(uint32_t)atom, 0u, (uint32_t)atom,"),
    "ramp_origin_sign": ("int64_t kr = k - t->ramp_origin;", "int64_t kr = k + t->ramp_origin;"),
    "rdf_bin_rounding": ("const double b = floor(r / dr);", "const double b = floor(r / dr + 0.5);"),
    "rdf_self_pair": ("            if (j == i) continue;\n            const double dx = pos[3 * i] - pos[3 * j];",
                      "            const double dx = pos[3 * i] - pos[3 * j];"),
    "rdf_centre_not_averaged": ("for (int d = 0; d < 3; ++d) c[d] /= (double)n;", "for (int d = 0; d < 3; ++d) c[d] /= 1.0;"),
    "ramp_index": ("t->T_start + (t->T_end - t->T_start) * (double)kk", "t->T_end + (t->T_start - t->T_end) * (double)kk"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    hdr = os.path.join(os.path.dirname(SRC), "sc_oracle.h")
    lib = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-I", os.path.dirname(hdr), str(path), "-o", str(lib), "-lm"], check=True)
    return oracle.load_variant(str(lib))


def _pin_calls():
    ball = (inputs.fcc_sphere(24.0, pins.A), 24.0)
    ni147 = (inputs.c1_icosahedron().pos, inputs.c1_icosahedron().vel)
    calls = [
        lambda o: pins.test_parameter_set_is_the_papers(o),
        lambda o: pins.test_dimer_closed_form(o, 2.49),
        lambda o: pins.test_dimer_equilibrium(o),
        lambda o: pins.test_equilateral_trimer(o),
        lambda o: pins.test_central_density_matches_fcc_lattice_sum(o, ball),
        lambda o: pins.test_central_site_energy_is_ni_cohesive_energy(o, ball),
        lambda o: pins.test_forces_are_minus_energy_gradient(o, None),
        lambda o: pins.test_forces_are_minus_energy_gradient(o, dict(rc=8.8)),
        lambda o: pins.test_net_force_and_torque_vanish(o),
        lambda o: pins.test_translation_rotation_permutation_scaling(o),
        lambda o: pins.test_mackay_icosahedron_symmetry(o),
        lambda o: pins.test_cutoff_dimer_and_limits(o),
        lambda o: pins.test_ndof_rule(o),
        lambda o: pins.test_maxwell_boltzmann_sample_has_its_temperature(o),
        lambda o: pins.test_berendsen_ramp_target(o),
        lambda o: pins.test_dimer_harmonic_period(o),
        lambda o: pins.test_berendsen_relaxes_to_target(o, ni147),
        lambda o: pins.test_time_reversibility(o, ni147),
        lambda o: rpins.test_fcc_central_atom_shells(o),
        lambda o: rpins.test_total_count_is_every_ordered_pair(o),
        lambda o: rpins.test_dimer_and_trimer(o),
        lambda o: rpins.test_mackay_selection(o),
        lambda o: rpins.test_invariant_under_rigid_motion_and_relabelling(o),
        lambda o: lpins.test_philox_known_answers(o),
        lambda o: lpins.test_noise_is_standard_normal(o),
        lambda o: lpins.test_noise_box_muller_structure(o),
        lambda o: lpins.test_zero_damping_is_velocity_verlet(o),
        lambda o: lpins.test_free_atom_decays_in_a_cold_bath(o, 1.0),
        lambda o: lpins.test_free_atoms_reach_bath_temperature(o),
        lambda o: lpins.test_noise_follows_the_step_count(o),
        lambda o: lpins.test_cluster_reaches_bath_temperature(o),
    ]
    return calls


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MUTANTS[name]
    mutant = _build(tmp_path, name, old, new)
    caught = None
    with np.errstate(all="ignore"):
        for i, call in enumerate(_pin_calls()):
            try:
                call(mutant)
            except (AssertionError, ValueError, FloatingPointError):
                caught = i
                break
    assert caught is not None, f"no pin caught mutant {name}"


def test_unmutated_copy_passes_every_pin(tmp_path):
    clean = _build(tmp_path, "clean", "#include <math.h>", "#include <math.h>")
    for call in _pin_calls():
        call(clean)
