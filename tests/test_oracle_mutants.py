"""The oracle's pins are sensitive: each test plants one plausible mistake in
a copy of the oracle's source, builds it, and checks that at least one of the
pins named for it fails (all on the CPU; the product library is not involved).
"""
import os
import tempfile

import pytest

import test_oracle as T
import test_oracle_buck as TB
import test_oracle_npt as TNP
import test_oracle_nvt as TN
import test_oracle_pressure as TP
import test_oracle_sc_vjp as TS
from paper_1009_4330_amd import inputs as I

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "md_oracle.c")

# name -> (original text, planted mistake, pins expected to catch it)
MUTANTS = {
    "virial_sign": ("wi[0] += 0.5 * d[0] * d[0] * g;", "wi[0] -= 0.5 * d[0] * d[0] * g;",
                    ["lattice", "brute_lj"]),
    "energy_half_dropped": ("ei += 0.5 * phi;", "ei += phi;", ["lattice", "two_atom"]),
    "no_minimum_image": ("return d - L * rint(d / L);", "return d;", ["brute_list"]),
    "lj_force_factor": ("double g = 24.0 * eps * sr6 * (2.0 * sr6 - 1.0) / s;",
                        "double g = 24.0 * eps * sr6 * (sr6 - 1.0) / s;", ["fd_lj", "two_atom"]),
    "sc_embedding_index": ("(em[i] + em[j])", "(em[i] + em[i])", ["fd_sc", "brute_sc"]),
    "sc_density_power": ("ri += pow(a2 / s, 0.5 * mexp);", "ri += pow(a2 / s, mexp);",
                         ["sc_lattice", "brute_sc"]),
    "vjp_second_term_sign": ("gi[q] += g * du[q] + 2.0 * gp * dud * d[q];",
                             "gi[q] += g * du[q] - 2.0 * gp * dud * d[q];", ["fd_vjp", "sym_vjp"]),
    "vjp_sigma_term": ("dsig += dg * (ui[0] * d[0] + ui[1] * d[1] + ui[2] * d[2]);",
                       "dsig += dg * (ui[0] * d[0] + ui[1] * d[1]);", ["fd_vjp"]),
    "full_kick_per_half": ("const double dtfm = (0.5 * p->dt * p->ftm2v) / p->mass;",
                           "const double dtfm = (p->dt * p->ftm2v) / p->mass;",
                           ["verlet_order", "reversible"]),
    "trigger_full_skin": ("int reb = dmax > trig2;", "int reb = dmax > 4.0 * trig2;",
                          ["schedule"]),
    "stencil_duplicates": ("if (!dup) out[k++] = v;", "out[k++] = v;", ["brute_list"]),
    "kinetic_half_dropped": ("double ke = 0.5 * p->mvv2e * p->mass * sv;",
                             "double ke = p->mvv2e * p->mass * sv;", ["temperature"]),
    "cell_index_scale": ("int c = (int)((r * (double)nc) / L);",
                         "int c = (int)((r * (double)(nc - 1)) / L);", ["bin_sort", "brute_list"]),
    "buck_species_pair": ("int ab = type[i] * 4 + type[j];", "int ab = type[i] * 4 + type[i];",
                          ["buck_brute_bm", "buck_symmetry"]),
    "buck_coulomb_force_power": ("- qq / s;", "- qq / r;", ["buck_fd", "buck_brute_coul"]),
    "buck_dispersion_factor": ("6.0 * C[ab] / (r6 * r)", "C[ab] / (r6 * r)",
                               ["buck_fd", "buck_brute_disp"]),
    "buck_energy_half_dropped": ("eb += 0.5 * phi;", "eb += phi;",
                                 ["buck_lattice", "buck_brute_disp"]),
    "scvjp_embedding_dropped": ("+ 2.0 * (lam[i] + lam[j]) * psip * d[q];",
                                "+ 0.0 * (lam[i] + lam[j]) * psip * d[q];", ["fd_scvjp"]),
    "scvjp_partner_lambda": ("(lam[i] + lam[j])", "(lam[i] + lam[i])",
                             ["fd_scvjp", "sym_scvjp"]),
    "scvjp_hprime_power": ("-(0.5 * nexp + 1.0) * A / s", "-(0.5 * nexp) * A / s",
                           ["fd_scvjp", "sym_scvjp"]),
    "scvjp_lambda_power": ("lam[i] = -0.5 * e[i] * e[i] * e[i] * (c * gci);",
                           "lam[i] = -0.5 * e[i] * e[i] * (c * gci);", ["fd_scvjp"]),
    "scvjp_da_factor": ("gparam[1] = (nexp * ta + 0.5 * mexp * c * tb) / a;",
                        "gparam[1] = (nexp * ta + mexp * c * tb) / a;", ["par_scvjp_a"]),
    "nvt_scale_quarter_step": ("double scale = exp(-dt2 * veta[0]);",
                               "double scale = exp(-dt4 * veta[0]);", ["nvt_conserved"]),
    "nvt_energy_dof": ("e += nf * kT * eta[0];", "e += kT * eta[0];", ["nvt_conserved"]),
    "nvt_ke_scaled_once": ("*ke2 = *ke2 * scale * scale;", "*ke2 = *ke2 * scale;",
                           ["nvt_conserved", "nvt_reversible"]),
    "nvt_eta_full_step": ("eta[j] = eta[j] + dt2 * veta[j];", "eta[j] = eta[j] + dt * veta[j];",
                          ["nvt_conserved"]),
    "pressure_volume_factor": ("/ (3.0 * vol);", "/ (2.0 * vol);",
                               ["ideal_gas", "pressure_dEdV"]),
    "pressure_kinetic_factor": ("row[5] = (2.0 * ke + ", "row[5] = (ke + ", ["ideal_gas"]),
    "pressure_virial_sign": ("(2.0 * ke + (vir[0] + vir[1] + vir[2]))",
                             "(2.0 * ke - (vir[0] + vir[1] + vir[2]))", ["pressure_dEdV"]),
    "pressure_virial_diagonal": ("(2.0 * ke + (vir[0] + vir[1] + vir[2]))",
                                 "(2.0 * ke + (vir[0] + vir[1] + vir[3]))", ["pressure_dEdV"]),
    "npt_barostat_force_kinetic": ("return alpha * ke2 + (vir[0] + vir[1] + vir[2])",
                                   "return ke2 + (vir[0] + vir[1] + vir[2])",
                                   ["npt_conserved"]),
    "npt_external_pressure_sign": ("- 3.0 * vol * p_target;", "+ 3.0 * vol * p_target;",
                                   ["npt_relax", "npt_conserved"]),
    "npt_drift_not_scaled": ("x[d * n + i] = x[d * n + i] * dc + de * v[d * n + i];",
                             "x[d * n + i] = x[d * n + i] + de * v[d * n + i];",
                             ["npt_conserved"]),
    "npt_kick_force_factor": ("const double kb = exp(-alpha * ve * 0.25 * p->dt) * sinhc",
                              "const double kb = exp(-alpha * ve * 0.5 * p->dt) * sinhc",
                              ["npt_conserved", "npt_reversible"]),
    "npt_energy_without_pv": ("0.5 * *peps * *peps / W + p_target * (L[0] * L[1] * L[2]))",
                              "0.5 * *peps * *peps / W)", ["npt_conserved"]),
}


def _scsys(o):
    x, box = TS.sc_system(5, 0.25, 81)
    nl, _ = o.build_nlist(x, box, TS.RC + 1.0)
    return x, box, nl


def _jittered():
    x, _, box = I.initial_state(TB.W8)
    return I.jitter(x, 0.08, 11), box

PINS = {
    "lattice": lambda o: T.test_lj_perfect_lattice_closed_form(o, 2.5),
    "two_atom": lambda o: T.test_lj_two_atom_golden(o),
    "brute_lj": lambda o: T.test_lj_equals_all_image_brute_force(o, 4, 0.3, 21),
    "brute_list": lambda o: T.test_nlist_equals_all_image_brute_force(o, 4, 0.3, 11, 0.0),
    "fd_lj": lambda o: T.test_lj_forces_are_minus_energy_gradient(o),
    "fd_sc": lambda o: T.test_sc_forces_are_minus_energy_gradient(o),
    "brute_sc": lambda o: T.test_sc_equals_all_image_brute_force(o),
    "sc_lattice": lambda o: T.test_sc_perfect_lattice_closed_form(o),
    "fd_vjp": lambda o: T.test_vjp_matches_central_differences(o),
    "sym_vjp": lambda o: T.test_vjp_symmetry_translation_and_linearity(o),
    "verlet_order": lambda o: T.test_nve_energy_error_is_second_order_in_dt(o),
    "reversible": lambda o: T.test_nve_time_reversible(o),
    "schedule": lambda o: T.test_rebuild_schedule_follows_half_skin(o),
    "temperature": lambda o: T.test_initial_temperature_and_momentum(o),
    "bin_sort": lambda o: T.test_bin_is_stable_counting_sort(o, 4, 1),
    "buck_symmetry": lambda o: TB.test_perfect_crystal_forces_vanish(o),
    "buck_brute_bm": lambda o: TB.test_each_term_against_brute_force(o, _jittered(), "born_mayer"),
    "buck_brute_disp": lambda o: TB.test_each_term_against_brute_force(o, _jittered(),
                                                                       "dispersion"),
    "buck_brute_coul": lambda o: TB.test_each_term_against_brute_force(o, _jittered(), "coulomb"),
    "buck_fd": lambda o: TB.test_forces_are_minus_energy_gradient(o, _jittered()),
    "buck_lattice": lambda o: TB.test_dispersion_lattice_sum(o),
    "fd_scvjp": lambda o: TS.test_sc_vjp_matches_central_differences_in_x(o, _scsys(o)),
    "sym_scvjp": lambda o: TS.test_sc_vjp_symmetry_translation_and_linearity(o, _scsys(o)),
    "par_scvjp_a": lambda o: TS.test_sc_vjp_parameter_gradients(o, _scsys(o), 1, "a"),
    "nvt_conserved": lambda o: TN.test_nvt_conserved_energy_is_second_order(o, 3),
    "nvt_reversible": lambda o: TN.test_nvt_time_reversible(o),
    "npt_conserved": lambda o: TNP.test_npt_conserved_energy_is_second_order(o),
    "npt_relax": lambda o: TNP.test_npt_relaxes_to_target_pressure(o),
    "npt_reversible": lambda o: TNP.test_npt_time_reversible(o),
    "ideal_gas": lambda o: TP.test_ideal_gas_law(o, TP.LJ, dict(lj_eps=0.0)),
    "pressure_dEdV": lambda o: TP.test_pressure_is_minus_energy_volume_derivative(o,
                                                                                  "lj_jittered"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(orc, name):
    original, planted, pins = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(original) == 1, f"mutation site for {name} not unique"
    with tempfile.TemporaryDirectory() as tmp:
        path = orc.oracle.build_variant(text.replace(original, planted),
                                        os.path.join(tmp, f"mut_{name}.so"))
        caught = []
        with orc.oracle.using(path):
            for pin in pins:
                try:
                    PINS[pin](orc)
                except (AssertionError, orc.OracleError):
                    caught.append(pin)
    assert caught, f"planted mistake {name!r} passed every pin in {pins}"
