"""The reference solver's pins catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, index or operand)
in a copy of ``oracle/oracle.c``, builds it on the CPU and runs a fast subset
of the pins against it: at least one pin must fail. The planted copies live in
a temporary directory and are never used for anything else.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_f2 as f2
import test_oracle_fofc as fofc
import test_oracle_physics as phys
import test_oracle_smr as smr
import test_oracle_units as units
from paper_2409_16053_amd import problems as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, planted text)
MUTANTS = [
    ("hllc_energy_star_sign", "(sstar - uk) * (sstar + pk", "(sstar + uk) * (sstar + pk"),
    ("hllc_right_speed_sign", "sr = ur + ar * qr", "sr = ur - ar * qr"),
    ("hllc_sstar_dropped_term", "pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)",
     "pr - pl + rl * ul * (sl - ul)"),
    ("hllc_pvrs_sign", "0.5 * (pl + pr) - 0.5 * (ur - ul)", "0.5 * (pl + pr) + 0.5 * (ur - ul)"),
    ("plm_half_slope", "*right = w0 + 0.5 * slope;", "*right = w0 + slope;"),
    ("plm_limiter_factor", "2.0 * prod / (dl + dr)", "prod / (dl + dr)"),
    ("ppm4_interface_sixth", "(sc1 - sc) / 6.0", "(sc1 - sc) / 3.0"),
    ("ppm4_monotone_swap", "aL = 3.0 * a - 2.0 * aR", "aL = 3.0 * a - 2.0 * aL"),
    ("c2p_kinetic_half", "u[4] - 0.5 * ke2 / rho", "u[4] - ke2 / rho"),
    ("c2p_wrong_velocity", "w[2] = u[2] / rho;", "w[2] = u[3] / rho;"),
    ("divergence_wrong_width", "l -= (Fy[ym + nx] - Fy[ym]) / p->dx[1];",
     "l -= (Fy[ym + nx] - Fy[ym]) / p->dx[0];"),
    ("divergence_sign", "l -= (Fz[zm + (size_t)nx * ny] - Fz[zm]) / p->dx[2];",
     "l += (Fz[zm + (size_t)nx * ny] - Fz[zm]) / p->dx[2];"),
    ("rk2_stage2_weight", "k.a = 0.5; k.b = 0.5; k.c = 0.5;", "k.a = 0.5; k.b = 0.5; k.c = 1.0;"),
    ("rk3_stage2_weights", "k.a = 0.75; k.b = 0.25; k.c = 0.25;", "k.a = 0.25; k.b = 0.75; k.c = 0.25;"),
    ("rk3_stage3_step", "k.c = 2.0 / 3.0;", "k.c = 1.0 / 3.0;"),
    ("wenoz_linear_weights", "const double d[3] = {0.1, 0.6, 0.3};", "const double d[3] = {0.3, 0.6, 0.1};"),
    ("wenoz_candidate_sign", "(2.0 * (w[3] - w[2]) - (w[1] - w[2])) / 6.0",
     "(2.0 * (w[3] - w[2]) + (w[1] - w[2])) / 6.0"),
    ("wenoz_indicator_index", "0.25 * (w[1] - w[3]) * (w[1] - w[3])", "0.25 * (w[1] - w[2]) * (w[1] - w[2])"),
    ("wenoz_left_not_mirrored", "const double m[5] = {w[4], w[3], w[2], w[1], w[0]};",
     "const double m[5] = {w[0], w[1], w[2], w[3], w[4]};"),
    ("ppmx_second_order_interface", "0.5 * (b + c) - ((a - b) + (d - c)) / 12.0",
     "0.5 * (b + c) - 0.0 * ((a - b) + (d - c)) / 12.0"),
    ("ppmx_ratio_sign", "aL = a - ratio * dm;", "aL = a + ratio * dm;"),
    ("ppmx_overshoot_factor", "aR = a + 2.0 * dm;", "aR = a + 3.0 * dm;"),
    ("ppmx_limiter_constant", "#define OR_PPMX_C 1.25", "#define OR_PPMX_C 0.75"),
    ("rk4_combine_weight", "Q2[c] = Q2[c] / 25.0 + 9.0 / 25.0 * q1[c];", "Q2[c] = Q2[c] / 25.0 + 9.0 / 24.0 * q1[c];"),
    ("rk4_last_step", "RK4_LAST = {1.0, 3.0 / 5.0, 1.0 / 10.0}", "RK4_LAST = {1.0, 3.0 / 5.0, 1.0 / 6.0}"),
    ("ghost_periodic_offset", "return bchi == OR_PERIODIC ? c % n : n - 1;",
     "return bchi == OR_PERIODIC ? (c + 1) % n : n - 1;"),
    ("ghost_outflow_index", "return bclo == OR_PERIODIC ? ((c % n) + n) % n : 0;",
     "return bclo == OR_PERIODIC ? ((c % n) + n) % n : 1;"),
    ("unrotate_transposed", "  out[t1] = f[2];\n  out[t2] = f[3];", "  out[t1] = f[3];\n  out[t2] = f[2];"),
    ("dt_signed_velocity", "p->dx[d] / (fabs(q[1 + d]) + cs)", "p->dx[d] / (q[1 + d] + cs)"),
    ("dt_sound_speed_gamma", "sqrt(p->gamma * pr / q[0])", "sqrt(pr / q[0])"),
    ("face_state_shift", "s[o + 2] = w->W[at(G, v, i + o * di", "s[o + 2] = w->W[at(G, v, i + (o + 1) * di"),
    ("llf_dissipation_sign", "0.5 * (fl[q] + fr[q]) - 0.5 * a * (ur[q] - ul[q])",
     "0.5 * (fl[q] + fr[q]) + 0.5 * a * (ur[q] - ul[q])"),
    ("fofc_wrong_cell_side", "const int li = i - di * (1 - side)", "const int li = i - di * side"),
    ("smr_restriction_weight", "((f[4] + f[5]) + (f[6] + f[7]))) * 0.125;", "((f[4] + f[5]) + (f[6] + f[7]))) * 0.12;"),
    ("smr_prolongation_child_sign", "t[d] = (f[d] & 1) ? sd : -sd;", "t[d] = (f[d] & 1) ? -sd : sd;"),
    ("smr_prolongation_offset", "return C + 0.25 * ((t[0] + t[1]) + t[2]);", "return C + 0.5 * ((t[0] + t[1]) + t[2]);"),
    ("smr_prolongation_unlimited_slope", "return fabs(a) < fabs(b) ? a : b;", "return 0.5 * (a + b) + 0.0 * fabs(a);"),
    ("smr_child_order", "const int q = m->rleaf[r] + (lx & 1) + 2 * (ly & 1) + 4 * (lz & 1);",
     "const int q = m->rleaf[r] + (lx & 1) + 2 * (lz & 1) + 4 * (ly & 1);"),
    ("smr_flux_correction_dropped", "*smr_face(m, &w[q], d, v, cf[0], cf[1], cf[2]) = ((f[0] + f[1]) + (f[2] + f[3])) * 0.25;",
     "(void)f;"),
    ("smr_fine_face_side", "lf[d] = side ? 0 : m->b[d];", "lf[d] = side ? m->b[d] : 0;"),
    ("smr_fofc_twin_dropped", "for (int v = 0; v < 5; ++v) *smr_face(m, &w[qn], d, v, fc[0], fc[1], fc[2]) = f[v];",
     "(void)qn;"),
    ("smr_fofc_level_faces_not_corrected", "  long long flagged = smr_fofc_level(m, w, k, U0, Ust, h, Uout, 1);\n  smr_correct_fluxes(m, w);",
     "  long long flagged = smr_fofc_level(m, w, k, U0, Ust, h, Uout, 1);"),
    ("smr_fofc_coarse_level_first",
     "smr_fofc_level(m, w, k, U0, Ust, h, Uout, 1);\n  smr_correct_fluxes(m, w);\n  flagged += smr_fofc_level(m, w, k, U0, Ust, h, Uout, 0);",
     "smr_fofc_level(m, w, k, U0, Ust, h, Uout, 0);\n  smr_correct_fluxes(m, w);\n  flagged += smr_fofc_level(m, w, k, U0, Ust, h, Uout, 1);"),
    ("smr_fine_cell_width", "pl.dx[d] = m->lev[q] ? 0.5 * m->p.dx[d] : m->p.dx[d];", "pl.dx[d] = m->p.dx[d];"),
]


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11", "-shared",
                           "-fPIC", str(path), "-o", str(lib), "-lm"])
    return oracle.Oracle.from_path(str(lib))


def _fast_pins(O):
    """A quick subset of the pins, each given the planted build."""
    yield lambda: units.test_plm_harmonic_mean_worked_example(O)
    yield lambda: units.test_ppm4_cubic_interfaces_exact(O)
    yield lambda: units.test_ppm4_overshoot_worked_example(O)
    yield lambda: units.test_hllc_consistency(O, 5.0 / 3.0)
    yield lambda: units.test_hllc_contact_resolution(O, 5.0 / 3.0)
    yield lambda: units.test_hllc_mirror_symmetry(O, 5.0 / 3.0)
    yield lambda: units.test_hllc_weak_jumps_match_godunov_to_second_order(O, 1.4)
    yield lambda: units.test_c2p_roundtrip(O)
    yield lambda: units.test_new_dt_closed_form(O)
    for bcs in (((0, 0), (0, 0), (0, 0)), ((1, 1), (1, 1), (1, 1))):
        yield lambda bcs=bcs: units.test_ghost_fill_matches_numpy_pad(O, P.PLM, bcs)
    yield lambda: phys.test_uniform_state_preserved_bitwise(O, P.PLM, P.PERIODIC)
    yield lambda: phys.test_periodic_conservation(O, P.PLM, "kh")
    yield lambda: phys.test_sound_wave_second_order_1d_plm(O, 0)
    yield lambda: phys.test_sod_converges_to_exact(O, 1.4, P.PLM)
    yield lambda: phys.test_sod_axis_symmetry_bitwise(O, P.PLM)
    yield lambda: phys.test_colliding_streams_two_shocks(O, P.PLM)
    yield lambda: phys.test_shear_wave_advection(O, 0)
    yield lambda: fofc.test_llf_is_hll_with_symmetric_speeds(O, 1.4)
    yield lambda: fofc.test_fofc_restores_positivity_hypersonic_turbulence(O, P.PLM)
    yield lambda: f2.test_wenoz_exact_for_quadratics(O)
    yield lambda: f2.test_wenoz_matches_its_definition(O)
    yield lambda: f2.test_wenoz_fifth_order_on_smooth_data(O)
    yield lambda: f2.test_wenoz_takes_the_smooth_side_of_a_jump(O)
    yield lambda: f2.test_ppmx_keeps_a_smooth_extremum(O)
    yield lambda: f2.test_ppmx_exact_for_monotone_cubics(O)
    yield lambda: f2.test_ppmx_no_new_extremum_at_a_jump(O)
    yield lambda: f2.test_ppmx_parabola_monotone_on_monotone_data(O)
    yield lambda: f2.test_time_order_of_the_integrators(O, P.WENOZ, 3, 256, (0.8, 0.4), 2.75, 3.3)
    yield lambda: f2.test_time_order_by_richardson(O, 4, 4.0)
    yield lambda: smr.test_face_ghosts_exact_for_linear_fields(O, P.PLM)
    yield lambda: smr.test_face_ghosts_match_independent_restriction_and_prolongation(
        O, (32, 24, 24), (8, 6, 12), ((1, 1, 0), (3, 3, 1)))
    yield lambda: smr.test_uniform_state_stays_uniform_bitwise(O, P.PERIODIC, P.PLM)
    yield lambda: smr.test_periodic_refined_mesh_conserves(O, P.PLM, 2)
    yield lambda: smr.test_full_refinement_equals_uniform_fine_grid_bitwise(O, P.PERIODIC)
    yield lambda: smr.test_fofc_empty_refinement_equals_uniform_bitwise(O, P.PLM, 2)
    yield lambda: smr.test_fofc_refined_hypersonic_turbulence(O, P.PLM, 2)
    yield lambda: smr.test_fofc_refined_hypersonic_turbulence(O, P.PPM4, 3)


def test_unplanted_build_passes_fast_pins(tmp_path):
    O = _build(tmp_path, "clean", "int or_nghost", "int or_nghost")
    for pin in _fast_pins(O):
        pin()


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    O = _build(tmp_path, name, old, new)
    caught = []
    for n, pin in enumerate(_fast_pins(O)):
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError) as e:
            caught.append((n, type(e).__name__))
            break
    assert caught, f"no pin caught the planted mistake {name}"
