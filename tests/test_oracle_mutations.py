"""The pins must bite: plant plausible mistakes in a copy of the oracle (CPU
only), rebuild it, and check that every mutant fails at least one pin."""
import os
import shutil
import subprocess
import tempfile

import pytest

from oracle import oracle as O
import tests.test_oracle_elements as TE
import tests.test_oracle_assembly as TA
import tests.test_oracle_shell as TS
import tests.test_oracle_cloth as TC
import tests.test_oracle_residual as TR

MUTANTS = {
    "product_rule_drops_cross_term": ("+ a.g[i] * b.g[j] + b.g[i] * a.g[j];", "+ a.g[i] * b.g[j];"),
    "unary_drops_second_derivative": ("f1 * a.h[i][j] + f2 * a.g[i] * a.g[j]", "f1 * a.h[i][j]"),
    "atan2_wrong_sign_dx": ("x.v / r2, -y.v / r2,", "x.v / r2, y.v / r2,"),
    "atan2_wrong_mixed_second": ("(y.v * y.v - x.v * x.v) / r4", "(x.v * x.v - y.v * y.v) / r4"),
    "sqrt_wrong_second": ("-0.25 / (s * a.v)", "-0.5 / (s * a.v)"),
    "recip_wrong_second": ("2.0 / (v * v * v)", "1.0 / (v * v * v)"),
    "cross_wrong_index": ("r.c[1] = hd_sub(hd_mul(a.c[2], b.c[0]), hd_mul(a.c[0], b.c[2]));",
                          "r.c[1] = hd_sub(hd_mul(a.c[2], b.c[0]), hd_mul(a.c[0], b.c[1]));"),
    "stvk_transposed_dminv": ("F[i][j] = hd_add(hd_scale(d1.c[i], mi[0 * 2 + j]), hd_scale(d2.c[i], mi[1 * 2 + j]));",
                              "F[i][j] = hd_add(hd_scale(d1.c[i], mi[j * 2 + 0]), hd_scale(d2.c[i], mi[j * 2 + 1]));"),
    "stvk_drops_lambda_half": ("hd_scale(hd_sq(trE), 0.5 * lam)", "hd_scale(hd_sq(trE), lam)"),
    "bending_flipped_n2": ("hd3 n2 = hd3_cross(hd3_sub(x3, x0), e);", "hd3 n2 = hd3_cross(e, hd3_sub(x3, x0));"),
    "bending_area_not_third": ("kb * abar / 3.0 * ht * ht", "kb * abar / 2.0 * ht * ht"),
    "dirichlet_dm_not_transposed": ("hd g0 = hd_add(hd_scale(d1, mi[0]), hd_scale(d2, mi[2]));",
                                    "hd g0 = hd_add(hd_scale(d1, mi[0]), hd_scale(d2, mi[1]));"),
    "symdir_wrong_inverse_entry": ("Ji[0][0] = hd_mul(J[1][1], idet);", "Ji[0][0] = hd_mul(J[0][0], idet);"),
    "rest_frame_sign": ("dm01 = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / l1;",
                        "dm01 = -(e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / l1;"),
    "jacobi_wrong_rotation_sign": ("A[r][p] = c * ap - s * aq;\n                    A[r][q] = s * ap + c * aq;\n                }\n                for (int r = 0; r < n; ++r) {\n                    double ap = A[p][r]",
                                   "A[r][p] = c * ap + s * aq;\n                    A[r][q] = s * ap + c * aq;\n                }\n                for (int r = 0; r < n; ++r) {\n                    double ap = A[p][r]"),
    "clamp_uses_abs": ("double lam = A[m][m] > eps ? A[m][m] : eps;", "double lam = fabs(A[m][m]);"),
    "pattern_drops_diagonal": ("keys[m++] = i * nv + i;", "keys[m++] = 0;"),
    "assembly_transposes_block": ("Hp[(a * d + i) * k + (b * d + j)]", "Hp[(a * d + j) * k + (b * d + i)]"),
    "diamond_wrong_wing": ("d[3] = rec[i + 1].opp;", "d[3] = rec[i].opp;"),
    "neumaier_wrong_sign": ("c += (s - t) + v[i];", "c += (s - t) - v[i];"),
    "shell_ii_wrong_sign": ("z[3 + q] = hd_addc(hd_scale(ii, -0.5), -rest[5 + q]);",
                            "z[3 + q] = hd_addc(hd_scale(ii, 0.5), -rest[5 + q]);"),
    "shell_ii_drops_symmetric_part": ("ii = hd_add(ii, hd_add(hd_scale(F[i][b], N[i][a]), hd_scale(F[i][a], N[i][b])));",
                                      "ii = hd_add(ii, hd_scale(hd_scale(F[i][b], N[i][a]), 2.0));"),
    "shell_n_transposed_dminv": ("N[i][j] = dn1 * mi[0 * 2 + j] + dn2 * mi[1 * 2 + j];",
                                 "N[i][j] = dn1 * mi[j * 2 + 0] + dn2 * mi[j * 2 + 1];"),
    "shell_plain_ii_wrong_rest": ("z[6 * f + 3 + q] = -0.5 * ii - mi[5 + q];", "z[6 * f + 3 + q] = -0.5 * ii + mi[5 + q];"),
    "shell_density_drops_factor_two": ("hd b2 = hd_add(hd_add(hd_sq(z[3]), hd_sq(z[4])), hd_scale(hd_sq(z[5]), 2.0));",
                                       "hd b2 = hd_add(hd_add(hd_sq(z[3]), hd_sq(z[4])), hd_sq(z[5]));"),
    "softplus_wrong_second": ("return hd_unary(a, softplus(a.v), s, s * (1.0 - s));",
                              "return hd_unary(a, softplus(a.v), s, s * s);"),
    "mlp_transposed_w2": ("a = hd_add(a, hd_scale(h1[n], W2[m * H + n]));", "a = hd_add(a, hd_scale(h1[n], W2[n * H + m]));"),
    "mlp_input_scale_dropped": ("xin[i] = hd_scale(z[i], sin_[i]);", "xin[i] = z[i];"),
    "normals_not_normalized": ("for (int d = 0; d < 3; ++d) n[d] /= l;", "for (int d = 0; d < 3; ++d) n[d] /= 1.0;"),
    "spring_drops_rest_length_factor": ("return hd_scale(hd_sq(q), prm[1] * 0.5 * prm[0] * l2);",
                                        "return hd_scale(hd_sq(q), prm[1] * 0.5 * prm[0]);"),
    "spring_strain_not_normalised": ("hd q = hd_addc(hd_scale(hd3_dot(d, d), 1.0 / l2), -1.0);",
                                     "hd q = hd_addc(hd3_dot(d, d), -1.0);"),
    "inertia_gravity_wrong_sign": ("acc = hd_add(acc, hd_scale(x.c[c], -prm[0] * m * prm[1 + c]));",
                                   "acc = hd_add(acc, hd_scale(x.c[c], prm[0] * m * prm[1 + c]));"),
    "inertia_drops_half": ("acc = hd_add(acc, hd_scale(hd_sq(dc), 0.5 * m));", "acc = hd_add(acc, hd_scale(hd_sq(dc), m));"),
    "inertia_rest_stride_wrong": ("case OR_INERTIA: case OR_RES_POSITION: return 4;",
                                  "case OR_INERTIA: case OR_RES_POSITION: return 3;"),
    "res_edge_weight_not_sqrt": ("out[0] = hd_scale(hd_addc(hd_sqrt(hd3_dot(d, d)), -rest[0]), sqrt(prm[0]));",
                                 "out[0] = hd_scale(hd_addc(hd_sqrt(hd3_dot(d, d)), -rest[0]), prm[0]);"),
    "gauss_newton_drops_half": ("out.v += 0.5 * res[i].v * res[i].v;", "out.v += res[i].v * res[i].v;"),
}

PINS = [TE.test_edge_sqlen_closed_form, TE.test_area_gradient_matches_paper_closed_form,
        TE.test_dirichlet_is_cotangent_stiffness, TE.test_dirichlet_constant_field_and_linear_field,
        TE.test_stvk_rest_hessian_is_linear_elastic_cst, TE.test_stvk_rigid_motion_zero_and_invariances,
        TE.test_stvk_uniform_stretch_energy, TE.test_bending_wing_gradient_and_rank_one_at_rest_angle,
        TE.test_bending_fd_and_invariances, TE.test_symdir_identity_map_and_fd,
        TE.test_stvk_fd_large_deformation, TE.test_spd_projection_leaves_psd_unchanged_and_handles_repeated_eigs,
        TE.test_element_spd_mode_equals_projection_of_raw_hessian,
        lambda: TE.test_bending_hinge_angle_closed_form(0.3),
        lambda: TE.test_spd_projection_matches_lapack(6),
        TA.test_topology_two_triangles_diamond_order, lambda: TA.test_pattern_brute_force("grid3"),
        lambda: TA.test_pattern_brute_force("nonmanifold"),
        lambda: TA.test_assembly_equals_dense_sum("grid3", True), TA.test_dirichlet_assembly_is_cotangent_laplacian,
        TA.test_neumaier_matches_exact_sum,
        TS.test_features_vanish_at_rest_and_are_rigid_invariant, TS.test_membrane_part_equals_stvk_element,
        TS.test_sphere_normals_give_second_form_minus_first_over_radius,
        TS.test_cylinder_normals_second_form_closed_form, TS.test_plain_features_equal_hyper_dual_features,
        TS.test_vertex_normals_closed_forms, TS.test_shell_element_fd_and_invariance,
        TS.test_one_neuron_network_closed_form, TS.test_network_derivatives_fd_and_reverse_mode_agree,
        TS.test_mlp_element_is_area_times_network_of_features, TS.test_shell_density_closed_form_gradient_by_fd,
        lambda: TC.test_spring_matches_closed_form(0.95), TC.test_inertia_matches_closed_form,
        lambda: TC.test_cloth_step_assembly_matches_dense_closed_form(True, 0.0),
        TR.test_position_residual_closed_form, TR.test_edge_residual_closed_form_and_fd,
        lambda: TR.test_residual_kind_as_scalar_term_is_gauss_newton(O.RES_EDGE),
        TR.test_assembled_jacobian_is_the_stacked_local_jacobians]


def run_pins():
    failed = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, RuntimeError, ValueError, FloatingPointError):
            failed.append(getattr(pin, "__name__", "lambda"))
    return failed


@pytest.fixture(scope="module")
def mutant_dir():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_unmutated_oracle_passes_all_pins():
    assert run_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, mutant_dir):
    src = open(os.path.join(os.path.dirname(O.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(old, new, 1)
    cpath = os.path.join(mutant_dir, f"{name}.c")
    spath = os.path.join(mutant_dir, f"lib{name}.so")
    with open(cpath, "w") as fh:
        fh.write(mutated)
    shutil.copy(os.path.join(os.path.dirname(O.__file__), "oracle.h"), mutant_dir)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", spath, cpath, "-lm"])
    with O.using(O.load(spath)):
        failed = run_pins()
    assert failed, f"mutant {name} passed every pin"
