"""Plant plausible mistakes in a copy of the oracle and check that the pins in
test_oracle_pins.py catch each one (CPU only; the copies are built in a
temporary directory with gcc)."""
import os
import shutil
import subprocess

import pytest

import oracle
from oracle.oracle import Variant, build
from tests import test_oracle_pins as pins
from tests import test_oracle_pins_u as upins
from tests import test_oracle_pins_blip as bpins
from tests import test_oracle_pins_layers as lpins

SRC = os.path.join(os.path.dirname(oracle.lib_path()), "oracle.c")

# (name, original text, mutated text)
MUTATIONS = [
    ("drop_background", "parts[4] = e_real + e_recip + e_self + e_bg;",
     "parts[4] = e_real + e_recip + e_self;"),
    ("self_sign", "double e_self = -a / sqrt(O_PI) * q2;", "double e_self = a / sqrt(O_PI) * q2;"),
    ("gauss_exponent", "exp(-g2 / (4 * a * a))", "exp(-g2 / (2 * a * a))"),
    ("recip_prefactor", "return 2 * O_PI / measure * exp", "return 4 * O_PI / measure * exp"),
    ("recip_2d_transposed", "bm[1] = -2 * O_PI * a[3] / det;", "bm[1] = -2 * O_PI * a[1] / det;"),
    ("recip_3d_wrong_cross", "bm[3 + d] = 2 * O_PI * c31[d] / det;", "bm[3 + d] = 2 * O_PI * c23[d] / det;"),
    ("erfc_over_r2", "if (dist < rc) sum += erfc(a * dist) / dist;", "if (dist < rc) sum += erfc(a * dist) / d2;"),
    ("self_image_factor", "e_real += 0.5 * q2 * self_img;", "e_real += q2 * self_img;"),
    ("erfc_2d_argument", "erfc(g / (2 * a)) / g", "erfc(g / a) / g"),
    ("cutoff_shrunk", "if (dist < rc) sum +=", "if (dist < 0.9 * rc) sum +="),
    ("delta_drop_square", "double tt = 2 * (rre[t] * dre + rim[t] * dim_) + dre * dre + dim_ * dim_;",
     "double tt = 2 * (rre[t] * dre + rim[t] * dim_);"),
    ("delta_old_sign", "- real_image_sum(s, bm, dold, 0));", "+ real_image_sum(s, bm, dold, 0));"),
    ("rho_update_sign", "rre[t] += q[kk] * (cos(pn) - cos(po));", "rre[t] -= q[kk] * (cos(pn) - cos(po));"),
    ("jastrow_half", "jas += 0.5 * jastrow_coef(s, g.shell[t]) * r2;", "jas += jastrow_coef(s, g.shell[t]) * r2;"),
    ("shell_order_reversed", "{ sidx = u; break; }", "{ sidx = nu - 1 - u; break; }"),
    ("run_batch_k_transposed", "kw[m] = k[(size_t)m * n_walkers + w];", "kw[m] = k[(size_t)w * n_steps + m];"),
    ("jgrad_factor", "gr[e] += 2 * q[k] * q[j] * pg[e];", "gr[e] += q[k] * q[j] * pg[e];"),
    ("jgrad_cos", "pg[e] += -0.5 * a * g.g[3 * t + e] * sin(ph);", "pg[e] += -0.5 * a * g.g[3 * t + e] * cos(ph);"),
    ("jlap_norm", "pl += -0.5 * a * g.g2[t] * cos(ph);", "pl += -0.5 * a * sqrt(g.g2[t]) * cos(ph);"),
    ("jlap_sign", "lp += 2 * q[k] * q[j] * pl;", "lp -= 2 * q[k] * q[j] * pl;"),
    ("jderiv_old_position", "prop[dim * kk + e] = rn[e];", "prop[dim * kk + e] = ro[e];"),
    ("u_sign_convention", "double x = r - s->u_cut;", "double x = s->u_cut - r;"),
    ("u_power_index", "P += a[l] * pow(r, l);", "P += a[l] * pow(r, l + 1);"),
    ("u_dpoly_index", "if (l >= 1) dP += l * a[l] * pow(r, l - 1);", "if (l >= 1) dP += a[l] * pow(r, l - 1);"),
    ("u_channel_swapped", "return s->spin[i] == s->spin[j] ? 0 : 1;", "return s->spin[i] == s->spin[j] ? 1 : 0;"),
    ("u_ions_included", "if (s->n_u <= 0 || !s->spin || s->spin[i] < 0 || s->spin[j] < 0) return -1;",
     "if (s->n_u <= 0 || !s->spin) return -1;"),
    ("u_cutoff_widened", "if (rho >= s->u_cut) continue;", "if (rho >= 1.5 * s->u_cut) continue;"),
    ("u_d2_cross_term", "2.0 * C * dP * xc1", "C * dP * xc1"),
    ("u_lap_dim", "l += d2u + (dim - 1) * du / rho;", "l += d2u + dim * du / rho;"),
    ("u_grad_sign", "g[e] += du * r[e] / rho;", "g[e] -= du * r[e] / rho;"),
    ("u_delta_old_sign", "dj += un - uo;", "dj += un + uo;"),
    ("blip_inner_cubic", "return 1.0 - 1.5 * x * x + 0.75 * ax * ax * ax;", "return 1.0 - 1.5 * x * x + 0.5 * ax * ax * ax;"),
    ("blip_outer_power", "return 0.25 * t * t * t;", "return 0.25 * t * t;"),
    ("blip_d1_sign", "return -0.75 * sg * t * t;", "return 0.75 * sg * t * t;"),
    ("blip_d2_inner", "return -3.0 + 4.5 * ax;", "return -3.0 + 3.0 * ax;"),
    ("blip_jacobian_transposed", "J[3 * e + d] = ainv[3 * e + d] * nn[d];", "J[3 * e + d] = ainv[3 * d + e] * nn[d];"),
    ("blip_lap_diagonal_only", "lp += J[3 * e + d] * J[3 * e + d2] * hx[3 * d + d2];",
     "lp += (d == d2) * J[3 * e + d] * J[3 * e + d2] * hx[3 * d + d2];"),
    ("blip_no_wrap", "off[d] -= nn[d] * floor(off[d] / nn[d] + 0.5);", "off[d] -= 0.0;"),
    ("blip_grid_scale", "x[d] = nn[d] * s;", "x[d] = (nn[d] - 1) * s;"),
    ("blip_coef_index", "(((size_t)i * n2 + j) * n3 + k)", "(((size_t)i * n3 + j) * n2 + k)"),
    ("layer_exp_sign", "double f = exp(z * gg) * erfc(gg / (2 * a) + z * a)",
     "double f = exp(-z * gg) * erfc(gg / (2 * a) + z * a)"),
    ("layer_const_erf", "return -2 * O_PI / area * (z * erf(z * a)", "return -2 * O_PI / area * (z * erfc(z * a)"),
    ("layer_const_gauss", "exp(-a * a * z * z) / (a * sqrt(O_PI))", "exp(-a * z * z) / (a * sqrt(O_PI))"),
    ("layer_real_z_dropped", "double dist = sqrt(r0 * r0 + r1 * r1 + z * z);", "double dist = sqrt(r0 * r0 + r1 * r1);"),
    ("layer_recip_prefactor", "return O_PI / area * sum;", "return 2 * O_PI / area * sum;"),
    ("layer_delta_same_plane", "double z = s->z[k] - s->z[j];", "double z = 0.0;"),
    ("layer_madelung_factor", "e_recip += 0.5 * q2 * 2 * O_PI / area * vm_recip;",
     "e_recip += 0.5 * q2 * O_PI / area * vm_recip;"),
]

CHECKS = [
    lambda o: [pins.test_wigner_3d(o, n, 1.0) for n in ("sc", "fcc", "bcc")],
    lambda o: [pins.test_wigner_2d(o, n) for n in ("triangular", "square")],
    lambda o: pins.test_nacl_madelung(o),
    lambda o: [pins.test_alpha_independence(o, 3, True, False), pins.test_alpha_independence(o, 2, True, False)],
    lambda o: [pins.test_lattice_basis_invariance(o, d) for d in (2, 3)],
    lambda o: pins.test_cutoff_shells(o),
    lambda o: [pins.test_incremental_moves_match_recompute(o, c) for c in (1, 3)],
    lambda o: pins.test_jastrow_structure_factor_equals_pair_form(o),
    lambda o: [pins.test_jastrow_shells_cubic(o, d) for d in (3, 2)],
    lambda o: [pins.test_shell_index_order(o, c) for c in (1, 3)],
    lambda o: [pins.test_run_batch_matches_run(o, c) for c in (2, 3)],
    lambda o: [pins.test_jastrow_derivs_finite_differences(o, d) for d in (3, 2)],
    lambda o: pins.test_run_derivs_at_proposed_configuration(o),
    lambda o: upins.test_u_closed_form_values(o),
    lambda o: upins.test_u_minimum_image(o),
    lambda o: [upins.test_u_cusp(o, c, p) for c in (1, 3) for p in (True, False)],
    lambda o: upins.test_u_order_c_zero_at_cutoff(o),
    lambda o: [upins.test_u_derivs_finite_differences(o, d) for d in (3, 2)],
    lambda o: [upins.test_u_incremental_moves_and_invariance(o, c) for c in (1, 3)],
    lambda o: bpins.test_blip_partition_of_unity(o),
    lambda o: bpins.test_blip_linear_reproduction(o),
    lambda o: [bpins.test_blip_plane_wave_at_nodes(o, m) for m in ((1, 0, 0), (2, -3, 1), (0, 4, 5))],
    lambda o: bpins.test_blip_lattice_periodicity(o),
    lambda o: bpins.test_blip_derivs_finite_differences(o),
    lambda o: bpins.test_blip_function_values(o),
    lambda o: lpins.test_layers_zero_height_equals_2d(o),
    lambda o: [lpins.test_layers_alpha_independence(o, d) for d in (0.7, 2.5)],
    lambda o: lpins.test_layers_charged_sheets(o),
    lambda o: lpins.test_layers_invariances(o),
    lambda o: lpins.test_layers_incremental_moves(o),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,orig,mut", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutation(tmp_path, name, orig, mut):
    text = open(SRC).read()
    assert text.count(orig) >= 1, f"mutation anchor not found: {orig}"
    src = tmp_path / "oracle_mut.c"
    src.write_text(text.replace(orig, mut))
    so = build(str(src), str(tmp_path / "liboracle_mut.so"))
    variant = Variant(so)
    caught = []
    for i, check in enumerate(CHECKS):
        try:
            check(variant)
        except (AssertionError, subprocess.CalledProcessError):
            caught.append(i)
    assert caught, f"no pin caught the planted mistake {name}"
