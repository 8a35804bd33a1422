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
