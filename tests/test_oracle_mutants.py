"""Planted mistakes: each mutant of the oracle source (a dropped term, a
wrong sign or index, a transposed operand, an off-by-one stop) is compiled on
the CPU and must fail at least one of the pins.  This checks that the pins
constrain every step of the oracle, not only the ones that are easy to test.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import build as ob
from oracle import ref as oref

import test_oracle_fd as fd
import test_oracle_median as med
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(ob.__file__), "gsr_ref.c")

# (name, original snippet, planted mistake)
MUTANTS = [
    ("no_lowpass", "r->cov[0] = S2[0] + LOWPASS;", "r->cov[0] = S2[0];"),
    ("conic_B_sign", "r->conic[1] = -r->cov[1] / r->det;", "r->conic[1] = r->cov[1] / r->det;"),
    ("rot_transposed", "R[1] = 2.0 * (x * y - w * z);", "R[1] = 2.0 * (x * y + w * z);"),
    ("stop_off_by_one", "if (Tn < T_MIN) break;", "if (T < T_MIN) break;"),
    ("extent", "#define EXTENT 3.0", "#define EXTENT 3.5"),
    ("back_to_front", "if (da != db) return da < db ? -1 : 1;", "if (da != db) return da > db ? -1 : 1;"),
    ("depth_weight", "*Sz += r->z * w;", "*Sz += r->z * a;"),
    ("colour_offset", "r->raw[c] = s + 0.5;", "r->raw[c] = s;"),
    ("sh_sign", "Y[1] = -k1 * y;", "Y[1] = k1 * y;"),
    ("bwd_no_suffix", "dLda += GC[c] * (r->color[c] * b->Ti - accc[c] / om);",
     "dLda += GC[c] * (r->color[c] * b->Ti);"),
    ("bwd_alpha_grad", "dLda += GA * (Tf / om);", "dLda += GA * Tf;"),
    ("bwd_dq_half", "const double dLdq = -0.5 * b->a * dLda;", "const double dLdq = -b->a * dLda;"),
    ("twist_phi_sign", "twf[3] += ty * dt[2] - tz * dt[1];", "twf[3] += tz * dt[1] - ty * dt[2];"),
    ("twist_no_centre", "twf[a] += W[a * 3 + 0] * dd[0] + W[a * 3 + 1] * dd[1] + W[a * 3 + 2] * dd[2];",
     "(void)dd;"),
    ("twist_no_cov", "twf[3 + k] += s;", "(void)s;"),
    ("quat_no_projection", "g_quats[g * 4 + a] = (dqh[a] - G.qh[a] * proj) / G.qn;",
     "g_quats[g * 4 + a] = dqh[a] / G.qn;"),
    ("opacity_chain", "g_opac[g] = dsig * G.opacity * (1.0 - G.opacity);", "g_opac[g] = dsig * G.opacity;"),
    ("jacobian_tz", "dt[2] += GJ[0] * (-fx / (tz * tz));", "dt[2] += GJ[0] * (-fx / tz);"),
    ("scale_chain", "g_log_scales[g * 3 + a] = ds[a] * G.s[a];", "g_log_scales[g * 3 + a] = ds[a];"),
    ("sh_grad_dir", "dd[a] = (ddir[a] - r->dir[a] * dd0) / r->dist;", "dd[a] = ddir[a] / r->dist;"),
    ("jguard_tz_term", "dt[2] += GJ[2] * (fx * txc / (tz * tz * tz));", "(void)txc;"),
    ("jguard_txc_for_tx", "dt[2] += GJ[2] * (fx * txc / (tz * tz * tz));",
     "dt[2] += GJ[2] * (fx * tx / (tz * tz * tz));"),
    ("jguard_y_tz_term", "dt[2] += GJ[5] * (fy * tyc / (tz * tz * tz));",
     "dt[2] += GJ[5] * (fy * ty / (tz * tz * tz));"),
    ("jguard_width_for_height", "const double limy = JGUARD * (double)cam->height / (2.0 * fy);",
     "const double limy = JGUARD * (double)cam->width / (2.0 * fy);"),
    ("jguard_flag_without_clamp", "if (rx > limx) { rx = limx; r->clamp_x = 1; }",
     "if (rx > limx) { r->clamp_x = 1; }"),
    ("nonfinite_sh_unchecked", "if (!isfinite(st->sh[g * st->K_sh * 3 + i])) return 0;", "(void)0;"),
    ("nonfinite_grads_not_zeroed", "if (!kept) { /* no frame sees it", "if (0) { /* no frame sees it"),
    ("median_before_blend", "if (*med < 0 && Tn < 0.5) {", "if (*med < 0 && T < 0.5) {"),
    ("median_last_crossing", "if (*med < 0 && Tn < 0.5) {", "if (Tn < 0.5) {"),
    ("median_bwd_blended", "if (i == med) gr[9] += GD;", "gr[9] += GD * w;"),
]

CHECKS = [
    ("brute", lambda: pins.test_brute_force_matches_oracle(2, 150, 2, 2, (32, 8))),
    ("brute_sh3", lambda: pins.test_brute_force_matches_oracle(1, 120, 3, 1, (8, 8))),
    ("closed_form", lambda: pins.test_single_gaussian_closed_form(dict(o=4.0, ls=(-2.5, -2.9, -3.1)))),
    ("over", pins.test_over_operator_and_order),
    ("early_stop", pins.test_early_stop_excludes_the_crossing_entry),
    ("sh_scipy", lambda: pins.test_sh_basis_matches_scipy(3)),
    ("quat_scipy", pins.test_quaternion_matches_scipy),
    ("fd_params", lambda: fd.test_parameter_gradients_match_central_differences(11, 3, 2, (0.1, 0.2, 0.3))),
    ("fd_twist", lambda: fd.test_twist_gradient_matches_central_differences(21, 3)),
    ("fd_colour", fd.test_colour_clamp_and_direction_paths),
    ("guard_jacobian", lambda: pins.test_guard_is_the_jacobian_at_the_clamped_point(41)),
    ("fd_guard", lambda: fd.test_gradients_through_the_jacobian_guard(41, 2)),
    ("nonfinite_sh", lambda: pins.test_nonfinite_gaussian_is_removed("sh", (0, 0, 1), np.nan)),
    ("nonfinite_quat", lambda: pins.test_nonfinite_gaussian_is_removed("quats", (0, 0), np.nan)),
    ("median_brute", lambda: med.test_median_matches_brute_force(2, 150, 2, (32, 8))),
    ("median_layered", lambda: med.test_layered_closed_form([-0.9, -0.4, 2.0], [3.5, 2.0, 2.5])),
    ("median_grad", med.test_single_pixel_gradient_closed_form),
]


def _build_mutant(src_text, outdir, name):
    c = os.path.join(outdir, f"{name}.c")
    so = os.path.join(outdir, f"lib_{name}.so")
    with open(c, "w") as f:
        f.write(src_text)
    inc = os.path.dirname(SRC)
    subprocess.run(["gcc", "-O1", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp",
                    "-fPIC", "-shared", "-I", inc, c, "-o", so, "-lm"], check=True,
                   capture_output=True)
    return so


def _caught(so):
    prev = oref.use_library(so)
    try:
        for name, fn in CHECKS:
            try:
                fn()
            except (AssertionError, ValueError, FloatingPointError):
                return name
        return None
    finally:
        oref.use_library(prev)


def test_unmutated_oracle_passes_every_check():
    for name, fn in CHECKS:
        fn()


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, orig, bad):
    text = open(SRC).read()
    assert text.count(orig) == 1, f"snippet for {name} not unique in the oracle"
    with tempfile.TemporaryDirectory() as d:
        so = _build_mutant(text.replace(orig, bad), d, name)
        caught_by = _caught(so)
    assert caught_by is not None, f"mutant {name} passed every pin"
    print(f"mutant {name}: caught by {caught_by}")
