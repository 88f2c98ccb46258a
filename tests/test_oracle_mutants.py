"""The pins catch plausible mistakes: each case plants one mistake in a copy
of the oracle's source (CPU only), builds it, and runs the pins that must now
fail."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

MUTANTS = [
    ("conic cross term sign in the blend",
     "- r.bcon[1] * dx * dy;", "+ r.bcon[1] * dx * dy;",
     "test_anisotropic_gaussian_pixel_values"),
    ("colour not weighted by transmittance",
     "C[c] += r.brgb[c] * alpha * T;", "C[c] += r.brgb[c] * alpha;",
     "test_weights_plus_transmittance_sum_to_one or test_two_gaussians_front_to_back"),
    ("quaternion rotation transposed",
     "R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);",
     "R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y + w * z);",
     "test_quaternion_rotation_matches_scipy or test_rotated_anisotropic_on_axis_uses_R_S_S_R"),
    ("affine instead of perspective-correct mesh interpolation",
     "const double q0 = b0 / tv[0].p[2], q1 = b1 / tv[1].p[2], q2 = b2 / tv[2].p[2];",
     "const double q0 = b0 / 1.0, q1 = b1 / 1.0, q2 = b2 / 1.0;",
     "test_room_mesh_matches_analytic_raycast"),
    ("bilinear without the half-texel offset",
     "const double x = uv[0] * sc.tex_w - 0.5, y = uv[1] * sc.tex_h - 0.5;",
     "const double x = uv[0] * sc.tex_w, y = uv[1] * sc.tex_h;",
     "test_config1_quad_depth_and_bilinear_block_mean or test_bilinear_texel_centre_and_clamp"),
    ("dropped suffix product in dT/dalpha",
     "galpha += gT * (-st.T * P);", "galpha += gT * (-st.T);",
     "test_oracle_gradient_matches_finite_differences"),
    ("sign of the conic gradient",
     "H[2 * a + c] = -(QG[2 * a] * Q[c] + QG[2 * a + 1] * Q[2 + c]);",
     "H[2 * a + c] = (QG[2 * a] * Q[c] + QG[2 * a + 1] * Q[2 + c]);",
     "test_oracle_gradient_matches_finite_differences"),
    ("Jacobian taken at the unclamped direction",
     "r.xc = std::min(limx, std::max(-limx, xz));", "r.xc = xz;",
     "test_jacobian_clamp_outside_the_view"),
    ("tile rectangle one tile short",
     "r.x1 = clampi(std::floor(ex1) + 1, TX);", "r.x1 = clampi(std::floor(ex1), TX);",
     "test_rect_is_the_tile_cover_of_the_3sigma_box or test_keys_match_brute_force_lexsort"),
    ("transmittance stop removed",
     "if ((Tn < p.t_min) != flipped((int)k, 1)) {", "if (false) {",
     "stack or n_contrib_is"),
    ("the Gaussian that crosses t_min blended before the stop",
     "      *npro = (int)k + 1;\n      h = mix(h, 2);\n      break;",
     "      for (int c = 0; c < 3; ++c) C[c] += r.brgb[c] * alpha * T;\n"
     "      T = Tn; *nc = (int)k + 1; *nb += 1;\n"
     "      *npro = (int)k + 1;\n      h = mix(h, 2);\n      break;",
     "stack"),
    ("n_contrib counted from 0",
     "*nc = (int)k + 1;", "*nc = (int)k;",
     "stack or n_contrib_is or strict"),
    ("tile-ellipse cut without its FP32 growth margin",
     "const double rp = 1.01 * rr + 0.1 + 1e-5 * (a + c) * ext * ext;", "const double rp = rr;",
     "tile_ellipse_key_set"),
    ("tile-ellipse run one tile short on the right",
     "*x1 = std::min(*x1, (int)std::floor((r.bu + xmax - 0.5) / tile) + 1);",
     "*x1 = std::min(*x1, (int)std::floor((r.bu + xmax - 0.5) / tile));",
     "tile_ellipse_key_set"),
    ("SH degree-2 constant off",
     "const double a2 = 0.5 * std::sqrt(15.0 / PI), b2 = 0.25 * std::sqrt(5.0 / PI),\n               d2 = 0.25 * std::sqrt(15.0 / PI);\n  Y[4]",
     "const double a2 = 0.5 * std::sqrt(15.0 / PI), b2 = 0.25 * std::sqrt(3.0 / PI),\n               d2 = 0.25 * std::sqrt(15.0 / PI);\n  Y[4]",
     "test_sh_basis_orthonormal_by_exact_quadrature or test_sh_basis_matches_scipy_real_combination"),
]


@pytest.mark.parametrize("name, old, new, tests", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_fail_on_a_planted_mistake(name, old, new, tests):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique or missing: {name}"
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, "oracle_mutant.cpp")
        lib = os.path.join(d, "liboracle_mutant.so")
        open(cpp, "w").write(src.replace(old, new))
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c++17", "-o",
                               lib, cpp])
        env = dict(os.environ, ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", tests],
                           env=env, cwd=ROOT, capture_output=True, text=True)
        assert "passed" in r.stdout or "failed" in r.stdout, r.stdout + r.stderr
        assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"
