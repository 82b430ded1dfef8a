"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle's C source
(on the CPU, never on a GPU), builds it, and runs the pin suite against that
build; the suite must fail.  The list covers every step of the method: the
difference operators, the Kronecker ordering and transposes, the smoothed
norm and its weights, the Poisson ratio, the floor, the EM preconditioner and
its Lambda clamp, the momentum weight and extrapolation, the prox, and the
initial image; and, for the nonsmooth model, the reflection 2 f^{k+1} - f~, the
dual balls and their radii, the dual step sizes, the dual terms of the primal
step, Nesterov's recurrence and the HOITV group norm.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "appga_oracle.c")

MUTATIONS = {
    "em_uses_extrapolated": ("p[j] = beta * f[j] / lam[j];", "p[j] = beta * ft[j] / lam[j];"),
    "theta_index": ("double tkm1 = a * pow((double)(k - 1), omega) + b;",
                    "double tkm1 = a * pow((double)(k), omega) + b;"),
    "momentum_sign": ("ft[j] = f[j] + theta * (f[j] - fprev[j]);",
                      "ft[j] = f[j] - theta * (f[j] - fprev[j]);"),
    "b2_block_order": ("kron_apply(n, op_negDt, op_D, f, v + d, w);",
                       "kron_apply(n, op_D, op_negDt, f, v + d, w);"),
    "b2t_not_transposed": ("kron_accum(n, op_negD, op_Dt, q + d, out, w);",
                           "kron_accum(n, op_Dt, op_negD, q + d, out, w);"),
    "drop_second_order": ("if (st == ORC_OK) st = orc_b2t(n, v, tmp);",
                          "if (st == ORC_OK) { st = orc_b2t(n, v, tmp); "
                          "memset(tmp, 0, sizeof(double) * d); }"),
    "ratio_sign": ("e[i] = 1.0 - g[i] / y;", "e[i] = g[i] / y - 1.0;"),
    "lambda_clamp": ("lam[j] = 1.0;", "lam[j] = 1e-300;"),
    "gradient_at_f": ("orc_forward(m, row_ptr, col, val, ft, y);",
                      "orc_forward(m, row_ptr, col, val, f, y);"),
    "prox": ("fn[j] = z > 0.0 ? z : 0.0;", "fn[j] = z > 0.0 ? z : -z;"),
    "s_eps_offset": ("return nrm - eps / 2.0;", "return nrm - eps;"),
    "weight_form": ("double w1 = lambda1 / (n1 > eps ? n1 : eps);",
                    "double w1 = lambda1 / (n1 + eps);"),
    "d_first_row": ("    for (int j = 1; j < n; ++j) {\n        y[j * sy] += 1.0 * x[j * sx];\n"
                    "        y[j * sy] += -1.0 * x[(j - 1) * sx];",
                    "    y[0] += x[0];\n    for (int j = 1; j < n; ++j) {\n"
                    "        y[j * sy] += 1.0 * x[j * sx];\n"
                    "        y[j * sy] += -1.0 * x[(j - 1) * sx];"),
    "disk_radius": ("rad2 = (n / 2.0) * (n / 2.0);", "rad2 = (n / 2.0 - 0.5) * (n / 2.0 - 0.5);"),
    "actc_background": ("actc += g[i] - gamma[i];", "actc += g[i];"),
    "floor_missing": ("if (y < tau) {", "if (y < -1e300) {"),
    "log_without_background": ("s -= g[i] * log(ax[i] + gamma[i]);", "s -= g[i] * log(ax[i]);"),
}

# Mistakes in the nonsmooth-model code (FPPA / AFPPA); the AFPPA pins must catch each.
AFPPA_MUTATIONS = {
    "afppa_reflection": ("w[j] = 2.0 * fn[j] - ft[j];", "w[j] = fn[j];"),
    "afppa_ball_radius": ("orc_ball_projection(z1, 2, lambda1 / rho1);",
                          "orc_ball_projection(z1, 2, lambda1);"),
    "afppa_c_group_size": ("orc_ball_projection(z2, 4, lambda2 / rho2);",
                           "orc_ball_projection(z2, 2, lambda2 / rho2);"),
    "afppa_rho2_factor": ("rho2 = 1.0 / (2.0 * 64.0 * pmax);", "rho2 = 1.0 / (2.0 * 8.0 * pmax);"),
    "afppa_pmax_extrapolated": ("fixed_p_scalar : beta * f[j] / lam[j];",
                                "fixed_p_scalar : beta * ft[j] / lam[j];"),
    "afppa_drop_b1t": ("double z = ft[j] - p[j] * (gF[j] + t1[j] + t2[j]);",
                       "double z = ft[j] - p[j] * (gF[j] + t2[j]);"),
    "afppa_dual_sign": ("z2[c] = ct[c * d + i] / rho2 + v[c * d + i];",
                        "z2[c] = ct[c * d + i] / rho2 - v[c * d + i];"),
    "afppa_dual_scale": ("bq[d + i] = rho1 * z1[1];", "bq[d + i] = z1[1];"),
    "afppa_gradient_at_f": ("orc_forward(m, row_ptr, col, val, ft, y);\n        if (round_f32)\n"
                            "            for (int64_t i = 0; i < m; ++i) y[i] = (double)(float)y[i];\n"
                            "        orc_ratio(m, y, g, gamma, e, &nclamp);\n        if (round_f32)\n"
                            "            for (int64_t i = 0; i < m; ++i) e[i] = (double)(float)e[i];\n"
                            "        orc_back(m, (int64_t)d, row_ptr, col, val, e, gF);\n        st = orc_b1t",
                            "orc_forward(m, row_ptr, col, val, f, y);\n        if (round_f32)\n"
                            "            for (int64_t i = 0; i < m; ++i) y[i] = (double)(float)y[i];\n"
                            "        orc_ratio(m, y, g, gamma, e, &nclamp);\n        if (round_f32)\n"
                            "            for (int64_t i = 0; i < m; ++i) e[i] = (double)(float)e[i];\n"
                            "        orc_back(m, (int64_t)d, row_ptr, col, val, e, gF);\n        st = orc_b1t"),
    "afppa_adjoint_of_unextrapolated_dual": ("st = orc_b1t(n, bt, t1);", "st = orc_b1t(n, bq, t1);"),
    "nesterov_recurrence": ("t = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;",
                            "t = (1.0 + sqrt(1.0 + 2.0 * t * t)) / 2.0;"),
    "hoitv_group": ("s1 += sqrt(u[i] * u[i] + u[d + i] * u[d + i]);",
                    "s1 += fabs(u[i]) + fabs(u[d + i]);"),
}


# Mistakes in the factored forward model (PSF taps, blur, attenuation).
FACTORED_MUTATIONS = {
    "psf_sigma": ("double sigma = fwhm / (2.0 * sqrt(2.0 * log(2.0)));",
                  "double sigma = fwhm / (2.0 * sqrt(log(2.0)));"),
    "psf_unnormalised": ("w[t] /= s;", "w[t] /= 1.0;"),
    "psf_clamped_border": ("if (rr < 0 || rr >= n) continue;", "if (rr < 0 || rr >= n) rr = rr < 0 ? 0 : n - 1;"),
    "attenuation_sign": ("out[i] = exp(-out[i]);", "out[i] = exp(out[i]);"),
}


def _cases():
    return [(n, "test_oracle_pins.py") for n in sorted(MUTATIONS)] + \
        [(n, "test_oracle_afppa.py") for n in sorted(AFPPA_MUTATIONS)] + \
        [(n, "test_oracle_factored.py") for n in sorted(FACTORED_MUTATIONS)]


@pytest.mark.slow
@pytest.mark.parametrize("name,pins", _cases())
def test_pins_catch_planted_mistake(name, pins, tmp_path):
    src = open(SRC).read()
    old, new = dict(MUTATIONS, **AFPPA_MUTATIONS, **FACTORED_MUTATIONS)[name]
    assert src.count(old) >= 1, "mutation site not found: " + name
    c_file = tmp_path / (name + ".c")
    so_file = tmp_path / (name + ".so")
    c_file.write_text(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", str(so_file), str(c_file), "-lm"])
    env = dict(os.environ, APPGA_ORACLE_LIB=str(so_file))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pins)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutation %s:\n%s" % (name, r.stdout[-2000:])
