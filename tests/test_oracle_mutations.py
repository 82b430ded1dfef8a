"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle's C source
(on the CPU, never on a GPU), builds it, and runs the pin suite against that
build; the suite must fail.  The list covers every step of the method: the
difference operators, the Kronecker ordering and transposes, the smoothed
norm and its weights, the Poisson ratio, the floor, the EM preconditioner and
its Lambda clamp, the momentum weight and extrapolation, the prox, and the
initial image.
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


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTATIONS[name]
    assert src.count(old) >= 1, "mutation site not found: " + name
    c_file = tmp_path / (name + ".c")
    so_file = tmp_path / (name + ".so")
    c_file.write_text(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", str(so_file), str(c_file), "-lm"])
    env = dict(os.environ, APPGA_ORACLE_LIB=str(so_file))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutation %s:\n%s" % (name, r.stdout[-2000:])
