"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutation edits one plausible spot of potref.c (a dropped term, a wrong
sign or index, a swapped operand), builds the copy into a temporary library
and runs the pin suite against it in a subprocess.  The pins are adequate
only if every mutant is caught.  Runs on the CPU only.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "potref.c")

MUTATIONS = {
    "phi_drops_sum_exp_v": ("+ sum_exp(m, v) - dot_vec(n, u, rt)", "- dot_vec(n, u, rt)"),
    "phi_wrong_sign_ws": ("- dot_vec(m, v, ct) - w * s;", "- dot_vec(m, v, ct) + w * s;"),
    "smoothing_uses_n_for_c": ("et / (8.0 * m);", "et / (8.0 * n);"),
    "setup_cap_wrong_mass": ("double cap = 8.0 * (nc - s) / (nc - 1.0);",
                             "double cap = 8.0 * (nr - s) / (nc - 1.0);"),
    "stats_wrong_column_index": ("x[j] = u[i] + v[j] + w - Ci[j] * ig;",
                                 "x[j] = u[i] + v[j % (n < m ? n : m)] + w - Ci[j] * ig;"),
    "gk_u_step_drops_slack": ("u[i] = u[i] + log(rt[i]) - logaddexp(lR[i], u[i]);",
                              "u[i] = u[i] + log(rt[i]) - lR[i];"),
    "gk_w_step_sign": ("*w = *w + log(s) - lT;", "*w = *w - log(s) + lT;"),
    "gk_v_step_uses_rt": ("v[j] = v[j] + log(ct[j]) - logaddexp(lQ[j], v[j]);",
                          "v[j] = v[j] + log(rt[j % n]) - logaddexp(lQ[j], v[j]);"),
    "score_w_wrong": ("sc[2] = rho_log(s, lT);", "sc[2] = rho_log(s, lT) * 0.25;"),
    "grave_wrong_sign": ("zgrave.u[i] = zbar.u[i] + theta * d;", "zgrave.u[i] = zbar.u[i] - theta * d;"),
    "theta_recursion": ("theta = theta * (sqrt(theta * theta + 4.0) - theta) / 2.0;",
                        "theta = theta * (sqrt(theta * theta + 4.0) - theta) / 1.9;"),
    "argmin_reversed": ("int pick = phihat < phichk ? 1 : 0;", "int pick = phihat > phichk ? 1 : 0;"),
    "grad_drops_slack": ("gu[i] = exp(lR[i]) + exp(zbar.u[i]) - rt[i];", "gu[i] = exp(lR[i]) - rt[i];"),
    "error_drops_mass_term": ("double e = fabs(exp(lT) - s);", "double e = 0.0;"),
    "sinkhorn_dummy_mass_swapped": ("rh[n] = sum_vec(m, ct) - s;", "rh[n] = sum_vec(n, rt) - s;"),
    "sinkhorn_corner_zero": ("Ce[(size_t)n * m1 + m] = A;", "Ce[(size_t)n * m1 + m] = 0.0;"),
    "round_beta_uses_r": ("beta[j] = cs[j] > c[j] ? c[j] / cs[j] : 1.0;",
                          "beta[j] = cs[j] > c[j % n] ? c[j % n] / cs[j] : 1.0;"),
    "round_lambda_one_norm": ("lambda = np * nq > 0.0 ? (s - T2) / (np * nq) : 0.0;",
                              "lambda = np * nq > 0.0 ? (s - T2) / (np) : 0.0;"),
    "round_scale_direction": ("kappa = s / T2;", "kappa = T2 / s;"),
    "form_primal_sign": ("X[(size_t)i * m + j] = exp(f[i] + g[j] - C[(long)i * ldc + j] * ig);",
                         "X[(size_t)i * m + j] = exp(f[i] - g[j] - C[(long)i * ldc + j] * ig);"),
    "rho_series_sign": ("double add = ((k & 1) ? -term : term) / k;", "double add = term / k;"),
    "tuned_max_entropy": ("double h = hr < hc ? hr : hc;", "double h = hr > hc ? hr : hc;"),
    "tuned_missing_root": ("double gamma = pow(2.0 * eps / (49.0 * h), 1.0 / p);",
                           "double gamma = 2.0 * eps / (49.0 * h);"),
    "tuned_log2_entropy": ("if (r[i] > 0.0) hr -= r[i] * log(r[i]);", "if (r[i] > 0.0) hr -= r[i] * log2(r[i]);"),
    "tuned_threshold_p": ("out3[1] = h * pow(gamma, p);", "out3[1] = h * gamma;"),
    "sk_error_dummy_mass_swapped": ("double rh_d = sum_vec(m, ct) - s, ch_d = sum_vec(n, rt) - s;",
                                    "double rh_d = sum_vec(n, rt) - s, ch_d = sum_vec(m, ct) - s;"),
    "sk_error_corner_cost_zero": ("((i == n && j == m) ? A : 0.0);", "0.0;"),
    "plan_eval_drops_rank_one": ("double v = kappa * (alpha[i] * xt * beta[j]) + lambda * pp[i] * qq[j];",
                                 "double v = kappa * (alpha[i] * xt * beta[j]);"),
    "plan_eval_prices_with_plan_cost": ("cx[j] = Ce[(long)i * lde + j] * v;", "cx[j] = Cp[(long)i * ldp + j] * v;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {name}"
    mutated = src.replace(old, new)
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "potref.c")
        open(cpath, "w").write(mutated)
        import shutil
        shutil.copy(os.path.join(ROOT, "oracle", "potref.h"), d)
        lib = os.path.join(d, "libpotref_mut.so")
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", lib, cpath,
                        "-lm"], check=True)
        env = dict(os.environ, POTREF_LIB=lib, OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "--timeout", "120", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
