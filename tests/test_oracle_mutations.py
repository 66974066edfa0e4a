"""The oracle's pins catch plausible mistakes: each case plants one mistake in
a copy of oracle.c (a dropped term, a wrong sign, index or bound, swapped
operands), builds it on the CPU, and runs the oracle pin tests against it.
Every mutant must fail at least one pin."""
import os
import subprocess
import sys

import pytest

from helpers import ROOT

SRC = os.path.join(ROOT, "oracle", "oracle.c")
PIN_TESTS = ["tests/test_oracle_spmv.py", "tests/test_oracle_features.py",
             "tests/test_oracle_convert_tree.py", "tests/test_oracle_krylov.py",
             "tests/test_oracle_dia_hyb.py"]

MUTANTS = {
    "spmv_beta_sign": ("y[i] = alpha * s + beta * y[i];", "y[i] = alpha * s - beta * y[i];"),
    "spmv_dropped_last_term": ("for (int64_t k = rp[i]; k < rp[i + 1]; ++k)\n            s = s + val[k]",
                               "for (int64_t k = rp[i]; k < rp[i + 1] - 1; ++k)\n            s = s + val[k]"),
    "sd_radicand_sign": ("(__int128)n * (__int128)a[4] - (__int128)a[3]",
                         "(__int128)n * (__int128)a[4] + (__int128)a[3]"),
    "cluster_run_reset": ("                else\n                    run = 1;",
                          "                else\n                    run = 0;"),
    "span_off_by_one": ("out[7] += (int64_t)col[rp[i + 1] - 1] - (int64_t)col[rp[i]];",
                        "out[7] += (int64_t)col[rp[i + 1] - 1] - (int64_t)col[rp[i]] + 1;"),
    "hist_bin_bound": ("while (bin < 15 && r >= ((int64_t)1 << bin))",
                       "while (bin < 15 && r > ((int64_t)1 << bin))"),
    "ell_pitch": ("*pitch = (n + 63) / 64 * 64;", "*pitch = (n + 31) / 32 * 32;"),
    "dia_fill_limit": ("if (count * (*pitch) > 8 * (int64_t)rp[n])",
                       "if (count * (*pitch) >= 8 * (int64_t)rp[n])"),
    "dia_padding_sign": ("dia_val[t] = 0.0;", "dia_val[t] = -0.0;"),
    "hyb_third_rule": ("if (rows == 0 || 3 * rows < n)", "if (rows == 0 || 3 * rows <= n)"),
    "hyb_tail_bound": ("if (rp[i + 1] - rp[i] > K) {", "if (rp[i + 1] - rp[i] >= K) {"),
    "tree_strict_compare": ("if (v <= thr[t])", "if (v < thr[t])"),
    "cascade_gate": ("if (out[1] == 1)", "if (out[1] == 0)"),
    "cg_beta_inverted": ("double beta = rho_new / rho;", "double beta = rho / rho_new;"),
    "cg_residual_sign": ("r[i] = r[i] - alpha * q[i];", "r[i] = r[i] + alpha * q[i];"),
    "cg_restart_stale_p": ("        memcpy(p, r, bytes);\n        double rho = dot(n, r, r);",
                           "        if (restart == 0)\n            memcpy(p, r, bytes);\n"
                           "        double rho = dot(n, r, r);"),
    "cg_restart_stale_r": ("        memcpy(r, b, bytes);\n        orc_spmv(n, rp, col, val, -1.0, x, 1.0, r);\n        memcpy(p, r, bytes);",
                           "        if (restart == 0) {\n            memcpy(r, b, bytes);\n"
                           "            orc_spmv(n, rp, col, val, -1.0, x, 1.0, r);\n        }\n"
                           "        memcpy(p, r, bytes);"),
    "mgs_wrong_vector": ("w[t] = w[t] - h * V[i * n + t];", "w[t] = w[t] - h * V[t];"),
    "givens_sign": ("hj[i + 1] = -sn[i] * a + cs[i] * c;", "hj[i + 1] = sn[i] * a + cs[i] * c;"),
    "gmres_update_transposed": ("x[t] = x[t] + y[i] * V[i * n + t];",
                                "x[t] = x[t] + y[i] * V[t * (m + 1) % (n * (m + 1)) + 0 * i];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    from oracle import GCC_FLAGS
    subprocess.run(["gcc", *GCC_FLAGS, str(mutated), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *PIN_TESTS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
