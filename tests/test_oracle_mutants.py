"""Plant plausible mistakes in a copy of the C oracle and check that the pins catch each one.

Each mutation is a textual edit of ``oracle/pspec_oracle.c`` (a dropped term, a wrong sign,
exponent or index, swapped operands).  The mutant is compiled with gcc into a temporary
library and the whole pin battery of ``tests/pins.py`` runs against it; at least one pin must
fail.  Only the CPU is involved.
"""
import os
import shutil
import subprocess

import pytest

import oracle as orc
from tests import pins

MUTANTS = {
    "phi_exponent": ("double m = pow(fabs(x), p - 1.0);", "double m = pow(fabs(x), p - 2.0);"),
    "phi_drop_sign": ("return x > 0.0 ? m : -m;", "return m;"),
    "abs_pow_exponent": ("return pow(fabs(x), p);", "return pow(fabs(x), p - 1.0);"),
    "drop_half": ("N *= 0.5L;", ""),
    "denominator_power": ("D += (long double)abs_pow(U[i * ldu + l], p);",
                          "D += (long double)abs_pow(U[i * ldu + l], 2.0);"),
    "objective_wrong_neighbour_column": ("double uj = U[(int64_t)col[e] * ldu + l];\n                s += (long double)(w[e] * abs_pow",
                                         "double uj = U[(int64_t)col[e] * ldu + (k - 1 - l)];\n                s += (long double)(w[e] * abs_pow"),
    "plap_sign": ("s += (long double)(w[e] * phi_p(ui - uj, p));", "s += (long double)(w[e] * phi_p(uj - ui, p));"),
    "plap_drop_weight": ("s += (long double)(w[e] * phi_p(ui - uj, p));", "s += (long double)(phi_p(ui - uj, p));"),
    "grad_sign": ("(Lil - Fl[l] * phi_p(U[i * ldu + l], p))", "(Lil + Fl[l] * phi_p(U[i * ldu + l], p))"),
    "grad_scale": ("G[i * k + l] = (p / D[l]) * (Lil", "G[i * k + l] = (1.0 / D[l]) * (Lil"),
    "hvp_diff_sign": ("(vi - V[j * ldv + l])", "(V[j * ldv + l] - vi)"),
    "hvp_drop_p_minus_1": ("double JL = (p - 1.0) * (double)s;", "double JL = (double)s;"),
    "hvp_drop_diag": ("HV[i * k + l] = (p / D[l]) * (JL - diag - rank2);", "HV[i * k + l] = (p / D[l]) * (JL - rank2);"),
    "hvp_drop_rank2_second": ("double rank2 = g[i * k + l] * a[l] + phi_p(ui, p) * b[l];",
                              "double rank2 = g[i * k + l] * a[l];"),
    "hvp_swap_ab": ("double rank2 = g[i * k + l] * a[l] + phi_p(ui, p) * b[l];",
                    "double rank2 = g[i * k + l] * b[l] + phi_p(ui, p) * a[l];"),
    "hvp_psi_exponent": ("return pow(a, p - 2.0);", "return pow(a, p - 1.0);"),
    "hvp_eps_ignored": ("if (a < eps) a = eps;", ""),
    "hvp_a_uses_v_of_neighbour": ("sa += (long double)(phi_p(U[i * ldu + l], p) * vi);",
                                  "sa += (long double)(phi_p(U[i * ldu + l], p) * V[i * ldv + (k - 1 - l)]);"),
    "hvp_transposed_gradient_index": ("double rank2 = g[i * k + l] * a[l]",
                                      "double rank2 = g[((n - 1 - i) * k) + l] * a[l]"),
    "hvp_sparse_drop_diag": ("HV[i * k + l] = (p / D[l]) * (JL - Fl[l] * Jphi);", "HV[i * k + l] = (p / D[l]) * JL;"),
    "hvp_sparse_diag_sign": ("HV[i * k + l] = (p / D[l]) * (JL - Fl[l] * Jphi);",
                             "HV[i * k + l] = (p / D[l]) * (JL + Fl[l] * Jphi);"),
    "hvp_sparse_psi_at_neighbour": ("double Jphi = (p - 1.0) * psi_eps(ui, p, eps) * vi;",
                                    "double Jphi = (p - 1.0) * psi_eps(U[col[rowptr[i]] * ldu + l], p, eps) * vi;"),
}


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_mutants")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, mutant_dir):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(orc.SRC).read()
    find, repl = MUTANTS[name]
    assert src.count(find) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(find, repl)
    assert mutated != src
    csrc = os.path.join(mutant_dir, f"{name}.c")
    so = os.path.join(mutant_dir, f"{name}.so")
    with open(csrc, "w") as f:
        f.write(mutated)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c99", csrc, "-o", so, "-lm"], check=True)
    bad = pins.failing_pins(orc.Oracle(so))
    assert bad, f"no pin caught mutant {name}"
