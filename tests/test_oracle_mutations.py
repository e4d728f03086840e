"""Each plausible mistake planted in a copy of the oracle must fail a pin.

The copies are made on the CPU from oracle/oracle.c by one textual
substitution each (a dropped term, a wrong sign, a wrong index or operand, a
wrong test), compiled with the oracle's own build, and run against every
pin of oracle_pins.py.  A mutant that passes all pins would mean the pins
leave that part of the oracle unchecked.
"""
import os

import pytest

import oracle
from oracle.build import build
from oracle_pins import PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, replacement, which occurrence (None = all))
MUTATIONS = [
    ("spmv_wrong_column", "acc = acc + vals[j] * p[col_idx[j]];", "acc = acc + vals[j] * p[i];", None),
    ("dot_drops_error_term", "s = s + (q + r);", "s = s + q;", None),
    ("dot_product_error_sign", "*e = fma(a, b, -x);", "*e = fma(a, b, x);", None),
    ("residual0_sign", "r[i] = b[i] - ax[i];", "r[i] = b[i] + ax[i];", None),
    ("cg_x_update_sign", "x[j] = x[j] + alpha * p[j];", "x[j] = x[j] - alpha * p[j];", 0),
    ("cg_beta_inverted", "double beta = rr_new / rr;", "double beta = rr / rr_new;", None),
    ("cg_converged_on_squared_norm", "if (sqrt(rr_new) <= tol)", "if (rr_new <= tol)", 0),
    ("eq3_drops_alpha_factor", "alpha * alpha * apap / rr - 1.0", "alpha * apap / rr - 1.0", None),
    ("pcg_residual_wrong_operand", "r[j] = r[j] - alpha * ap[j];", "r[j] = r[j] - alpha * p[j];", None),
    ("pcg_direction_sign", "p[j] = r[j] + beta * p[j];", "p[j] = r[j] - beta * p[j];", 1),
    ("bicg_direction_sign", "p[j] = r[j] + beta * (p[j] - omega * v[j]);",
     "p[j] = r[j] + beta * (p[j] + omega * v[j]);", None),
    ("bicg_omega_inverted", "double omega = ts / tt;", "double omega = tt / ts;", None),
    ("pbicg_beta_sign", "double beta = -asr / apr;", "double beta = asr / apr;", None),
    ("pbicg_residual_wrong_operand", "r[j] = s[j] - omega * as[j];", "r[j] = s[j] - omega * ap[j];", None),
    ("pbicg_expanded_norm_drops_factor", "ss - 2.0 * omega * ass", "ss - omega * ass", None),
    ("pbicg_x_update_wrong_operand", "x[j] = x[j] + alpha * p[j] + omega * s[j];",
     "x[j] = x[j] + alpha * p[j] + omega * as[j];", 1),
    ("pbicg_rho_wrong_vector", "rho = oracle_dot(n, r, rs);                        /* <r_{i+1}, r0*> */",
     "rho = oracle_dot(n, r, r);", None),
    ("half_step_wrong_vector", "x[j] = x[j] + alpha * p[j];", "x[j] = x[j] + alpha * s[j];", 3),
    ("gmres_gs_update_sign", "w[t] = w[t] - rj * vj[t];", "w[t] = w[t] + rj * vj[t];", None),
    ("gmres_normalise_wrong", "vi[t] = w[t] / rii;", "vi[t] = w[t] * rii;", None),
    ("gmres_backsub_order", "s = s - R[i * (m + 1) + j] * eta[j];", "s = s - R[j * (m + 1) + i] * eta[j];", None),
    ("gmres_update_drops_v0", "double s = eta[1] * V[t];", "double s = 0.0;", None),
    ("gmres_update_unscaled", "x[t] = x[t] + rho0 * s;", "x[t] = x[t] + s;", None),
    ("gmres_monitor_drops_xi", "zeta2 = zeta2 - xi[i] * xi[i];", "zeta2 = zeta2 - xi[i];", None),
    ("gmres_xi_unnormalised", "xi[i] = oracle_dot(n, rr, vi);", "xi[i] = oracle_dot(n, rr, w);", None),
    ("f32_spmv_wrong_column", "acc = acc + v[j] * p[ci[j]];", "acc = acc + v[j] * p[i];", None),
    ("f32_dot_drops_compensation", "        s = s + q;\n", "", None),
    ("f32_cg_residual_wrong_operand", "r[j] = r[j] - af * ap[j];", "r[j] = r[j] - af * p[j];", None),
    ("f32_cg_direction_sign", "p[j] = r[j] + bf * p[j];", "p[j] = r[j] - bf * p[j];", None),
    ("f32_cg_beta_unrounded_alpha", "const float af = (float)alpha, bf = (float)beta;",
     "const float af = (float)(0.5 * alpha), bf = (float)beta;", None),
    ("f32acc_dot_wide_accumulator", "float acc = 0.0f;", "double acc = 0.0;", 0),
    ("f32acc_dot_unrounded_product", "const float prod = a[i] * b[i];",
     "const double prod = (double)a[i] * b[i];", None),
    ("f32acc_cg_residual_wrong_operand", "r[j] = r[j] - alpha * ap[j];", "r[j] = r[j] - alpha * p[j];", 1),
    ("f32acc_cg_direction_sign", "p[j] = r[j] + beta * p[j];", "p[j] = r[j] - beta * p[j];", 2),
    ("f32acc_cg_correction_sign", "d[j] = d[j] + alpha * p[j];", "d[j] = d[j] - alpha * p[j];", None),
    ("f32acc_eq3_drops_alpha", "beta = alpha * alpha * apap / rr - 1.0f;", "beta = alpha * apap / rr - 1.0f;",
     None),
    ("f32acc_converged_on_squared_norm", "if (sqrtf(rr) <= tol)", "if (rr <= tol)", None),
    ("mixed_update_sign", "x[j] = x[j] + (double)d[j];", "x[j] = x[j] - (double)d[j];", None),
    ("mixed_solves_b_not_residual", "r32[j] = (float)r[j];", "r32[j] = (float)b[j];", None),
    ("mixed_inner_tol_absolute", "double tol = rtol * sqrt(rr);", "double tol = rtol;", None),
    ("mixed_values_perturbed", "v32[j] = (float)vals[j];", "v32[j] = (float)(vals[j] * 1.0000001);", None),
]


def _mutate(text, old, new, which):
    count = text.count(old)
    assert count >= 1, f"mutation target not found: {old!r}"
    if which is None:
        return text.replace(old, new)
    assert which < count, (old, which, count)
    idx = -1
    for _ in range(which + 1):
        idx = text.index(old, idx + 1)
    return text[:idx] + new + text[idx + len(old):]


@pytest.mark.parametrize("name,old,new,which", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutant_is_caught(name, old, new, which, tmp_path):
    text = open(SRC).read()
    src = tmp_path / f"oracle_{name}.c"
    src.write_text(_mutate(text, old, new, which))
    lib = build(src=str(src), out=str(tmp_path / f"liboracle_{name}.so"))
    O = oracle.Oracle(lib)
    failed = []
    for pin in PINS:
        try:
            pin(O)
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError, OverflowError):
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passes every pin"
