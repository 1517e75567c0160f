"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/oracle.c``, plants one plausible mistake (a dropped
term, a wrong sign, a wrong operand or index, a transposed product), builds the
copy with gcc into a temporary directory and runs the pin checks of
``test_oracle_pins`` against it: at least one must fail.  CPU only.
"""
import os
import re
import tempfile

import pytest

import oracle as O

import test_oracle_pins as pins

SPMV_BODY = ("    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) two_sum_acc(&s, &c, A->val[k] * x[A->col[k]]);\n"
             "    y[i] = s + c;\n")
SPMV_TRANSPOSED = (SPMV_BODY + "  }\n  { double *yt = (double *)calloc((size_t)A->n, sizeof(double));\n"
                   "    for (int64_t i2 = 0; i2 < A->n; ++i2)\n"
                   "      for (int64_t k = A->rowptr[i2]; k < A->rowptr[i2 + 1]; ++k) yt[A->col[k]] += A->val[k] * x[i2];\n"
                   "    memcpy(y, yt, sizeof(double) * (size_t)A->n); free(yt);\n")

MUTANTS = {
    "r_update_sign": ("r[k] - al * o[k] - y[k]", "r[k] - al * o[k] + y[k]"),
    "p_update_plus_u": ("be * (p[k] - u[k])", "be * (p[k] + u[k])"),
    "o_drops_beta_t": ("o[k] = s[k] + be * t[k]", "o[k] = s[k]"),
    "u_drops_beta": ("et * (y[k] + be * u[k])", "et * (y[k] + u[k])"),
    "q_drops_l": ("q[k] = As[k] + be * l[k]", "q[k] = As[k]"),
    "w_wrong_sign": ("et * (g[k] + be * w[k])", "et * (g[k] - be * w[k])"),
    "z_update_sign": ("et * z[k] - al * u[k]", "et * z[k] + al * u[k]"),
    "y_uses_r_for_s": ("y[k] = ze * s[k] + et * y[k]", "y[k] = ze * r[k] + et * y[k]"),
    "x_drops_z": ("x[k] = x[k] + al * p[k] + z[k]", "x[k] = x[k] + al * p[k]"),
    "l_sign": ("l[k] = q[k] - Aw[k]", "l[k] = q[k] + Aw[k]"),
    "g_drops_eta": ("g[k] = ze * As[k] + et * g[k] - al * Aw[k]", "g[k] = ze * As[k] - al * Aw[k]"),
    "s_drops_g": ("s[k] = s[k] - al * q[k] - g[k]", "s[k] = s[k] - al * q[k]"),
    "zeta_numerator_swapped": ("zeta = (bb * d - c * e) / den_ze", "zeta = (bb * e - c * d) / den_ze"),
    "eta_numerator_swapped": ("eta = (a * e - c * d) / den_ze", "eta = (a * d - c * e) / den_ze"),
    "beta_inverted": ("beta = (S[S_ALPHA] * f) / den_beta", "beta = (S[S_ALPHA] * S[S_F]) / (S[S_ZETA] * f)"),
    "alpha_den_sign": ("den_alpha = gh + beta * h", "den_alpha = gh - beta * h"),
    "h_uses_s": ("h = dot(n, rs, t, S)", "h = dot(n, rs, s, S)"),
    "c_uses_r": ("c = dot(n, s, y, S)", "c = dot(n, r, y, S)"),
    "e_uses_s": ("e = dot(n, y, r, S)", "e = dot(n, y, s, S)"),
    "no_initial_s": ("spmv(&A, r, v[VS], S);                       /* R2", "(void)0;                       /* R2"),
    "spmv_transposed": (SPMV_BODY, SPMV_TRANSPOSED),
    "spmv_drops_compensation": ("    y[i] = s + c;", "    y[i] = s;"),
    "dot_drops_product_error": ("xsum_add(&T, fma(u[k], v[k], -p));", "(void)0;"),
    "dot_drops_carries": ("    X->d[i + 1] += c;", "    X->d[i + 1] += 0 * c;"),
    "dot_ties_away": ("(rem == half && (sticky || (M & 1)))", "(rem == half)"),
    "dot_ignores_sticky": ("(rem == half && (sticky || (M & 1)))", "(rem == half && (M & 1))"),
    "rr_l_from_y": ("spmv(A, t, l, S);", "spmv(A, y, l, S);"),
    "rr_residual_sign": ("r[k] = b[k] - tmp[k]", "r[k] = b[k] + tmp[k]"),
    "pbicgstab_w_sign": ("om * (t[k] - al * vv[k])", "om * (t[k] + al * vv[k])"),
    "pbicgstab_z_drops_v": ("z[k] = t[k] + be * (z[k] - omp * vv[k])", "z[k] = t[k] + be * z[k]"),
    "pbicgstab_alpha_drops_gz": ("den_alpha = gw + beta * gs - beta * om * gz", "den_alpha = gw + beta * gs"),
    "pbicgstab_y_uses_s": ("y[k] = w[k] - al * z[k]", "y[k] = w[k] - al * s[k]"),
    "pbicgstab_omega_inverted": ("qy / yy", "yy / qy"),
    "prec_no_rounding": ("v[k] = (double)(float)A->val[k];", "v[k] = A->val[k];"),
    "prec_residual_rounded": ("  if (precision == 1) Ar->val = v;", "  Ar->val = v;"),
    "prec_krylov_fp64": ("  Ak->val = v;\n", "\n"),
    "prec_setup_residual_rounded": ("spmv(&Ares, x, tmp, S);", "spmv(&A, x, tmp, S);"),
    "prec_rr_residual_rounded": ("spmv(Ares, x, tmp, S);", "spmv(A, x, tmp, S);"),
    "prec_setup_s_fp64": ("spmv(&A, r, v[VS], S);", "spmv(&Ares, r, v[VS], S);"),
    "spmv_fast_two_sum": ("const double e = (*s - (t - z)) + (v - z);", "const double e = v - z;"),
    "dot_merge_drops_threads": ("      for (int i = 0; i < XDIG; ++i) X.d[i] += T.d[i];",
                                "      if (omp_get_thread_num() == 0) for (int i = 0; i < XDIG; ++i) X.d[i] += T.d[i];"),
    "x0_scale_inverted": ("const double c = num / den;", "const double c = den / num;"),
    "x0_scale_uses_x0": ("dot(n, tmp, b, S), den", "dot(n, x, b, S), den"),
    "x0_rule_reversed": ("if (!(rr <= bb)) {", "if (!(rr >= bb)) {"),
    "x0_rule_keeps_r": ("      for (int64_t k = 0; k < n; ++k) r[k] = b[k]; /* b - A 0 */", "      (void)0;"),
    "f32_z_not_held": ("z[k] = held(f32v, ze * r[k] + et * z[k] - al * u[k]);",
                       "z[k] = ze * r[k] + et * z[k] - al * u[k];"),
    "f32_p_not_held": ("p[k] = held(f32v, r[k] + be * (p[k] - u[k]));", "p[k] = r[k] + be * (p[k] - u[k]);"),
    "f32_x_held": ("    x[k] = x[k] + al * p[k] + z[k];\n    if (!replace)",
                   "    x[k] = held(f32v, x[k] + al * p[k] + z[k]);\n    if (!replace)"),
    "f32_u_not_held": ("u[k] = held(f32v, ze * o[k] + et * (y[k] + be * u[k]));",
                       "u[k] = ze * o[k] + et * (y[k] + be * u[k]);"),
}


@pytest.fixture(scope="module")
def source():
    return open(O.SRC).read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / f"{name}.c"
    src.write_text(source.replace(old, new))
    lib = O.build(str(src), str(tmp_path / f"lib{name}.so"))
    orc = O.Oracle(lib)
    failures = []
    for check in pins.CHECKS:
        try:
            msg = check(orc)
        except Exception as exc:  # a mutant may also make a check raise
            msg = f"{check.__name__}: {exc!r}"
        if msg is not None:
            failures.append(msg)
            break
    assert failures, f"planted mistake {name} passed every pin"
