"""Planted mistakes in the oracle's C source must each fail at least one pin.

Every mutant is a copy of oracle/snlm_oracle.c with one plausible mistake (a
dropped tap, a wrong extension, a wrong sign or index, swapped passes), built
into a temporary library on the CPU.  The real oracle is never modified."""
import os

import pytest

import oracle
import oracle_pin_checks as pc

MUTANTS = {
    "drop_last_tap": ("for (int k = -K; k <= K; ++k)", "for (int k = -K; k < K; ++k)"),
    "periodic_instead_of_reflect": ("return m < n ? m : p - 1 - m;", "return m < n ? m : m - n;"),
    "exp_wrong_scale": ("w = exp(-d2 / (h * h));", "w = exp(-d2 / h);"),
    "exp_wrong_sign": ("w = exp(-d2 / (h * h));", "w = exp(d2 / (h * h));"),
    "value_from_centre": ("P += w * x[refl(j, n) * stride];", "P += w * x[refl(i, n) * stride];"),
    "mirrored_partner_tap": ("double b = x[refl(j + k, n) * stride];",
                             "double b = x[refl(j - k, n) * stride];"),
    "gauss_width": ("(2.0 * beta * beta)", "(beta * beta)"),
    "window_one_short": ("for (long j = i - S; j <= i + S; ++j)", "for (long j = i - S; j < i + S; ++j)"),
    "second_pass_reads_input": (
        "filter_lines(mid, H, W, W, !first_rows, S, K, h, kernel, beta, out, W, nthreads);",
        "filter_lines(f, H, W, ld, !first_rows, S, K, h, kernel, beta, out, W, nthreads);"),
    "orders_swapped": ("int first_rows = (order == ORACLE_ROW_COL);",
                       "int first_rows = (order != ORACLE_ROW_COL);"),
    "normaliser_off_by_one": ("return P / Q;", "return P / (Q + 1.0);"),
    "tap_difference_unsquared": ("d2 += tap(k, kernel, beta) * (a - b) * (a - b);",
                                 "d2 += tap(k, kernel, beta) * (a - b);"),
    "div_mirror_index": ("refl(2 * i - j, n)", "refl(2 * j - i, n)"),
    "div_drops_partner_tap": ("if (labs(i - j) <= K) dd +=", "if (0) dd +="),
    "div_quotient_sign": ("acc += (xj - y) * dw;", "acc += (y - xj) * dw;"),
    "div_wii_missing": ("*divi = (1.0 + acc) / W;", "*divi = acc / W;"),
    "div_factor_two": ("const double dw = 2.0 * wt", "const double dw = wt"),
    "div_centre_term_sign": ("double dd = xj - xi;", "double dd = xi - xj;"),
    # a mistake confined to the first and last K samples of a line
    "div_mirror_clamped_at_ends": ("x[refl(2 * i - j, n) * stride] - xi",
                                   "x[(2 * i - j < 0 ? 0 : (2 * i - j >= n ? n - 1 : 2 * i - j)) * stride] - xi"),
    "div_not_chained": ("(din ? din[i * dstride] : 1.0) * di", "di"),
    "sure_b_sign": ("double b1 = c1 - sg2 * s1", "double b1 = c1 + sg2 * s1"),
    "sure_second_pass_reads_input": ("div_lines(mid, W, dmid, H, W, 0,", "div_lines(f, ld, dmid, H, W, 0,"),
    "sure_offdiag": ("a12 += f_rc[i] * f_cr[i];", "a12 += f_rc[i] * f_rc[i];"),
    "bf_support_ceil": ("long R = (long)floor(3.0 * sigma_s);", "long R = (long)ceil(3.0 * sigma_s);"),
    "bf_spatial_unsquared": ("exp(-(double)(dy * dy + dx * dx) / (2.0 * sigma_s * sigma_s))",
                             "exp(-(double)(labs(dy) + labs(dx)) / (2.0 * sigma_s * sigma_s))"),
    "bf_range_against_centre_missing": ("exp(-(u - v) * (u - v) / (2.0 * sigma_r * sigma_r))",
                                        "exp(-u * u / (2.0 * sigma_r * sigma_r))"),
    "bf_rule_coefficient": ("- 0.088 * s2", "- 0.088 * s3"),
    "bf_value_from_centre": ("num += ws * g * u;", "num += ws * g * v;"),
    "vol_z_stride": ("long stride = ax == 0 ? 1 : (ax == 1 ? W : H * W);",
                     "long stride = ax == 0 ? 1 : (ax == 1 ? W : H);"),
    "vol_y_line_base": ("base = (l / W) * H * W + (l % W);", "base = l;"),
    "iir_forward_drops_b3": ("(b[1] * w1 + b[2] * w2 + b[3] * w3) / b[0]", "(b[1] * w1 + b[2] * w2) / b[0]"),
    "iir_backward_taps_swapped": ("(b[1] * y1 + b[2] * y2 + b[3] * y3) / b[0]",
                                  "(b[3] * y1 + b[2] * y2 + b[1] * y3) / b[0]"),
    "iir_backward_reads_input": ("double y = B * out[v] +", "double y = B * in[v] +"),
    "iir_cold_backward_start": ("double y1 = out[n - 1], y2 = out[n - 1], y3 = out[n - 1];",
                                "double y1 = 0.0, y2 = 0.0, y3 = 0.0;"),
    "iir_q_branch": ("double q = beta >= 2.5 ?", "double q = beta >= 25.0 ?"),
    "iir_scale_missing": ("= scale * D[u + L];", "= D[u + L];"),
    "iir_partner_behind": ("x[refl(v + s, n) * stride];", "x[refl(v - s, n) * stride];"),
    "iir_pair_index": ("d2[(size_t)(s - 1) * (n + S) + (lo + S)];", "d2[(size_t)(s - 1) * (n + S) + (i + S)];"),
    "vol_passes_not_chained": ("        double *t = a;\n        a = b;\n        b = t;\n", ""),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(oracle.SOURCE).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new)
    srcp = os.path.join(tmp_path, "mutant.c")
    open(srcp, "w").write(mutated)
    lib = oracle.build(force=True, src=srcp, out=os.path.join(tmp_path, "libmutant.so"))
    orc = oracle.load(lib)
    failed = []
    for check in pc.ALL_CHECKS:
        try:
            check(orc)
        except (AssertionError, ValueError, IndexError):
            failed.append(check.__name__)
    assert failed, "mutant %s passed every pin" % name
