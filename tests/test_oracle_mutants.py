"""Planted mistakes: each edit below is a plausible slip in the oracle (a
dropped term, a wrong sign, index or constant).  A copy of the oracle with the
edit is compiled on the CPU and the pins are run against it; at least one pin
must fail, otherwise the pins would not have caught that mistake."""
import math

import pytest

import oracle
from tests import test_oracle_end_to_end as E2E
from tests import test_oracle_pins as PINS
from tests import test_oracle_dedisperse as DD
from tests import test_oracle_distill as DS
from tests import test_oracle_ell as ELL
from tests import test_oracle_series_whitening as SW
from tests import test_oracle_zap as ZP

MUTANTS = {
    "kepler_step_sign": ("E -= step;", "E += step;"),
    "kepler_denominator": ("(1.0 - e * cos(E))", "(1.0 + e * cos(E))"),
    "mean_anomaly_alg1_garble": ("Omega * time_s + t->alpha_rad", "Omega * (time_s + t->alpha_rad)"),
    "sqrt_one_minus_e2": ("sqrt(1.0 - e * e) * sin(E)", "sqrt(1.0 + e * e) * sin(E)"),
    "sin_cos_psi_swapped": ("* sin(t->omega_rad)\n", "* cos(t->omega_rad)\n"),
    "no_zero_offset": ("double d0 = tbo_roemer_delay(t, 0.0);", "double d0 = 0.0;"),
    "index_sign": ("src[j] = j - (int64_t)rint(dj);", "src[j] = j + (int64_t)rint(dj);"),
    "index_floor": ("src[j] = j - (int64_t)rint(dj);", "src[j] = j - (int64_t)floor(dj);"),
    "oob_clamps": ("(double)x0[s] : 0.0;", "(double)x0[s] : (double)x0[s < 0 ? 0 : n - 1];"),
    "mean_divisor": ("double mean = sum / (double)n;", "double mean = sum / (double)(n - 1);"),
    "dft_sign": ("ai -= y[j] * s[r];", "ai += y[j] * s[r];"),
    "fft_twiddle_sign": ("double wr = c[q * step], wi = -s[q * step];", "double wr = c[q * step], wi = s[q * step];"),
    "fft_twiddle_index": ("double wr = c[q * step], wi = -s[q * step];", "double wr = c[q], wi = -s[q];"),
    "power_drops_imag": ("p[k] = re[k] * re[k] + im[k] * im[k];", "p[k] = re[k] * re[k];"),
    "median_rank": ("meds[b] = tmp[(cnt - 1) / 2];", "meds[b] = tmp[cnt / 2];"),
    "block_centre": ("cent[b] = (double)start + (double)(cnt - 1) / 2.0;", "cent[b] = (double)start + (double)cnt / 2.0;"),
    "whiten_ln2": ("p[k] * M_LN2 / level", "p[k] / level"),
    "whiten_no_interp": ("level = meds[b] + (meds[b + 1] - meds[b]) * f;", "level = meds[b];"),
    "harmsum_rounding": ("acc += phat[(2 * mm * k + 2 * h) / (4 * h)];", "acc += phat[(2 * mm * k) / (4 * h)];"),
    "harmsum_even_terms": ("for (int64_t mm = 1; mm < h2; mm += 2)", "for (int64_t mm = 1; mm < h2; mm += 1)"),
    "tail_missing_term": ("for (int32_t k = 0; k < h; ++k) acc +=", "for (int32_t k = 0; k + 1 < h; ++k) acc +="),
    "gauss_tail_two_sided": ("return log(0.5 * erfc(z / sqrt(2.0)));", "return log(erfc(z / sqrt(2.0)));"),
    "fmin_not_scaled_by_fold": ("int64_t klo = h * J->kmin;", "int64_t klo = J->kmin;"),
    "series_mode_ignored": ("if (lev) whiten_apply(w->p, nb, lev, w->phat);",
                            "if (0) whiten_apply(w->p, nb, lev, w->phat);"),
    "series_levels_window": ("whiten_levels(p, nb, cfg->whiten_window, med, lev);",
                             "whiten_levels(p, nb, cfg->whiten_window + 1, med, lev);"),
    "series_search_drops_levels": ("        J.lev = lev;\n", ""),
    "distill_tol_not_at_ratio": ("if (1000000 * d <= 1000000 * q * tol + ppm * p * fa) return 1;",
                                 "if (1000000 * d <= 1000000 * tol + ppm * p * fa) return 1;"),
    "distill_ppm_of_source": ("if (1000000 * d <= 1000000 * q * tol + ppm * p * fa) return 1;",
                              "if (1000000 * d <= 1000000 * q * tol + ppm * q * fa) return 1;"),
    "distill_across_series": ("    if (a->series_id != b->series_id) return 0;\n    int64_t fa = cand_F(a)",
                              "    int64_t fa = cand_F(a)"),
    "distill_weakest_first": ("if (a->sigma != b->sigma) return a->sigma > b->sigma;",
                              "if (a->sigma != b->sigma) return a->sigma < b->sigma;"),
    "distill_absorbed_kept": ("        if (absorbed[a]) continue;\n", ""),
    "distill_fold_shift": ("return (int64_t)c->bin << (4 - c->log2_harm);", "return (int64_t)c->bin << c->log2_harm;"),
    "appb_C1_e6_sign": ("- 7.0 / 9216.0 * e6;", "+ 7.0 / 9216.0 * e6;"),
    "appb_S3_e4": ("S[3] = 3.0 / 8.0 * e2 - 51.0 / 128.0 * e4", "S[3] = 3.0 / 8.0 * e2 - 45.0 / 128.0 * e4"),
    "appb_C0_dropped": ("    for (int k = 0; k <= 7; ++k) {\n        cosE", "    for (int k = 1; k <= 7; ++k) {\n        cosE"),
    "appb_sin_cos_swapped": ("sinE_b += S[k] * sin((double)k * M);", "sinE_b += S[k] * cos((double)k * M);"),
    "series_no_zero_offset": ("double d0 = tbo_roemer_delay_series(t, 0.0);", "double d0 = 0.0;"),
    "zap_floor_low_end": ("double lo = ceil(lo_hz[i] * T), hi = floor(hi_hz[i] * T);",
                          "double lo = floor(lo_hz[i] * T), hi = floor(hi_hz[i] * T);"),
    "zap_open_high_end": ("if ((double)k >= lo && (double)k <= hi) phat[k] = 0.0;",
                          "if ((double)k >= lo && (double)k < hi) phat[k] = 0.0;"),
    "zap_not_applied": ("    tbo_zap(w->phat, nb, (double)n * c->tsamp, c->zap_lo_hz, c->zap_hi_hz, c->nzap);\n", ""),
    "dedisp_delay_from_bottom": ("(1.0 / (f * f) - 1.0 / (ftop * ftop))", "(1.0 / (ftop * ftop) - 1.0 / (f * f))"),
    "dedisp_truncated_delay": ("int64_t v = (int64_t)rint(delay / tsamp);", "int64_t v = (int64_t)(delay / tsamp);"),
    "dedisp_read_backwards": ("fb_sample(data, nbits, nchan, t + s[(size_t)d * nchan + c], c)",
                              "fb_sample(data, nbits, nchan, t + smax - s[(size_t)d * nchan + c], c)"),
    "dedisp_nibble_order": ("return (c % 2 == 0) ? (b & 15u) : (b >> 4);", "return (c % 2 == 0) ? (b >> 4) : (b & 15u);"),
    "dedisp_constant": ("return 4.148808e3;", "return 4.148808e3 * 1.0005;"),
    "fold_pick_index": ("for (int64_t mm = 1; mm < h; mm += 2) acc += w->phat[(2 * mm * k + 2 * hp) / (4 * hp)];",
                        "for (int64_t mm = 1; mm < h; mm += 2) acc += w->phat[(2 * mm * k + 2 * hp) / (4 * h)];"),
}


def _pins():
    """Every pin as a zero-argument callable."""
    out = []
    for e in [0.02, 0.1]:
        out.append(lambda e=e: PINS.test_kepler_matches_appendix_b_series(None, e))
    for e in [0.1, 0.5]:
        out.append(lambda e=e: PINS.test_kepler_against_high_precision(None, e))
    for tm in PINS.TEMPLATES:
        out.append(lambda tm=tm: PINS.test_resample_index_hand_values(None, tm))
    for f in [PINS.test_zero_orbit_is_identity, PINS.test_circular_equals_elliptical_limit_and_phase_flip,
              PINS.test_out_of_range_reads_zero, PINS.test_mean_subtract, PINS.test_naive_dft_brute_force_2_10,
              PINS.test_parseval_and_pure_tone, PINS.test_whiten_constant_spectrum,
              PINS.test_whiten_linear_ramp_odd_window, PINS.test_whiten_medians_brute_force,
              PINS.test_harmsum_comb_closed_form, PINS.test_harmsum_direct_brute_force, PINS.test_thresholds,
              PINS.test_sigma_conversion, E2E.test_search_output_sorted_and_consistent,
              E2E.test_injected_binary_peaks_at_true_template_and_frequency]:
        out.append(lambda f=f: f(None))
    out.append(lambda: PINS.test_fft_against_library(None, 14))
    out.append(lambda: ELL.test_appendix_b_coefficients_are_the_bessel_taylor_polynomials(None, 0.3))
    out.append(lambda: ELL.test_series_delay_within_truncation_of_exact(None, 0.1))
    for f in [ELL.test_zero_eccentricity_is_the_circular_bt_delay, ELL.test_series_indices_follow_the_exact_delay]:
        out.append(lambda f=f: f(None))
    for f in [ZP.test_zapped_bins_are_zero_and_the_rest_untouched, ZP.test_zap_function_edges]:
        out.append(lambda f=f: f(None))
    for f in [DD.test_dispersion_constant_from_codata, DD.test_zero_dm_is_the_channel_sum,
              DD.test_impulse_lands_at_its_delay, DD.test_band_order_does_not_matter,
              DD.test_four_bit_samples_unpack_to_the_eight_bit_result]:
        out.append(lambda f=f: f(None))
    for f in [DS.test_hand_worked_example, DS.test_tolerance_is_measured_at_the_ratio,
              DS.test_relative_tolerance_scales_with_the_target, DS.test_same_frequency_only]:
        out.append(lambda f=f: f(None))
    out.append(lambda: DS.test_greedy_matches_declarative_rule(None, 1, 16, 16, 0))
    for f in [SW.test_series_levels_of_an_impulse_are_flat, SW.test_series_levels_of_a_silent_series_are_zero,
              SW.test_series_medians_against_library_spectrum, SW.test_zero_orbit_matches_per_template_whitening,
              SW.test_levels_do_not_depend_on_the_template,
              SW.test_series_search_thresholds_the_series_whitened_sums]:
        out.append(lambda f=f: f(None))
    return out


def _caught(path):
    with oracle.use_library(path):
        for pin in _pins():
            try:
                pin()
            except (AssertionError, ValueError, ZeroDivisionError, OverflowError):
                return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle_lib, name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) >= 1, "mutation site vanished: " + name
    path = oracle.build_variant(src.replace(old, new), str(tmp_path))
    assert _caught(path), "no pin caught: " + name


def test_unmodified_oracle_passes_every_pin(oracle_lib, tmp_path):
    path = oracle.build_variant(oracle.source_text(), str(tmp_path))
    assert not _caught(path)
