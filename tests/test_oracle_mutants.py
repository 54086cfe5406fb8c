"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the pin tests against it: at
least one pin must fail.  The unmodified source must pass them all.
"""
import os

import pytest

import oracle
from oracle import build as obuild
from tests import test_oracle_fp8_pins as fp8pins
from tests import test_oracle_freeze_pins as frpins
from tests import test_oracle_penalty_pins as penpins
from tests import test_oracle_sample_pins as smpins
from tests import test_oracle_pins as pins

PIN_TESTS = [
    pins.test_hand_examples,
    pins.test_hand_example_coefficients,
    lambda o: pins.test_log_transform_closed_form(o, 0),
    lambda o: pins.test_log_transform_closed_form(o, 1),
    pins.test_log1p_matches_math_over_range,
    pins.test_stage_permutation_invariance,
    pins.test_coefficients_nonnegative,
    pins.test_split_stages_sum,
    pins.test_candidate_permutation,
    pins.test_unit_coefficients_reduce_to_fsum,
    pins.test_constant_embeddings,
    pins.test_positive_model_is_a_matmul_chain,
    pins.test_select_all_equal,
    pins.test_select_signed_zero_tie,
    pins.test_select_nan_last_and_padding,
    pins.test_select_brute_force_tiny,
    pins.test_relu_clips_negative_and_passes_nan,
    fp8pins.test_e4m3_decode_table,
    fp8pins.test_e4m3_codes_are_ordered_and_round_trip,
    fp8pins.test_e4m3_encode_rounding_and_saturation,
    fp8pins.test_fp8_scale_is_largest_power_of_two,
    fp8pins.test_fp8_form_hand_examples_exact,
    fp8pins.test_fp8_form_quantizes_hidden_and_inputs,
    fp8pins.test_fp8_form_invariants,
    fp8pins.test_fp8_form_close_to_fp64_model,
    fp8pins.test_fp8_input_codes,
    fp8pins.test_fp8_error_bound,
    frpins.test_freeze_counts,
    frpins.test_freeze_hand_cases,
    frpins.test_freeze_brute_force,
    penpins.test_penalty_hand_cases,
    penpins.test_penalty_is_float32_addition,
    penpins.test_penalty_moves_candidates_back,
    smpins.test_splitmix64_reference_outputs,
    smpins.test_representatives_per_bucket,
    smpins.test_sample_brute_force,
    smpins.test_draws_are_uniform,
]

# (name, text in cm_oracle.c, replacement)
MUTANTS = [
    ("stack order swapped", "z[E + e] = a;", "z[e] = a; z[E + e] = z[E + e];"),
    ("no hidden ReLU", "h[j] = a < 0.0 ? 0.0 : a;", "h[j] = a;"),
    ("no output ReLU", "c[m] = a < 0.0 ? 0.0 : a;", "c[m] = a;"),
    ("log instead of log1p", "x[f] = log1p((double)sched_si[f]);",
     "x[f] = log((double)sched_si[f] + 1e-300);"),
    ("pipeline features not logged", "p[f] = log1p((double)pipe_s[f]);",
     "p[f] = (double)pipe_s[f];"),
    ("W_1 transposed", "P->W1[j * 2 * E + k]", "P->W1[(k % H) * 2 * E + (j + k / H * H) % (2 * E)]"),
    ("W_s transposed", "P->Ws[e * FS + f]", "P->Ws[(f % E) * FS + (e + f / E * E) % FS]"),
    ("b_s dropped", "double a = (double)P->bs[e];", "double a = 0.0;"),
    ("b_1 dropped", "double a = (double)P->b1[j];", "double a = 0.0;"),
    ("b_2 dropped", "double a = (double)P->b2[m];", "double a = 0.0;"),
    ("terms shifted", "c[m] * (double)terms_si[m]", "c[m] * (double)terms_si[(m + 1) % C]"),
    ("last stage only", "total += v;", "total = v;"),
    ("ties to higher index", "return (A->idx > B->idx) - (A->idx < B->idx);",
     "return (A->idx < B->idx) - (A->idx > B->idx);"),
    ("NaN first", "return A->nan - B->nan;", "return B->nan - A->nan;"),
    ("padding index 0", "idx_out[j] = -1;", "idx_out[j] = 0;"),
    ("ReLU maps NaN to 0", "h[j] = a < 0.0 ? 0.0 : a;", "h[j] = a > 0.0 ? a : 0.0;"),
    ("descending order", "if (A->key < B->key) return -1;", "if (A->key > B->key) return -1;"),
    ("e4m3 subnormals scaled by 2^-10", "ldexp((double)m, -9)", "ldexp((double)m, -10)"),
    ("e4m3 exponent bias 8", "ldexp(1.0 + m / 8.0, e - 7)", "ldexp(1.0 + m / 8.0, e - 8)"),
    ("e4m3 ties to the larger code", "(d == bd && (c & 1) == 0)", "(d == bd)"),
    ("e4m3 no saturation", "if (a >= 448.0) return sign | 0x7E;", "if (a >= 480.0) return sign | 0x7F;"),
    ("fp8 scale rounds up", "return ldexp(1.0, e - 1);", "return ldexp(1.0, e);"),
    ("fp8 input scale not undone", "const double pre = a / s1;", "const double pre = a / sw1;"),
    ("fp8 activation scale not undone", "a = a / s2 + (double)P.b2[c];",
     "a = a / (s2 / act_scale) + (double)P.b2[c];"),
    ("fp8 hidden activations not quantized", "hq[h] = q8(x);", "hq[h] = x;"),
    ("fp8 inputs decoded as zero", "const double prod = Wq1[h][f] * cmo_e4m3_decode(q[f]);",
     "const double prod = Wq1[h][f] * cmo_e4m3_decode(q[f]) * 0.0;"),
    ("fp8 bound ignores rounding swings", "flips += fabs(Wq2[c][h]) * swing[h];",
     "flips += 0.0 * swing[h];"),
    ("fp8 bound ignores coefficient sums", "bound += (flips + acc_tol * pmax) / s2",
     "bound += (flips + 0.0 * pmax) / s2"),
    ("fp8 bound ignores the hoisted row", "+ 1e-5 * uabs[s * H + h]) * act_scale;",
     "+ 0.0 * uabs[s * H + h]) * act_scale;"),
    ("freeze leaves floor(log2 S) free", "while (((int64_t)1 << unfrozen) < (int64_t)S) ++unfrozen;",
     "while (((int64_t)2 << unfrozen) <= (int64_t)S) ++unfrozen;"),
    ("freeze takes the costliest stages", "frozen_out[it[j].idx] = j < S - unfrozen ? 1 : 0;",
     "frozen_out[it[j].idx] = j >= unfrozen ? 1 : 0;"),
    ("penalty ignores the last bad hash", "for (int64_t j = 0; j < n_bad && !seen; ++j) seen",
     "for (int64_t j = 0; j + 1 < n_bad && !seen; ++j) seen"),
    ("penalty matches every hash", "for (int64_t j = 0; j < n_bad && !seen; ++j) seen = hashes[i] == bad[j];",
     "for (int64_t j = 0; j < n_bad && !seen; ++j) seen = hashes[i] == bad[j] || n_bad > 0;"),
    ("splitmix64 wrong shift", "z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;",
     "z = (z ^ (z >> 28)) * 0x94D049BB133111EBull;"),
    ("sample keeps floor(log2 B)", "while (((int64_t)1 << reps) < B) ++reps;",
     "while (((int64_t)2 << reps) <= B) ++reps;"),
    ("sample keeps the largest keys", "if (A->key != B->key) return A->key < B->key ? -1 : 1;",
     "if (A->key != B->key) return A->key > B->key ? -1 : 1;"),
    ("fp8 folded bias dropped", "u[s * H + h] = a + beta[h];", "u[s * H + h] = a + 0.0 * beta[h];"),
    ("fp8 stage costs cumulative", "if (stage_cost_out != NULL) stage_cost_out[row] = v;",
     "if (stage_cost_out != NULL) stage_cost_out[row] = stage_sum + v;"),
    ("fp8 stage bound of the whole candidate",
     "if (stage_bound_out != NULL) stage_bound_out[row] = sbound;",
     "if (stage_bound_out != NULL) stage_bound_out[row] = bound + sbound;"),
]


def _failures(orc):
    failed = 0
    for t in PIN_TESTS:
        try:
            t(orc)
        except (AssertionError, ValueError):
            failed += 1
    return failed


def _build_variant(tmp_path, name, src_text):
    d = tmp_path / name.replace(" ", "_")
    d.mkdir()
    src = d / "cm_oracle.c"
    src.write_text(src_text)
    out = str(d / "libcm_oracle_variant.so")
    obuild.compile_lib(str(src), out)
    return oracle.Oracle(out)


def test_unmodified_source_passes(tmp_path):
    with open(obuild.SRC) as f:
        text = f.read()
    assert _failures(_build_variant(tmp_path, "clean", text)) == 0


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    with open(obuild.SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site not unique: {old!r}"
    orc = _build_variant(tmp_path, name, text.replace(old, new))
    assert _failures(orc) > 0, f"no pin caught mutant: {name}"
