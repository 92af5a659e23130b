"""Plant plausible mistakes in copies of the application oracles (on the CPU)
and check that the pins catch every one of them."""
import pytest

import ml_pins
from oracle import ml

MUTANTS = {
    # the last writer wins instead of the first (a set density is overwritten)
    "spade_last_writer": ("if (dens[near[t]] == 0) dens[near[t]] = c;", "dens[near[t]] = c;"),
    # a sample exactly at the approximation width counts as approximated
    "spade_le_apprx": ("if (dij < apprx_width) {", "if (dij <= apprx_width) {"),
    # a sample exactly at the kernel width is counted
    "spade_le_kernel": ("} else if (dij < kernel_width) {", "} else if (dij <= kernel_width) {"),
    # approximated samples are not counted (the count's first branch dropped)
    "spade_count_branch": ("near[nnear++] = (int32_t)j;\n                c++;", "near[nnear++] = (int32_t)j;"),
    # skipped rows are visited anyway
    "spade_no_skip": ("if (dens[i] > 0) continue;", "if (dens[i] > 1 << 30) continue;"),
    # the row itself is not counted
    "spade_self": ("for (int64_t j = 0; j < n; ++j) {\n            double dij",
                   "for (int64_t j = 0; j < n; ++j) {\n            if (j == i) continue;\n            double dij"),
    # the L1 distance loses its absolute value
    "l1_abs": ("s += metric == 0 ? fabs(diff) : diff * diff;\n    }\n    return s;\n}\n\n/* distance between an FP32 sample",
               "s += metric == 0 ? diff : diff * diff;\n    }\n    return s;\n}\n\n/* distance between an FP32 sample"),
    # the centroid L1 distance loses its absolute value
    "cen_l1_abs": ("double diff = (double)x[f] - c[f];\n        s += metric == 0 ? fabs(diff) : diff * diff;",
                   "double diff = (double)x[f] - c[f];\n        s += metric == 0 ? diff : diff * diff;"),
    # ties go to the highest centroid index
    "assign_tie": ("if (j1 < 0 || dij < b1) {", "if (j1 < 0 || dij <= b1) {"),
    # naive Bayes smoothing denominator without the feature count
    "nb_denominator": ("/ (T + (double)d);", "/ (T + 1.0);"),
    # naive Bayes prior as a count, not a fraction
    "nb_prior": ("prior[c] = (double)cnt[c] / (double)n;\n        for (int f = 0; f < d; ++f)\n            phi",
                 "prior[c] = (double)cnt[c];\n        for (int f = 0; f < d; ++f)\n            phi"),
    # GDA centres on the global class 0 mean
    "gda_wrong_mean": ("const double *m = mu + (size_t)y[i] * (size_t)d;", "const double *m = mu;"),
    # GDA covariance divided by n - 1
    "gda_unbiased": ("sigma[o] /= (double)n;", "sigma[o] /= (double)(n - 1);"),
    # GDA covariance transposed index (only the diagonal survives)
    "gda_outer": ("sigma[(size_t)a * d + b] += z[a] * z[b];", "sigma[(size_t)a * d + b] += z[a] * z[a];"),
    # per-class sums into the wrong class
    "sums_index": ("double *s = S + (size_t)c * (size_t)d;", "double *s = S + (size_t)((c + 1) % C) * (size_t)d;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(ml.SRC_PATH).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = ml.build(str(path), str(tmp_path / f"libmut_{name}.so"))
    caught = []
    for pin in ml_pins.ALL_ML_PINS:
        try:
            pin(lib)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin catches mutant {name}"
