"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
the pins catch every one of them."""
import os

import pytest

import oracle
import oracle_pins

MUTANTS = {
    # dropped term: the last feature never enters the distance
    "dropped_feature": ("for (int f = 0; f < d; ++f) {\n        double diff",
                        "for (int f = 0; f + 1 < d; ++f) {\n        double diff"),
    # wrong sign inside the difference
    "wrong_sign": ("double diff = (double)x[f] - c[f];", "double diff = (double)x[f] + c[f];"),
    # ties go to the highest index
    "tie_rule": ("if (j1 < 0 || dij < b1) {", "if (j1 < 0 || dij <= b1) {"),
    # off-by-one mean
    "mean_length": ("S[o] / (double)counts[j]", "S[o] / (double)(counts[j] + 1)"),
    # empty cluster collapses to the origin
    "empty_rule": (": C_old[o];", ": 0.0;"),
    # transposed centroid indexing
    "transposed": ("C + (size_t)j * (size_t)d, d);", "C + (size_t)j, d);"),
    # objective taken from the second-nearest centroid
    "objective_term": ("best[i] = b1;", "best[i] = (k > 1) ? b2 : b1;"),
    # tolerance rule relative to the new objective instead of the previous one
    "tol_denominator": ("(J_prev - J) <= tol * J_prev", "(J_prev - J) <= tol * J"),
    # tolerance rule with a strict comparison (an exact equality no longer stops)
    "tol_strict": ("(J_prev - J) <= tol * J_prev", "(J_prev - J) < tol * J_prev"),
    # the previous objective is never advanced
    "tol_stale_prev": ("        J_prev = J;\n", "\n"),
    # the objective of given labels uses the wrong centroid row
    "objective_index": ("const double *cj = C + (size_t)j * (size_t)d;",
                        "const double *cj = C + (size_t)((j + 1) % k) * (size_t)d;"),
    # the update sums into the wrong label
    "update_index": ("double *s = S + (size_t)j * (size_t)d;",
                     "double *s = S + (size_t)((j + 1) % k) * (size_t)d;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.oracle.SRC_PATH).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.build(str(path), str(tmp_path / f"libmut_{name}.so"))
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin catches mutant {name}"


# Mistakes in the near-tie margin (Python side of the oracle): each replaces
# one expression inside near_tie_margin.
PY_MUTANTS = {
    "margin_sign": ("(d2nd - dmin) / den", "(dmin - d2nd) / den"),
    "margin_half": ("den = dmin + d2nd", "den = 2.0 * (dmin + d2nd)"),
    "margin_relative_to_d2": ("den = dmin + d2nd", "den = d2nd"),
    "margin_zero_case": ("m = np.where(den == 0.0, 0.0, m)", "m = m"),
    "margin_inf_case": ("m = np.where(np.isinf(d2nd), np.inf, m)", "m = m"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_margin_mutant_is_caught(name):
    import inspect
    old, new = PY_MUTANTS[name]
    src = inspect.getsource(oracle.oracle.near_tie_margin)
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    ns = {"np": __import__("numpy")}
    exec(src.replace(old, new), ns)
    with pytest.raises(AssertionError):
        oracle_pins.pin_near_tie_margin(None, margin_fn=ns["near_tie_margin"])
