"""The FP64 oracle against its pins (arXiv 2005.10123, Section 2.1), and planted mistakes that the
pins must catch.  CPU only."""
import os
import subprocess

import pytest

import oracle
import oracle_pins as P


@pytest.fixture(scope="module")
def lib():
    oracle.build()
    return oracle.load(oracle.LIBRARY)


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=[p.__name__ for p in P.ALL_PINS])
def test_pin(lib, pin):
    pin(lib)


# (description, text in hawkes_oracle.c, replacement).  Each is a plausible slip in the oracle.
MUTANTS = [
    ("background normaliser (2 pi)^1 instead of (2 pi)^(3/2)",
     "pow(ORACLE_TWO_PI, 1.5)", "pow(ORACLE_TWO_PI, 1.0)"),
    ("trigger coefficient theta/omega as printed",
     "const double ce = theta * omega /", "const double ce = theta / omega /"),
    ("ties counted as causal", "if (t[j] < t[i]) {", "if (t[j] <= t[i]) {"),
    ("diagonal background term dropped",
     "for (long j = 0; j < n; ++j) {\n        const double dx",
     "for (long j = 0; j < n; ++j) {\n        if (j == i) continue;\n        const double dx"),
    ("temporal bandwidth replaced by the spatial one",
     "dt * dt / (2.0 * tt * tt)", "dt * dt / (2.0 * tx * tx)"),
    ("trigger delay sign flipped", "exp(-omega * dt - r2", "exp(omega * dt - r2"),
    ("sign of the trigger part of Lambda",
     ") - theta * expm1(-omega * u);", ") + theta * expm1(-omega * u);"),
    ("lower limit of the background integral dropped",
     "norm_cdf(u / tt) - norm_cdf(-t[i] / tt)) - theta", "norm_cdf(u / tt) - 0.5) - theta"),
    ("tau_t gradient without its Sbt term", "cb * (-Sb / tt + Sbt / (tt * tt * tt)),", "cb * (-Sb / tt),"),
    ("omega gradient sign", "(Se - omega * Set)", "(Se + omega * Set)"),
    ("h gradient power", "Ser / (h * h * h)", "Ser / (h * h)"),
    ("T taken as the last time, not the largest", "if (t[k] > T) T = t[k];", "T = t[k];"),
    ("x and y mixed up", "const double dy = y[i] - y[j];", "const double dy = y[i] - x[j];"),
    ("d Lambda / d omega without u", "theta * u * exp(-omega * u)", "theta * exp(-omega * u)"),
    ("d Lambda / d tau_t sign of the lower-limit term",
     "(u * norm_pdf(u / tt) + t[i] * norm_pdf(t[i] / tt))",
     "(u * norm_pdf(u / tt) - t[i] * norm_pdf(t[i] / tt))"),
    ("pi from the background part", "out->pi = ce * Se / lambda;", "out->pi = cb * Sb / lambda;"),
    ("Sbr weighted by dt", "Sbr += r2 * b;", "Sbr += dt * b;"),
    ("Set weighted by r2", "Set += dt * e;", "Set += r2 * e;"),
    ("Ser weighted by dt", "Ser += r2 * e;", "Ser += dt * e;"),
    ("pi without the trigger coefficient", "out->pi = ce * Se / lambda;", "out->pi = Se / lambda;"),
    ("pi over the background part of lambda", "out->pi = ce * Se / lambda;", "out->pi = ce * Se / (cb * Sb);"),
    ("two per-event sums swapped", "out->sums[1] = Sbr;\n    out->sums[2] = Sbt;",
     "out->sums[1] = Sbt;\n    out->sums[2] = Sbr;"),
    ("trigger sums written in the wrong order", "out->sums[4] = Set;\n    out->sums[5] = Ser;",
     "out->sums[4] = Ser;\n    out->sums[5] = Set;"),
    ("row layout: lambda and Lambda swapped", "o[0] = r.lambda;\n        o[1] = r.Lambda;",
     "o[0] = r.Lambda;\n        o[1] = r.lambda;"),
    ("row layout: ell and pi swapped", "o[2] = r.ell;\n        o[3] = r.pi;", "o[2] = r.pi;\n        o[3] = r.ell;"),
    ("row layout: sums one slot early", "o[10 + p] = r.sums[p];", "o[9 + p] = r.sums[p];"),
]


@pytest.mark.parametrize("desc,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, desc, old, new):
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    oracle.build(str(path), so)
    lib = oracle.load(so)
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, ValueError, FloatingPointError) as exc:
            caught.append((pin.__name__, str(exc)[:80]))
            break
    assert caught, f"no pin catches: {desc}"


def test_parallel_driver_matches_whole_evaluation(lib):
    """The threaded whole-workload driver (row ranges through hawkes_oracle_rows, totals by exact
    summation) reproduces evaluate(rows=True) row by row and in total."""
    import numpy as np

    x, y, t = P.random_events(300, 77, L=2.0, T=50.0)
    th = [1.0, 0.4, 6.0, 0.5, 0.8, 0.15]
    whole = oracle.evaluate(x, y, t, th, lib=lib, rows=True)
    for threads in (1, 3, 7):
        par = oracle.evaluate_parallel(x, y, t, th, threads=threads, lib=lib)
        for k in ("row_ell", "row_Lambda", "row_pi", "row_grad"):
            assert np.array_equal(par[k], whole[k]), (threads, k)
        assert abs(par["ell"] - whole["ell"]) <= 1e-13 * np.abs(whole["row_ell"]).sum()
        assert np.all(np.abs(par["grad"] - whole["grad"]) <= 1e-13 * np.abs(whole["row_grad"]).sum(axis=0))
