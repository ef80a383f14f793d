"""The host multi-core SIMD evaluation (hawkes_host_eval, the paper's CPU design of Section 2.3)
against the FP64 oracle: log-likelihood, every gradient component and every self-excitation
probability, on the 2,000-event workload, ragged sizes, ties and degenerate inputs; independent of
the thread count (bitwise) and of the input order.  CPU only: it needs no GPU."""
import numpy as np
import pytest

import oracle
import oracle_pins as P
from gpu_util import TOL, assert_close
from paper_2005_10123_amd import binding, synth

TOL_HOST = TOL["fp64"]


def check(x, y, t, th, what, threads=4):
    ref = oracle.evaluate(x, y, t, th, rows=True)
    ell, g, pi = binding.host_eval(x, y, t, th, threads=threads, want_pi=True)
    assert_close(ell, g, ref, "fp64", what, th)
    assert np.max(np.abs(pi - ref["row_pi"])) <= TOL_HOST, (what, np.max(np.abs(pi - ref["row_pi"])))
    return ell, g, pi


@pytest.mark.parametrize("case", ["E1_single", "E2_pair", "E3_tie", "E4_five", "E5_unsorted"])
@pytest.mark.parametrize("thn", ["theta_small", "theta_posterior_regime"])
def test_small_fixtures(case, thn):
    x, y, t = P._case(case)
    check(x, y, t, P._theta(thn), case)


@pytest.mark.parametrize("n", [2, 3, 7, 63, 65, 257, 1025])
def test_ragged_sizes(n):
    x, y, t = synth.simulate(synth.SimSpec(n, 4.0, 200.0, 3, 0.5, 0.1, 0.4, (7, n, 2)))
    perm = np.random.default_rng(n).permutation(n)
    check(x[perm], y[perm], t[perm], (1.0, 0.5, 20.0, 0.4, 0.5, 0.1), f"n={n}")


def test_small_workload_and_thread_count():
    (x, y, t), th = synth.config_events("small_2k")
    a = check(x, y, t, th, "small_2k", threads=1)
    for threads in (3, 8):
        b = binding.host_eval(x, y, t, th, threads=threads, want_pi=True)
        assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), threads


def test_ties_and_degenerate():
    rng = np.random.default_rng(5)
    n = 500
    x, y = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    t = np.round(rng.uniform(0, 30, n))
    check(x, y, t, (1.0, 0.3, 5.0, 0.5, 0.8, 0.2), "ties")
    check(x, y, np.full(n, 7.0), (1.0, 0.3, 5.0, 0.5, 0.8, 0.2), "all one time")
    check(x, y, t, (1.0, 0.3, 5.0, 0.0, 0.8, 0.2), "theta=0")
    check(x, y, t, (1.0, 0.3, 5.0, 0.5, 1440.0, 0.0695), "minute-scale trigger")


def test_invalid_input_is_refused():
    with pytest.raises(binding.HawkesError):
        binding.host_eval([0.0], [0.0], [-1.0], (1, 0.5, 20, 0.3, 0.5, 0.1))
    with pytest.raises(binding.HawkesError):
        binding.host_eval([0.0], [0.0], [1.0], (1, -0.5, 20, 0.3, 0.5, 0.1))
