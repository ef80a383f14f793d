"""Algorithm 1 (adaptive random-scan MH with truncated-normal proposals) on a target whose answer
is known: the log-likelihood is chosen so that the posterior is a product of gamma densities with
mass near 0, where the truncation correction of the proposal matters.  CPU only."""
import math

import numpy as np
from scipy import stats

from paper_2005_10123_amd import mcmc

SHAPE = {0: 1.5, 3: 1.0, 4: 1.2, 5: 3.0}
SCALE = {0: 0.4, 3: 0.1, 4: 2.0, 5: 0.05}


def loglik(theta):
    # posterior = prior * likelihood = prod_d Gamma(theta_d; k_d, s_d)
    v = -mcmc.log_prior(theta)
    for d in mcmc.FREE:
        k, s, x = SHAPE[d], SCALE[d], theta[d]
        v += (k - 1) * math.log(x) - x / s - math.lgamma(k) - k * math.log(s)
    return v


def z_scores(ch, burn=5000):
    samples = np.array(ch.samples[burn:])
    z = {}
    for d in mcmc.FREE:
        x = samples[:, d]
        ess = mcmc.effective_sample_size(x)
        mean, sd = SHAPE[d] * SCALE[d], math.sqrt(SHAPE[d]) * SCALE[d]
        z[d] = (x.mean() - mean) / (sd / math.sqrt(ess))
    return z, samples


def test_gamma_logpdf_matches_library():
    th = np.array([0.7, 0.5, 20.0, 0.2, 1.3, 0.12])
    want = -mcmc.log_prior(th) + sum(stats.gamma.logpdf(th[d], SHAPE[d], scale=SCALE[d]) for d in mcmc.FREE)
    assert abs(loglik(th) - want) < 1e-10


def test_log_prior():
    th = np.array([1.0, 0.5, 20.0, 0.3, 0.5, 0.1])
    want = -0.5 - 0.5 * 0.0009 - 0.5 * 0.0025 - 0.5 * 1.0 - 2 * math.log(0.1)
    assert abs(mcmc.log_prior(th) - want) < 1e-12
    th[3] = 0.0
    assert mcmc.log_prior(th) == -math.inf


def test_mh_recovers_known_posterior():
    theta0 = np.array([1.0, 0.5, 20.0, 0.3, 0.5, 0.1])
    ch = mcmc.run_local(loglik, theta0, 40000, seed=3)
    z, samples = z_scores(ch)
    assert all(abs(v) < 4 for v in z.values()), z
    assert all(mcmc.effective_sample_size(samples[:, d]) > 500 for d in mcmc.FREE)
    # fixed coordinates never move
    assert np.all(samples[:, 1] == 0.5) and np.all(samples[:, 2] == 20.0)
    # adaptation drives the per-coordinate acceptance towards 0.44
    rate = ch.accepted / ch.steps
    assert 0.25 < rate < 0.65, rate


def test_truncation_correction_matters():
    """Without the Phi(x/v) ratio the chain targets the wrong density near 0 (planted mistake)."""
    theta0 = np.array([1.0, 0.5, 20.0, 0.3, 0.5, 0.1])
    orig = mcmc._log_norm_cdf
    try:
        mcmc._log_norm_cdf = lambda z: 0.0
        ch = mcmc.run_local(loglik, theta0, 40000, seed=3)
    finally:
        mcmc._log_norm_cdf = orig
    z, _ = z_scores(ch)
    assert max(abs(v) for v in z.values()) > 4.5, z


def test_ess_of_iid_and_ar1():
    rng = np.random.default_rng(0)
    assert 8000 < mcmc.effective_sample_size(rng.standard_normal(10000)) <= 10000 * 1.2
    x = np.zeros(20000)
    for k in range(1, x.size):
        x[k] = 0.9 * x[k - 1] + rng.standard_normal()
    ess = mcmc.effective_sample_size(x)
    assert 20000 * 0.03 < ess < 20000 * 0.08  # (1 - 0.9) / (1 + 0.9) = 0.053


def loglik_grad(theta):
    """(ell, d ell / d Theta) with the gamma-product posterior of the MH test."""
    g = -mcmc.log_prior_grad(theta)
    for d in mcmc.FREE:
        k, s, x = SHAPE[d], SCALE[d], theta[d]
        g[d] += (k - 1) / x - 1 / s
    return loglik(theta), g


def test_log_prior_grad_matches_finite_differences():
    th = np.array([0.7, 0.5, 20.0, 0.2, 1.3, 0.12])
    g = mcmc.log_prior_grad(th)
    for d in mcmc.FREE:
        e = np.zeros(6)
        e[d] = 1e-6 * th[d]
        fd = (mcmc.log_prior(th + e) - mcmc.log_prior(th - e)) / (2 * e[d])
        assert abs(fd - g[d]) <= 1e-6 * max(1.0, abs(g[d]))


def test_hmc_recovers_known_posterior():
    theta0 = np.array([1.0, 0.5, 20.0, 0.3, 0.5, 0.1])
    ch = mcmc.run_hmc_local(loglik_grad, theta0, 4000, seed=5, warmup=300)
    samples = np.array(ch.samples)
    for d in mcmc.FREE:
        x = samples[:, d]
        ess = mcmc.effective_sample_size(x)
        mean, sd = SHAPE[d] * SCALE[d], math.sqrt(SHAPE[d]) * SCALE[d]
        assert abs(x.mean() - mean) < 4.5 * sd / math.sqrt(ess), (d, x.mean(), mean, ess)
    assert 0.5 < ch.accepted / ch.iters < 0.95
