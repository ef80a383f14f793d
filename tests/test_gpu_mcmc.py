"""Algorithm 1 chains driven through the serving API: many chains in flight, each result equal to
the blocking evaluation (with shared passes on: to the multi-parameter pass's value for its
vector, within rounding of the blocking evaluation), and the whole run reproducible from the
seeds."""
import numpy as np
import pytest

from paper_2005_10123_amd import binding, mcmc, synth

pytestmark = pytest.mark.gpu


def run(ctx, dss, seeds, steps):
    theta0 = np.array(synth.THETA_CFG1)
    chains = [mcmc.ChainState(theta0.copy(), np.random.default_rng(s)) for s in seeds]
    served = mcmc.run_served(ctx, chains, [dss[k % len(dss)] for k in range(len(chains))], steps)
    return chains, served


@pytest.mark.parametrize("shared", [False, True])
def test_served_chains_reproducible_and_exact(shared):
    ctx = binding.Context(0)
    ctx.set_shared_passes(shared)
    dss = [ctx.dataset(*synth.simulate(synth.SimSpec(n, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 50, k))))
           for k, n in enumerate([2000, 3000])]
    seeds = list(range(100, 108))
    a, served = run(ctx, dss, seeds, 60)
    assert served == len(seeds) * 61
    b, _ = run(ctx, dss, seeds, 60)
    for ca, cb in zip(a, b):
        assert ca.steps == 60
        assert np.array_equal(np.array(ca.samples), np.array(cb.samples))
        assert 0 < ca.accepted < 60
    for k, ch in enumerate(a):
        blocking = ctx.loglik(dss[k % 2], ch.theta, "fp32c")
        if shared:
            assert ch.loglik == ctx.loglik_multi(dss[k % 2], [ch.theta], "fp32c", want_pi=False)[0]
            assert abs(ch.loglik - blocking) <= 1e-7 * abs(blocking)
        else:
            assert ch.loglik == blocking
    for d in dss:
        d.close()
    ctx.close()


def test_served_hmc_chains():
    """HMC chains using the fused gradient through the serving API: reproducible, and the final
    gradient of each chain equals the blocking evaluation."""
    ctx = binding.Context(0)
    dss = [ctx.dataset(*synth.simulate(synth.SimSpec(n, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 51, k))))
           for k, n in enumerate([1500, 2500])]
    theta0 = np.array(synth.THETA_CFG1)

    def go():
        chains = [mcmc.HMCChain(theta0.copy(), np.random.default_rng(200 + k), leapfrog=4, warmup=10)
                  for k in range(4)]
        served = mcmc.run_hmc_served(ctx, chains, [dss[k % 2] for k in range(4)], 20)
        return chains, served

    a, served = go()
    b, _ = go()
    assert served == sum(ch.evals for ch in a)
    for ca, cb in zip(a, b):
        assert ca.iters == 20 and ca.accepted > 0
        assert np.array_equal(np.array(ca.samples), np.array(cb.samples))
        assert np.all(np.isfinite(ca.theta))
    for d in dss:
        d.close()
    ctx.close()
