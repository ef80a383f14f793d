"""Batched serving through hawkes_submit / hawkes_poll: each result matches the FP64 oracle and
is bitwise the same alone and whatever it is batched with: equal to the blocking evaluation (same
plan, same arithmetic), or, with shared passes on, for FP32C log-likelihoods (evaluated in shared
multi-parameter passes) to hawkes_loglik_multi's value for that vector; invalid requests fail
alone; a small HBM budget queues work instead of failing; destroying a busy dataset is refused;
destroying the context with requests in flight is clean; several threads may submit at once."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, assert_close, rel
from paper_2005_10123_amd import binding, synth

pytestmark = pytest.mark.gpu


def datasets(ctx, sizes, seed0=40, events=False):
    out, evs = [], []
    for k, n in enumerate(sizes):
        spec = synth.SimSpec(n, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, seed0, k))
        ev = synth.simulate(spec)
        evs.append(ev)
        out.append(ctx.dataset(*ev))
    return (out, evs) if events else out


def drain(ctx, count, timeout_s=60.0):
    import time

    got = {}
    end = time.time() + timeout_s
    while len(got) < count:
        assert time.time() < end, "serving did not complete in time"
        for r in ctx.poll(cap=256, timeout_us=100000):
            got[r.tag] = r
    return got


def test_alone_equals_mix():
    """48 requests over four datasets, both precisions, with and without the gradient, submitted in
    bursts so that launches hold several requests: every served result against the oracle's
    evaluation of its own dataset and parameters, and bitwise equal to the blocking call."""
    ctx = binding.Context(0)
    dss, evs = datasets(ctx, [3000, 700, 9000, 1500], events=True)
    rng = np.random.default_rng(1)
    theta0 = np.array(synth.THETA_CFG1)
    reqs = []
    for k in range(48):
        th = theta0 * np.exp(0.1 * rng.standard_normal(6))
        prec = "fp32c" if k % 3 else "fp64"
        reqs.append(binding.request(dss[k % 4], th, prec, want_grad=(k % 5 != 0), tag=k))
    # Submitted in several bursts so later requests join while earlier launches run.
    ctx.submit(reqs[:5])
    ctx.submit(reqs[5:20])
    ctx.submit(reqs[20:])
    got = drain(ctx, len(reqs))
    for k, r in enumerate(reqs):
        res = got[r.tag]
        assert res.status == 0
        prec = "fp64" if r.precision == binding.FP64 else "fp32c"
        th = [getattr(r.p, name) for name in binding.PARAM_NAMES]
        ref = oracle.evaluate_parallel(*evs[k % 4], th)
        if r.want_grad:
            assert_close(res.loglik, np.array(res.grad[:]), ref, prec, ("served", r.tag), th)
        else:
            assert rel(res.loglik, ref["ell"]) <= TOL[prec], (r.tag, prec, res.loglik, ref["ell"])
        if r.want_grad:
            ell, g = ctx.grad(r.dataset, r.p, prec)
            assert res.loglik == ell and np.array_equal(np.array(res.grad[:]), g), r.tag
        else:
            ell = ctx.loglik(r.dataset, r.p, prec)
            assert res.loglik == ell and all(v == 0.0 for v in res.grad), r.tag
        assert res.t_done_ns >= res.t_submit_ns
    assert ctx.outstanding() == 0
    for d in dss:
        d.close()
    ctx.close()


def test_bad_requests_fail_alone():
    ctx = binding.Context(0)
    (ds,) = datasets(ctx, [1200])
    good = binding.request(ds, synth.THETA_CFG1, "fp32c", True, tag=1)
    bad_theta = binding.request(ds, (1.0, -0.5, 20.0, 0.3, 0.5, 0.1), "fp32c", True, tag=2)
    bad_ds = binding.request(9999, synth.THETA_CFG1, "fp32c", True, tag=3)
    bad_prec = binding.request(ds, synth.THETA_CFG1, 7, True, tag=4)
    ctx.submit([good, bad_theta, bad_ds, bad_prec])
    got = drain(ctx, 4)
    assert got[1].status == 0
    assert got[2].status == binding.HAWKES_EINVAL
    assert got[3].status == binding.HAWKES_ENOTFOUND
    assert got[4].status == binding.HAWKES_EINVAL
    ell, g = ctx.grad(ds, synth.THETA_CFG1, "fp32c")
    assert got[1].loglik == ell
    ds.close()
    ctx.close()


def test_budget_queues_instead_of_failing():
    # A budget that holds the datasets and roughly one request's scratch at a time.
    ctx = binding.Context(0, hbm_budget=48 << 20)
    dss = datasets(ctx, [20000, 20000], seed0=41)
    reqs = [binding.request(dss[k % 2], synth.THETA_CFG1, "fp32c", True, tag=k) for k in range(12)]
    ctx.submit(reqs)
    got = drain(ctx, len(reqs))
    ref = [ctx.grad(d, synth.THETA_CFG1, "fp32c")[0] for d in dss]
    for k in range(12):
        assert got[k].status == 0
        assert got[k].loglik == ref[k % 2]
    for d in dss:
        d.close()
    ctx.close()


def test_request_that_can_never_fit():
    ctx = binding.Context(0, hbm_budget=12 << 20)
    (ds,) = datasets(ctx, [60000], seed0=42)
    ctx.submit([binding.request(ds, synth.THETA_CFG1, "fp32c", True, tag=5)])
    got = drain(ctx, 1)
    assert got[5].status == binding.HAWKES_ENOMEM
    ds.close()
    ctx.close()


def test_dataset_busy_while_requests_in_flight():
    ctx = binding.Context(0)
    (ds,) = datasets(ctx, [40000], seed0=43)
    ctx.submit([binding.request(ds, synth.THETA_CFG1, "fp64", True, tag=k) for k in range(8)])
    with pytest.raises(binding.HawkesError) as e:
        ds.close()
    assert e.value.status == binding.HAWKES_EBUSY
    drain(ctx, 8)
    ds.close()
    ctx.close()


def test_destroy_with_requests_in_flight():
    """Destroying a context while its requests are queued or running waits for the device, drops
    them and frees everything; the device is usable afterwards."""
    import time

    ctx = binding.Context(0)
    (ds,) = datasets(ctx, [20000], seed0=44)
    theta0 = np.array(synth.THETA_CFG1)
    ctx.submit([binding.request(ds, theta0 * (1.0 + 0.01 * k), "fp32c", True, k) for k in range(40)])
    a = time.time()
    ctx.close()
    assert time.time() - a < 30.0
    ctx2 = binding.Context(0)
    (ds2,) = datasets(ctx2, [700], seed0=45)
    ell, g = ctx2.grad(ds2, theta0, "fp64")
    assert np.isfinite(ell) and np.all(np.isfinite(g))
    ds2.close()
    ctx2.close()


def test_submit_from_many_threads():
    """One context shared by several submitting threads (as chains would): every request completes
    once, with the blocking result."""
    import threading

    ctx = binding.Context(0)
    dss = datasets(ctx, [2000, 5000], seed0=46)
    theta0 = np.array(synth.THETA_CFG1)
    rng = np.random.default_rng(9)
    thetas = theta0 * np.exp(0.1 * rng.standard_normal((64, 6)))
    want = [ctx.grad(dss[k % 2], thetas[k], "fp32c") for k in range(64)]

    def worker(w):
        for k in range(w, 64, 4):
            ctx.submit([binding.request(dss[k % 2], thetas[k], "fp32c", True, k)])

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    got = drain(ctx, 64)
    assert sorted(got) == list(range(64))
    for k in range(64):
        assert got[k].status == 0
        assert got[k].loglik == want[k][0] and np.array_equal(np.array(got[k].grad[:]), want[k][1]), k
    for d in dss:
        d.close()
    ctx.close()


def test_shared_passes_alone_equal_grouped():
    """FP32C log-likelihood requests (the requests of Algorithm 1's chains) on one dataset share
    multi-parameter passes: 4 requests on each of two datasets submitted at once (grouped four per
    pass), then each again alone; every result is bitwise the same both ways, equal to
    hawkes_loglik_multi for its vector, and within the FP32C tolerance of the oracle."""
    ctx = binding.Context(0)
    ctx.set_shared_passes(True)
    dss, evs = datasets(ctx, [6000, 11000], seed0=47, events=True)
    rng = np.random.default_rng(12)
    thetas = np.array(synth.THETA_CFG1) * np.exp(0.1 * rng.standard_normal((8, 6)))
    reqs = [binding.request(dss[k % 2], thetas[k], "fp32c", False, tag=k) for k in range(8)]
    ctx.submit(reqs)
    grouped = drain(ctx, 8)
    alone = {}
    for k in range(8):
        ctx.submit([binding.request(dss[k % 2], thetas[k], "fp32c", False, tag=100 + k)])
        alone.update(drain(ctx, 1))
    for k in range(8):
        a, g = alone[100 + k], grouped[k]
        assert a.status == 0 and g.status == 0
        assert a.loglik == g.loglik, (k, a.loglik, g.loglik)
        assert g.loglik == ctx.loglik_multi(dss[k % 2], [thetas[k]], "fp32c", want_pi=False)[0]
        ref = oracle.evaluate_parallel(*evs[k % 2], thetas[k])
        assert rel(g.loglik, ref["ell"]) <= TOL["fp32c"], (k, g.loglik, ref["ell"])
        assert rel(g.loglik, ctx.loglik(dss[k % 2], thetas[k], "fp32c")) <= 1e-7, k
    # Shared passes off (the default): the single-parameter pass, bitwise the blocking call.
    ctx.set_shared_passes(False)
    ctx.submit(reqs)
    plain = drain(ctx, 8)
    for k in range(8):
        assert plain[k].loglik == ctx.loglik(dss[k % 2], thetas[k], "fp32c"), k
    for d in dss:
        d.close()
    ctx.close()
