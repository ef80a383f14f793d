"""Pins that fix the FP64 oracle against the paper and the mathematics, not against itself.

Each ``pin_*`` function takes a loaded oracle library (the real one or a planted-mistake copy) and
raises ``AssertionError`` when the oracle disagrees with an independent evaluation:

* ``pin_n1``          N = 1 closed form of the log-likelihood and its gradient;
* ``pin_library``     per-event lambda_n, Lambda_n and pi_n = xi_n / lambda_n from scipy.stats
                      probability densities (3-D normal background kernel, exponential x 2-D
                      normal trigger; xi_n the trigger part of lambda_n);
* ``pin_rows``        the selected-rows entry point against the whole evaluation, and its six
                      per-event sums against density ratios of scipy.stats kernels summed in numpy;
* ``pin_mpmath``      40-digit brute-force sums of mpmath normal densities on the small fixtures,
                      with the gradient from mpmath's numerical differentiation;
* ``pin_quadrature``  adaptive quadrature of the intensity over [0, T] against the closed-form
                      integrated intensity;
* ``pin_fd``          central finite differences of the oracle's own log-likelihood against its
                      analytic gradient;
* ``pin_identity``    mu0 dl/dmu0 + theta dl/dtheta = N - Lambda (linearity of lambda, Lambda
                      in mu0 and theta), per event and in total;
* ``pin_invariants``  theta = 0, all-ties, permutation, spatial translation, 0 <= pi <= 1.

Model: arXiv 2005.10123 Section 2.1 (intensity, background, trigger, likelihood, integrated
intensity, self-excitation probability).  The excitation coefficient is read as theta*omega/h^d, the
one consistent with the paper's closed-form temporal integral.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_cases.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _case(name):
    c = golden()["cases"][name]
    return np.array(c["x"], float), np.array(c["y"], float), np.array(c["t"], float)


def _theta(name="theta_small"):
    return np.array(golden()[name]["value"], float)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def random_events(n, seed, L=3.0, T=30.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, L, n), rng.uniform(0, L, n), np.sort(rng.uniform(0, T, n))


# ----------------------------------------------------------------------------------------------
def pin_n1(lib):
    """N = 1: lambda_1 is the diagonal background term alone and T = t_1, so
    ell = log(mu0 (2 pi)^(-3/2) tau_x^-2 tau_t^-1) - mu0 (1/2 - Phi(-t_1/tau_t))."""
    from scipy.stats import norm

    rng = np.random.default_rng(7)
    for _ in range(8):
        mu0, tx, tt, th, om, h = rng.uniform([0.2, 0.1, 1, 0.0, 0.05, 0.01], [3, 2, 40, 0.9, 5, 0.5])
        t1 = rng.uniform(0, 100)
        ell, g = oracle.evaluate([0.3], [-1.2], [t1], [mu0, tx, tt, th, om, h], lib=lib)
        want = math.log(mu0 / ((2 * math.pi) ** 1.5 * tx * tx * tt)) - mu0 * (0.5 - norm.cdf(-t1 / tt))
        assert _rel(ell, want) < 1e-13, ("N=1 ell", ell, want)
        g_mu = 1 / mu0 - (0.5 - norm.cdf(-t1 / tt))
        g_tt = -1 / tt + mu0 * t1 * norm.pdf(t1 / tt) / tt**2
        assert _rel(g[0], g_mu) < 1e-12, ("N=1 dmu0", g[0], g_mu)
        assert _rel(g[1], -2 / tx) < 1e-13, ("N=1 dtau_x", g[1], -2 / tx)
        assert _rel(g[2], g_tt) < 1e-11, ("N=1 dtau_t", g[2], g_tt)
        assert g[3] == 0.0 and g[4] == 0.0 and g[5] == 0.0, ("N=1 excitation grads", g)


# ----------------------------------------------------------------------------------------------
def library_rows(x, y, t, th, with_trigger=False):
    """lambda_n and Lambda_n from scipy.stats densities (independent of the oracle's algebra);
    with ``with_trigger`` also xi_n, the trigger (self-excitation) part of lambda_n."""
    from scipy.stats import expon, multivariate_normal, norm

    mu0, tx, tt, theta, omega, h = th
    pts = np.stack([x, y, t], axis=1)
    T = t.max()
    lam = np.empty(x.size)
    Lam = np.empty(x.size)
    xi = np.zeros(x.size)
    for i in range(x.size):
        bg = multivariate_normal(mean=pts[i], cov=np.diag([tx**2, tx**2, tt**2])).pdf(pts)
        bg = np.atleast_1d(bg)
        causal = t < t[i]
        ex = 0.0
        if causal.any():
            sp = multivariate_normal(mean=pts[i, :2], cov=h**2 * np.eye(2)).pdf(pts[causal, :2])
            ex = np.sum(np.atleast_1d(sp) * expon(scale=1 / omega).pdf(t[i] - t[causal]))
        xi[i] = theta * ex
        lam[i] = mu0 * bg.sum() + xi[i]
        Lam[i] = (mu0 * (norm.cdf(T, loc=t[i], scale=tt) - norm.cdf(0.0, loc=t[i], scale=tt))
                  + theta * expon(scale=1 / omega).cdf(T - t[i]))
    if with_trigger:
        return lam, Lam, xi
    return lam, Lam


def pin_library(lib):
    rng = np.random.default_rng(11)
    for k in range(4):
        n = [7, 19, 30, 12][k]
        x, y, t = random_events(n, 100 + k, L=[1.0, 3.0, 0.6, 2.0][k], T=[5.0, 40.0, 10.0, 3.0][k])
        if k == 3:
            t[3] = t[4]  # a tie
        th = rng.uniform([0.3, 0.2, 1.0, 0.05, 0.2, 0.05], [2.0, 1.5, 10.0, 0.9, 3.0, 0.6])
        res = oracle.evaluate(x, y, t, th, lib=lib, rows=True)
        lam, Lam, xi = library_rows(x, y, t, th, with_trigger=True)
        ell_lib = np.log(lam) - Lam
        assert np.max(np.abs(res["row_ell"] - ell_lib) / np.abs(ell_lib)) < 1e-12, "row ell vs scipy"
        assert np.max(np.abs(res["row_Lambda"] - Lam) / np.abs(Lam)) < 1e-12, "Lambda vs scipy"
        assert _rel(res["ell"], ell_lib.sum()) < 1e-12, "ell vs scipy"
        # Self-excitation probability (Section 2.1, probability equation): the trigger part of
        # lambda_n over lambda_n.  Events with no causal predecessor have pi_n = 0 exactly.
        pi_lib = xi / lam
        assert np.all(res["row_pi"][xi == 0] == 0.0), "pi of untriggerable events"
        pos = xi > 0
        assert pos.sum() >= n // 2, "the case must hold triggerable events"
        assert np.max(np.abs(res["row_pi"][pos] - pi_lib[pos]) / pi_lib[pos]) < 1e-12, "pi vs scipy"


# ----------------------------------------------------------------------------------------------
def library_sums(x, y, t, th):
    """The six per-event sums S_b, S_br, S_bt, S_e, S_et, S_er of the unnormalised kernels, each
    kernel value taken as a scipy.stats density divided by the same density at its own mean (so no
    normalising constant is retyped here): B_ij = N3(p_j; p_i, diag(tx^2, tx^2, tt^2)) / peak and,
    for t_j < t_i, E_ij = Exp(t_i - t_j; omega) N2(x_j; x_i, h^2 I) / (Exp(0; omega) N2 peak).
    The moments weight them by r^2 = |x_i - x_j|^2 and dt = t_i - t_j (dt^2 for the background)."""
    from scipy.stats import expon, multivariate_normal

    _, tx, tt, _, omega, h = th
    pts = np.stack([x, y, t], axis=1)
    out = np.zeros((x.size, 6))
    for i in range(x.size):
        bmv = multivariate_normal(mean=pts[i], cov=np.diag([tx**2, tx**2, tt**2]))
        B = np.atleast_1d(bmv.pdf(pts)) / bmv.pdf(pts[i])
        r2 = (x[i] - x) ** 2 + (y[i] - y) ** 2
        dt = t[i] - t
        out[i, 0] = B.sum()
        out[i, 1] = (r2 * B).sum()
        out[i, 2] = (dt * dt * B).sum()
        causal = t < t[i]
        if causal.any():
            smv = multivariate_normal(mean=pts[i, :2], cov=h**2 * np.eye(2))
            ex = expon(scale=1 / omega)
            E = (np.atleast_1d(smv.pdf(pts[causal, :2])) * ex.pdf(dt[causal])) / (smv.pdf(pts[i, :2]) * ex.pdf(0.0))
            out[i, 3] = E.sum()
            out[i, 4] = (dt[causal] * E).sum()
            out[i, 5] = (r2[causal] * E).sum()
    return out


def pin_rows(lib):
    """``hawkes_oracle_rows`` (16 doubles per selected event) against the whole evaluation and
    against the library densities: every field in its documented slot, for rows in any order."""
    rng = np.random.default_rng(21)
    x, y, t = random_events(30, 2100, L=0.8, T=6.0)
    t[7] = t[8]  # a tie
    th = np.array([1.1, 0.45, 1.5, 0.6, 0.9, 0.3])
    full = oracle.evaluate(x, y, t, th, lib=lib, rows=True)
    idx = rng.permutation(x.size)[:23]
    r = oracle.rows(x, y, t, th, idx, lib=lib)
    assert np.array_equal(r["ell"], full["row_ell"][idx]), "rows: ell slot"
    assert np.array_equal(r["Lambda"], full["row_Lambda"][idx]), "rows: Lambda slot"
    assert np.array_equal(r["pi"], full["row_pi"][idx]), "rows: pi slot"
    assert np.array_equal(r["grad"], full["row_grad"][idx]), "rows: gradient slots"
    lam_lib, Lam_lib, xi_lib = library_rows(x, y, t, th, with_trigger=True)
    assert np.max(np.abs(r["lambda"] - lam_lib[idx]) / lam_lib[idx]) < 1e-12, "rows: lambda slot"
    sums = library_sums(x, y, t, th)[idx]
    assert np.all(sums[:, 3:] > 0) or np.any(xi_lib[idx] == 0), "the case must exercise the trigger sums"
    scale = np.maximum(np.abs(sums), 1e-300)
    nz = np.abs(sums) > 0
    assert np.all(r["sums"][~nz] == 0.0), "rows: sums of events without causal predecessors"
    err = np.abs(r["sums"] - sums) / scale
    assert np.max(err[nz]) < 1e-12, ("rows: sums vs scipy", err.max(axis=0))


# ----------------------------------------------------------------------------------------------
def mp_loglik(x, y, t, th):
    """Brute-force log-likelihood from mpmath normal densities and CDFs, at the working precision
    of the caller (``mpmath.workdps``)."""
    import mpmath as mp

    mu0, tx, tt, theta, omega, h = [mp.mpf(v) for v in th]
    X = [mp.mpf(v) for v in x]
    Y = [mp.mpf(v) for v in y]
    Tt = [mp.mpf(v) for v in t]
    T = max(Tt)
    total = mp.mpf(0)
    for i in range(len(X)):
        lam = mp.mpf(0)
        for j in range(len(X)):
            lam += mu0 * (mp.npdf(X[i] - X[j], 0, tx) * mp.npdf(Y[i] - Y[j], 0, tx)
                          * mp.npdf(Tt[i] - Tt[j], 0, tt))
            if Tt[j] < Tt[i]:
                dt = Tt[i] - Tt[j]
                lam += theta * omega * mp.exp(-omega * dt) * (mp.npdf(X[i] - X[j], 0, h)
                                                              * mp.npdf(Y[i] - Y[j], 0, h))
        Lam = (mu0 * (mp.ncdf(T, Tt[i], tt) - mp.ncdf(0, Tt[i], tt))
               + theta * (1 - mp.exp(-omega * (T - Tt[i]))))
        total += mp.log(lam) - Lam
    return total


def pin_mpmath(lib, grad=True):
    import mpmath as mp

    with mp.workdps(40):
        _pin_mpmath(lib, grad)


def _pin_mpmath(lib, grad):
    import mpmath as mp

    for name in ["E1_single", "E2_pair", "E3_tie", "E4_five", "E5_unsorted"]:
        x, y, t = _case(name)
        for thn in ["theta_small", "theta_posterior_regime"]:
            th = _theta(thn)
            ell, g = oracle.evaluate(x, y, t, th, lib=lib)
            want = mp_loglik(x, y, t, th)
            assert _rel(ell, float(want)) < 1e-14, (name, thn, ell, float(want))
            if not grad or thn != "theta_small":
                continue
            for p in range(6):
                def f(v, p=p):
                    q = [mp.mpf(c) for c in th]
                    q[p] = v
                    return mp_loglik(x, y, t, q)
                gp = float(mp.diff(f, mp.mpf(th[p])))
                assert abs(g[p] - gp) <= 1e-11 * max(1.0, abs(gp)), (name, p, g[p], gp)


# ----------------------------------------------------------------------------------------------
def pin_quadrature(lib):
    """int_0^T int_R2 lambda(x, t) dx dt == sum_n Lambda_n.  The spatial integral of each kernel is
    1 (normalised densities), so the space-integrated intensity is
    mu0 sum_n N(t; t_n, tau_t^2) + theta sum_{t_n < t} omega exp(-omega (t - t_n)); it is
    integrated by adaptive quadrature split at every event time (the trigger jumps there)."""
    from scipy.integrate import quad
    from scipy.stats import expon, norm

    for k, (n, th) in enumerate([(4, [1.3, 0.4, 2.0, 0.4, 0.7, 0.2]),
                                 (5, [0.6, 1.0, 0.5, 0.8, 3.0, 0.1]),
                                 (3, [2.0, 0.3, 8.0, 0.1, 0.05, 0.3])]):
        x, y, t = random_events(n, 300 + k, L=2.0, T=12.0)
        res = oracle.evaluate(x, y, t, th, lib=lib, rows=True)
        mu0, tx, tt, theta, omega, h = th

        def rate(s):
            bg = mu0 * np.sum(norm.pdf(s, loc=t, scale=tt))
            past = t < s
            return bg + theta * np.sum(expon(scale=1 / omega).pdf(s - t[past]))

        knots = np.concatenate([[0.0], np.sort(t)])
        total = 0.0
        for a, b in zip(knots[:-1], knots[1:]):
            if b > a:
                total += quad(rate, a, b, epsabs=1e-13, epsrel=1e-13, limit=200)[0]
        Lam = res["row_Lambda"].sum()
        assert _rel(Lam, total) < 1e-9, ("quadrature", Lam, total)


# ----------------------------------------------------------------------------------------------
def pin_fd(lib, n=120):
    x, y, t = random_events(n, 17, L=2.0, T=60.0)
    th = np.array([1.0, 0.5, 20.0, 0.3, 0.5, 0.1])
    res = oracle.evaluate(x, y, t, th, lib=lib, rows=True)
    g = res["grad"]
    l1 = np.abs(res["row_grad"]).sum(axis=0)
    for p in range(6):
        step = 1e-6 * th[p]
        tp, tm = th.copy(), th.copy()
        tp[p] += step
        tm[p] -= step
        fd = (oracle.evaluate(x, y, t, tp, lib=lib)[0] - oracle.evaluate(x, y, t, tm, lib=lib)[0]) / (2 * step)
        assert abs(fd - g[p]) <= 1e-6 * l1[p], ("FD", p, fd, g[p], l1[p])


# ----------------------------------------------------------------------------------------------
def pin_identity(lib):
    for k in range(3):
        x, y, t = random_events(60, 500 + k, L=1.5, T=20.0)
        th = np.array([0.8 + k, 0.4, 5.0, 0.2 + 0.3 * k, 1.5, 0.15])
        res = oracle.evaluate(x, y, t, th, lib=lib, rows=True)
        rg = res["row_grad"]
        per_row = th[0] * rg[:, 0] + th[3] * rg[:, 3]
        assert np.max(np.abs(per_row - (1 - res["row_Lambda"]))) < 1e-12, "row identity"
        total = th[0] * res["grad"][0] + th[3] * res["grad"][3]
        want = x.size - res["row_Lambda"].sum()
        assert abs(total - want) < 1e-11 * x.size, ("identity", total, want)


# ----------------------------------------------------------------------------------------------
def pin_invariants(lib):
    x, y, t = random_events(40, 900, L=1.0, T=15.0)
    # theta = 0: background only, independent of (omega, h), zero omega/h gradient.
    a = oracle.evaluate(x, y, t, [1.0, 0.5, 3.0, 0.0, 0.5, 0.1], lib=lib)
    b = oracle.evaluate(x, y, t, [1.0, 0.5, 3.0, 0.0, 3.0, 0.7], lib=lib)
    assert a[0] == b[0], "theta=0 must not depend on omega, h"
    assert a[1][4] == 0.0 and a[1][5] == 0.0, "theta=0: d/domega = d/dh = 0"
    # All events at one time: no excitation anywhere, Lambda has no trigger part (u = 0).
    tt = np.full(x.size, 4.0)
    c = oracle.evaluate(x, y, tt, [1.0, 0.5, 3.0, 0.3, 0.5, 0.1], lib=lib)
    d = oracle.evaluate(x, y, tt, [1.0, 0.5, 3.0, 0.9, 2.0, 0.4], lib=lib)
    assert c[0] == d[0], "all ties: independent of theta, omega, h"
    assert c[1][3] == 0.0 and c[1][4] == 0.0 and c[1][5] == 0.0, "all ties: zero trigger gradient"
    # Permutation of the input and translation in space.
    th = [1.2, 0.6, 4.0, 0.4, 0.8, 0.2]
    ref = oracle.evaluate(x, y, t, th, lib=lib, rows=True)
    perm = np.random.default_rng(3).permutation(x.size)
    p = oracle.evaluate(x[perm], y[perm], t[perm], th, lib=lib)
    assert _rel(p[0], ref["ell"]) < 1e-13 and np.allclose(p[1], ref["grad"], rtol=1e-11, atol=1e-11)
    s = oracle.evaluate(x + 3.7, y - 12.25, t, th, lib=lib)
    assert _rel(s[0], ref["ell"]) < 1e-12 and np.allclose(s[1], ref["grad"], rtol=1e-9, atol=1e-9)
    # Self-excitation probabilities.
    pi = ref["row_pi"]
    assert np.all(pi >= 0) and np.all(pi <= 1)
    assert pi[np.argmin(t)] == 0.0, "the earliest event cannot be triggered"


ALL_PINS = [pin_n1, pin_library, pin_rows, pin_mpmath, pin_quadrature, pin_fd, pin_identity, pin_invariants]
