"""Adaptive random-scan Metropolis-Hastings chains (the paper's Algorithm 1) driven by the batched
serving API: every chain's likelihood evaluation is a request to ``hawkes_submit``, many chains are
in flight at once, and a chain advances as soon as its own result is polled.

Algorithm 1 (Section 2.2): pick a coordinate d uniformly; propose theta*_d from a normal centred at
the current value with scale v_d, truncated to theta*_d > 0; accept with the Metropolis-Hastings
ratio (prior x likelihood x the ratio of the truncated proposals' normalising constants); every
b_d updates of coordinate d, multiply v_d by the acceptance proportion over 0.44 clamped to
[0.5, 2], raise b_d to b_d^1.1 and reset the counters.  Because b_d^1.1 is not an integer, the
interval ends when the counter reaches b_d or more.

Priors (Section 2.1): truncated normals with lower bound 0 (half-normals) with standard deviation 1
on mu0, 10 on theta, 10 on omega, and 10 on 1/h; tau_x and tau_t are held fixed.  The chain moves h
itself, so the prior density of h carries the Jacobian |d(1/h)/dh| = 1/h^2 (a reading: the paper
does not say on which scale the chain moves).

Pure host logic: the log-likelihood comes from the library (or, in tests, from any callable).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Coordinates of Theta = (mu0, tau_x, tau_t, theta, omega, h) that the chain updates.
FREE = (0, 3, 4, 5)
PRIOR_SD = {0: 1.0, 3: 10.0, 4: 10.0, 5: 10.0}


def log_prior(theta) -> float:
    """Half-normal priors of Section 2.1 (up to a constant); -inf outside the positive orthant."""
    mu0, _, _, th, om, h = theta
    if mu0 <= 0 or th <= 0 or om <= 0 or h <= 0:
        return -math.inf
    lp = -0.5 * (mu0 / PRIOR_SD[0]) ** 2 - 0.5 * (th / PRIOR_SD[3]) ** 2 - 0.5 * (om / PRIOR_SD[4]) ** 2
    inv_h = 1.0 / h
    lp += -0.5 * (inv_h / PRIOR_SD[5]) ** 2 - 2.0 * math.log(h)  # density of 1/h, moved to h
    return lp


def _log_norm_cdf(z: float) -> float:
    return math.log(0.5 * math.erfc(-z / math.sqrt(2.0)))


@dataclass
class ChainState:
    """One chain of Algorithm 1."""

    theta: np.ndarray
    rng: np.random.Generator
    loglik: float = math.nan
    b: np.ndarray = field(default_factory=lambda: np.full(6, 5.0))
    l: np.ndarray = field(default_factory=lambda: np.zeros(6))
    a: np.ndarray = field(default_factory=lambda: np.zeros(6))
    v: np.ndarray = field(default_factory=lambda: np.ones(6))
    proposal: np.ndarray | None = None
    coord: int = -1
    samples: list = field(default_factory=list)
    accepted: int = 0
    steps: int = 0

    def propose(self) -> np.ndarray:
        """Steps 3a-3b: choose d and draw theta*_d ~ Normal(theta_d, v_d) restricted to > 0."""
        d = FREE[self.rng.integers(len(FREE))]
        cur = self.theta[d]
        while True:
            x = cur + self.v[d] * self.rng.standard_normal()
            if x > 0:
                break
        prop = self.theta.copy()
        prop[d] = x
        self.coord = d
        self.proposal = prop
        return prop

    def log_ratio(self, loglik_prop: float) -> float:
        """Step 4a in logs: target ratio times q(Theta | Theta*) / q(Theta* | Theta).  For normals
        truncated at 0 the kernels' Gaussian parts cancel and the normalisers Phi(x / v) remain."""
        d = self.coord
        v = self.v[d]
        x_old, x_new = self.theta[d], self.proposal[d]
        lq = _log_norm_cdf(x_old / v) - _log_norm_cdf(x_new / v)
        return (loglik_prop + log_prior(self.proposal)) - (self.loglik + log_prior(self.theta)) + lq

    def accept_reject(self, loglik_prop: float):
        """Steps 4b-4c (accept/reject) and 5 (adaptation)."""
        d = self.coord
        if math.log(self.rng.uniform()) < self.log_ratio(loglik_prop):
            self.theta = self.proposal
            self.loglik = loglik_prop
            self.a[d] += 1
            self.accepted += 1
        self.l[d] += 1
        if self.l[d] >= self.b[d]:
            r3 = min(2.0, max(0.5, (self.a[d] / self.b[d]) / 0.44))
            self.v[d] *= r3
            self.b[d] = self.b[d] ** 1.1
            self.l[d] = 0
            self.a[d] = 0
        self.proposal = None
        self.steps += 1
        self.samples.append(self.theta.copy())


def run_local(loglik, theta0, steps: int, seed: int) -> ChainState:
    """One chain with a synchronous log-likelihood callable (for tests and small runs)."""
    ch = ChainState(np.array(theta0, float), np.random.default_rng(seed))
    ch.loglik = loglik(ch.theta)
    for _ in range(steps):
        ch.accept_reject(loglik(ch.propose()))
    return ch


def run_served(ctx, chains: list, datasets: list, steps: int, precision="fp32c", poll_us=200, on_result=None):
    """Advance many chains through the serving API until each has taken `steps` MH steps.

    chains[k] runs on datasets[k].  Each chain keeps one request in flight; a chain's next proposal
    is submitted as soon as its previous result is polled, so requests of different chains overlap
    on the device.  ``on_result(k, result)``, if given, sees every polled result of chain k.
    Returns the number of requests served.
    """
    from . import binding

    tag_of = {}
    pending = []
    for k, (ch, ds) in enumerate(zip(chains, datasets)):
        tag_of[k] = ("init", k)
        pending.append(binding.request(ds, ch.theta, precision, want_grad=False, tag=2 * k))
    ctx.submit(pending)
    waiting = len(chains)
    served = 0
    while waiting:
        for r in ctx.poll(cap=512, timeout_us=poll_us):
            served += 1
            if r.status != 0:
                raise RuntimeError(f"request {r.tag} failed with status {r.status}")
            k, is_prop = divmod(int(r.tag), 2)
            if on_result is not None:
                on_result(k, r)
            ch = chains[k]
            if is_prop:
                ch.accept_reject(r.loglik)
            else:
                ch.loglik = r.loglik
            if ch.steps >= steps:
                waiting -= 1
                continue
            ctx.submit([binding.request(datasets[k], ch.propose(), precision, want_grad=False, tag=2 * k + 1)])
    return served


def chain_ess(chains: list, burn_fraction: float = 0.5) -> dict:
    """ESS of each free coordinate summed over chains, each chain's samples after discarding the
    first ``burn_fraction`` of them."""
    out = {}
    for d in FREE:
        tot = 0.0
        for ch in chains:
            xs = np.array([s[d] for s in ch.samples])
            tot += effective_sample_size(xs[int(burn_fraction * xs.size):])
        out[d] = tot
    return out


def effective_sample_size(x: np.ndarray) -> float:
    """ESS = n / tau with tau = 1 + 2 sum_k rho_k, the sum truncated at the first negative pair of
    consecutive autocorrelations (Geyer's initial positive sequence)."""
    x = np.asarray(x, float)
    n = x.size
    if n < 4 or np.var(x) == 0:
        return float(n)
    xc = x - x.mean()
    f = np.fft.rfft(xc, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    acf /= acf[0]
    tau = -1.0
    for m in range(0, n // 2):
        pair = acf[2 * m] + acf[2 * m + 1]
        if pair <= 0:
            break
        tau += 2.0 * pair
    return n / max(1.0, tau)


# ----------------------------------------------------------------------------------------------
# Hamiltonian Monte Carlo on q = log(Theta_free), using the fused log-likelihood gradient.
#
# The target in q is ell(Theta) + log prior(Theta) + sum_d q_d (Jacobian of Theta_d = exp(q_d)).
# Leapfrog integration with a diagonal unit mass, a fixed number of steps, and a step size tuned
# during warm-up by dual averaging (Hoffman and Gelman, 2014, Algorithm 5) towards a target mean
# acceptance probability; frozen afterwards.

def log_prior_grad(theta) -> np.ndarray:
    """d log_prior / d Theta for the free coordinates (zeros elsewhere)."""
    g = np.zeros(6)
    g[0] = -theta[0] / PRIOR_SD[0] ** 2
    g[3] = -theta[3] / PRIOR_SD[3] ** 2
    g[4] = -theta[4] / PRIOR_SD[4] ** 2
    h = theta[5]
    g[5] = 1.0 / (h ** 3 * PRIOR_SD[5] ** 2) - 2.0 / h
    return g


@dataclass
class HMCChain:
    theta: np.ndarray
    rng: np.random.Generator
    leapfrog: int = 8
    eps: float = 0.05
    warmup: int = 100
    target_accept: float = 0.75
    samples: list = field(default_factory=list)
    accepted: int = 0
    iters: int = 0
    evals: int = 0
    # dual averaging state
    _mu: float = 0.0
    _hbar: float = 0.0
    _log_eps_bar: float = 0.0

    def __post_init__(self):
        self._mu = math.log(10.0 * self.eps)

    @staticmethod
    def _q(theta):
        return np.log(theta[list(FREE)])

    def _theta(self, q):
        th = self.theta.copy()
        th[list(FREE)] = np.exp(q)
        return th

    def _logp_grad(self, theta, ell, grad):
        """Target and its gradient in q from (ell, d ell / d Theta)."""
        q = self._q(theta)
        lp = ell + log_prior(theta) + float(q.sum())
        g_theta = grad + log_prior_grad(theta)
        gq = theta[list(FREE)] * g_theta[list(FREE)] + 1.0
        return lp, gq

    def run(self, iterations: int):
        """Generator: yields a Theta to evaluate and receives (ell, grad) for it."""
        ell, grad = yield self.theta.copy()
        self.evals += 1
        lp, gq = self._logp_grad(self.theta, ell, grad)
        for it in range(iterations):
            q0 = self._q(self.theta)
            p0 = self.rng.standard_normal(q0.size)
            q, p, g = q0.copy(), p0.copy(), gq.copy()
            lp_new, ok = lp, True
            theta_new = self.theta
            for _ in range(self.leapfrog):
                p = p + 0.5 * self.eps * g
                q = q + self.eps * p
                theta_new = self._theta(q)
                free = theta_new[list(FREE)]
                if not np.all(np.isfinite(free)) or np.any(free > 1e12) or np.any(free < 1e-12):
                    ok = False  # left the region the likelihood accepts: a divergent trajectory
                    break
                ell_n, grad_n = yield theta_new
                self.evals += 1
                lp_new, g = self._logp_grad(theta_new, ell_n, grad_n)
                if not (math.isfinite(lp_new) and np.all(np.isfinite(g))):
                    ok = False
                    break
                p = p + 0.5 * self.eps * g
            alpha = 0.0
            if ok:
                log_alpha = (lp_new - 0.5 * p @ p) - (lp - 0.5 * p0 @ p0)
                if math.isfinite(log_alpha):
                    alpha = 1.0 if log_alpha >= 0 else math.exp(log_alpha)
            if self.rng.uniform() < alpha:
                self.theta, lp, gq = theta_new, lp_new, g
                self.accepted += 1
            self.iters += 1
            if it < self.warmup:
                m = it + 1
                t0, gamma, kappa = 10.0, 0.05, 0.75
                self._hbar = (1 - 1 / (m + t0)) * self._hbar + (self.target_accept - alpha) / (m + t0)
                log_eps = self._mu - math.sqrt(m) / gamma * self._hbar
                w = m ** (-kappa)
                self._log_eps_bar = w * log_eps + (1 - w) * self._log_eps_bar
                self.eps = math.exp(log_eps)
                if it == self.warmup - 1:
                    self.eps = math.exp(self._log_eps_bar)
            else:
                self.samples.append(self.theta.copy())


def run_hmc_local(loglik_grad, theta0, iterations: int, seed: int, **kw) -> HMCChain:
    """One HMC chain with a synchronous (ell, grad) callable."""
    ch = HMCChain(np.array(theta0, float), np.random.default_rng(seed), **kw)
    gen = ch.run(iterations)
    th = next(gen)
    try:
        while True:
            th = gen.send(loglik_grad(th))
    except StopIteration:
        pass
    return ch


def run_hmc_served(ctx, chains: list, datasets: list, iterations: int, precision="fp32c", poll_us=200,
                   on_result=None):
    """Advance HMC chains through the serving API (one gradient request in flight per chain);
    ``on_result(k, result)``, if given, sees every polled result of chain k."""
    from . import binding

    gens = [ch.run(iterations) for ch in chains]
    ctx.submit([binding.request(datasets[k], next(g), precision, want_grad=True, tag=k) for k, g in enumerate(gens)])
    live = len(chains)
    served = 0
    while live:
        for r in ctx.poll(cap=512, timeout_us=poll_us):
            served += 1
            if r.status != 0:
                raise RuntimeError(f"request {r.tag} failed with status {r.status}")
            k = int(r.tag)
            if on_result is not None:
                on_result(k, r)
            try:
                th = gens[k].send((r.loglik, np.array(r.grad[:])))
            except StopIteration:
                live -= 1
                continue
            ctx.submit([binding.request(datasets[k], th, precision, want_grad=True, tag=k)])
    return served
