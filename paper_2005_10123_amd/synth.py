"""Seeded synthetic event sets shaped like the paper's city-scale workloads.

This module simulates a spatiotemporal Hawkes process by its branching (cluster) representation
and returns event coordinates.  It holds none of the likelihood arithmetic: both the FP64 oracle
(test infrastructure) and the GPU library consume what it produces, so it is the only code the
two sides share.

Model being simulated (the paper's Section 2.1 "Model"): immigrants arrive uniformly in time on
[0, T_end] at locations drawn from a K-component isotropic Gaussian mixture on the square
[0, L]^2 (rejection-sampled into the square); every event independently has Poisson(theta)
children, each delayed by an Exponential(rate omega) time and displaced by N(0, h^2 I).  Children
past T_end are dropped; children are not clipped in space.

The mixture layout (K means uniform on [0.2L, 0.8L]^2, sd 0.1L, equal weights) is a reading: the
paper's data are the Washington D.C. gunfire records, which are not available, and its timing runs
use unspecified "randomly generated observations" (Section 3.1).  Seeds follow
``numpy.random.PCG64(SeedSequence([10123, config, dataset]))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["SimSpec", "simulate", "CONFIGS", "config_events", "subsample", "loguniform_sizes"]


@dataclass(frozen=True)
class SimSpec:
    """Parameters of one synthetic workload (lengths in km, times in days)."""

    n: int
    L: float
    T_end: float
    K: int
    omega: float
    h: float
    theta: float
    seed: tuple = field(default=(10123, 0, 0))


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(int(s) for s in seed))))


def _immigrants(rng, m, means, sd, L, T_end):
    """m background events: mixture locations rejection-sampled into [0, L]^2, uniform times."""
    K = means.shape[0]
    xy = np.empty((m, 2))
    todo = np.arange(m)
    while todo.size:
        comp = rng.integers(0, K, size=todo.size)
        cand = means[comp] + sd * rng.standard_normal((todo.size, 2))
        ok = np.all((cand >= 0.0) & (cand <= L), axis=1)
        xy[todo[ok]] = cand[ok]
        todo = todo[~ok]
    t = rng.uniform(0.0, T_end, size=m)
    return xy[:, 0], xy[:, 1], t


def _cascade(rng, x, y, t, theta, omega, h, T_end):
    """All descendants of the given events, generation by generation."""
    out_x, out_y, out_t = [], [], []
    gx, gy, gt = x, y, t
    while gt.size:
        nchild = rng.poisson(theta, size=gt.size)
        parent = np.repeat(np.arange(gt.size), nchild)
        if parent.size == 0:
            break
        cx = gx[parent] + h * rng.standard_normal(parent.size)
        cy = gy[parent] + h * rng.standard_normal(parent.size)
        ct = gt[parent] + rng.exponential(1.0 / omega, size=parent.size)
        keep = ct <= T_end
        gx, gy, gt = cx[keep], cy[keep], ct[keep]
        out_x.append(gx)
        out_y.append(gy)
        out_t.append(gt)
    if not out_t:
        return np.empty(0), np.empty(0), np.empty(0)
    return np.concatenate(out_x), np.concatenate(out_y), np.concatenate(out_t)


def simulate(spec: SimSpec):
    """Return (x, y, t) float64 arrays of exactly ``spec.n`` events, stably sorted by t."""
    if spec.n < 1:
        raise ValueError("n must be >= 1")
    if not (0.0 <= spec.theta < 1.0):
        raise ValueError("branching ratio theta must be in [0, 1)")
    rng = _rng(spec.seed)
    means = rng.uniform(0.2 * spec.L, 0.8 * spec.L, size=(spec.K, 2))
    sd = 0.1 * spec.L
    xs, ys, ts = [], [], []
    total = 0
    m = math.ceil(spec.n * (1.0 - spec.theta))
    while total < spec.n:
        ix, iy, it = _immigrants(rng, m, means, sd, spec.L, spec.T_end)
        cx, cy, ct = _cascade(rng, ix, iy, it, spec.theta, spec.omega, spec.h, spec.T_end)
        xs += [ix, cx]
        ys += [iy, cy]
        ts += [it, ct]
        total += ix.size + cx.size
        m = math.ceil((spec.n - total) * (1.0 - spec.theta)) + 1
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    t = np.concatenate(ts)
    pick = np.sort(rng.choice(x.size, size=spec.n, replace=False))
    x, y, t = x[pick], y[pick], t[pick]
    order = np.argsort(t, kind="stable")
    return (np.ascontiguousarray(x[order]), np.ascontiguousarray(y[order]),
            np.ascontiguousarray(t[order]))


# Parameter vector order (mu0, tau_x, tau_t, theta, omega, h), as in the paper's Section 2.1.
THETA_CFG1 = (1.0, 0.5, 20.0, 0.3, 0.5, 0.1)

# The benchmark workloads.  Each entry: (generator spec, parameter vector evaluated).
CONFIGS = {
    # N=2,000 on a 10 km square over 1,000 days, 3-component background.
    "small_2k": (SimSpec(2000, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 1, 0)), THETA_CFG1),
    # N=85,000 on a 15 km square over 5,000 days, 5-component background (loglik workload).
    "city_85k_15km": (SimSpec(85000, 15.0, 5000.0, 5, 0.2, 0.05, 0.5, (10123, 2, 0)),
                      (1.0, 0.5, 20.0, 0.5, 0.2, 0.05)),
    # N=85,000 with the small-workload generator (loglik + gradient workload).
    "city_85k_10km": (SimSpec(85000, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 3, 0)), THETA_CFG1),
    # N=1,000,000 on a 40 km square over 20,000 days, 10-component background.
    "stress_1m": (SimSpec(1000000, 40.0, 20000.0, 10, 0.1, 0.08, 0.6, (10123, 5, 0)),
                  (1.0, 0.5, 20.0, 0.6, 0.1, 0.08)),
}


def config_events(name: str, n: int | None = None):
    """Events of a named workload; ``n`` overrides the size (same generator, same seed)."""
    spec, theta = CONFIGS[name]
    if n is not None:
        spec = SimSpec(n, spec.L, spec.T_end, spec.K, spec.omega, spec.h, spec.theta, spec.seed)
    return simulate(spec), theta


def subsample(x, y, t, m: int, seed=(10123, 5, 1)):
    """Seeded uniform subset of m events (kept in time order)."""
    rng = _rng(seed)
    pick = np.sort(rng.choice(x.size, size=m, replace=False))
    return x[pick].copy(), y[pick].copy(), t[pick].copy()


def loguniform_sizes(count: int, lo: float, hi: float, seed=(10123, 4, 999)):
    """Dataset sizes N = round(exp(U[ln lo, ln hi])) for the serving workload."""
    rng = _rng(seed)
    return [int(round(math.exp(v))) for v in rng.uniform(math.log(lo), math.log(hi), size=count)]
