"""Seeded branching generator: reproducible, exact size, sorted, plausible branching ratio."""
import numpy as np

from paper_2005_10123_amd import synth


def test_reproducible_and_sorted():
    spec = synth.SimSpec(3000, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 1, 0))
    a = synth.simulate(spec)
    b = synth.simulate(spec)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    x, y, t = a
    assert x.size == 3000 and x.dtype == np.float64
    assert np.all(np.diff(t) >= 0)
    assert t.min() >= 0 and t.max() <= 1000.0
    c = synth.simulate(synth.SimSpec(3000, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 1, 1)))
    assert not np.array_equal(c[0], x)


def test_branching_structure():
    # With theta = 0 every event is an immigrant inside the square.
    x, y, t = synth.simulate(synth.SimSpec(5000, 10.0, 100.0, 3, 0.5, 0.1, 0.0, (1, 2, 3)))
    assert x.min() >= 0 and x.max() <= 10 and y.min() >= 0 and y.max() <= 10
    # With theta = 0.5 and a short trigger, many events have a close earlier neighbour.
    x2, y2, t2 = synth.simulate(synth.SimSpec(5000, 10.0, 1000.0, 3, 5.0, 0.01, 0.5, (1, 2, 4)))
    close = 0
    for i in range(1, 2000):
        j = max(0, i - 50)
        d = (np.abs(t2[j:i] - t2[i]) < 2.0) & (np.hypot(x2[j:i] - x2[i], y2[j:i] - y2[i]) < 0.05)
        close += bool(d.any())
    frac = close / 1999
    assert 0.3 < frac < 0.7, frac


def test_named_configs_small():
    (x, y, t), th = synth.config_events("small_2k")
    assert x.size == 2000 and len(th) == 6
    sizes = synth.loguniform_sizes(16, 5e3, 1.2e5)
    assert len(sizes) == 16 and min(sizes) >= 5000 and max(sizes) <= 120000
