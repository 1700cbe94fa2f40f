"""The seeded workloads satisfy the gauge conditions Eq. (1) assumes
(transverse temporal gauge Xdot.X' = 0, footnote of Sec. II.A) and the
conformal normalisation Xdot^2 + X'^2 = 1, and have the stated
distributions."""
import math

import numpy as np
from scipy import stats

import synth


def test_constraints_fp64():
    x, xd, xp, ds = synth.segments(20000, 0, np.float64)
    assert np.max(np.abs(np.sum(xd * xp, 1))) < 1e-14
    assert np.max(np.abs(np.sum(xd * xd, 1) + np.sum(xp * xp, 1) - 1.0)) < 1e-14
    assert x.min() >= 0.0 and x.max() < 1.0


def test_constraints_fp32_quantised():
    x, xd, xp, ds = synth.segments(20000, 1, np.float32)
    xd64, xp64 = xd.astype(np.float64), xp.astype(np.float64)
    assert np.max(np.abs(np.sum(xd64 * xp64, 1))) < 2e-7
    assert np.max(np.abs(np.sum(xd64 * xd64, 1) + np.sum(xp64 * xp64, 1) - 1.0)) < 4e-7


def test_distributions():
    x, xd, xp, ds = synth.segments(50000, 2, np.float64)
    v = np.linalg.norm(xd, axis=1)
    assert stats.kstest(v, stats.uniform(loc=0.2, scale=0.6).cdf).pvalue > 1e-3
    assert stats.kstest(ds, stats.uniform(loc=0.001, scale=0.009).cdf).pvalue > 1e-3
    s_hat = xp / np.linalg.norm(xp, axis=1, keepdims=True)
    # isotropy: z component of a uniform unit vector is U(-1, 1)
    assert stats.kstest(s_hat[:, 2], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    for c in range(3):
        assert stats.kstest(x[:, c], stats.uniform.cdf).pvalue > 1e-3


def test_seeds_reproducible():
    a = synth.segments(100, 7, np.float32)
    b = synth.segments(100, 7, np.float32)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_workload_geometry():
    w1 = synth.config1(nseg=10)
    cent = np.array([b.origin + 0.5 for b in w1.boxes])
    assert len(cent) == 24 and np.allclose(np.linalg.norm(cent, axis=1), math.sqrt(5))
    assert len({tuple(c) for c in cent}) == 24
    g2 = synth.config2_geometry()
    near = [np.min(np.linalg.norm(o + np.array([[i, j, k] for i in (0, 1) for j in (0, 1)
                                                 for k in (0, 1)]), axis=1)) for o in g2]
    assert 0.09 < min(near) and max(np.linalg.norm(np.array(g2) + 0.5, axis=1)) < 16
    counts, r, dirs, frac = synth.config3_geometry()
    assert counts.min() >= 1000 and counts.max() <= 2_000_000
    assert 0.001 <= frac.min() and frac.max() <= 0.05
