"""Pins for the oracle's counter-based Gaussian generator."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox as ph


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((3, 4), (4, 7, 9, 11)),
                                     ((2212031370, 5), (123456789, 4095, 31, 0)),
                                     ((2**64 - 1, 2**63), (2**64 - 2, 2**64 - 1, 5, 2**40))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox (4x64, 10 rounds) emits the block of counter+1
    ref = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64)).random_raw(4)
    c = list(ctr)
    c0 = (c[0] + 1) % 2**64
    carry = c0 == 0
    c1 = (c[1] + carry) % 2**64
    got = ph.philox4x64_10(([c0], [c1], [c[2]], [c[3]]), key)
    assert [int(g[0]) for g in got] == [int(r) for r in ref]


def test_philox_vectorised_equals_scalar():
    ctr = np.arange(50, dtype=np.uint64)
    v = ph.philox4x64_10((ctr, 3, 2, 1), (9, 8))
    for k in (0, 17, 49):
        s = ph.philox4x64_10(([ctr[k]], [3], [2], [1]), (9, 8))
        assert [int(a[k]) for a in v] == [int(a[0]) for a in s]


def test_uniform_range():
    x = np.array([0, 2**64 - 1, 2**11 - 1, 2**11], dtype=np.uint64)
    u = ph.uniform(x)
    assert u[0] == 0.5 * 2.0**-53 and u[1] == 1.0 - 0.5 * 2.0**-53
    assert u[2] == u[0] and u[3] == 1.5 * 2.0**-53


def test_own_log_accuracy():
    rng = np.random.default_rng(0)
    u = np.concatenate([rng.random(200000), [2.0**-54, 0.5, ph.SQRT_HALF, np.nextafter(ph.SQRT_HALF, 0),
                                             1.0 - 2.0**-53, 0.75, 1e-300]])
    ref = np.array([math.log(v) for v in u])
    err = np.abs(ph.own_log(u) - ref) / np.maximum(np.abs(ref), 1e-300)
    # near u = 1 the value is tiny; compare with an absolute floor there
    assert np.all(np.abs(ph.own_log(u) - ref) <= 4e-16 * np.maximum(np.abs(ref), 1.0))
    assert np.median(err) < 2e-16


def test_own_sincos_accuracy():
    rng = np.random.default_rng(1)
    u = np.concatenate([rng.random(200000), [0.0, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 0.999999]])
    s, c = ph.own_sincos_2pi(u)
    rs = np.array([math.sin(2 * math.pi * v) for v in u])
    rc = np.array([math.cos(2 * math.pi * v) for v in u])
    assert np.max(np.abs(s - rs)) < 2e-15 and np.max(np.abs(c - rc)) < 2e-15
    assert np.max(np.abs(s * s + c * c - 1.0)) < 1e-15


def test_gaussian_distribution():
    g = ph.gaussians4(2212031370, 5, np.arange(250000, dtype=np.uint64), 7, 3).ravel()
    assert abs(g.mean()) < 5 * 1.0 / math.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2.0 / g.size)
    assert abs(stats.kurtosis(g, fisher=False) - 3.0) < 0.03
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # components of one call and neighbouring counters are uncorrelated
    G = ph.gaussians4(1, 6, np.arange(100000, dtype=np.uint64), 0, 0)
    C = np.corrcoef(G.T)
    assert np.max(np.abs(C - np.eye(4))) < 0.02


def test_noise_layout():
    xi = ph.rpmd_noise(11, 5, n_atoms=6, n_beads=4)
    assert xi.shape == (4, 6, 3)
    one = ph.gaussians4(11, ph.STREAM_RPMD_O, np.uint64(5), np.uint64(2), np.uint64(3))
    assert np.array_equal(xi[3, 2], one[:3])
    w = ph.qtb_white(11, -8, 24, 5, 8)
    one = ph.gaussians4(11, ph.STREAM_QTB_WHITE, np.uint64(-8 + 3 + 8), np.uint64(4), np.uint64(0))
    assert np.array_equal(w[3, 4], one[:3])
