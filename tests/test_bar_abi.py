"""The library's BAR solver (host code behind the C ABI, no device needed) against the
oracle's, and its argument checks."""
import os

import numpy as np
import pytest

from oracle import bar as obar


def _lib():
    import paper_2212_03137_amd as q
    if not os.path.exists(q.LIB_PATH):
        pytest.skip("libqhp.so not built")
    return q


@pytest.mark.parametrize("seed,na,nb,beta", [(0, 400, 400, 1.0), (1, 57, 1300, 1.68),
                                              (2, 2000, 31, 0.4), (3, 1, 1, 2.0)])
def test_bar_matches_the_oracle(seed, na, nb, beta):
    q = _lib()
    rng = np.random.default_rng(seed)
    du_a = rng.normal(1.2, 1.1, na)
    du_b = rng.normal(-0.3, 0.9, nb)
    want, _ = obar.bar(du_a, du_b, beta)
    got, it = q.bar(du_a, du_b, beta)
    assert it >= 1
    assert got == pytest.approx(want, abs=1e-9 * max(1.0, abs(want)))


def test_bar_constant_shift_and_argument_checks():
    q = _lib()
    got, _ = q.bar(np.full(10, 0.75), np.full(3, 0.75), 1.3)
    assert got == pytest.approx(0.75, abs=1e-12)
    with pytest.raises(q.QhpError) as e:
        q.bar(np.zeros(0), np.zeros(3), 1.0)
    assert e.value.code == q.EINVAL
    with pytest.raises(q.QhpError) as e:
        q.bar(np.zeros(2), np.zeros(3), -1.0)
    assert e.value.code == q.EINVAL
    with pytest.raises(q.QhpError) as e:
        q.bar(np.array([0.0, np.nan]), np.zeros(3), 1.0)
    assert e.value.code == q.ENONFINITE
