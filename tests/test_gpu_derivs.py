"""Parity of the HIP path's parameter gradients (and Hessian-vector products) with the FP64
oracle's, through the C ABI."""
import sys

import numpy as np
import pytest

import synth
from helpers import has_gpu, medium_box
from oracle import derivs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ctx_for(s, **kw):
    import paper_2212_03137_amd as q
    return q.Context.from_system(s, **kw)


def _small():
    return synth.water_box(27, 2, 10.5, seed=21, cutoff=5.0, ewald_alpha=0.4, pme_grid=16,
                           pme_order=5)


@pytest.mark.parametrize("which", ["small", "medium"])
def test_parameter_gradients_match_the_oracle(which):
    import paper_2212_03137_amd as q
    s = _small() if which == "small" else medium_box(P=4)
    say("param grad", which, s.n_atoms, s.n_beads)
    dq_r, de_r, ds_r = derivs.param_gradients(s.pos, s)
    for prec in (q.FP64, q.FP32_PAIRS):
        with ctx_for(s, precision=prec) as c:
            c.set_state(s.pos, s.vel, 0)
            dq, de, ds = c.param_grad(s.pos)
            x, _, _ = c.get_state()
        assert np.abs(dq - dq_r).max() <= 1e-10 * np.abs(dq_r).max(), prec
        assert np.allclose(de, de_r, rtol=1e-10, atol=1e-10 * np.abs(de_r).max())
        assert np.allclose(ds, ds_r, rtol=1e-10, atol=1e-10 * np.abs(ds_r).max())
        # the propagated state is left alone
        assert np.abs(x - s.pos).max() <= 1e-12 * np.abs(s.pos).max()
