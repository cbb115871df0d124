"""The adQTB workload at full size (21,952 waters, P = 1, 128^3 grid, 1,024-step segments)
in the configuration the library uses for it: forces on sampled atoms against the oracle,
the first coloured-noise segment of sampled atoms against the oracle's direct sum, and a
few steps that stay finite."""
import numpy as np
import pytest

import synth
from helpers import has_gpu, oracle_forces_on, rel_max
from oracle import philox as oph
from oracle import qtb as oq

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


@pytest.fixture(scope="module")
def box():
    return synth.adqtb_box()


def test_full_box_forces_noise_and_steps(box):
    import paper_2212_03137_amd as q
    s = box
    print("adqtb box", s.n_atoms, flush=True)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(s.n_atoms, 48, replace=False))
    with q.Context.from_system(s, thermostat=q.ADQTB, precision=q.FP32_PAIRS) as c:
        E, F = c.eval(s.pos)
        Fref, e_rec = oracle_forces_on(s, s.pos[0], sample)
        assert np.sqrt(np.mean((F[0, sample] - Fref) ** 2)) / np.sqrt(np.mean(Fref ** 2)) <= 1e-5
        assert abs(E[0, 6] - e_rec) <= 1e-11 * abs(e_rec)
        c.set_state(s.pos, s.vel, 0)
        noise = c.qtb_noise()
        # oracle: first segment of the sampled atoms by the direct convolution sum
        Q = oq.QTB(s.mass, s.types, s.n_types, s.kT, s.hbar, s.dt, s.qtb_gamma0, s.qtb_nseg,
                   s.qtb_adapt_rate, s.qtb_gamma_min_frac, s.seed, None)
        h = Q.kernels()
        nseg = s.qtb_nseg
        w = oph.qtb_white(s.seed, -nseg, 3 * nseg, s.n_atoms, nseg, atoms=sample)
        ref = np.zeros((nseg, len(sample), 3))
        hs = h[s.types[sample]]
        for jj, j in enumerate(range(-nseg, nseg)):
            ref += hs[None, :, jj, None] * w[nseg - j:2 * nseg - j]
        assert np.abs(noise[:, sample] - ref).max() <= 1e-11 * np.abs(ref).max()
        c.step(8)
        x, v, st = c.get_state()
        assert st == 8 and np.all(np.isfinite(x)) and np.all(np.isfinite(v))


def test_full_box_fp64_forces(box):
    import paper_2212_03137_amd as q
    s = box
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(s.n_atoms, 32, replace=False))
    with q.Context.from_system(s, thermostat=q.ADQTB, precision=q.FP64) as c:
        E, F = c.eval(s.pos)
    Fref, _ = oracle_forces_on(s, s.pos[0], sample)
    scale = np.sqrt(np.mean(Fref ** 2))
    assert np.abs(F[0, sample] - Fref).max() / scale <= 1e-11
