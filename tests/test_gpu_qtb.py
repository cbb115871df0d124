"""Parity of the adaptive quantum thermal bath on the GPU with the FP64 oracle."""
import numpy as np
import pytest

import synth
from helpers import has_gpu, oracle_grad_fn
from oracle import qtb as oq

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def _system(nseg=64, n_w=27, L=12.0, rate=1e-3):
    return synth.water_box(n_w, 1, L, seed=9, cutoff=5.5, ewald_alpha=0.4, pme_grid=16,
                           pme_order=4, qtb_gamma0=0.02, qtb_nseg=nseg, qtb_adapt_rate=rate,
                           name="qtb_small")


def _ctx(s, **kw):
    import paper_2212_03137_amd as q
    return q.Context.from_system(s, thermostat=q.ADQTB, **kw)


def _oracle(s, classical=False):
    Q = oq.QTB(s.mass, s.types, s.n_types, s.kT, s.hbar, s.dt, s.qtb_gamma0, s.qtb_nseg,
               s.qtb_adapt_rate, s.qtb_gamma_min_frac, s.seed, oracle_grad_fn(s),
               classical_theta=classical)
    Q.set_state(s.pos, s.vel, 0)
    return Q


@pytest.mark.parametrize("nseg", [16, 64, 256, 24, 40, 56, 120, 1000])
def test_first_noise_segment(nseg):
    # powers of two and segment lengths with factors 3, 5 and 7 (mixed-radix transforms)
    s = _system(nseg)
    print("qtb segment", nseg, flush=True)
    Q = _oracle(s)
    with _ctx(s) as c:
        c.set_state(s.pos, s.vel, 0)
        F = c.qtb_noise()
        g = c.qtb_gamma()
    assert np.all(g == s.qtb_gamma0)
    # FFT convolution against the oracle's direct sum
    assert np.abs(F - Q.noise).max() <= 1e-11 * np.abs(Q.noise).max()


def test_classical_limit_trajectory_matches_oracle():
    s = _system(32)
    Q = _oracle(s, classical=True)
    Q.step(96)
    xr, vr, _ = Q.get_state()
    with _ctx(s, qtb_classical=True) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(96)
        x, v, st = c.get_state()
    assert st == 96
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-9
    assert np.abs(v - vr).max() / np.abs(vr).max() < 1e-7


@pytest.mark.parametrize("nseg", [64, 120])
def test_adaptation_over_segments_matches_oracle(nseg):
    s = _system(nseg, rate=5e-3)
    print("qtb adaptation", nseg, flush=True)
    Q = _oracle(s)
    with _ctx(s) as c:
        c.set_state(s.pos, s.vel, 0)
        for seg in range(3):
            Q.step(nseg)
            c.step(nseg)
            g, d = c.qtb_gamma(), c.qtb_delta()
            scale = np.abs(Q.last_delta).max()
            assert np.abs(d - Q.last_delta).max() <= 1e-7 * scale, seg
            assert np.abs(g - Q.gamma).max() <= 1e-9 * np.abs(Q.gamma).max(), seg
            assert np.abs(c.qtb_noise() - Q.noise).max() <= 1e-8 * np.abs(Q.noise).max()
        x, v, _ = c.get_state()
    xr, vr, _ = Q.get_state()
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-8


def test_segment_end_at_the_workload_segment_length():
    """N_seg = 1,024 (the adQTB workload's segments: 2,048-point spectra and 4,096-point
    noise convolutions held in LDS): one full segment of 64 waters, then the segment-end
    spectra, type-averaged Delta_FDT, SIMPLE update and the next segment's noise against
    the oracle."""
    s = _system(1024, n_w=64, L=12.42, rate=5e-3)
    print("qtb segment end at N_seg 1024", flush=True)
    Q = _oracle(s)
    with _ctx(s) as c:
        c.set_state(s.pos, s.vel, 0)
        assert np.abs(c.qtb_noise() - Q.noise).max() <= 1e-11 * np.abs(Q.noise).max()
        Q.step(1024)
        c.step(1024)
        g, d = c.qtb_gamma(), c.qtb_delta()
        F = c.qtb_noise()
        x, v, st = c.get_state()
    assert st == 1024
    scale = np.abs(Q.last_delta).max()
    assert np.abs(d - Q.last_delta).max() <= 1e-7 * scale
    assert np.abs(g - Q.gamma).max() <= 1e-9 * np.abs(Q.gamma).max()
    assert np.any(g != s.qtb_gamma0)
    assert np.abs(F - Q.noise).max() <= 1e-8 * np.abs(Q.noise).max()
    xr, vr, _ = Q.get_state()
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-8


def test_ratio_with_eight_types_at_the_workload_segment_length():
    """RATIO keeps three per-type spectra accumulators next to the transform in LDS; with
    eight types at N_seg = 1,024 they do not fit together and are accumulated by several
    launches. Molecules cycle through four copies of the water's (O, H) type pair."""
    import dataclasses
    import paper_2212_03137_amd as q
    s = _system(1024, n_w=64, L=12.42, rate=5e-3)
    mol = np.arange(s.n_atoms) // 3
    types = (2 * (mol % 4) + (np.arange(s.n_atoms) % 3 != 0)).astype(np.int32)
    s = dataclasses.replace(s, types=types, lj_sigma=np.tile(s.lj_sigma, 4),
                            lj_epsilon=np.tile(s.lj_epsilon, 4))
    assert s.n_types == 8
    print("ratio with 8 types at N_seg 1024", flush=True)
    tau = 800.0
    Q = oq.QTB(s.mass, s.types, s.n_types, s.kT, s.hbar, s.dt, s.qtb_gamma0, s.qtb_nseg,
               s.qtb_adapt_rate, s.qtb_gamma_min_frac, s.seed, oracle_grad_fn(s),
               scheme="RATIO", tau=tau)
    Q.set_state(s.pos, s.vel, 0)
    with _ctx(s, qtb_adapt_scheme=q.QTB_RATIO, qtb_tau=tau) as c:
        c.set_state(s.pos, s.vel, 0)
        Q.step(1024)
        c.step(1024)
        g, d = c.qtb_gamma(), c.qtb_delta()
    assert np.abs(d - Q.last_delta).max() <= 1e-7 * np.abs(Q.last_delta).max()
    assert np.abs(g - Q.gamma).max() <= 1e-7 * np.abs(Q.gamma).max()


def test_gamma_min_clamp_and_set_gamma():
    s = _system(32, rate=1e6)
    with _ctx(s) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(32)
        g = c.qtb_gamma()
        assert np.all(g >= 0.01 * s.qtb_gamma0 - 1e-18)
        assert np.any(g == 0.01 * s.qtb_gamma0)
        g2 = np.full_like(g, 0.03)
        c.qtb_set_gamma(g2)
        assert np.array_equal(c.qtb_gamma(), g2)


def test_state_must_start_on_a_segment_boundary():
    import paper_2212_03137_amd as q
    s = _system(32)
    with _ctx(s) as c:
        with pytest.raises(q.QhpError):
            c.set_state(s.pos, s.vel, 5)


@pytest.mark.parametrize("nseg", [64, 56])
def test_ratio_adaptation_over_segments_matches_oracle(nseg):
    import paper_2212_03137_amd as q
    s = _system(nseg)
    print("qtb ratio", nseg, flush=True)
    tau = 150.0
    Q = oq.QTB(s.mass, s.types, s.n_types, s.kT, s.hbar, s.dt, s.qtb_gamma0, s.qtb_nseg,
               s.qtb_adapt_rate, s.qtb_gamma_min_frac, s.seed, oracle_grad_fn(s),
               scheme="RATIO", tau=tau)
    Q.set_state(s.pos, s.vel, 0)
    with _ctx(s, qtb_adapt_scheme=q.QTB_RATIO, qtb_tau=tau) as c:
        c.set_state(s.pos, s.vel, 0)
        for seg in range(3):
            Q.step(nseg)
            c.step(nseg)
            g = c.qtb_gamma()
            assert np.abs(g - Q.gamma).max() <= 1e-7 * np.abs(Q.gamma).max(), seg
            assert np.abs(c.qtb_noise() - Q.noise).max() <= 1e-6 * np.abs(Q.noise).max()
        x, v, _ = c.get_state()
    xr, vr, _ = Q.get_state()
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-7


def test_per_type_schemes_and_times_match_oracle():
    """SIMPLE for the oxygens and RATIO for the hydrogens, then RATIO for both with a time
    of its own per type (Sec. "Computation of the adQTB Spectra and Adaptation
    Procedure"): gamma and the noise over three segments against the oracle."""
    import paper_2212_03137_amd as q
    s = _system(64, rate=2e-3)
    for schemes, taus in ((["SIMPLE", "RATIO"], [150.0, 150.0]), (["RATIO", "RATIO"], [60.0, 400.0])):
        print("per-type adaptation", schemes, taus, flush=True)
        Q = oq.QTB(s.mass, s.types, s.n_types, s.kT, s.hbar, s.dt, s.qtb_gamma0, s.qtb_nseg,
                   s.qtb_adapt_rate, s.qtb_gamma_min_frac, s.seed, oracle_grad_fn(s),
                   scheme=schemes, tau=taus)
        Q.set_state(s.pos, s.vel, 0)
        code = {"SIMPLE": q.QTB_SIMPLE, "RATIO": q.QTB_RATIO}
        with _ctx(s, qtb_scheme_of=[code[x] for x in schemes], qtb_tau_of=taus) as c:
            c.set_state(s.pos, s.vel, 0)
            for seg in range(3):
                Q.step(64)
                c.step(64)
                g = c.qtb_gamma()
                assert np.abs(g - Q.gamma).max() <= 1e-7 * np.abs(Q.gamma).max(), seg
                assert np.abs(c.qtb_noise() - Q.noise).max() <= 1e-6 * np.abs(Q.noise).max()
            x, v, _ = c.get_state()
        xr, vr, _ = Q.get_state()
        assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-7


def test_a_simple_type_needs_no_time():
    import paper_2212_03137_amd as q
    s = _system(32)
    with _ctx(s, qtb_scheme_of=[q.QTB_SIMPLE, q.QTB_RATIO], qtb_tau_of=[0.0, 50.0]) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(32)
        assert np.all(np.isfinite(c.qtb_gamma()))


def test_ratio_needs_a_positive_tau():
    import paper_2212_03137_amd as q
    s = _system(32)
    with pytest.raises(q.QhpError):
        _ctx(s, qtb_adapt_scheme=q.QTB_RATIO, qtb_tau=0.0)
