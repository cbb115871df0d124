"""Pins for the oracle's ring-polymer BAOAB (Sec. "Integration Scheme")."""
import math

import numpy as np
import pytest

import synth
from oracle import normal_modes as nm
from oracle import philox as ph
from oracle import rpmd

KT = synth.KB * 300.0
HBAR = synth.HBAR
MH = 1.008 * synth.AMU


def harmonic(m, w):
    def gf(x):
        return None, m[None, :, None] * w * w * x
    return gf


def test_single_bead_is_textbook_langevin_baoab():
    # P = 1: the scheme reduces to classical BAOAB (Leimkuhler & Matthews 2013)
    rng = np.random.default_rng(0)
    N = 7
    m = rng.uniform(1.0, 16.0, N) * synth.AMU
    k = rng.uniform(50.0, 200.0, N)

    def grad(x):                                    # anharmonic tether, [N][3]
        return k[:, None] * x + 0.3 * k[:, None] * x ** 3

    x0 = rng.standard_normal((1, N, 3)) * 0.1
    v0 = rng.standard_normal((1, N, 3)) * 0.01
    dt, g0, seed = 0.5, 0.01, 42
    R = rpmd.RPMD(1, m, KT, HBAR, dt, g0, 2.0, seed, lambda x: (None, grad(x[0])[None]))
    R.set_state(x0, v0)
    R.step(25)
    x, v = x0[0].copy(), v0[0].copy()
    c1 = math.exp(-g0 * dt)
    for n in range(25):
        v = v - 0.5 * dt * grad(x) / m[:, None]
        x = x + 0.5 * dt * v
        xi = ph.rpmd_noise(seed, n, N, 1)[0]
        v = c1 * v + math.sqrt(1 - c1 * c1) * np.sqrt(KT / m)[:, None] * xi
        x = x + 0.5 * dt * v
        v = v - 0.5 * dt * grad(x) / m[:, None]
    xr, vr, step = R.get_state()
    assert step == 25
    assert np.allclose(xr[0], x, rtol=1e-12, atol=1e-14)
    assert np.allclose(vr[0], v, rtol=1e-12, atol=1e-14)


def test_harmonic_closed_form_sum():
    # the P-bead closed form tends to the quantum result hbar/(2 m w) coth(beta hbar w / 2)
    w, beta = 0.05, 1.0 / KT
    for P, tol in ((256, 2e-3), (2048, 3e-5)):
        wk = nm.mode_frequencies(P, beta, HBAR)
        x2 = (1.0 / (beta * MH)) * np.sum(1.0 / (w * w + wk * wk))
        q = HBAR / (2 * MH * w) / math.tanh(beta * HBAR * w / 2)
        assert abs(x2 / q - 1) < tol
    assert math.isclose((1.0 / (beta * MH)) / (w * w), 1.0 / (beta * MH * w * w))


@pytest.mark.slow
def test_harmonic_ring_polymer_sampling():
    # <x^2> averaged over beads = (1 / beta m) sum_k 1 / (w^2 + w_k^2); <P_n^2> = m kT
    P, N, w = 8, 400, 0.05
    m = np.full(N, MH)
    R = rpmd.RPMD(P, m, KT, HBAR, 0.5, 0.05, 2.0, 7, harmonic(m, w))
    rng = np.random.default_rng(1)
    R.set_state(rng.standard_normal((P, N, 3)) * 0.05, rng.standard_normal((P, N, 3)) * 0.01)
    R.step(300)
    x2, p2, n = 0.0, np.zeros(P), 0
    for _ in range(2700):
        R.step(1)
        x, _, _ = R.get_state()
        x2 += (x ** 2).mean()
        p2 += (R.Pm ** 2 / MH).mean(axis=(1, 2))
        n += 1
    x2 /= n; p2 /= n
    wk = nm.mode_frequencies(P, 1.0 / KT, HBAR)
    ref = KT / MH * np.sum(1.0 / (w * w + wk * wk))
    assert abs(x2 / ref - 1) < 0.025
    assert np.all(np.abs(p2 / KT - 1) < 0.03)


def test_microcanonical_limit_conserves_energy():
    P, N, w = 8, 20, 0.05
    m = np.full(N, MH)
    R = rpmd.RPMD(P, m, KT, HBAR, 0.5, 0.0, 0.0, 1, harmonic(m, w))
    rng = np.random.default_rng(2)
    R.set_state(rng.standard_normal((P, N, 3)) * 0.1, rng.standard_normal((P, N, 3)) * 0.02)

    def H():
        x, _, _ = R.get_state()
        return R.kinetic() + R.spring() + (0.5 * MH * w * w * x ** 2).sum() / P
    H0 = H()
    hs = []
    for _ in range(40):
        R.step(50)
        hs.append(H())
    hs = np.array(hs)
    assert np.max(np.abs(hs - H0)) / H0 < 2e-3
    assert abs(hs[-10:].mean() - hs[:10].mean()) / H0 < 5e-4


def test_A_block_is_exact_free_ring_polymer():
    # with no external force and no friction, A(t) is the exact harmonic flow of each mode
    P, N = 4, 3
    m = np.full(N, MH)
    R = rpmd.RPMD(P, m, KT, HBAR, 0.5, 0.0, 0.0, 1, lambda x: (None, np.zeros_like(x)))
    rng = np.random.default_rng(4)
    R.set_state(rng.standard_normal((P, N, 3)), rng.standard_normal((P, N, 3)) * 0.01)
    Q0, P0 = R.Q.copy(), R.Pm.copy()
    R.A(3.7)
    for n in range(1, P):
        wn = R.omega[n]
        amp = Q0[n] + 1j * P0[n] / (MH * wn)
        exact = amp * np.exp(-1j * wn * 3.7)
        assert np.allclose(R.Q[n], exact.real, atol=1e-12)
        assert np.allclose(R.Pm[n] / (MH * wn), exact.imag, atol=1e-12)
    assert np.allclose(R.Q[0], Q0[0] + 3.7 * P0[0] / MH)


# ---------------------------------------------------------------- BCOCB (Cayley A step)
def _free_modes(P=8, N=5, seed=4):
    rng = np.random.default_rng(seed)
    m = rng.uniform(1.0, 16.0, N) * synth.AMU
    R = rpmd.RPMD(P, m, KT, HBAR, 0.5, 0.001, 2.0, 1, lambda x: (None, np.zeros_like(x)),
                  integrator="BCOCB")
    R.Q = rng.standard_normal((P, N, 3)) * 0.1
    R.Pm = rng.standard_normal((P, N, 3)) * np.sqrt(m * KT)[None, :, None]
    return R, m


def test_cayley_step_is_the_implicit_midpoint_rule():
    # Q' - Q = h (P + P') / 2m and P' - P = -h m w^2 (Q + Q') / 2 for every internal mode
    R, m = _free_modes()
    h = 0.7
    Q0, P0 = R.Q.copy(), R.Pm.copy()
    R.A(h)
    w = R.omega[:, None, None]
    mm = m[None, :, None]
    lhs_q, rhs_q = R.Q - Q0, h * (P0 + R.Pm) / (2 * mm)
    lhs_p, rhs_p = R.Pm - P0, -h * mm * w * w * (Q0 + R.Q) / 2
    assert np.allclose(lhs_q, rhs_q, rtol=1e-12, atol=1e-15)
    assert np.allclose(lhs_p[1:], rhs_p[1:], rtol=1e-12, atol=1e-15 * np.abs(P0).max())
    assert np.allclose(lhs_p[0], 0.0) and np.allclose(R.Q[0], Q0[0] + h * P0[0] / m[:, None])


def test_cayley_step_conserves_each_mode_energy_even_for_large_steps():
    # the implicit midpoint rule conserves the quadratic invariant of a linear flow exactly,
    # whatever w h is (where the exact rotation would simply be periodic)
    R, m = _free_modes(P=32)
    w = R.omega[:, None, None]
    mm = m[None, :, None]

    def energy():
        return R.Pm ** 2 / (2 * mm) + 0.5 * mm * (w * R.Q) ** 2

    e0 = energy()
    for h in (0.1, 3.0, 50.0):
        R.A(h)
        assert np.allclose(energy()[1:], e0[1:], rtol=1e-12)


def test_bcocb_samples_the_free_ring_polymer_exactly():
    # C preserves the mode energy and O is exact: the internal modes sample kT / (m w^2)
    P, N = 8, 1500
    kT, hbar = 1.0, 1.0
    m = np.ones(N)
    R = rpmd.RPMD(P, m, kT, hbar, 0.4, 1.0, 2.0, 77, lambda x: (None, np.zeros_like(x)),
                  integrator="BCOCB")
    rng = np.random.default_rng(2)
    R.set_state(rng.standard_normal((P, N, 3)) * 0.1, rng.standard_normal((P, N, 3)))
    R.step(200)
    acc = np.zeros(P)
    for _ in range(40):
        R.step(5)
        acc += (R.Q ** 2).mean(axis=(1, 2))
    got = acc / 40 * R.omega ** 2 / kT
    assert np.allclose(got[1:], 1.0, atol=0.04), got
