"""Pins for the oracle's BAOAB-RESPA with ring-polymer contraction (Sec. "Multi-timestep
Methods")."""
import math

import numpy as np
import pytest

import synth
from oracle import forces
from oracle import normal_modes as nm
from oracle import respa
from oracle import rpmd


def bandlimited(P, kmax, rng, n_atoms=5):
    """Beads x_i = a + sum_{k<=kmax} (b_k cos 2 pi k i/P + c_k sin 2 pi k i/P), [P][n][3],
    and the interpolant as a function of tau in [0, 1)."""
    a = rng.standard_normal((n_atoms, 3))
    b = rng.standard_normal((kmax + 1, n_atoms, 3))
    c = rng.standard_normal((kmax + 1, n_atoms, 3))

    def curve(tau):
        out = np.repeat(a[None], len(tau), axis=0)
        for k in range(1, kmax + 1):
            out += np.cos(2 * math.pi * k * tau)[:, None, None] * b[k]
            out += np.sin(2 * math.pi * k * tau)[:, None, None] * c[k]
        return out
    return curve(np.arange(P) / P), curve


@pytest.mark.parametrize("P,Pc", [(16, 1), (16, 2), (16, 3), (16, 4), (16, 5), (16, 8),
                                  (32, 4), (32, 5), (32, 7), (8, 8)])
def test_contraction_samples_the_bandlimited_polymer(P, Pc):
    # a polymer made of harmonics below Pc/2 is reproduced exactly at tau_j = j / Pc
    rng = np.random.default_rng(P * 100 + Pc)
    x, curve = bandlimited(P, (Pc - 1) // 2, rng)
    Q = nm.modes_from_beads(x, nm.transfer_matrix(P))
    xc = respa.contract(Q, Pc)
    assert np.allclose(xc, curve(np.arange(Pc) / Pc), rtol=0, atol=1e-12)


@pytest.mark.parametrize("P,Pc", [(8, 1), (8, 2), (8, 3), (8, 4), (8, 5), (8, 6), (8, 7),
                                  (32, 5), (32, 12), (32, 32)])
def test_every_kept_mode_enters_with_unit_weight(P, Pc):
    # x~_j = Q_0 + sqrt(P~) sum_{1<=n<P~} T~_jn Q_n with T~ orthogonal: a unit amplitude on
    # mode n < P~ gives contracted beads of mean square 1 (so (1/P~) sum_j x~_j^2 equals the
    # sum of the kept modes' squares for any polymer), and modes n >= P~ do not enter
    for n in range(P):
        Q = np.zeros((P, 1, 1))
        Q[n] = 1.0
        xc = respa.contract(Q, Pc)
        assert np.isclose((xc ** 2).mean(), 1.0 if n < Pc else 0.0, rtol=0, atol=1e-14), n
    rng = np.random.default_rng(P + 7 * Pc)
    Q = rng.standard_normal((P, 4, 3))
    xc = respa.contract(Q, Pc)
    assert np.allclose((xc ** 2).mean(axis=0), (Q[:Pc] ** 2).sum(axis=0), rtol=1e-13, atol=0)


def test_even_contraction_keeps_the_full_polymers_cosine_mode_once():
    # P = 8, P~ = 4: the kept modes are the centroid, (cos, sin) of harmonic 1 and the
    # cosine of harmonic 2 of the full polymer; the contracted beads at tau_j = j/4 are
    # Q_0 + sqrt(2) (Q_1 cos(pi j/2) + Q_2 sin(pi j/2)) + (-1)^j Q_3 (transfer matrix of 4
    # beads: columns 1/2, (1/sqrt 2)(cos, sin)(pi j / 2), (-1)^j / 2, times sqrt(4))
    rng = np.random.default_rng(5)
    Q = rng.standard_normal((8, 3, 3))
    j = np.arange(4)[:, None, None]
    expect = (Q[0] + math.sqrt(2.0) * (Q[1] * np.cos(math.pi * j / 2) + Q[2] * np.sin(math.pi * j / 2))
              + (-1.0) ** j * Q[3])
    assert np.allclose(respa.contract(Q, 4), expect, rtol=0, atol=1e-14)


def test_contraction_limits():
    rng = np.random.default_rng(3)
    P = 8
    x = rng.standard_normal((P, 6, 3))
    Q = nm.modes_from_beads(x, nm.transfer_matrix(P))
    assert np.allclose(respa.contract(Q, P), x, atol=1e-13)            # no contraction
    assert np.allclose(respa.contract(Q, 1)[0], x.mean(axis=0), atol=1e-14)  # centroid


@pytest.mark.parametrize("P,Pc", [(8, 1), (8, 2), (8, 3), (8, 4), (8, 5), (8, 8), (16, 4),
                                  (16, 6)])
def test_slow_mode_forces_are_the_gradient(P, Pc):
    # central differences of U_s(Q) = (1/Pc) sum_j V_s(x~_j(Q)) for an anharmonic V_s
    rng = np.random.default_rng(7 + P + Pc)
    n = 3
    A = rng.uniform(0.5, 2.0, (n, 3))

    def vs(xc):
        return (A * xc ** 2 + 0.1 * xc ** 4).sum(axis=(1, 2)) + 0.2 * (xc[:, :, 0] * xc[:, :, 1]).sum(axis=1)

    def grad(xc):
        g = 2 * A * xc + 0.4 * xc ** 3
        g[:, :, 0] += 0.2 * xc[:, :, 1]
        g[:, :, 1] += 0.2 * xc[:, :, 0]
        return g

    def U(Q):
        return vs(respa.contract(Q, Pc)).sum() / Pc

    Q = rng.standard_normal((P, n, 3)) * 0.3
    f = respa.slow_mode_forces(grad(respa.contract(Q, Pc)), P)
    h = 1e-6
    fd = np.zeros_like(Q)
    for idx in np.ndindex(Q.shape):
        Qp, Qm = Q.copy(), Q.copy()
        Qp[idx] += h
        Qm[idx] -= h
        fd[idx] = -(U(Qp) - U(Qm)) / (2 * h)
    assert np.allclose(f, fd, rtol=0, atol=2e-8)
    assert np.all(f[Pc:] == 0.0)


def toy(n=6, seed=11):
    rng = np.random.default_rng(seed)
    m = rng.uniform(1.0, 16.0, n) * synth.AMU
    kf = rng.uniform(100.0, 300.0, n)
    ks = rng.uniform(5.0, 20.0, n)

    def gfast(x):
        return None, kf[None, :, None] * x + 0.2 * kf[None, :, None] * x ** 3

    def gslow(x):
        return None, ks[None, :, None] * x + 0.5 * ks[None, :, None] * x ** 3

    def gsum(x):
        return None, gfast(x)[1] + gslow(x)[1]

    return m, gfast, gslow, gsum, rng


KT = synth.KB * 300.0


def test_no_contraction_single_inner_step_is_baoab():
    P = 8
    m, gfast, gslow, gsum, rng = toy()
    x0 = rng.standard_normal((P, len(m), 3)) * 0.05
    v0 = rng.standard_normal((P, len(m), 3)) * 0.01
    args = (P, m, KT, synth.HBAR, 0.25, 0.002, 2.0, 99)
    R = rpmd.RPMD(*args, gsum)
    S = respa.RPMDRespa(*args, gfast, gslow, n_contract=P, n_alt=1)
    R.set_state(x0, v0)
    S.set_state(x0, v0)
    R.step(30)
    S.step(30)
    xr, vr, nr = R.get_state()
    xs, vs, ns = S.get_state()
    assert nr == ns == 30
    assert np.allclose(xs, xr, rtol=0, atol=1e-12)
    assert np.allclose(vs, vr, rtol=0, atol=1e-12)


def test_zero_slow_force_is_n_alt_plain_steps():
    P, nalt = 4, 3
    m, gfast, _, _, rng = toy(seed=12)

    def zero(x):
        return None, np.zeros_like(x)

    x0 = rng.standard_normal((P, len(m), 3)) * 0.05
    v0 = rng.standard_normal((P, len(m), 3)) * 0.01
    args = (P, m, KT, synth.HBAR, 0.25, 0.002, 2.0, 5)
    R = rpmd.RPMD(*args, gfast)
    S = respa.RPMDRespa(*args, gfast, zero, n_contract=2, n_alt=nalt)
    R.set_state(x0, v0)
    S.set_state(x0, v0)
    R.step(5 * nalt)
    S.step(5)
    xr, vr, nr = R.get_state()
    xs, vs, ns = S.get_state()
    assert nr == ns == 5 * nalt
    assert np.allclose(xs, xr, rtol=0, atol=1e-12)
    assert np.allclose(vs, vr, rtol=0, atol=1e-12)


def test_frictionless_respa_is_time_reversible():
    # with gamma = 0 the outer step is a symmetric composition of exact flows
    P, nalt = 8, 4
    m, gfast, gslow, _, rng = toy(seed=13)
    x0 = rng.standard_normal((P, len(m), 3)) * 0.05
    v0 = rng.standard_normal((P, len(m), 3)) * 0.01
    S = respa.RPMDRespa(P, m, KT, synth.HBAR, 0.25, 0.0, 0.0, 1, gfast, gslow,
                        n_contract=4, n_alt=nalt)
    S.set_state(x0, v0)
    S.step(10)
    x1, v1, _ = S.get_state()
    assert not np.allclose(x1, x0)
    S.set_state(x1, -v1)
    S.step(10)
    x2, v2, _ = S.get_state()
    assert np.allclose(x2, x0, rtol=0, atol=1e-11)
    assert np.allclose(-v2, v0, rtol=0, atol=1e-11)


def test_harmonic_mode_variances_under_contraction():
    # V_f = kf x^2/2 on the P beads and V_s = ks x^2/2 on the P~ contracted beads make every
    # mode an independent oscillator: <Q_n^2> = kT / (kf + ks w_n + m omega_n^2), with
    # w_n = 1 for n < P~ and 0 for n >= P~
    # (hbar large enough that the spring stiffness m omega_n^2 of the kept modes does not
    # swamp ks, so a wrong weight w_n would show)
    P, Pc, nalt, N = 8, 4, 2, 1500
    kT, hbar, m0 = 1.0, 4.0, 1.0
    kf, ks = 1.0, 1.5
    m = np.full(N, m0)

    def gfast(x):
        return None, kf * x

    def gslow(x):
        return None, ks * x

    S = respa.RPMDRespa(P, m, kT, hbar, 0.05, 1.0, 2.0, 2024, gfast, gslow,
                        n_contract=Pc, n_alt=nalt)
    w = nm.mode_frequencies(P, 1.0 / kT, hbar)
    wn = np.zeros(P)
    wn[:Pc] = 1.0
    expect = kT / (kf + ks * wn + m0 * w * w)
    rng = np.random.default_rng(1)
    T = nm.transfer_matrix(P)
    Q0 = rng.standard_normal((P, N, 3)) * np.sqrt(expect)[:, None, None]
    P0 = rng.standard_normal((P, N, 3)) * math.sqrt(m0 * kT)
    S.set_state(nm.beads_from_modes(Q0, T), nm.beads_from_modes(P0, T) / m0)
    S.step(100)
    acc = np.zeros(P)
    n_samp = 0
    for _ in range(60):
        S.step(10)
        acc += (S.Q ** 2).mean(axis=(1, 2))
        n_samp += 1
    got = acc / n_samp
    assert np.allclose(got / expect, 1.0, atol=0.03), got / expect


def test_fast_plus_slow_is_the_full_potential():
    s = synth.small_rpmd()
    Ef, Gf = forces.evaluate_fast(s.pos, s)
    Es, Gs = forces.evaluate_slow(s.pos, s)
    E, F = forces.evaluate(s.pos, s)
    assert np.allclose(Ef + Es, E, rtol=1e-13, atol=1e-9)
    assert np.allclose(-(Gf + Gs), F, rtol=0, atol=1e-9 * np.abs(F).max())
    assert np.all(Ef[:, 2:] == 0) and np.all(Es[:, :2] == 0)
