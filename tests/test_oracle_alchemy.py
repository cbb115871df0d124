"""Pins for the oracle's alchemical coupling (scaled solute charges, soft-core LJ) and for
its Bennett acceptance ratio estimators."""
import dataclasses
import math

import numpy as np
import pytest

import synth
from oracle import bar, forces, normal_modes


@pytest.fixture(scope="module")
def box():
    # 27 molecules of which 4 form the solute, two beads, small box and cutoff
    s = synth.water_box(27, 2, 10.5, seed=31, cutoff=5.0, ewald_alpha=0.4, pme_grid=16,
                        pme_order=5, solute=4)
    return s


def with_lambda(s, le, lv):
    return dataclasses.replace(s, lambda_elec=le, lambda_vdw=lv)


def test_solute_recipe(box):
    s = box
    sol = s.types >= 2
    assert sol.sum() == 12
    assert abs(s.charge[sol].sum()) < 1e-12 and np.abs(s.charge[sol]).max() <= 0.6
    assert np.all((s.lj_sigma[2:] >= 2.5) & (s.lj_sigma[2:] <= 3.8))
    assert np.all((s.lj_epsilon[2:] >= 0.05) & (s.lj_epsilon[2:] <= 0.2))
    assert list(s.type_soft) == [0, 0, 1, 1, 1, 1, 1, 1]
    # whole molecules
    assert np.all(sol.reshape(-1, 3).all(axis=1) == sol.reshape(-1, 3).any(axis=1))


def test_full_coupling_is_the_plain_potential(box):
    s = with_lambda(box, 1.0, 1.0)
    E1, F1 = forces.evaluate(s.pos, s)
    E0, F0 = forces.evaluate(s.pos, dataclasses.replace(s, type_soft=None))
    # same terms, the soft-core form evaluated at lambda = 1 (rounding differs only)
    assert np.allclose(E1, E0, rtol=1e-13, atol=1e-11)
    assert np.abs(F1 - F0).max() <= 1e-12 * np.abs(F0).max()


def test_soft_core_well_depth_and_position():
    # E(D) = lam 4 e (1/D^2 - 1/D) is least at D = 2: r* = s (2 - a)^(1/6), E* = -lam e
    s_, e_, alpha = 3.1, 0.15, 0.5
    for lam in (0.25, 0.6, 1.0):
        a = alpha * (1.0 - lam)
        r = np.linspace(0.5, 6.0, 200001)
        E, dE = forces.soft_core(r, s_, e_, lam, alpha)
        k = int(np.argmin(E))
        assert r[k] == pytest.approx(s_ * (2.0 - a) ** (1.0 / 6.0), abs=1e-4)
        assert E[k] == pytest.approx(-lam * e_, rel=1e-8)
        assert abs(dE[k]) < 1e-3
    # finite at contact for lam < 1: the limit lam 4 e (1/a^2 - 1/a)
    lam = 0.5
    a = alpha * (1.0 - lam)
    E0, _ = forces.soft_core(np.array([1e-6]), s_, e_, lam, alpha)
    assert E0[0] == pytest.approx(lam * 4 * e_ * (1 / a ** 2 - 1 / a), rel=1e-9)


def test_decoupled_solute_reduces_to_separate_terms(box):
    # lambda_vdw = 0: LJ = the plain LJ over pairs that are not solute-solvent;
    # lambda_elec = 0: electrostatics = those of the system with the solute's charges zeroed
    s = with_lambda(box, 0.0, 0.0)
    E, _ = forces.evaluate(s.pos, s)
    pairs = forces.pair_list(forces.centroids_of(s.pos), s.box, s.cutoff + s.skin)
    sol = s.types >= 2
    keep = pairs[sol[pairs[:, 0]] == sol[pairs[:, 1]]]
    q0 = np.where(sol, 0.0, s.charge)
    plain = dataclasses.replace(s, type_soft=None, charge=q0)
    Ep, _ = forces.evaluate(s.pos, plain)
    for b in range(s.n_beads):
        _, e_lj, _ = forces.real_space(s.pos[b], keep, s.charge, s.types, s.lj_sigma,
                                       s.lj_epsilon, s.box, s.ewald_alpha, s.cutoff, s.coulomb)
        assert E[b, 3] == pytest.approx(e_lj, rel=1e-13)
    coul = [2, 4, 5, 6]
    assert np.allclose(E[:, coul], Ep[:, coul], rtol=1e-13, atol=1e-12)
    # the solute's internal terms keep their full strength: bonded terms unchanged
    assert np.allclose(E[:, :2], Ep[:, :2], rtol=1e-14)


def test_forces_are_minus_the_energy_gradient_at_partial_coupling(box):
    s = with_lambda(box, 0.3, 0.45)
    E, F = forces.evaluate(s.pos, s)
    h = 1e-5
    sol_atoms = np.nonzero(s.types >= 2)[0]
    for a in (int(sol_atoms[0]), int(sol_atoms[4]), 0, 13):
        for d in range(3):
            p, m = s.pos.copy(), s.pos.copy()
            p[1, a, d] += h
            m[1, a, d] -= h
            # same pair list as at s.pos (the displacement is far inside the skin)
            fd = -(forces.evaluate(p, s, r_list=s.cutoff + s.skin)[0][1].sum()
                   - forces.evaluate(m, s, r_list=s.cutoff + s.skin)[0][1].sum()) / (2 * h)
            assert fd == pytest.approx(F[1, a, d], rel=1e-6, abs=1e-6)


def test_coupling_is_monotone_in_the_soft_core_energy_at_overlap():
    # at a near-overlap distance the soft-core energy grows with lambda
    r = np.array([1.0])
    vals = [forces.soft_core(r, 3.0, 0.1, lam, 0.5)[0][0] for lam in (0.1, 0.3, 0.5, 0.7, 0.9)]
    assert all(b > a for a, b in zip(vals, vals[1:]))


# ---- BAR -------------------------------------------------------------------------------
def test_bar_of_a_constant_shift_is_the_shift():
    # U_B = U_A + c on every sample: Delta F_AB = c exactly, for any sample sizes
    rng = np.random.default_rng(1)
    for c in (-3.0, 0.0, 0.7):
        du_a = np.full(37, c)
        du_b = np.full(91, c)
        dF, _ = bar.bar(du_a + 0 * rng.standard_normal(37), du_b, beta=1.7)
        assert dF == pytest.approx(c, abs=1e-10)


def test_bar_is_antisymmetric_in_the_states():
    rng = np.random.default_rng(2)
    du_a = rng.normal(1.0, 0.8, 500)
    du_b = rng.normal(0.4, 0.7, 300)
    f_ab, _ = bar.bar(du_a, du_b, beta=1.3)
    f_ba, _ = bar.bar(-du_b, -du_a, beta=1.3)
    assert f_ab == pytest.approx(-f_ba, abs=1e-10)


def test_bar_recovers_the_classical_harmonic_free_energy():
    # V = k x^2 / 2 in 3 dimensions: Delta F_AB = (3 / 2 beta) ln(k_B / k_A)
    rng = np.random.default_rng(3)
    beta, kA, kB, n = 1.6, 1.0, 1.5, 200000
    xa = rng.standard_normal((n, 3)) / math.sqrt(beta * kA)
    xb = rng.standard_normal((n, 3)) / math.sqrt(beta * kB)
    du_a = 0.5 * (kB - kA) * (xa ** 2).sum(axis=1)
    du_b = 0.5 * (kB - kA) * (xb ** 2).sum(axis=1)
    dF, _ = bar.bar(du_a, du_b, beta)
    assert dF == pytest.approx(1.5 / beta * math.log(kB / kA), abs=3e-3)


@pytest.mark.parametrize("P", [4, 16])
def test_pi_bar_recovers_the_ring_polymer_free_energy(P):
    # harmonic oscillator, P beads sampled exactly in normal modes: U_P = m w^2/2 sum Q_n^2,
    # Q_n ~ N(0, 1/(beta m (w^2 + w_n^2))); Delta F_AB = (1/2 beta) sum_n ln((wB^2 + w_n^2) /
    # (wA^2 + w_n^2)) with w_n the free ring polymer's frequencies
    rng = np.random.default_rng(4 + P)
    beta, hbar, m, n = 1.0, 1.0, 1.0, 100000
    wA, wB = 3.0, 3.6
    wn = normal_modes.mode_frequencies(P, beta, hbar)
    T = normal_modes.transfer_matrix(P)

    def sample(w):
        Q = rng.standard_normal((n, P)) / np.sqrt(beta * m * (w * w + wn * wn))[None, :]
        return Q @ (math.sqrt(P) * T.T)          # x_j = sqrt(P) sum_n T_jn Q_n (T_j0 = 1/sqrt P)

    def V(x, w):
        return 0.5 * m * w * w * x * x          # per bead

    xa, xb = sample(wA), sample(wB)
    EA_a, EB_a, EA_b, EB_b = V(xa, wA), V(xa, wB), V(xb, wA), V(xb, wB)
    du_a, du_b = bar.window_differences(EA_a, EB_a, EA_b, EB_b, "pi")
    dF, _ = bar.bar(du_a, du_b, beta)
    exact = 0.5 / beta * np.log((wB ** 2 + wn ** 2) / (wA ** 2 + wn ** 2)).sum()
    assert dF == pytest.approx(exact, abs=5e-3)
    # the single-bead estimator agrees to first order in the (small) difference V_B - V_A
    du1_a, du1_b = bar.window_differences(EA_a, EB_a, EA_b, EB_b, "single")
    d1, _ = bar.bar(du1_a, du1_b, beta)
    assert d1 == pytest.approx(exact, abs=0.05 * abs(exact) + 5e-3)


def test_fermi_identity():
    # f(x) = f(-x) exp(-beta x), the property the estimators' derivation rests on
    x = np.linspace(-30.0, 30.0, 601)
    for beta in (0.3, 1.0, 1.7):
        lhs = bar.fermi(x, beta)
        rhs = bar.fermi(-x, beta) * np.exp(-beta * x)
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-300)


def test_estimators_under_cyclic_relabelling_of_the_beads():
    # the bead average is invariant under a cyclic shift of the bead labels, and the
    # single-bead estimator on bead k of shifted samples is the bead-0 estimator of the
    # originals when the shift brings bead k to 0
    rng = np.random.default_rng(9)
    n, P = 400, 8
    EA_a, EB_a = rng.normal(0, 1, (n, P)), rng.normal(0.3, 1, (n, P))
    EA_b, EB_b = rng.normal(0.1, 1, (n, P)), rng.normal(0.2, 1, (n, P))
    roll = lambda E, k: np.roll(E, k, axis=1)
    d_pi, _ = bar.bar(*bar.window_differences(EA_a, EB_a, EA_b, EB_b, "pi"), 1.0)
    d_pi3, _ = bar.bar(*bar.window_differences(roll(EA_a, 3), roll(EB_a, 3), roll(EA_b, 3),
                                               roll(EB_b, 3), "pi"), 1.0)
    assert d_pi == pytest.approx(d_pi3, abs=1e-12)
    d_1, _ = bar.bar(*bar.window_differences(EA_a, EB_a, EA_b, EB_b, "single"), 1.0)
    d_1k, _ = bar.bar(*bar.window_differences(roll(EA_a, 5), roll(EB_a, 5), roll(EA_b, 5),
                                              roll(EB_b, 5), "single"), 1.0)
    d_1ref, _ = bar.bar(EB_a[:, -5] - EA_a[:, -5], EB_b[:, -5] - EA_b[:, -5], 1.0)
    assert d_1k == pytest.approx(d_1ref, abs=1e-12)
    assert d_1 != pytest.approx(d_1k, abs=1e-6)       # a different bead: a different sample
