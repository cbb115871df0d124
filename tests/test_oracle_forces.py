"""Pins for the per-bead potential of the oracle: pair list, real space, intramolecular,
exclusion and self corrections, SPME."""
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import forces as fo
from oracle import spme as sp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kdtree_pairs(c, L, r, n_per_mol=3):
    w = np.mod(c, L)
    w[w >= L] = 0.0
    pr = cKDTree(w, boxsize=L).query_pairs(r, output_type="ndarray")
    pr = np.sort(pr, axis=1)
    pr = pr[pr[:, 0] // n_per_mol != pr[:, 1] // n_per_mol]
    return pr[np.lexsort((pr[:, 1], pr[:, 0]))]


@pytest.mark.parametrize("n_w,L,r", [(64, 12.42, 8.0), (64, 12.42, 5.0), (216, 18.7, 7.5),
                                     (343, 21.8, 11.0)])
def test_pair_list_equals_kdtree(n_w, L, r):
    s = synth.water_box(n_w, 4, L, seed=n_w)
    c = fo.centroids_of(s.pos)
    mine = fo.pair_list(c, s.box, r)
    ref = _kdtree_pairs(c, L, r)
    assert np.array_equal(mine, ref)


@pytest.mark.parametrize("n_w,L,r", [(216, 18.7, 7.5), (343, 21.8, 11.0)])
def test_pair_list_rows_are_the_kdtree_pairs_of_the_rows(n_w, L, r):
    # the sampled variant against the k-d tree's pairs that involve the sampled atoms
    s = synth.water_box(n_w, 4, L, seed=n_w + 1)
    c = fo.centroids_of(s.pos)
    rows = np.random.default_rng(n_w).choice(len(c), 40, replace=False)
    ref = _kdtree_pairs(c, L, r)
    ref = ref[np.isin(ref[:, 0], rows) | np.isin(ref[:, 1], rows)]
    assert np.array_equal(fo.pair_list_rows(c, s.box, r, rows), ref)


def test_tether_is_zero_at_the_anchors_and_its_gradient_is_the_energy_derivative():
    rng = np.random.default_rng(5)
    a = rng.uniform(0, 10, (12, 3))
    e0, g0 = fo.tether(a, a, 3.0)
    assert e0 == 0.0 and np.all(g0 == 0.0)
    x = a + rng.normal(0, 0.3, a.shape)
    e, g = fo.tether(x, a, 3.0)
    h = 1e-6
    for i in (0, 5, 11):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, d] += h; xm[i, d] -= h
            fd = (fo.tether(xp, a, 3.0)[0] - fo.tether(xm, a, 3.0)[0]) / (2 * h)
            assert math.isclose(g[i, d], fd, rel_tol=1e-7, abs_tol=1e-9)


def _fd_check(energy_fn, grad, x, atoms, h=1e-5, rtol=1e-6, atol=1e-7):
    for a in atoms:
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a, d] += h; xm[a, d] -= h
            fd = (energy_fn(xp) - energy_fn(xm)) / (2 * h)
            assert math.isclose(grad[a, d], fd, rel_tol=rtol, abs_tol=atol), (a, d, grad[a, d], fd)


@pytest.fixture(scope="module")
def box64():
    return synth.small_rpmd()


def test_real_space_gradient(box64):
    s = box64
    x = s.pos[3]
    pairs = fo.pair_list(fo.centroids_of(s.pos), s.box, s.cutoff + s.skin)

    def E(xx):
        a, b, _ = fo.real_space(xx, pairs, s.charge, s.types, s.lj_sigma, s.lj_epsilon, s.box,
                                s.ewald_alpha, s.cutoff, s.coulomb)
        return a + b
    _, _, g = fo.real_space(x, pairs, s.charge, s.types, s.lj_sigma, s.lj_epsilon, s.box,
                            s.ewald_alpha, s.cutoff, s.coulomb)
    _fd_check(E, g, x, [0, 1, 2, 50, 191])
    assert np.allclose(g.sum(axis=0), 0.0, atol=1e-10)


def test_intramolecular_gradient_and_closed_form(box64):
    s = box64
    x = s.pos[1]
    E = lambda xx: sum(fo.intramolecular(xx, s.box, s.bond_r0, s.bond_k, s.angle_theta0, s.angle_k)[:2])
    g = fo.intramolecular(x, s.box, s.bond_r0, s.bond_k, s.angle_theta0, s.angle_k)[2]
    _fd_check(E, g, x, [0, 1, 2, 30, 31, 32])
    assert np.allclose(g.sum(axis=0), 0.0, atol=1e-10)
    # one molecule with bond 1 stretched by 0.1 and the angle opened by 0.2 rad
    th = s.angle_theta0 + 0.2
    m = np.array([[5.0, 5.0, 5.0],
                  [5.0 + (s.bond_r0 + 0.1), 5.0, 5.0],
                  [5.0 + s.bond_r0 * math.cos(th), 5.0 + s.bond_r0 * math.sin(th), 5.0]])
    eb, ea, _ = fo.intramolecular(m, np.array([20.0] * 3), s.bond_r0, s.bond_k, s.angle_theta0, s.angle_k)
    assert math.isclose(eb, 0.5 * s.bond_k * 0.01, rel_tol=1e-12)
    assert math.isclose(ea, 0.5 * s.angle_k * 0.04, rel_tol=1e-9)


def test_lennard_jones_minimum():
    # two waters, O atoms at the LJ minimum 2^(1/6) sigma: energy -epsilon, zero O-O force
    s = synth.water_box(8, 1, 40.0, seed=3)
    x = np.zeros((6, 3)) + 10.0
    rmin = 2.0 ** (1.0 / 6.0) * s.lj_sigma[0]
    x[3:, 0] += rmin
    x[1] += [0.0, 1.0, 0.0]; x[2] += [0.0, 0.0, 1.0]
    x[4] += [0.0, 1.0, 0.0]; x[5] += [0.0, 0.0, 1.0]
    pairs = np.array([[0, 3], [0, 4], [0, 5], [1, 3], [1, 4], [1, 5], [2, 3], [2, 4], [2, 5]])
    zero_q = np.zeros(6)
    ec, elj, g = fo.real_space(x, pairs, zero_q, s.types[:6], s.lj_sigma, s.lj_epsilon, np.array([40.0] * 3),
                               0.35, 9.0, s.coulomb)
    assert ec == 0.0
    assert math.isclose(elj, -s.lj_epsilon[0], rel_tol=1e-12)
    assert np.allclose(g, 0.0, atol=1e-12)


def test_exclusion_gradient(box64):
    s = box64
    x = s.pos[2]
    E = lambda xx: fo.excluded_correction(xx, s.charge, s.box, s.ewald_alpha, s.coulomb)[0]
    g = fo.excluded_correction(x, s.charge, s.box, s.ewald_alpha, s.coulomb)[1]
    _fd_check(E, g, x, [0, 1, 2, 99])
    assert np.allclose(g.sum(axis=0), 0.0, atol=1e-10)


def test_isolated_molecule_ewald_self_consistency():
    # One neutral molecule with its intramolecular pairs excluded: the reciprocal sum, the
    # self term and the exclusion correction add up to the energy of the molecule's
    # interaction with its periodic images, which for a cubic lattice under tin-foil
    # boundary conditions is -2 pi mu^2 / (3 V) to leading order (de Leeuw, Perram & Smith
    # 1980).
    s = synth.water_box(1, 1, 40.0, seed=1)
    x = s.pos[0]
    q = s.charge
    for L in (30.0, 60.0):
        box = np.array([L] * 3)
        erec, _ = sp.ewald_recip_direct(x, q, box, 0.35, int(0.6 * L), s.coulomb)
        eself = fo.self_energy(q, 0.35, s.coulomb)
        eexcl, _ = fo.excluded_correction(x, q, box, 0.35, s.coulomb)
        mu = (q[:, None] * x).sum(0)
        image = -2.0 * math.pi / 3.0 / L ** 3 * s.coulomb * (mu @ mu)
        assert abs((erec + eself + eexcl) - image) < 0.02 * abs(image)
        assert abs(eself) > 1000 * abs(image)


def _nacl(ncell, a):
    pts, qs = [], []
    for i in range(2 * ncell):
        for j in range(2 * ncell):
            for k in range(2 * ncell):
                pts.append([i, j, k]); qs.append(1.0 if (i + j + k) % 2 == 0 else -1.0)
    return np.array(pts, dtype=float) * (a / 2.0), np.array(qs)


@pytest.mark.parametrize("use_spme", [False, True])
def test_madelung_constant_nacl(use_spme):
    M_ref = float(open(os.path.join(GOLDEN, "madelung_nacl.txt")).read().split()[-1])
    a = 5.64
    x, q = _nacl(2, a)
    L = 2 * a
    box = np.array([L, L, L])
    alpha, rc, C = 1.0, 5.5, 1.0
    n = len(x)
    pairs = np.array([(i, j) for i in range(n) for j in range(i + 1, n)])
    types = np.zeros(n, dtype=int)
    ereal, _, _ = fo.real_space(x, pairs, q, types, np.zeros(1), np.zeros(1), box, alpha, rc, C)
    if use_spme:
        erec, _ = sp.spme(x, q, box, (48, 48, 48), 8, alpha, C)
    else:
        erec, _ = sp.ewald_recip_direct(x, q, box, alpha, 24, C)
    E = ereal + erec + fo.self_energy(q, alpha, C)
    M = -E * (a / 2.0) / (n / 2.0)
    assert abs(M - M_ref) < (1e-10 if not use_spme else 1e-7)


def test_bspline_partition_of_unity():
    for n in (3, 4, 5, 6, 8):
        f = np.random.default_rng(n).random(50)
        t = np.arange(n)
        w = sp.bspline(n, f[:, None] + t[None, :])
        dw = sp.bspline_deriv(n, f[:, None] + t[None, :])
        assert np.allclose(w.sum(1), 1.0, atol=1e-14)
        assert np.allclose(dw.sum(1), 0.0, atol=1e-14)
        assert np.all(w >= 0)


@pytest.mark.parametrize("K,n,tol", [((16, 16, 16), 4, 5e-3), ((32, 32, 32), 6, 2e-6),
                                     ((40, 36, 32), 8, 1e-6), ((56, 24, 40), 6, 1e-6),
                                     ((24, 24, 24), 4, 5e-4)])
def test_spme_converges_to_classic_ewald(box64, K, n, tol):
    s = box64
    x = s.pos[0]
    e, g = sp.spme(x, s.charge, s.box, K, n, s.ewald_alpha, s.coulomb)
    e2, g2 = sp.ewald_recip_direct(x, s.charge, s.box, s.ewald_alpha, 20, s.coulomb)
    assert abs(e - e2) / abs(e2) < tol
    assert np.abs(g - g2).max() / np.abs(g2).max() < 20 * tol


def test_spme_gradient_is_exact(box64):
    s = box64
    x = s.pos[5]
    E = lambda xx: sp.spme(xx, s.charge, s.box, s.pme_grid, s.pme_order, s.ewald_alpha, s.coulomb)[0]
    g = sp.spme(x, s.charge, s.box, s.pme_grid, s.pme_order, s.ewald_alpha, s.coulomb)[1]
    _fd_check(E, g, x, [0, 1, 2, 77], h=1e-5, rtol=1e-6, atol=1e-7)


def test_spme_odd_order_moduli_finite():
    mod = sp.bspline_moduli(64, 5)
    assert np.all(np.isfinite(mod)) and mod[32] == mod[31]
    # even order has no vanishing denominator
    assert np.all(np.isfinite(sp.bspline_moduli(16, 4)))


def test_total_forces_finite_difference(box64):
    s = box64
    pos = s.pos[:2].copy()
    E0, F = fo.evaluate(pos, s, r_list=s.cutoff + s.skin)
    pairs = fo.pair_list(fo.centroids_of(pos), s.box, s.cutoff + s.skin)

    def Etot(xx):
        return fo.bead_potential(xx, s, pairs)[0].sum()
    _fd_check(Etot, -F[1], pos[1], [0, 4, 100], h=1e-5, rtol=2e-6, atol=2e-6)
