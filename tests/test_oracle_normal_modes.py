"""Pins for the normal-mode transform (eqs. matrix_free_RP, beads_positions,
force_normal_modes)."""
import math

import numpy as np
import pytest

from oracle import normal_modes as nm

BETA, HBAR = 1.0 / 0.596, 15.18


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 8, 16, 32, 64])
def test_transfer_matrix_orthogonal(P):
    T = nm.transfer_matrix(P)
    assert np.allclose(T.T @ T, np.eye(P), atol=1e-14)
    assert np.allclose(T[:, 0], 1.0 / math.sqrt(P))


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 8, 16, 32])
def test_eigenpairs_of_free_ring_matrix(P):
    A = nm.free_ring_matrix(P, BETA, HBAR)
    T = nm.transfer_matrix(P)
    w = nm.mode_frequencies(P, BETA, HBAR)
    D = T.T @ A @ T
    scale = max(1.0, np.abs(A).max())
    assert np.allclose(D, np.diag(w ** 2), atol=1e-12 * scale)
    # independently: the library eigen-solver on the matrix definition
    ev = np.sort(np.linalg.eigvalsh(A))
    assert np.allclose(ev, np.sort(w ** 2), atol=1e-12 * scale)
    assert np.all(np.diff(w) >= -1e-12) and w[0] == 0.0


@pytest.mark.parametrize("P", [1, 4, 7, 32])
def test_round_trip_and_centroid(P):
    rng = np.random.default_rng(P)
    x = rng.standard_normal((P, 10, 3))
    T = nm.transfer_matrix(P)
    Q = nm.modes_from_beads(x, T)
    assert np.allclose(nm.beads_from_modes(Q, T), x, atol=1e-13)
    assert np.allclose(Q[0], x.mean(axis=0), atol=1e-14)


@pytest.mark.parametrize("P", [2, 5, 8])
def test_spring_energy_in_modes(P):
    # (1/P) sum_i 1/2 m wP^2 (x_i - x_{i+1})^2 == sum_n 1/2 m w_n^2 Q_n^2
    rng = np.random.default_rng(3)
    m = 2.0
    x = rng.standard_normal((P, 4, 3))
    T = nm.transfer_matrix(P)
    Q = nm.modes_from_beads(x, T)
    wP = P / (BETA * HBAR)
    lhs = sum(0.5 * m * wP ** 2 * ((x[i] - x[(i + 1) % P]) ** 2).sum() for i in range(P)) / P
    rhs = (0.5 * m * nm.mode_frequencies(P, BETA, HBAR)[:, None, None] ** 2 * Q ** 2).sum()
    assert math.isclose(lhs, rhs, rel_tol=1e-12)


@pytest.mark.parametrize("P", [1, 3, 8])
def test_mode_forces_are_gradient_of_bead_average(P):
    # U_P(Q) = (1/P) sum_i V(x_i(Q)) with an anharmonic V; f_n = -dU_P/dQ_n
    rng = np.random.default_rng(5)
    T = nm.transfer_matrix(P)
    Q = rng.standard_normal((P, 3, 3)) * 0.3

    def V(x):
        return (0.7 * x ** 4 - 0.3 * x ** 3 + 0.2 * x ** 2).sum(axis=(-1, -2))

    def gradV(x):
        return 2.8 * x ** 3 - 0.9 * x ** 2 + 0.4 * x

    def U(Q):
        return V(nm.beads_from_modes(Q, T)).sum() / P

    f = nm.forces_on_modes(gradV(nm.beads_from_modes(Q, T)), T)
    h = 1e-6
    for idx in [(0, 0, 0), (P - 1, 2, 1), (P // 2, 1, 2)]:
        Qp, Qm = Q.copy(), Q.copy()
        Qp[idx] += h; Qm[idx] -= h
        fd = -(U(Qp) - U(Qm)) / (2 * h)
        assert math.isclose(f[idx], fd, rel_tol=1e-7, abs_tol=1e-8)
