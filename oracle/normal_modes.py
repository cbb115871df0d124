"""Scaled normal modes of the free ring polymer (Sec. "Ring-Polymer Molecular Dynamics").

* The free ring-polymer matrix is (P / (hbar beta))^2 times the cyclic second-difference
  matrix (2 on the diagonal, -1 on the two cyclic off-diagonals), eq. matrix_free_RP.
* omega_n are the square roots of its eigenvalues, in increasing order; the columns of
  the orthogonal transfer matrix T are its eigenvectors; mode 0 is the centroid with
  omega_0 = 0 (text after eq. beads_positions).
* Beads from modes: x_i = Q_0 + sqrt(P) sum_{n>=1} T_in Q_n (eq. beads_positions).
* Forces on modes: f_0 = -(1/P) sum_i grad V(x_i), f_n = -(1/sqrt(P)) sum_i T_in grad V(x_i)
  (eq. force_normal_modes).

Reading where the paper is silent: eigenvalues of the matrix come in equal pairs, so the
eigenvectors are fixed here as the real Fourier basis: column 0 = 1/sqrt(P); for
1 <= k < P/2 the pair (2k-1, 2k) = sqrt(2/P) (cos, sin)(2 pi j k / P); for even P the last
column is (-1)^j / sqrt(P). Any orthonormal eigenbasis is equally valid physically.
"""
import math

import numpy as np


def free_ring_matrix(P, beta, hbar):
    """Omega_P^2 of eq. matrix_free_RP, as a dense P x P matrix."""
    A = 2.0 * np.eye(P)
    for j in range(P):
        A[j, (j + 1) % P] -= 1.0
        A[j, (j - 1) % P] -= 1.0
    if P == 1:
        A[:] = 0.0
    return (P / (hbar * beta)) ** 2 * A


def transfer_matrix(P):
    """T[j, n]: bead j, mode n (real Fourier basis, see module docstring)."""
    T = np.zeros((P, P))
    j = np.arange(P)
    T[:, 0] = 1.0 / math.sqrt(P)
    for k in range(1, (P + 1) // 2):
        T[:, 2 * k - 1] = math.sqrt(2.0 / P) * np.cos(2.0 * math.pi * j * k / P)
        T[:, 2 * k] = math.sqrt(2.0 / P) * np.sin(2.0 * math.pi * j * k / P)
    if P % 2 == 0 and P > 1:
        T[:, P - 1] = (-1.0) ** j / math.sqrt(P)
    return T


def mode_frequencies(P, beta, hbar):
    """omega_n matching the columns of transfer_matrix: 2 (P / (beta hbar)) sin(pi k / P)."""
    w = np.zeros(P)
    wP = P / (beta * hbar)
    for k in range(1, (P + 1) // 2):
        w[2 * k - 1] = w[2 * k] = 2.0 * wP * math.sin(math.pi * k / P)
    if P % 2 == 0 and P > 1:
        w[P - 1] = 2.0 * wP
    return w


def beads_from_modes(Q, T):
    """eq. beads_positions. Q: [P][...] mode amplitudes -> x: [P][...] bead positions."""
    P = T.shape[0]
    x = np.repeat(Q[0:1], P, axis=0).astype(np.float64)
    if P > 1:
        x = x + math.sqrt(P) * np.tensordot(T[:, 1:], Q[1:], axes=(1, 0))
    return x


def modes_from_beads(x, T):
    """Inverse of beads_from_modes (T is orthogonal): Q = T^T x / sqrt(P)."""
    P = T.shape[0]
    return np.tensordot(T.T, x, axes=(1, 0)) / math.sqrt(P)


def forces_on_modes(grad, T):
    """eq. force_normal_modes. grad: [P][...] = grad V at each bead -> f: [P][...]."""
    P = T.shape[0]
    f = np.empty_like(grad)
    f[0] = -grad.sum(axis=0) / P
    if P > 1:
        f[1:] = -np.tensordot(T[:, 1:].T, grad, axes=(1, 0)) / math.sqrt(P)
    return f
