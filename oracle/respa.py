"""Multiple time stepping with ring-polymer contraction (Sec. "Multi-timestep Methods").

The potential is split as V = V_f + V_s (eq. splitting_sf): a cheap, quickly varying part
V_f and an expensive, slowly varying part V_s.

Ring-polymer contraction (paragraph "Ring-polymer Contractions", unlabelled equation for
U_P): V_f is evaluated on the P beads and V_s on P~ <= P contracted beads built, as in
eq. beads_positions, from the P~ lowest-frequency modes only,

    x~_j = Q_0 + sqrt(P~) sum_{n=1}^{P~-1} T~_jn Q_n,        T~ = transfer matrix of P~,

    U_P(Q) ~ (1/P) sum_i V_f(x_i) + (1/P~) sum_j V_s(x~_j).

The chain rule gives the slow force on mode n < P~ as -(1/sqrt(P~)) sum_j C_jn grad V_s(x~_j)
(C = T~: eq. force_normal_modes with P~ in place of P) and zero on modes n >= P~.

BAOAB-RESPA (paragraph "Path-integral RESPA integrator", the two-stage Trotter splitting):
one outer step of length n_alt dt is

    Bs(n_alt dt/2) [ Bf(dt/2) A(dt/2) O(dt) A(dt/2) Bf(dt/2) ]^n_alt  Bs(n_alt dt/2).

Readings (where the paper leaves the choice open):
* V_f = the O-H bonds and the H-O-H angle; V_s = everything else (real-space Coulomb and
  LJ, the intramolecular exclusion correction of the Ewald sum, the self term, the
  reciprocal sum). The exclusion correction stays with the rest of the electrostatics so
  that all of it is evaluated on the same (contracted) beads.
* The n-th contracted mode is the n-th lowest of the full polymer in the ordering of
  ``normal_modes.transfer_matrix`` (cos before sin within a pair). For even P~ < P the
  last kept mode is therefore the cosine of harmonic P~/2 of the full polymer, which the
  transfer matrix of P~ beads places on its alternating column (-1)^j / sqrt(P~): every
  kept mode enters the contracted beads with unit weight, so that
  (1/P~) sum_j x~_j^2 = sum_{n<P~} Q_n^2 for any polymer.
* The step counter of the O-step noise counts inner steps (time = counter x dt).
* With P~ = P and n_alt = 1 the scheme is the plain BAOAB step of ``oracle/rpmd.py``
  with the kick split in two, which the tests use as one of the pins.
"""
import math

import numpy as np

from . import normal_modes as nm
from .rpmd import RPMD


def contraction_matrix(P_full, P_c):
    """C [P~][P~]: x~_j = sqrt(P~) sum_n C_jn Q_n over the P~ lowest modes; C is the
    transfer matrix of P~ beads (eq. beads_positions with P~ in place of P)."""
    if not 1 <= P_c <= P_full:
        raise ValueError("the contracted polymer needs 1 <= P~ <= P")
    return nm.transfer_matrix(P_c)


def contract(Q, P_c):
    """Contracted beads x~ [P~][...] from the full polymer's modes Q [P][...]."""
    C = contraction_matrix(Q.shape[0], P_c)
    return math.sqrt(P_c) * np.tensordot(C, Q[:P_c], axes=(1, 0))


def slow_mode_forces(grad_c, P_full):
    """Forces on the P full modes from grad V_s at the P~ contracted beads (chain rule
    through ``contract``): -(1/sqrt(P~)) sum_j C_jn grad_j for n < P~, zero for the rest.
    With C = T~ this is eq. force_normal_modes with P~ beads."""
    P_c = grad_c.shape[0]
    C = contraction_matrix(P_full, P_c)
    f = np.zeros((P_full,) + grad_c.shape[1:])
    f[:P_c] = -np.tensordot(C.T, grad_c, axes=(1, 0)) / math.sqrt(P_c)
    return f


class RPMDRespa(RPMD):
    """RPMD with BAOAB-RESPA and ring-polymer contraction.

    ``grad_fast(x [P][N][3]) -> (E [P][T], grad [P][N][3])`` and
    ``grad_slow(x~ [P~][N][3]) -> (E [P~][T], grad [P~][N][3])``.
    ``step(n)`` advances n outer steps (n * n_alt inner steps of length dt).
    """

    def __init__(self, n_beads, mass, kT, hbar, dt, gamma0, trpmd_c, seed, grad_fast,
                 grad_slow, n_contract, n_alt, integrator="BAOAB"):
        if not 1 <= n_contract <= n_beads:
            raise ValueError("n_contract must be in 1..P")
        if n_alt < 1:
            raise ValueError("n_alt must be >= 1")
        super().__init__(n_beads, mass, kT, hbar, dt, gamma0, trpmd_c, seed, grad_fn=None,
                         integrator=integrator)
        self.grad_fast, self.grad_slow = grad_fast, grad_slow
        self.Pc, self.n_alt = n_contract, n_alt

    def _forces(self):
        self._fast_forces()
        self._slow_forces()

    def _fast_forces(self):
        x = nm.beads_from_modes(self.Q, self.T)
        self.E_fast, g = self.grad_fast(x)
        self.f_fast = nm.forces_on_modes(g, self.T)

    def _slow_forces(self):
        xc = contract(self.Q, self.Pc)
        self.E_slow, gc = self.grad_slow(xc)
        self.f_slow = slow_mode_forces(gc, self.P)

    def Bf(self, h):
        self.Pm = self.Pm + h * self.f_fast

    def Bs(self, h):
        self.Pm = self.Pm + h * self.f_slow

    def step(self, n=1):
        h = 0.5 * self.dt
        H = 0.5 * self.n_alt * self.dt
        for _ in range(n):
            self.Bs(H)
            for _ in range(self.n_alt):
                self.Bf(h)
                self.A(h)
                self.O()
                self.A(h)
                self._fast_forces()
                self.Bf(h)
                self.step_index += 1
            self._slow_forces()
            self.Bs(H)

    def potential_estimator(self):
        """U_P of the contraction equation: (1/P) sum V_f + (1/P~) sum V_s."""
        return float(self.E_fast.sum() / self.P + self.E_slow.sum() / self.Pc)
