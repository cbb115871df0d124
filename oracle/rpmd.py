"""Ring-polymer BAOAB in scaled normal modes (Sec. "Integration Scheme").

One step is B(dt/2) A(dt/2) O(dt) A(dt/2) B(dt/2) (the symmetric splitting of the TRPMD
propagator, eq. RPMD_EOM):

* B: P_n += dt/2 f_n with f from eq. force_normal_modes;
* A: exact free ring-polymer evolution: a rotation of (Q_n, P_n) at frequency omega_n for
  n > 0, free flight of the centroid (omega_0 = 0);
* O: exact Ornstein-Uhlenbeck step per mode, P_n <- c1 P_n + sqrt(m kT) c2 xi,
  c1 = exp(-gamma_n dt), c2 = sqrt(1 - c1^2), with the physical mass and temperature for
  every mode (the joint density, eq. distrib_RPMD).

Readings: the friction is gamma_n = max(gamma_0, c omega_n); the paper writes c = 1 and
calls it critical damping, the workloads ask for the optimal value 2 omega_n, so c is a
parameter (2 in every workload). xi is the Philox noise of ``oracle/philox.py`` with
counter (step, atom, mode). The first B of a step uses the forces of the current state,
which are computed once when the state is set.

BCOCB variant (the option named at the end of Sec. "Integration Scheme", after Korol,
Bou-Rabee and Miller): the exact A(h) rotation of each internal mode is replaced by its
Cayley form, the implicit midpoint rule of the free ring-polymer flow,
    Q' - Q = h (P + P') / (2m),   P' - P = -h m omega^2 (Q + Q') / 2,
i.e. with a = omega h / 2: Q' = ((1 - a^2) Q + (h/m) P) / (1 + a^2),
P' = (-m omega^2 h Q + (1 - a^2) P) / (1 + a^2). The centroid still moves freely.
"""
import math

import numpy as np

from . import normal_modes as nm
from . import philox


class RPMD:
    """State (Q, P) in modes, [P][N][3]; ``grad_fn(x) -> (E[P][T], grad[P][N][3])``."""

    def __init__(self, n_beads, mass, kT, hbar, dt, gamma0, trpmd_c, seed, grad_fn,
                 integrator="BAOAB"):
        self.P = n_beads
        self.m = np.asarray(mass, dtype=np.float64)
        self.kT, self.hbar, self.dt = kT, hbar, dt
        self.seed = seed
        self.grad_fn = grad_fn
        beta = 1.0 / kT
        self.T = nm.transfer_matrix(n_beads)
        self.omega = nm.mode_frequencies(n_beads, beta, hbar)
        self.gamma = np.maximum(gamma0, trpmd_c * self.omega)
        self.c1 = np.exp(-self.gamma * dt)
        self.c2 = np.sqrt(1.0 - self.c1 * self.c1)
        if integrator not in ("BAOAB", "BCOCB"):
            raise ValueError(integrator)
        self.cayley = integrator == "BCOCB"
        self.step_index = 0

    # -- state --------------------------------------------------------------------
    def set_state(self, pos, vel, step=0):
        m = self.m[None, :, None]
        self.Q = nm.modes_from_beads(pos, self.T)
        self.Pm = m * nm.modes_from_beads(vel, self.T)
        self.step_index = step
        self._forces()

    def get_state(self):
        x = nm.beads_from_modes(self.Q, self.T)
        v = nm.beads_from_modes(self.Pm, self.T) / self.m[None, :, None]
        return x, v, self.step_index

    def _forces(self):
        x = nm.beads_from_modes(self.Q, self.T)
        self.E, g = self.grad_fn(x)
        self.f = nm.forces_on_modes(g, self.T)

    # -- blocks -------------------------------------------------------------------
    def B(self, h):
        self.Pm = self.Pm + h * self.f

    def A(self, h):
        m = self.m[None, :, None]
        Q, Pm = self.Q.copy(), self.Pm.copy()
        Q[0] = self.Q[0] + h * self.Pm[0] / self.m[:, None]
        for n in range(1, self.P):
            w = self.omega[n]
            if self.cayley:
                a2 = (0.5 * w * h) ** 2
                Q[n] = ((1.0 - a2) * self.Q[n] + h / m[0] * self.Pm[n]) / (1.0 + a2)
                Pm[n] = (-m[0] * w * w * h * self.Q[n] + (1.0 - a2) * self.Pm[n]) / (1.0 + a2)
                continue
            c, s = math.cos(w * h), math.sin(w * h)
            Q[n] = c * self.Q[n] + s / (m[0] * w) * self.Pm[n]
            Pm[n] = -m[0] * w * s * self.Q[n] + c * self.Pm[n]
        self.Q, self.Pm = Q, Pm

    def O(self):
        xi = philox.rpmd_noise(self.seed, self.step_index, self.Q.shape[1], self.P)
        sd = np.sqrt(self.m * self.kT)[None, :, None]
        self.Pm = self.c1[:, None, None] * self.Pm + self.c2[:, None, None] * sd * xi

    def step(self, n=1):
        for _ in range(n):
            h = 0.5 * self.dt
            self.B(h)
            self.A(h)
            self.O()
            self.A(h)
            self._forces()
            self.B(h)
            self.step_index += 1

    # -- observables ----------------------------------------------------------------
    def kinetic(self):
        return float((self.Pm ** 2 / (2.0 * self.m[None, :, None])).sum())

    def spring(self):
        return float((0.5 * self.m[None, :, None] * (self.omega[:, None, None] * self.Q) ** 2).sum())
