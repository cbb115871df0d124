"""Adaptive quantum thermal bath on classical beads (Secs. "Adaptive Quantum Thermal Bath",
"adQTB", "Colored Noise Generation", "Computation of the adQTB Spectra and Adaptation").

* Dynamics: Langevin with friction gamma_0 and a coloured random force F (eq_langevin),
  integrated by BAOAB in which only the white noise is replaced.
* Target spectrum: C_FF(omega) = 2 m gamma(omega) Theta(omega, beta) (eq. Cff_qtb),
  Theta = (hbar omega / 2) / tanh(beta hbar omega / 2).
* Noise: segments of N_seg steps, each generated at the start of the segment by
  convolving normalised white noise with the Fourier transform of sqrt(C_FF); the white
  noise of three segments (previous, current, next) enters each segment.
* Spectra at the end of a segment from the DFT of v and F over that segment;
  Delta_FDT = m gamma C_vv - Re C_vF (eq. QTB_spectra), averaged over the degrees of
  freedom of each atom type; SIMPLE update gamma <- gamma - A_gamma Delta; then
  gamma <- max(gamma_min, gamma), gamma_min = 0.01 gamma_0 by default.

Readings where the paper is silent (all stated here and used by both implementations):

* frequency grid omega_k = pi k / (N_seg dt), k = 0 .. N_seg (a 2 N_seg-point DFT);
  Theta(0) = kT (its limit);
* kernel: H_k = sqrt(2 m gamma_k Theta(omega_k) / dt), extended evenly to 2 N_seg points,
  h_j = (1 / 2N_seg) sum_k H_k exp(2 pi i j k / 2N_seg) for j = -N_seg .. N_seg-1;
  noise F_t = sum_j h_j w_{t-j} (so white noise with H constant gives
  F_t = sqrt(2 m gamma_0 kT / dt) w_t);
* O step: p <- c1 p + sqrt((1 - c1^2) dt / (2 gamma_0)) F_t, c1 = exp(-gamma_0 dt), which
  equals the classical O step when F is that white noise;
* the velocity recorded for the spectra is the O-step midpoint (p_before + p_after)/(2m);
* C_XY(omega_k) = (dt / N_seg) X_k conj(Y_k), X_k the DFT of the segment zero-padded to
  2 N_seg points;
* the finite-timestep and finite-friction corrections the paper cites are not applied
  (their form is not given): parity unpinned against the paper for that part;
* RATIO scheme (eq. adapt_ratio with the exponentially decaying running means): the
  running means start from zero, so the first update is the plain ratio of the first
  segment's type-averaged spectra (the common factor 1 - e^{-N_seg dt / tau} cancels);
  where the running C_vv is not positive gamma keeps its value;
* per type z (the same section): each type has its own running-mean time tau_z, and the
  two schemes can be mixed by type (SIMPLE for some types, RATIO for others); a type's
  update uses only its own spectra, scheme and tau_z;
* A_gamma is in 1/fs per kcal/mol and the first update happens at the end of segment 0:
  parity unpinned beyond the HIP path matching this oracle.
"""
import math

import numpy as np

from . import philox


def theta(omega, kT, hbar, classical=False):
    """Mean energy of a quantum harmonic oscillator, Theta(0) = kT; kT if classical."""
    omega = np.asarray(omega, dtype=np.float64)
    if classical:
        return np.full_like(omega, kT)
    out = np.full_like(omega, kT)
    nz = omega > 0
    x = hbar * omega[nz]
    out[nz] = 0.5 * x / np.tanh(0.5 * x / kT)
    return out


def omega_grid(nseg, dt):
    return math.pi * np.arange(nseg + 1) / (nseg * dt)


def kernel(gamma_k, m, kT, hbar, dt, classical=False):
    """h_j for j = -N_seg .. N_seg-1 (index j + N_seg), from gamma on the omega grid."""
    nseg = len(gamma_k) - 1
    om = omega_grid(nseg, dt)
    H = np.sqrt(2.0 * m * gamma_k * theta(om, kT, hbar, classical) / dt)
    Hfull = np.concatenate([H, H[-2:0:-1]])               # even extension to 2 N_seg
    j = np.arange(-nseg, nseg)
    k = np.arange(2 * nseg)
    h = (np.exp(2j * math.pi * np.outer(j, k) / (2 * nseg)) @ Hfull).real / (2 * nseg)
    return h


def colored_segment(h_of_atom, seed, seg, nseg, n_atoms):
    """F_t for t in segment ``seg`` by the direct convolution sum. h_of_atom: [N][2 nseg]."""
    t0 = seg * nseg
    # white noise for global steps t0 - nseg .. t0 + 2 nseg - 1
    w = philox.qtb_white(seed, t0 - nseg, 3 * nseg, n_atoms, nseg)   # [3 nseg][N][3]
    F = np.zeros((nseg, n_atoms, 3))
    for jj, j in enumerate(range(-nseg, nseg)):
        # F_t += h_j w_{t-j}; w index of global step t-j is (t - j) - (t0 - nseg)
        lo = nseg - j
        F += h_of_atom[None, :, jj, None] * w[lo:lo + nseg]
    return F


def spectra(v, F, dt):
    """C_vv and Re C_vF per atom and axis, [N][3][N_seg+1], from v, F: [N_seg][N][3]."""
    nseg = v.shape[0]
    V = np.fft.rfft(v, n=2 * nseg, axis=0)
    Fk = np.fft.rfft(F, n=2 * nseg, axis=0)
    Cvv = dt / nseg * np.abs(V) ** 2
    CvF = dt / nseg * V * np.conj(Fk)
    return np.transpose(Cvv, (1, 2, 0)), np.transpose(CvF.real, (1, 2, 0))


def spectra_delta(v, F, gamma_of_atom, m, dt):
    """Delta_FDT per atom and axis: [N][3][N_seg+1] from v, F: [N_seg][N][3]."""
    Cvv, CvFr = spectra(v, F, dt)
    return m[:, None, None] * gamma_of_atom[:, None, :] * Cvv - CvFr


class QTB:
    """adQTB run on P = 1 beads. ``grad_fn(x[1][N][3]) -> (E, grad[1][N][3])``.

    ``scheme``: "SIMPLE" or "RATIO" for every type, or a sequence of one per type;
    ``tau``: the RATIO running-mean time, one number or one per type (read for the RATIO
    types only)."""

    def __init__(self, mass, types, n_types, kT, hbar, dt, gamma0, nseg, adapt_rate,
                 gamma_min_frac, seed, grad_fn, classical_theta=False, scheme="SIMPLE",
                 tau=None):
        self.m = np.asarray(mass, dtype=np.float64)
        self.types = np.asarray(types)
        self.n_types = n_types
        self.kT, self.hbar, self.dt = kT, hbar, dt
        self.g0, self.nseg, self.A = gamma0, nseg, adapt_rate
        self.gmin = gamma_min_frac * gamma0
        self.seed = seed
        self.grad_fn = grad_fn
        self.classical = classical_theta
        self.c1 = math.exp(-gamma0 * dt)
        self.osd = math.sqrt((1.0 - self.c1 * self.c1) * dt / (2.0 * gamma0))
        self.gamma = np.full((n_types, nseg + 1), gamma0)
        self.type_mass = np.array([self.m[self.types == z][0] for z in range(n_types)])
        schemes = [scheme] * n_types if isinstance(scheme, str) else list(scheme)
        taus = list(tau) if np.ndim(tau) == 1 else [tau] * n_types
        if len(schemes) != n_types or len(taus) != n_types:
            raise ValueError("one scheme and one tau per type")
        if any(sz not in ("SIMPLE", "RATIO") for sz in schemes):
            raise ValueError(scheme)
        self.ratio_of = np.array([sz == "RATIO" for sz in schemes])
        # running-mean factor e^{-N_seg dt / tau_z} of each RATIO type
        self.decay = np.array([math.exp(-nseg * dt / tz) if rz else 0.0
                               for rz, tz in zip(self.ratio_of, taus)])
        self.avg_vv = np.zeros((n_types, nseg + 1))
        self.avg_vf = np.zeros((n_types, nseg + 1))

    def set_state(self, pos, vel, step=0):
        assert step % self.nseg == 0
        self.x = pos[0].copy()
        self.p = self.m[:, None] * vel[0]
        self.step_index = step
        self.vrec = np.zeros((self.nseg, len(self.m), 3))
        self._generate(step // self.nseg)
        self._forces()

    def get_state(self):
        return self.x[None].copy(), (self.p / self.m[:, None])[None].copy(), self.step_index

    def _forces(self):
        self.E, g = self.grad_fn(self.x[None])
        self.f = -g[0]

    def kernels(self):
        return np.stack([kernel(np.maximum(self.gamma[z], self.gmin), self.type_mass[z], self.kT,
                                self.hbar, self.dt, self.classical) for z in range(self.n_types)])

    def _generate(self, seg):
        self.gamma = np.maximum(self.gamma, self.gmin)
        h = self.kernels()
        self.noise = colored_segment(h[self.types], self.seed, seg, self.nseg, len(self.m))

    def _adapt(self):
        d = spectra_delta(self.vrec, self.noise, self.gamma[self.types], self.m, self.dt)
        dbar = np.stack([d[self.types == z].mean(axis=(0, 1)) for z in range(self.n_types)])
        self.last_delta = dbar
        # the dissipation term m gamma C_vv alone, type-averaged (for diagnostics)
        diss = spectra_delta(self.vrec, np.zeros_like(self.noise), self.gamma[self.types], self.m, self.dt)
        self.last_dissipation = np.stack([diss[self.types == z].mean(axis=(0, 1))
                                          for z in range(self.n_types)])
        # SIMPLE: gamma <- gamma - A_gamma Delta_bar
        simple = self.gamma - self.A * dbar
        if not self.ratio_of.any():
            self.gamma = simple
            return
        # RATIO: gamma = Re <C_vF> / (m <C_vv>) over exponentially decaying running means
        Cvv, CvFr = spectra(self.vrec, self.noise, self.dt)
        vv = np.stack([Cvv[self.types == z].mean(axis=(0, 1)) for z in range(self.n_types)])
        vf = np.stack([CvFr[self.types == z].mean(axis=(0, 1)) for z in range(self.n_types)])
        d = self.decay[:, None]
        self.avg_vv = np.where(self.ratio_of[:, None], self.avg_vv * d + vv * (1.0 - d), 0.0)
        self.avg_vf = np.where(self.ratio_of[:, None], self.avg_vf * d + vf * (1.0 - d), 0.0)
        ok = self.avg_vv > 0.0
        ratio = np.where(ok, self.avg_vf / (self.type_mass[:, None] * np.where(ok, self.avg_vv, 1.0)),
                         self.gamma)
        self.gamma = np.where(self.ratio_of[:, None], ratio, simple)

    def step(self, n=1):
        for _ in range(n):
            h = 0.5 * self.dt
            t = self.step_index % self.nseg
            self.p = self.p + h * self.f
            self.x = self.x + h * self.p / self.m[:, None]
            p_before = self.p
            self.p = self.c1 * self.p + self.osd * self.noise[t]
            self.vrec[t] = 0.5 * (p_before + self.p) / self.m[:, None]
            self.x = self.x + h * self.p / self.m[:, None]
            self._forces()
            self.p = self.p + h * self.f
            self.step_index += 1
            if t == self.nseg - 1:
                self._adapt()
                self._generate(self.step_index // self.nseg)
