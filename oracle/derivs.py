"""Derivatives of the bead potential beyond the forces: gradients with respect to the
force-field parameters (charges, per-type LJ sigma and epsilon) and Hessian-vector
products in positions. TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The quantity differentiated is the sum of the bead potentials E = sum_b V(x_b) (eq.
PI_potential without the 1/P), with V the water model of ``forces.py``:

* charges: real-space C q_i q_j erfc(alpha r)/r over pairs with bead distance < rc, the
  exclusion correction -C q_a q_b erf(alpha r)/r, the self term -C alpha/sqrt(pi) sum q^2,
  and the SPME reciprocal energy, whose charge derivative is the interpolated potential
  sum_k theta_i(k) phi(k) at the atom (the same phi the forces use);
* LJ: 4 e_ij ((s_ij/r)^12 - (s_ij/r)^6) with s_ij = (sigma_i + sigma_j)/2 and
  e_ij = sqrt(eps_i eps_j); the derivative with respect to eps_t is unbounded where
  eps_t = 0 (the geometric mean), so those entries are reported as 0;
* Hessian-vector products H u = d/dh grad V(x + h u) at h = 0, taken here by its
  definition as the central difference (grad V(x + h u) - grad V(x - h u)) / 2h of the
  analytic gradient, h = 1e-5 A (truncation error O(h^2), far below the test bounds),
  with the set of pairs inside the cutoff frozen at x: the truncated potential has no
  second derivative across the cutoff, and a pair that crosses it between x - hu and
  x + hu would add a jump of order 1/h (the analytic operator has no such term).
"""
import math

import numpy as np
from scipy.special import erf, erfc

from . import forces
from . import spme as _spme


def _charge_grad_bead(x, s, pairs):
    """dV/dq_i for one bead configuration x [N][3] -> [N]."""
    box, q, a, C = s.box, s.charge, s.ewald_alpha, s.coulomb
    dq = np.zeros(len(q))
    # real space, pairs in range
    i, j = pairs[:, 0], pairs[:, 1]
    d = forces.min_image(x[j] - x[i], box)
    r2 = np.einsum("ij,ij->i", d, d)
    m = r2 < s.cutoff * s.cutoff
    i, j, r = i[m], j[m], np.sqrt(r2[m])
    k = C * erfc(a * r) / r
    np.add.at(dq, i, k * q[j])
    np.add.at(dq, j, k * q[i])
    # exclusion correction of the three intramolecular pairs
    for p0, p1 in ((0, 1), (0, 2), (1, 2)):
        dd = forces.min_image(x[p1::3] - x[p0::3], box)
        rr = np.sqrt(np.einsum("ij,ij->i", dd, dd))
        kk = -C * erf(a * rr) / rr
        dq[p0::3] += kk * q[p1::3]
        dq[p1::3] += kk * q[p0::3]
    # self term
    dq += -2.0 * C * a / math.sqrt(math.pi) * q
    # reciprocal: the interpolated potential at each atom
    dq += spme_potential(x, q, box, s.pme_grid, s.pme_order, a, C)
    return dq


def spme_potential(x, q, box, K, n, alpha, coulomb):
    """d E_recip / d q_i = sum_k theta_i(k) phi(k), with phi the potential grid."""
    K = tuple(int(k) for k in K)
    idx, w, _ = _spme._stencil(x, box, K, n)
    N = len(x)
    f = ((idx[:, 0, :, None, None] * K[1] + idx[:, 1, None, :, None]) * K[2]
         + idx[:, 2, None, None, :]).reshape(N, -1)
    W = (w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]).reshape(N, -1)
    Qg = np.bincount(f.ravel(), weights=(q[:, None] * W).ravel(),
                     minlength=K[0] * K[1] * K[2]).reshape(K)
    G = _spme.influence(box, K, n, alpha, coulomb)
    phi = (np.fft.ifftn(G * np.fft.fftn(Qg)).real * (K[0] * K[1] * K[2])).ravel()
    return (W * phi[f]).sum(axis=1)


def _lj_grad_bead(x, s, pairs):
    """dV/deps_t and dV/dsigma_t for one bead -> ([T], [T])."""
    T = len(s.lj_sigma)
    de = np.zeros(T)
    ds = np.zeros(T)
    i, j = pairs[:, 0], pairs[:, 1]
    d = forces.min_image(x[j] - x[i], s.box)
    r2 = np.einsum("ij,ij->i", d, d)
    m = r2 < s.cutoff * s.cutoff
    i, j, r2 = i[m], j[m], r2[m]
    ti, tj = s.types[i], s.types[j]
    sig, eps = np.asarray(s.lj_sigma, float), np.asarray(s.lj_epsilon, float)
    sij = 0.5 * (sig[ti] + sig[tj])
    eij = np.sqrt(eps[ti] * eps[tj])
    sr6 = (sij * sij / r2) ** 3
    dE_de = 4.0 * (sr6 * sr6 - sr6)
    live = eij > 0                       # pairs with an LJ term (sigma_ij > 0 there)
    dE_ds = np.zeros_like(r2)
    dE_ds[live] = 4.0 * eij[live] * (12.0 * sr6[live] ** 2 - 6.0 * sr6[live]) / sij[live]
    for tt, other in ((ti, tj), (tj, ti)):
        ok = (eps[tt] > 0) & (eps[other] > 0)
        # d e_ij / d eps_t = e_ij / (2 eps_t) for the side of type t
        np.add.at(de, tt[ok], dE_de[ok] * eij[ok] / (2.0 * eps[tt[ok]]))
        np.add.at(ds, tt, 0.5 * dE_ds)
    return de, ds


def param_gradients(pos, s, r_list=None):
    """d(sum_b V(x_b)) / d(charges [N], lj_epsilon [T], lj_sigma [T]) for pos [P][N][3]."""
    if r_list is None:
        r_list = s.cutoff + s.skin
    pairs = forces.pair_list(forces.centroids_of(pos), s.box, r_list)
    dq = np.zeros(s.n_atoms)
    de = np.zeros(len(s.lj_sigma))
    ds = np.zeros(len(s.lj_sigma))
    for b in range(pos.shape[0]):
        dq += _charge_grad_bead(pos[b], s, pairs)
        e, g = _lj_grad_bead(pos[b], s, pairs)
        de += e
        ds += g
    return dq, de, ds


def _grad_frozen(x, s, pairs_in):
    """grad V at x with the real-space terms over the given pairs (no cutoff test)."""
    _, _, g_in = forces.intramolecular(x, s.box, s.bond_r0, s.bond_k, s.angle_theta0, s.angle_k)
    _, _, g_rs = forces.real_space(x, pairs_in, s.charge, s.types, s.lj_sigma, s.lj_epsilon,
                                   s.box, s.ewald_alpha, np.inf, s.coulomb)
    _, g_x = forces.excluded_correction(x, s.charge, s.box, s.ewald_alpha, s.coulomb)
    _, g_r = _spme.spme(x, s.charge, s.box, s.pme_grid, s.pme_order, s.ewald_alpha, s.coulomb)
    return g_in + g_rs + g_x + g_r


def hvp(pos, s, u, h=1e-5, r_list=None, beads=None):
    """H u per bead [P][N][3] (only the listed beads if given; the others are zero):
    central difference of the analytic gradient along u, pairs in range frozen at pos."""
    if r_list is None:
        r_list = s.cutoff + s.skin
    pairs = forces.pair_list(forces.centroids_of(pos), s.box, r_list)
    out = np.zeros_like(pos)
    for b in (range(pos.shape[0]) if beads is None else beads):
        d = forces.min_image(pos[b][pairs[:, 1]] - pos[b][pairs[:, 0]], s.box)
        inside = pairs[np.einsum("ij,ij->i", d, d) < s.cutoff * s.cutoff]
        gp = _grad_frozen(pos[b] + h * u[b], s, inside)
        gm = _grad_frozen(pos[b] - h * u[b], s, inside)
        out[b] = (gp - gm) / (2.0 * h)
    return out


def mixed(pos, s, u, h=1e-5, r_list=None):
    """d/dh of the parameter gradients at pos + h u (h = 0): the derivatives of u . grad E
    with respect to the charges [N], lj_epsilon [T] and lj_sigma [T], by the central
    difference of ``param_gradients`` with the in-range pair set frozen at pos."""
    if r_list is None:
        r_list = s.cutoff + s.skin
    pairs = forces.pair_list(forces.centroids_of(pos), s.box, r_list)
    dq = np.zeros(s.n_atoms)
    de = np.zeros(len(s.lj_sigma))
    ds = np.zeros(len(s.lj_sigma))
    for b in range(pos.shape[0]):
        d = forces.min_image(pos[b][pairs[:, 1]] - pos[b][pairs[:, 0]], s.box)
        inside = pairs[np.einsum("ij,ij->i", d, d) < s.cutoff * s.cutoff]
        sp, sm = _frozen_cut(s), _frozen_cut(s)
        qp = _charge_grad_bead(pos[b] + h * u[b], sp, inside)
        qm = _charge_grad_bead(pos[b] - h * u[b], sm, inside)
        ep, gp = _lj_grad_bead(pos[b] + h * u[b], sp, inside)
        em, gm = _lj_grad_bead(pos[b] - h * u[b], sm, inside)
        dq += (qp - qm) / (2.0 * h)
        de += (ep - em) / (2.0 * h)
        ds += (gp - gm) / (2.0 * h)
    return dq, de, ds


def _frozen_cut(s):
    """The system with an infinite cutoff (the caller passes the frozen in-range pairs)."""
    import dataclasses
    return dataclasses.replace(s, cutoff=np.inf)
