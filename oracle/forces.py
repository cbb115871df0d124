"""Per-bead potential V(x) of the flexible 3-site water model and its gradient (with, for
alchemical runs, a solute coupled to the water through scaled charges and soft-core LJ).

The paper leaves V to the force field (Sec. "Massively Parallel Implementation": the
force evaluation is done independently on each bead). The model here is the one the
workloads fix: harmonic O-H bonds and H-O-H angle, Ewald electrostatics (real space with
erfc screening inside the cutoff, reciprocal space by SPME in ``oracle/spme.py``, the
self term and the correction for the three excluded intramolecular pairs) and an O-O
Lennard-Jones term, all pairs truncated at the cutoff with no shift or tail.

Neighbour pairs are found on ring-polymer *centroids*: two atoms are neighbours for every
bead if their centroids are (Sec. "Massively Parallel Implementation"). The list is
defined here by brute force: all intermolecular (i < j) with minimum-image centroid
distance squared strictly below r_list^2, the squared distance evaluated as
dx - L rint(dx * (1/L)) per axis then (dx*dx + dy*dy) + dz*dz, with no fused operations.

Energies are returned per term in the order
[bond, angle, coulomb_real, lennard_jones, coulomb_excluded, coulomb_self, coulomb_recip].
"""
import math

import numpy as np
from scipy.special import erf, erfc

from . import spme as _spme

TERMS = ("bond", "angle", "coul_real", "lj", "coul_excl", "coul_self", "coul_recip")


def min_image(d, box):
    """Minimum-image displacement, axis by axis, round-half-even."""
    return d - box * np.rint(d / box)


def pair_list(centroids, box, r_list, n_per_mol=3):
    """Brute-force centroid pair list: sorted (i, j) with i < j, different molecules.

    Canonical arithmetic (a reading: the paper fixes no rounding): d = c_j - c_i,
    d <- d - L rint(d * (1/L)) per axis with 1/L rounded once, d2 = (dx*dx + dy*dy) + dz*dz,
    kept when d2 < r_list * r_list.
    """
    N = len(centroids)
    mol = np.arange(N) // n_per_mol
    r2max = r_list * r_list
    inv = 1.0 / box
    I_all, J_all = [], []
    chunk = max(1, 4_000_000 // max(N, 1))
    for i0 in range(0, N, chunk):
        i = np.arange(i0, min(N, i0 + chunk))
        d = centroids[None, :, :] - centroids[i, None, :]
        d = d - box * np.rint(d * inv)
        d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]
        d2 = d2 + d[..., 2] * d[..., 2]
        ii, jj = np.nonzero(d2 < r2max)
        ii = i[ii]
        keep = (jj > ii) & (mol[jj] != mol[ii])
        I_all.append(ii[keep]); J_all.append(jj[keep])
    I = np.concatenate(I_all); J = np.concatenate(J_all)
    order = np.lexsort((J, I))
    return np.stack([I[order], J[order]], axis=1).astype(np.int64)


def pair_list_rows(centroids, box, r_list, rows, n_per_mol=3):
    """The pairs of ``pair_list`` that involve any atom of ``rows`` (sorted (i, j), i < j),
    by the same canonical arithmetic (d = c_j - c_i for i < j), for sampled checks of
    large systems."""
    N = len(centroids)
    mol = np.arange(N) // n_per_mol
    r2max = r_list * r_list
    inv = 1.0 / box
    out = set()
    for a in np.unique(np.asarray(rows, dtype=np.int64)):
        j = np.arange(N)
        lo = np.minimum(a, j)
        hi = np.maximum(a, j)
        d = centroids[hi] - centroids[lo]
        d = d - box * np.rint(d * inv)
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
        d2 = d2 + d[:, 2] * d[:, 2]
        keep = (d2 < r2max) & (mol != mol[a]) & (j != a)
        out.update(zip(lo[keep].tolist(), hi[keep].tolist()))
    P = np.array(sorted(out), dtype=np.int64).reshape(-1, 2)
    return P


def centroids_of(pos):
    """Centroid of each atom's beads: beads summed in bead order, then divided by P."""
    c = pos[0].copy()
    for b in range(1, pos.shape[0]):
        c = c + pos[b]
    return c / pos.shape[0]


def real_space(x, pairs, charge, types, sigma, eps, box, alpha, rc, coulomb, soft=None,
               lam_vdw=1.0, sc_alpha=0.5):
    """Ewald real-space Coulomb and LJ over listed pairs whose bead distance < rc.

    ``soft`` (per type, optional) marks the solute types of an alchemical run: a pair with
    exactly one solute atom takes the soft-core form of its LJ term (see ``soft_core``)
    at coupling ``lam_vdw``; every other pair keeps the plain form."""
    i, j = pairs[:, 0], pairs[:, 1]
    d = min_image(x[j] - x[i], box)
    r2 = np.einsum("ij,ij->i", d, d)
    m = r2 < rc * rc
    i, j, d, r2 = i[m], j[m], d[m], r2[m]
    r = np.sqrt(r2)
    qq = coulomb * charge[i] * charge[j]
    e_c = qq * erfc(alpha * r) / r
    # dE/dr for the screened Coulomb pair
    de_c = -qq * (erfc(alpha * r) / r2 + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-alpha * alpha * r2) / r)
    s = 0.5 * (sigma[types[i]] + sigma[types[j]])
    e = np.sqrt(eps[types[i]] * eps[types[j]])
    sr6 = (s * s / r2) ** 3
    e_lj = 4.0 * e * (sr6 * sr6 - sr6)
    de_lj = 4.0 * e * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r
    if soft is not None:
        soft = np.asarray(soft, dtype=bool)
        mixed = (soft[types[i]] != soft[types[j]]) & (e > 0)
        e_lj[mixed], de_lj[mixed] = soft_core(r[mixed], s[mixed], e[mixed], lam_vdw, sc_alpha)
    # gradient wrt x_j is dE/dr * d/r, wrt x_i the opposite
    gj = ((de_c + de_lj) / r)[:, None] * d
    grad = np.zeros_like(x)
    np.add.at(grad, j, gj)
    np.add.at(grad, i, -gj)
    return e_c.sum(), e_lj.sum(), grad


def soft_core(r, s, e, lam, sc_alpha):
    """Soft-core LJ of a solute-environment pair (the free-energy decoupling path of Sec.
    "Hydration free energies", soft-core van der Waals with Beutler's form):
    E = lam 4 e [1/D^2 - 1/D] with D = sc_alpha (1 - lam) + (r/s)^6; at lam = 1 this is
    plain LJ, at lam = 0 it vanishes, and for lam < 1 it stays finite as r -> 0.
    -> (E, dE/dr) per pair."""
    x6 = (r / s) ** 6
    D = sc_alpha * (1.0 - lam) + x6
    E = lam * 4.0 * e * (1.0 / (D * D) - 1.0 / D)
    dE_dD = lam * 4.0 * e * (-2.0 / D ** 3 + 1.0 / (D * D))
    return E, dE_dD * 6.0 * x6 / r


def charges_of(s):
    """Charges entering every electrostatic term: a solute atom's charge is scaled by the
    electrostatic coupling lambda_elec (the solute's charges are scaled down, Sec.
    "Hydration free energies"), so solute-solvent terms scale with lambda_elec and the
    solute's internal ones with its square; no solute -> the charges as given."""
    soft = getattr(s, "type_soft", None)
    if soft is None:
        return s.charge
    return s.charge * np.where(np.asarray(soft, dtype=bool)[s.types], s.lambda_elec, 1.0)


def _lj_soft(s):
    soft = getattr(s, "type_soft", None)
    return dict(soft=soft, lam_vdw=getattr(s, "lambda_vdw", 1.0),
                sc_alpha=getattr(s, "sc_alpha", 0.5))


def intramolecular(x, box, r0, kb, theta0, ktheta):
    """Harmonic O-H bonds and H-O-H angle of every water (atoms 3w, 3w+1, 3w+2 = O, H, H)."""
    O, H1, H2 = x[0::3], x[1::3], x[2::3]
    grad = np.zeros_like(x)
    e_bond = 0.0
    unit = []
    lens = []
    for k, H in ((1, H1), (2, H2)):
        d = min_image(H - O, box)
        r = np.linalg.norm(d, axis=1)
        e_bond += (0.5 * kb * (r - r0) ** 2).sum()
        g = (kb * (r - r0) / r)[:, None] * d       # dE/dx_H
        grad[k::3] += g
        grad[0::3] -= g
        unit.append(d / r[:, None]); lens.append(r)
    u1, u2 = unit
    r1, r2 = lens
    cos = np.clip(np.einsum("ij,ij->i", u1, u2), -1.0, 1.0)
    th = np.arccos(cos)
    e_angle = (0.5 * ktheta * (th - theta0) ** 2).sum()
    dE_dth = ktheta * (th - theta0)
    sin = np.sqrt(1.0 - cos * cos)
    # d theta / d x_H1 = -(u2 - cos u1) / (r1 sin)
    g1 = (-dE_dth / (r1 * sin))[:, None] * (u2 - cos[:, None] * u1)
    g2 = (-dE_dth / (r2 * sin))[:, None] * (u1 - cos[:, None] * u2)
    grad[1::3] += g1
    grad[2::3] += g2
    grad[0::3] -= g1 + g2
    return e_bond, e_angle, grad


def excluded_correction(x, charge, box, alpha, coulomb):
    """Remove the screened-Gaussian interaction of the 3 intramolecular pairs that the
    reciprocal sum includes: -C q_a q_b erf(alpha r) / r per pair."""
    grad = np.zeros_like(x)
    e_tot = 0.0
    for a, b in ((0, 1), (0, 2), (1, 2)):
        d = min_image(x[b::3] - x[a::3], box)
        r2 = np.einsum("ij,ij->i", d, d)
        r = np.sqrt(r2)
        qq = coulomb * charge[a::3] * charge[b::3]
        e_tot += (-qq * erf(alpha * r) / r).sum()
        de = -qq * (2.0 * alpha / math.sqrt(math.pi) * np.exp(-alpha * alpha * r2) / r - erf(alpha * r) / r2)
        g = (de / r)[:, None] * d
        grad[b::3] += g
        grad[a::3] -= g
    return e_tot, grad


def self_energy(charge, alpha, coulomb):
    """Ewald self term -C alpha / sqrt(pi) sum q^2."""
    return -coulomb * alpha / math.sqrt(math.pi) * float(np.sum(charge * charge))


def bead_potential(x, s, pairs):
    """All terms of V at one bead configuration x [N][3] -> (energies[7], grad [N][3])."""
    box = s.box
    q = charges_of(s)
    e_b, e_a, g_in = intramolecular(x, box, s.bond_r0, s.bond_k, s.angle_theta0, s.angle_k)
    e_c, e_lj, g_rs = real_space(x, pairs, q, s.types, s.lj_sigma, s.lj_epsilon,
                                 box, s.ewald_alpha, s.cutoff, s.coulomb, **_lj_soft(s))
    e_x, g_x = excluded_correction(x, q, box, s.ewald_alpha, s.coulomb)
    e_s = self_energy(q, s.ewald_alpha, s.coulomb)
    e_r, g_r = _spme.spme(x, q, box, s.pme_grid, s.pme_order, s.ewald_alpha, s.coulomb)
    E = np.array([e_b, e_a, e_c, e_lj, e_x, e_s, e_r])
    return E, g_in + g_rs + g_x + g_r


def tether(x, anchor, k):
    """Test-only harmonic tether of one bead (not part of the paper's potential; it turns
    free atoms into the harmonic oscillators of the closed-form checks): V = (k/2) sum over
    atoms of |x - a|^2, the plain Cartesian difference. -> (energy, grad [N][3])."""
    d = x - anchor
    return 0.5 * k * float(np.sum(d * d)), k * d


def evaluate(pos, s, r_list=None):
    """Energies [P][7] and forces -grad V [P][N][3] of every bead, pair list built on the
    centroids of ``pos`` with r_list = cutoff + skin (or the given r_list)."""
    if r_list is None:
        r_list = s.cutoff + s.skin
    pairs = pair_list(centroids_of(pos), s.box, r_list)
    P = pos.shape[0]
    E = np.zeros((P, len(TERMS)))
    F = np.zeros_like(pos)
    k = getattr(s, "tether_k", 0.0)
    for b in range(P):
        E[b], g = bead_potential(pos[b], s, pairs)
        if k:
            e_t, g_t = tether(pos[b], s.tether_anchor, k)
            E[b, 0] += e_t
            g = g + g_t
        F[b] = -g
    return E, F


def evaluate_fast(pos, s):
    """The quickly varying part V_f of the potential (Sec. "Multi-timestep Methods", eq.
    splitting_sf): O-H bonds and H-O-H angles of every bead. -> (E [P][7], grad [P][N][3]),
    with the other terms' columns zero."""
    P = pos.shape[0]
    E = np.zeros((P, len(TERMS)))
    G = np.zeros_like(pos)
    for b in range(P):
        e_b, e_a, G[b] = intramolecular(pos[b], s.box, s.bond_r0, s.bond_k, s.angle_theta0,
                                        s.angle_k)
        E[b, 0], E[b, 1] = e_b, e_a
    return E, G


def evaluate_slow(pos, s, r_list=None):
    """The slowly varying part V_s = V - V_f: real-space Coulomb and LJ over the centroid
    list, exclusion correction, self term and reciprocal sum, for every bead of ``pos``
    (the contracted beads under ring-polymer contraction; their centroid is the full
    polymer's). -> (E [P][7] with the bond and angle columns zero, grad [P][N][3])."""
    if r_list is None:
        r_list = s.cutoff + s.skin
    pairs = pair_list(centroids_of(pos), s.box, r_list)
    P = pos.shape[0]
    E = np.zeros((P, len(TERMS)))
    G = np.zeros_like(pos)
    q = charges_of(s)
    for b in range(P):
        x = pos[b]
        e_c, e_lj, g_rs = real_space(x, pairs, q, s.types, s.lj_sigma, s.lj_epsilon,
                                     s.box, s.ewald_alpha, s.cutoff, s.coulomb, **_lj_soft(s))
        e_x, g_x = excluded_correction(x, q, s.box, s.ewald_alpha, s.coulomb)
        e_s = self_energy(q, s.ewald_alpha, s.coulomb)
        e_r, g_r = _spme.spme(x, q, s.box, s.pme_grid, s.pme_order, s.ewald_alpha,
                              s.coulomb)
        E[b] = [0.0, 0.0, e_c, e_lj, e_x, e_s, e_r]
        G[b] = g_rs + g_x + g_r
    return E, G
