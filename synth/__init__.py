"""Seeded synthetic inputs: water boxes, ring-polymer initial conditions, run settings.

This module only *draws inputs*. It holds no arithmetic of the ring-polymer / adQTB
method itself (no normal-mode transform, no force, no thermostat): both the oracle and
the HIP path receive the arrays and scalars produced here and nothing else.

Units used throughout: Angstrom, fs, e, K, kcal/mol. Masses are handed out already
converted to kcal/mol * fs^2 / Angstrom^2 so that p^2/(2m) is in kcal/mol.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# --- physical constants (CODATA 2018, converted to kcal/mol, Angstrom, fs) -------------
_NA = 6.02214076e23
_KCAL = 4184.0
KB = 1.380649e-23 * _NA / _KCAL                      # kcal/mol/K
HBAR = 1.054571817e-34 * _NA / _KCAL * 1e15          # kcal/mol * fs
AMU = 1.66053906660e-27 * 1e-20 / 1e-30 * _NA / _KCAL  # (amu*A^2/fs^2) in kcal/mol
COULOMB = (1.602176634e-19 ** 2 / (4.0 * math.pi * 8.8541878128e-12)
           * _NA / _KCAL * 1e10)                     # kcal*A/(mol*e^2)

# --- flexible 3-site water (geometry, charges and O-O LJ as given for the workloads;
#     force constants chosen as in SPC/Fw, Wu, Tepper & Voth, JCP 124, 024503, 2006) ---
MASS_O_AMU = 15.999
MASS_H_AMU = 1.008
Q_O = -0.82
Q_H = 0.41
SIGMA_OO = 3.165
EPS_OO = 0.1554
BOND_R0 = 1.012
BOND_K = 1059.162                 # kcal/mol/A^2,   E = k/2 (r - r0)^2
ANGLE_THETA0 = math.radians(113.24)
ANGLE_K = 75.90                   # kcal/mol/rad^2, E = k/2 (theta - theta0)^2

WATER_DENSITY = 0.03337           # molecules / A^3 (used when a box edge is not given)
SEED_BASE = 2212031370


@dataclasses.dataclass
class System:
    """Everything a run needs: topology, parameters and the initial bead state.

    Molecules are 3 consecutive atoms (O, H, H). ``pos``/``vel`` are bead positions and
    bead velocities, shape [P][N][3], FP64.
    """
    n_waters: int
    n_beads: int
    box: np.ndarray            # [3] A
    types: np.ndarray          # [N] int32 (0 = O, 1 = H)
    mass: np.ndarray           # [N] kcal/mol fs^2/A^2
    charge: np.ndarray         # [N] e
    lj_sigma: np.ndarray       # [n_types] A
    lj_epsilon: np.ndarray     # [n_types] kcal/mol
    bond_r0: float
    bond_k: float
    angle_theta0: float
    angle_k: float
    coulomb: float
    ewald_alpha: float
    cutoff: float
    skin: float
    pme_grid: tuple
    pme_order: int
    dt: float                  # fs
    temperature: float         # K
    kT: float                  # kcal/mol
    hbar: float                # kcal/mol fs
    gamma_centroid: float      # 1/fs
    trpmd_c: float             # internal-mode friction = max(gamma_centroid, c * omega_n)
    seed: int
    qtb_gamma0: float = 0.0    # 1/fs (adQTB friction; 0 = not an adQTB run)
    qtb_nseg: int = 1024
    qtb_adapt_rate: float = 1e-3
    qtb_gamma_min_frac: float = 0.01
    pos: np.ndarray = None     # [P][N][3]
    vel: np.ndarray = None     # [P][N][3]
    name: str = ""
    # alchemical runs: per-type solute flags (None: no solute), couplings, soft-core alpha
    type_soft: np.ndarray = None
    lambda_elec: float = 1.0
    lambda_vdw: float = 1.0
    sc_alpha: float = 0.5
    # test-only harmonic tether: spring constant (0 = off) and per-atom anchors [N][3]
    tether_k: float = 0.0
    tether_anchor: np.ndarray = None

    @property
    def n_atoms(self) -> int:
        return 3 * self.n_waters

    @property
    def n_types(self) -> int:
        return len(self.lj_sigma)


def _rotation_matrices(rng, n):
    """Uniform random rotations from normalised 4-Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _min_intermolecular_distance(xyz, box, mol):
    from scipy.spatial import cKDTree
    L = float(box[0])
    wrapped = np.mod(xyz, L)
    wrapped[wrapped >= L] = 0.0
    tree = cKDTree(wrapped, boxsize=L)
    pairs = tree.query_pairs(1.5, output_type="ndarray")
    if len(pairs) == 0:
        return []
    inter = mol[pairs[:, 0]] != mol[pairs[:, 1]]
    return np.unique(np.concatenate([mol[pairs[inter, 0]], mol[pairs[inter, 1]]]))


def water_box(n_waters, n_beads, box_edge=None, seed=0, temperature=300.0, *,
              cutoff=9.0, ewald_alpha=0.35, pme_grid=64, pme_order=5, skin=2.0,
              dt=0.5, gamma_centroid=1e-3, trpmd_c=2.0, qtb_gamma0=0.0,
              qtb_nseg=1024, qtb_adapt_rate=1e-3, bead_spread=True, name="", solute=0):
    """Jittered-lattice water box with random orientations and thermal beads.

    Recipe: molecules on the first ``n_waters`` sites (seeded permutation when the cube is
    not full) of an ``ceil(n^(1/3))``^3 lattice, jitter U(-0.05a, 0.05a), uniform random
    orientation (redrawn when two molecules come closer than 1.5 A); each atom's beads are
    a closed Gaussian random walk with link variance hbar^2/(m kT P) (a free ring polymer);
    bead velocities are Maxwell at P*T, then the total centroid momentum is removed.
    """
    rng = np.random.Generator(np.random.Philox(seed))
    L = float(box_edge) if box_edge is not None else (n_waters / WATER_DENSITY) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    n_side = int(math.ceil(round(n_waters ** (1.0 / 3.0), 9)))
    sites = np.arange(n_side ** 3)
    if n_side ** 3 > n_waters:
        sites = np.sort(rng.permutation(sites)[:n_waters])
    a = L / n_side
    ijk = np.stack([sites % n_side, (sites // n_side) % n_side, sites // (n_side * n_side)], axis=1)
    O = (ijk + 0.5) * a + rng.uniform(-0.05 * a, 0.05 * a, size=(n_waters, 3))

    half = 0.5 * ANGLE_THETA0
    ref = np.array([[0.0, 0.0, 0.0],
                    [BOND_R0 * math.sin(half), 0.0, BOND_R0 * math.cos(half)],
                    [-BOND_R0 * math.sin(half), 0.0, BOND_R0 * math.cos(half)]])
    mol = np.repeat(np.arange(n_waters), 3)
    R = _rotation_matrices(rng, n_waters)
    for _ in range(100):
        xyz = (O[:, None, :] + np.einsum("wij,aj->wai", R, ref)).reshape(-1, 3)
        bad = _min_intermolecular_distance(xyz, box, mol)
        if len(bad) == 0:
            break
        R[bad] = _rotation_matrices(rng, len(bad))
    else:
        raise RuntimeError("could not place molecules without overlap")

    N = 3 * n_waters
    types = np.tile(np.array([0, 1, 1], dtype=np.int32), n_waters)
    mass_amu = np.where(types == 0, MASS_O_AMU, MASS_H_AMU)
    charge = np.where(types == 0, Q_O, Q_H).astype(np.float64)
    lj_sigma, lj_epsilon, type_soft = np.array([SIGMA_OO, 0.0]), np.array([EPS_OO, 0.0]), None
    if solute:
        types, mass_amu, charge, lj_sigma, lj_epsilon, type_soft = _solute(
            rng, xyz, box, solute, types, mass_amu, charge)
    mass = mass_amu * AMU
    kT = KB * temperature
    P = n_beads

    pos = np.repeat(xyz[None], P, axis=0).copy()
    if P > 1 and bead_spread:
        link_sd = np.sqrt(HBAR ** 2 / (mass * kT * P))               # [N]
        steps = rng.standard_normal((P, N, 3)) * link_sd[None, :, None]
        steps -= steps.mean(axis=0, keepdims=True)                   # close the loop
        walk = np.cumsum(steps, axis=0)
        walk -= walk.mean(axis=0, keepdims=True)                     # keep the centroid
        pos += walk
    vel = rng.standard_normal((P, N, 3)) * np.sqrt(P * kT / mass)[None, :, None]
    vcm = (mass[None, :, None] * vel).sum(axis=(0, 1)) / (P * mass.sum())
    vel -= vcm

    return System(n_waters=n_waters, n_beads=P, box=box, types=types, mass=mass,
                  charge=charge, lj_sigma=lj_sigma, type_soft=type_soft,
                  lj_epsilon=lj_epsilon, bond_r0=BOND_R0, bond_k=BOND_K,
                  angle_theta0=ANGLE_THETA0, angle_k=ANGLE_K, coulomb=COULOMB,
                  ewald_alpha=ewald_alpha, cutoff=cutoff, skin=skin,
                  pme_grid=(pme_grid,) * 3 if np.isscalar(pme_grid) else tuple(pme_grid),
                  pme_order=pme_order, dt=dt, temperature=temperature, kT=kT, hbar=HBAR,
                  gamma_centroid=gamma_centroid, trpmd_c=trpmd_c, seed=seed,
                  qtb_gamma0=qtb_gamma0, qtb_nseg=qtb_nseg, qtb_adapt_rate=qtb_adapt_rate,
                  pos=pos, vel=vel, name=name)


# --- alchemical solute ------------------------------------------------------------------
SOLUTE_TYPES = 6                  # types 2..7; type t + 2 is solute type t
SOLUTE_MASS_AMU = (12.011, 14.007, 15.999)   # centre, first and second outer atom


def _solute(rng, xyz, box, n_mol, types, mass_amu, charge):
    """Turn the ``n_mol`` molecules nearest the box centre into the solute: triatomic
    fragments (the water's bonded geometry and force constants) whose 3 n_mol atoms take
    solute types 2.. (molecule k uses types 2 + 3 (k % 2) + {0, 1, 2}); per type a sigma
    U(2.5, 3.8) A and an epsilon U(0.05, 0.2) kcal/mol; per atom a charge U(-0.6, 0.6),
    shifted to a zero total and scaled back into the range if the shift left it."""
    O = xyz[0::3]
    d = O - 0.5 * box
    pick = np.sort(np.argsort(np.einsum("ij,ij->i", d, d), kind="stable")[:n_mol])
    types = types.copy(); mass_amu = mass_amu.astype(np.float64).copy(); charge = charge.copy()
    sig = np.concatenate([[SIGMA_OO, 0.0], rng.uniform(2.5, 3.8, SOLUTE_TYPES)])
    eps = np.concatenate([[EPS_OO, 0.0], rng.uniform(0.05, 0.2, SOLUTE_TYPES)])
    q = rng.uniform(-0.6, 0.6, 3 * n_mol)
    q -= q.mean()
    if np.abs(q).max() > 0.6:
        q *= 0.6 / np.abs(q).max()
    for k, m in enumerate(pick):
        for a in range(3):
            types[3 * m + a] = 2 + 3 * (k % 2) + a
            mass_amu[3 * m + a] = SOLUTE_MASS_AMU[a]
            charge[3 * m + a] = q[3 * k + a]
    soft = np.zeros(2 + SOLUTE_TYPES, dtype=np.int32)
    soft[2:] = 1
    return types, mass_amu, charge, sig, eps, soft


def alchemical_window(i, n_windows=16, n_beads=None, n_waters=None):
    """Instance i of the batched free-energy workload: 16 windows lambda = i / 15 of a
    12-atom solute (4 triatomic fragments) in n_w = [256, 512, 1024, 2048][i % 4] waters
    with P = [8, 16, 32][i % 3]; lambda_elec = max(0, 2 lambda - 1), lambda_vdw =
    min(1, 2 lambda) (lambda = 1 fully coupled), soft-core alpha 0.5. Box edge
    (n_w / 0.03337)^(1/3) (19.7 to 39.4 A) holding the n_w + 4 molecules, rc 7.8 A (so that
    rc + skin stays below half the smallest edge), alpha 0.35 /A, SPME order 5 on a 32^3
    grid (64^3 for 2,048 waters): 0.6 to 1 A spacing."""
    n_w = [256, 512, 1024, 2048][i % 4] if n_waters is None else n_waters
    P = [8, 16, 32][i % 3] if n_beads is None else n_beads
    lam = i / (n_windows - 1)
    L = (n_w / WATER_DENSITY) ** (1.0 / 3.0)
    grid = 32 if n_w <= 1024 else 64
    s = water_box(n_w + 4, P, L, SEED_BASE + 3 + 1000 * i, cutoff=7.8, ewald_alpha=0.35,
                  pme_grid=grid, pme_order=5, solute=4, name=f"alchem{i}_w{n_w}_P{P}")
    s.lambda_elec = max(0.0, 2.0 * lam - 1.0)
    s.lambda_vdw = min(1.0, 2.0 * lam)
    return s


# --- the named workloads ---------------------------------------------------------------
def small_rpmd(seed_offset=0):
    """64 waters, 12.42 A cube, rc 6 A, SPME 16^3 order 4, P = 8, 300 K, dt 0.5 fs."""
    return water_box(64, 8, 12.42, SEED_BASE + 0 + seed_offset, cutoff=6.0, ewald_alpha=0.35,
                     pme_grid=16, pme_order=4, name="water64_P8")


def large_rpmd(seed_offset=0, n_beads=32):
    """4,096 waters, 49.7 A cube, rc 9 A, SPME 64^3 order 5, P = 32, 300 K, dt 0.5 fs."""
    return water_box(4096, n_beads, 49.7, SEED_BASE + 1 + seed_offset, cutoff=9.0,
                     ewald_alpha=0.35, pme_grid=64, pme_order=5, name="water4096_P32")


def adqtb_box(seed_offset=0, n_waters=21952, edge=87.3):
    """21,952 waters, 87.3 A cube, P = 1, gamma0 20 /ps, 1,024-step segments, rate 1e-3.

    The paper and workload leave the cutoff and grid of this box open: rc = 9 A,
    alpha = 0.35 /A, order 5 and a 128^3 grid (0.68 A spacing) are used, dt = 0.5 fs.
    """
    return water_box(n_waters, 1, edge, SEED_BASE + 2 + seed_offset, cutoff=9.0,
                     ewald_alpha=0.35, pme_grid=128, pme_order=5, qtb_gamma0=0.02,
                     qtb_nseg=1024, qtb_adapt_rate=1e-3, name=f"water{n_waters}_adqtb")


def diff_box(config=0):
    """One of the seeded configurations of the differentiation workload: 1,024 waters
    (3,072 atoms), 31.3 A cube, P = 16; rc 9 A, alpha 0.35 /A, SPME 32^3 order 5 (about
    1 A spacing: the workload leaves the grid open)."""
    return water_box(1024, 16, 31.3, SEED_BASE + 4 + 1000 * config, cutoff=9.0,
                     ewald_alpha=0.35, pme_grid=32, pme_order=5, name=f"water1024_P16_c{config}")


def perturbed_parameters(s, seed):
    """The workload's reference parameters: charges scaled by U(-5%, +5%) per atom (then
    shifted to keep the total at zero), LJ sigma and epsilon by U(-3%, +3%) per type."""
    rng = np.random.default_rng([seed, 77])
    q = s.charge * (1.0 + rng.uniform(-0.05, 0.05, s.n_atoms))
    q = q - q.mean()
    sig = s.lj_sigma * (1.0 + rng.uniform(-0.03, 0.03, len(s.lj_sigma)))
    eps = s.lj_epsilon * (1.0 + rng.uniform(-0.03, 0.03, len(s.lj_epsilon)))
    return q, sig, eps
