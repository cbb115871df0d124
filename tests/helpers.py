"""Shared test helpers: building contexts and oracle runs from a synthetic system."""
import numpy as np

import synth


def has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def oracle_grad_fn(s, r_list=None):
    from oracle import forces
    rl = s.cutoff + s.skin if r_list is None else r_list

    def gf(x):
        E, F = forces.evaluate(x, s, r_list=rl)
        return E, -F
    return gf


def rel_max(a, b):
    """max |a - b| / RMS(b)"""
    return float(np.abs(a - b).max() / np.sqrt(np.mean(b * b)))


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b * b)))


def medium_box(P=4, seed=5, n_w=343, L=None, K=32, order=5, rc=8.0):
    """A box spanning several tiles with a ragged tail: 343 waters (1,029 atoms)."""
    return synth.water_box(n_w, P, L, seed=seed, cutoff=rc, ewald_alpha=0.35, pme_grid=K,
                           pme_order=order, name=f"water{n_w}_P{P}")


def oracle_forces_on(s, x, sample):
    """-grad V at the sampled atoms: all real-space partners of the sample by brute force,
    full intramolecular, exclusion and SPME terms."""
    from oracle import forces, spme
    N = len(x)
    mol = np.arange(N) // 3
    I, J = [], []
    for i in sample:
        j = np.arange(N)
        j = j[(mol[j] != mol[i]) & (j != i)]
        I.append(np.full(len(j), i)); J.append(j)
    I = np.concatenate(I); J = np.concatenate(J)
    both = np.isin(J, sample)
    keep = ~both | (I < J)
    pairs = np.stack([I[keep], J[keep]], axis=1)
    _, _, g_rs = forces.real_space(x, pairs, s.charge, s.types, s.lj_sigma, s.lj_epsilon,
                                   s.box, s.ewald_alpha, s.cutoff, s.coulomb)
    _, _, g_in = forces.intramolecular(x, s.box, s.bond_r0, s.bond_k, s.angle_theta0,
                                       s.angle_k)
    _, g_x = forces.excluded_correction(x, s.charge, s.box, s.ewald_alpha, s.coulomb)
    e_r, g_r = spme.spme(x, s.charge, s.box, s.pme_grid, s.pme_order, s.ewald_alpha, s.coulomb)
    return -(g_rs + g_in + g_x + g_r)[sample], e_r
