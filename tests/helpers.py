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
