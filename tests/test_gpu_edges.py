"""Edge cases of the HIP path against the FP64 oracle: the largest bead count (P = 64, one
atom per wavefront in the pair and gather kernels), the classical P = 1 case, a single
molecule (empty neighbour list), and host inputs rejected before any device work."""
import sys

import numpy as np
import pytest

import synth
from helpers import has_gpu, oracle_grad_fn, rel_max, rel_rms
from oracle import forces, rpmd

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ctx_for(s, **kw):
    import paper_2212_03137_amd as q
    return q.Context.from_system(s, **kw)


def _trajectory(s, nsteps, **kw):
    R = rpmd.RPMD(s.n_beads, s.mass, s.kT, s.hbar, s.dt, s.gamma_centroid, s.trpmd_c, s.seed,
                  oracle_grad_fn(s))
    R.set_state(s.pos, s.vel)
    R.step(nsteps)
    xr, vr, _ = R.get_state()
    with ctx_for(s, **kw) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(nsteps)
        x, v, st = c.get_state()
    assert st == nsteps
    return np.abs(x - xr).max() / np.abs(xr).max(), np.abs(v - vr).max() / np.abs(vr).max()


def test_sixty_four_beads_fp64_eval_and_trajectory():
    s = synth.water_box(64, 64, 12.42, seed=61, cutoff=6.0, pme_grid=16, pme_order=4)
    say("P=64 small", s.n_atoms)
    E_r, F_r = forces.evaluate(s.pos, s)
    with ctx_for(s) as c:
        E, F = c.eval(s.pos)
    assert rel_max(F, F_r) <= 1e-11
    assert np.allclose(E, E_r, rtol=1e-11, atol=1e-9)
    ex, ev = _trajectory(s, 3)
    assert ex < 1e-10 and ev < 1e-8, (ex, ev)


def test_sixty_four_beads_fp32_pairs():
    # 216 waters, 18.7 A: 2 (rc + skin) < L, so the FP32 pair kernel runs with one slot
    s = synth.water_box(216, 64, 18.7, seed=62, cutoff=6.5, pme_grid=32, pme_order=5)
    say("P=64 FP32", s.n_atoms)
    import paper_2212_03137_amd as q
    F_r = np.empty_like(s.pos)
    E_r = np.empty((s.n_beads, 7))
    for b in (0, 17, 63):                    # the oracle on three beads
        e, f = forces.evaluate(s.pos[b:b + 1], s)
        E_r[b], F_r[b] = e[0], f[0]
    with ctx_for(s, precision=q.FP32_PAIRS) as c:
        E, F = c.eval(s.pos)
        c.set_state(s.pos, s.vel, 0)
        c.step(5)
        x, _, _ = c.get_state()
    for b in (0, 17, 63):
        assert rel_rms(F[b], F_r[b]) <= 1e-5, b
        assert np.allclose(E[b], E_r[b], rtol=1e-5, atol=1e-4 * np.abs(E_r[b]).max())
    assert np.all(np.isfinite(x))


def test_classical_single_bead_eval_and_trajectory():
    s = synth.water_box(64, 1, 12.42, seed=63, cutoff=6.0, pme_grid=16, pme_order=4)
    E_r, F_r = forces.evaluate(s.pos, s)
    with ctx_for(s) as c:
        E, F = c.eval(s.pos)
    assert rel_max(F, F_r) <= 1e-11
    assert np.allclose(E, E_r, rtol=1e-11, atol=1e-9)
    ex, ev = _trajectory(s, 3)
    assert ex < 1e-10 and ev < 1e-8, (ex, ev)


def test_classical_single_bead_fp32_pairs():
    # one bead, FP32 pairs (343 waters, 21.7 A: 2 (rc + skin) < L): the kernel evaluates
    # each lane's list entry in place; the bar of the FP32-pair mode against the oracle
    from helpers import medium_box
    import paper_2212_03137_amd as q
    s = medium_box(P=1)
    E_r, F_r = forces.evaluate(s.pos, s)
    with ctx_for(s, precision=q.FP32_PAIRS) as c:
        E, F = c.eval(s.pos)
        c.set_state(s.pos, s.vel, 0)
        c.step(20)
        x, _, st = c.get_state()
    assert rel_rms(F, F_r) <= 1e-5
    assert np.allclose(E, E_r, rtol=1e-5, atol=1e-4 * np.abs(E_r).max())
    assert st == 20 and np.all(np.isfinite(x))


def test_single_molecule_has_no_pairs():
    # one water in a 10 A box: the centroid list is empty; bonded, exclusion, self and
    # reciprocal terms remain
    s = synth.water_box(1, 4, 10.0, seed=64, cutoff=4.0, pme_grid=16, pme_order=4)
    E_r, F_r = forces.evaluate(s.pos, s)
    assert np.all(E_r[:, 2] == 0.0) and np.all(E_r[:, 3] == 0.0)
    with ctx_for(s) as c:
        E, F = c.eval(s.pos)
        assert c.nlist().shape[0] == 0
    assert rel_max(F, F_r) <= 1e-11
    assert np.allclose(E, E_r, rtol=1e-11, atol=1e-9)
    ex, ev = _trajectory(s, 3)
    assert ex < 1e-10 and ev < 1e-8, (ex, ev)


def test_non_finite_host_input_is_rejected_before_device_work():
    import paper_2212_03137_amd as q
    s = synth.water_box(8, 2, 10.0, seed=65, cutoff=4.0, pme_grid=16, pme_order=4)
    pos = s.pos.copy()
    pos[1, 5, 2] = np.nan
    with ctx_for(s) as c:
        with pytest.raises(q.QhpError) as e:
            c.eval(pos)
        assert e.value.code == q.ENONFINITE
        with pytest.raises(q.QhpError) as e:
            c.set_state(pos, s.vel, 0)
        assert e.value.code == q.ENONFINITE
        E, F = c.eval(s.pos)                 # the context still works
    assert np.all(np.isfinite(F))


def test_microcanonical_ring_polymer_conserves_energy():
    # no friction on any mode: BAOAB reduces to velocity Verlet in the normal modes, so
    # H = sum_n P_n^2/2m + sum_n m w_n^2 Q_n^2 / 2 + (1/P) sum_b V(x_b) stays near its
    # start (bounded O(dt^2) oscillation, no drift beyond the cutoff's small jumps)
    import dataclasses
    s = synth.water_box(64, 4, 12.42, seed=66, cutoff=6.0, pme_grid=16, pme_order=4, dt=0.25)
    s = dataclasses.replace(s, gamma_centroid=0.0, trpmd_c=0.0)
    hs, ks = [], []
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 0)
        for _ in range(20):
            E = c.step(20, energy=True)
            k, sp = c.mode_energies()
            hs.append(k + sp + E.sum() / s.n_beads)
            ks.append(k)
    hs, K = np.array(hs), float(np.mean(ks))
    say("NVE H", hs.min(), hs.max(), "K", K)
    assert np.max(np.abs(hs - hs[0])) <= 0.01 * K
    assert abs(hs[-5:].mean() - hs[:5].mean()) <= 0.003 * K


def _tethered(s, k, **zero):
    import dataclasses
    return dataclasses.replace(s, tether_k=k, tether_anchor=s.pos[0].copy(), **zero)


def test_tether_forces_and_energies_match_the_oracle():
    s = synth.water_box(27, 2, 10.5, seed=71, cutoff=5.0, ewald_alpha=0.4, pme_grid=16,
                        pme_order=5)
    s = _tethered(s, 7.5)
    s.tether_anchor = s.tether_anchor + 0.05          # the beads sit off their anchors
    E_r, F_r = forces.evaluate(s.pos, s)
    with ctx_for(s) as c:
        E, F = c.eval(s.pos)
    assert rel_max(F, F_r) <= 1e-11
    assert np.allclose(E, E_r, rtol=1e-11, atol=1e-9)


def test_tethered_free_atoms_sample_the_ring_polymer_oscillator():
    # every interaction switched off and a harmonic tether k on each atom: independent
    # 3-D oscillators, w^2 = k / m; per dof and bead <(x - a)^2> = (kT / m) sum_k
    # 1 / (w^2 + w_k^2) with the free ring polymer's w_k (the P-bead closed form)
    import dataclasses
    from oracle import normal_modes as nm
    s = synth.water_box(64, 8, 12.42, seed=72, cutoff=6.0, pme_grid=16, pme_order=4)
    mH = s.mass[1]
    w = 2.0 * s.kT / s.hbar                             # beta hbar w = 2 for hydrogen
    k = mH * w * w
    s = _tethered(s, k, charge=np.zeros_like(s.charge), lj_epsilon=np.zeros_like(s.lj_epsilon),
                  bond_k=0.0, angle_k=0.0)
    s = dataclasses.replace(s, gamma_centroid=0.01)
    wk = nm.mode_frequencies(s.n_beads, 1.0 / s.kT, s.hbar)
    acc = np.zeros(s.n_atoms)
    n = 0
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(2000)
        for _ in range(1000):
            c.step(20)
            x, _, _ = c.get_state()
            acc += ((x - s.tether_anchor[None]) ** 2).mean(axis=(0, 2))
            n += 1
    acc /= n
    for t in (0, 1):                                    # O, H
        m = s.mass[t]
        ref = s.kT / m * np.sum(1.0 / (k / m + wk * wk))
        got = acc[s.types == t].mean()
        say("tether", t, got, ref)
        assert abs(got / ref - 1) < 0.02
