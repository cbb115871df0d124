"""Parity of the HIP path's BAOAB-RESPA with ring-polymer contraction (Sec. "Multi-timestep
Methods") with the FP64 oracle, through the C ABI.

The oracle is ``oracle/respa.py`` with V_f = bonds + angles on the P beads and V_s = all
other terms on the contracted beads. Bars as for the plain RPMD trajectories: per-step
parity at FP64 rounding over short runs, and the FP32-pair tolerance of the workload
(1e-5 relative RMS force) for the FP32 path.
"""
import math
import sys

import numpy as np
import pytest

import synth
from helpers import has_gpu, medium_box
from oracle import forces as ofo
from oracle import respa

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ctx_for(s, **kw):
    import paper_2212_03137_amd as q
    return q.Context.from_system(s, **kw)


def oracle_respa(s, Pc, nalt):
    R = respa.RPMDRespa(s.n_beads, s.mass, s.kT, s.hbar, s.dt, s.gamma_centroid, s.trpmd_c,
                        s.seed, lambda x: ofo.evaluate_fast(x, s),
                        lambda x: ofo.evaluate_slow(x, s), n_contract=Pc, n_alt=nalt)
    R.set_state(s.pos, s.vel)
    return R


@pytest.fixture(scope="module")
def small():
    return synth.small_rpmd()


@pytest.fixture(scope="module")
def small32():
    """64 waters at P = 32: room for the paper's contraction to about five beads."""
    return synth.water_box(64, 32, 12.42, synth.SEED_BASE + 50, cutoff=6.0, ewald_alpha=0.35,
                           pme_grid=16, pme_order=4)


@pytest.mark.parametrize("Pc,nalt,nout", [(8, 2, 2), (4, 1, 2), (4, 3, 2), (2, 2, 2),
                                           (1, 4, 2), (4, 2, 15), (3, 2, 2), (5, 2, 2),
                                           (7, 1, 2), (5, 3, 15), (6, 2, 2)])
def test_respa_trajectory_small(small, Pc, nalt, nout):
    _respa_parity(small, Pc, nalt, nout)


@pytest.mark.parametrize("Pc,nalt,nout", [(5, 4, 2), (5, 2, 8), (3, 2, 2), (16, 2, 2)])
def test_respa_trajectory_32_beads(small32, Pc, nalt, nout):
    _respa_parity(small32, Pc, nalt, nout)


def _respa_parity(s, Pc, nalt, nout):
    say("respa trajectory", Pc, nalt, nout)
    R = oracle_respa(s, Pc, nalt)
    R.step(nout)
    xr, vr, nr = R.get_state()
    with ctx_for(s, rpc_beads=Pc, respa_nalt=nalt) as c:
        c.set_state(s.pos, s.vel, 0)
        E = c.step(nout, energy=True)
        x, v, st = c.get_state()
        kin, spr = c.mode_energies()
    assert st == nr == nout * nalt
    tol = 1e-10 if nout <= 2 else 1e-8
    assert np.abs(x - xr).max() / np.abs(xr).max() < tol
    assert np.abs(v - vr).max() / np.abs(vr).max() < tol * 100
    # energies: bond and angle on all beads, the rest on the contracted beads only
    Ef, Es = R.E_fast, R.E_slow
    assert np.abs(E[:, :2] - Ef[:, :2]).max() / np.abs(Ef[:, :2]).max() < tol * 100
    assert np.abs(E[:Pc, 2:] - Es[:, 2:]).max() / np.abs(Es[:, 2:]).max() < tol * 100
    assert np.all(E[Pc:, 2:] == 0.0)
    assert math.isclose(kin, R.kinetic(), rel_tol=tol * 100)
    assert math.isclose(spr, R.spring(), rel_tol=tol * 100)


def test_respa_state_round_trip_and_eval_leave_the_state(small):
    s = small
    with ctx_for(s, rpc_beads=2, respa_nalt=3) as c:
        c.set_state(s.pos, s.vel, 6)
        x, v, st = c.get_state()
        assert st == 6
        assert np.abs(x - s.pos).max() < 1e-12 * np.abs(s.pos).max()
        assert np.abs(v - s.vel).max() < 1e-12 * np.abs(s.vel).max()
        # eval is the full potential on every bead and does not change the propagated state
        E, F = c.eval(s.pos[::-1].copy())
        Eref, Fref = ofo.evaluate(s.pos[::-1].copy(), s)
        assert np.abs(F - Fref).max() / np.sqrt(np.mean(Fref ** 2)) <= 1e-11
        assert np.abs(E - Eref).max() <= 1e-11 * np.abs(Eref).max()
        c.step(3)
        x1, v1, _ = c.get_state()
    with ctx_for(s, rpc_beads=2, respa_nalt=3) as c:
        c.set_state(s.pos, s.vel, 6)
        c.step(3)
        x2, v2, _ = c.get_state()
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x2).max()
    assert np.abs(v1 - v2).max() <= 1e-12 * np.abs(v2).max()


def test_respa_graph_replay_equals_eager(small):
    s = small
    out = []
    for g in (True, False):
        with ctx_for(s, rpc_beads=4, respa_nalt=2, use_graph=g) as c:
            c.set_state(s.pos, s.vel, 0)
            c.step(12)
            out.append(c.get_state())
    assert out[0][2] == out[1][2] == 24
    assert np.abs(out[0][0] - out[1][0]).max() / np.abs(out[1][0]).max() < 1e-12


def test_respa_fp32_pairs_medium():
    import paper_2212_03137_amd as q
    s = medium_box(P=4)
    say("respa fp32 medium")
    R = oracle_respa(s, 2, 2)
    R.step(2)
    xr, vr, _ = R.get_state()
    with ctx_for(s, rpc_beads=2, respa_nalt=2, precision=q.FP32_PAIRS) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(2)
        x, v, st = c.get_state()
    assert st == 4
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-9
    dv = v - vr
    assert np.sqrt(np.mean(dv ** 2)) / np.sqrt(np.mean(vr ** 2)) < 1e-5


def test_rejects_unsupported_combinations(small):
    import paper_2212_03137_amd as q
    s = small
    for kw in (dict(rpc_beads=9), dict(rpc_beads=16), dict(rpc_beads=-1), dict(respa_nalt=-1),
               dict(respa_nalt=65)):
        with pytest.raises(q.QhpError):
            ctx_for(s, **kw)
    with pytest.raises(q.QhpError):
        ctx_for(s, rpc_beads=4, exec_mode=q.PLAIN)


@pytest.mark.parametrize("Pc", [4, 5])
def test_large_box_contracted_respa_energies(Pc):
    """4,096 waters, P = 32, FP32 pairs, n = 4: after 10 outer steps (the list rebuilt from
    the skin rule on the contracted beads) the step's energies are checked against the
    oracle at the GPU's final state: bonds and angles on the 32 beads, the other terms on
    the contracted beads the oracle builds from that state's modes."""
    import paper_2212_03137_amd as q
    from oracle import normal_modes as nm
    s = synth.large_rpmd()
    say("large respa", s.n_atoms, s.n_beads, Pc)
    with ctx_for(s, rpc_beads=Pc, respa_nalt=4, precision=q.FP32_PAIRS) as c:
        c.set_state(s.pos, s.vel, 0)
        E = c.step(10, energy=True)
        x, v, st = c.get_state()
        stats = c.nlist_stats()
    assert st == 40
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(v))
    assert np.all(E[Pc:, 2:] == 0.0) and np.all(np.isfinite(E))
    assert stats["max_count"] <= stats["capacity"] and stats["builds"] >= 1
    Ef, _ = ofo.evaluate_fast(x, s)
    assert np.abs(E[:, :2] - Ef[:, :2]).max() <= 1e-9 * np.abs(Ef[:, :2]).max()
    xc = respa.contract(nm.modes_from_beads(x, nm.transfer_matrix(s.n_beads)), Pc)
    say("oracle slow terms on", xc.shape)
    Es, _ = ofo.evaluate_slow(xc, s)
    for t in (4, 5, 6):                  # exclusion, self, reciprocal: FP64 on both sides
        assert np.abs(E[:Pc, t] - Es[:, t]).max() <= 1e-9 * np.abs(Es[:, t]).max(), t
    for t in (2, 3):                     # real-space Coulomb and LJ: FP32 pairs
        assert np.abs(E[:Pc, t] - Es[:, t]).max() <= 1e-5 * np.abs(Es[:, t]).max(), t
