"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Bars: bit-exact for the Philox/Gaussian noise streams and the centroid neighbour list;
forces <= 1e-11 (max abs error over RMS force) and per-term energies <= 1e-11 relative in
FP64; <= 1e-5 relative RMS for FP32 pairs (the tolerances of the workload definition).
"""
import math
import sys

import numpy as np
import pytest

import synth
from helpers import has_gpu, medium_box, oracle_forces_on, oracle_grad_fn, rel_max, rel_rms
from oracle import forces as ofo
from oracle import philox as oph

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ctx_for(s, **kw):
    import paper_2212_03137_amd as q
    return q.Context.from_system(s, **kw)


# ---------------------------------------------------------------------------- noise
@pytest.mark.parametrize("P,NW", [(1, 3), (6, 20), (8, 64), (32, 111)])
def test_rpmd_noise_bit_exact(P, NW):
    s = synth.water_box(NW, P, 20.0, seed=3)
    N = s.n_atoms
    say("noise", P, N)
    with ctx_for(s) as c:
        for step in (0, 1, 12345, 2 ** 40 + 7):
            got = c.noise(5, step)
            ref = oph.rpmd_noise(s.seed, step, N, P)
            assert np.array_equal(got, ref), (step, np.abs(got - ref).max())


def test_qtb_white_noise_bit_exact():
    s = synth.water_box(20, 1, 20.0, seed=4, qtb_gamma0=0.02, qtb_nseg=64)
    with ctx_for(s) as c:
        for tau in (-64, -1, 0, 5, 1000):
            got = c.noise(6, tau)
            ref = oph.qtb_white(s.seed, tau, 1, 60, 64)[0]
            assert np.array_equal(got, ref)


# ---------------------------------------------------------------------------- list
@pytest.mark.parametrize("n_w,L,P,rc", [(64, 12.42, 8, 6.0), (216, 18.7, 2, 6.5),
                                        (343, 21.8, 4, 8.0), (4096, 49.7, 1, 9.0)])
def test_neighbour_list_bit_exact(n_w, L, P, rc):
    s = synth.water_box(n_w, P, L, seed=n_w, cutoff=rc, pme_grid=16 if L < 15 else 32,
                        pme_order=4)
    say("nlist", n_w, L, P)
    with ctx_for(s) as c:
        c.eval(s.pos)
        got = c.nlist()
    ref = ofo.pair_list(ofo.centroids_of(s.pos), s.box, s.cutoff + s.skin)
    assert got.shape == ref.shape and np.array_equal(got, ref)


def test_list_and_forces_of_a_system_past_the_register_binning():
    # 6,000 waters = 18,000 atoms: more than 16 atoms per thread of the one-block
    # bookkeeping kernel, which then bins SPME tiles and list cells with its strided,
    # run-aggregated path; the list rows of 300 sampled atoms are compared bit for bit
    # with the oracle's (the full brute-force list takes the oracle minutes), the forces
    # (which use the tiles) at both beads
    s = synth.water_box(6000, 2, 56.4, seed=6000, cutoff=9.0, pme_grid=32, pme_order=4)
    say("strided binning", s.n_atoms)
    with ctx_for(s) as c:
        E, F = c.eval(s.pos)
        got = c.nlist()
    cen = ofo.centroids_of(s.pos)
    rows = np.random.default_rng(7).choice(s.n_atoms, 300, replace=False)
    ref = ofo.pair_list_rows(cen, s.box, s.cutoff + s.skin, rows)
    mine = got[np.isin(got[:, 0], rows) | np.isin(got[:, 1], rows)]
    assert np.array_equal(mine, ref)
    assert np.all(got[:, 0] < got[:, 1])
    assert np.all(np.diff(got[:, 0] * s.n_atoms + got[:, 1]) > 0)
    sample = np.sort(np.random.default_rng(8).choice(s.n_atoms, 32, replace=False))
    for b in range(2):
        Fref, e_rec = oracle_forces_on(s, s.pos[b], sample)
        assert rel_max(F[b, sample], Fref) <= 1e-11
        assert abs(E[b, 6] - e_rec) <= 1e-11 * abs(e_rec)


# ---------------------------------------------------------------------------- forces
def _oracle_eval(s, beads=None):
    pos = s.pos if beads is None else s.pos
    return ofo.evaluate(pos, s)


@pytest.fixture(scope="module")
def small():
    s = synth.small_rpmd()
    return s, ofo.evaluate(s.pos, s)


@pytest.fixture(scope="module")
def medium():
    s = medium_box()
    return s, ofo.evaluate(s.pos, s)


def _check_fp64(E, F, Eref, Fref):
    assert rel_max(F, Fref) <= 1e-11, rel_max(F, Fref)
    scale = np.abs(Eref).max(axis=0) + 1e-300
    err = np.abs(E - Eref) / scale
    assert err.max() <= 1e-11, err.max(axis=0)


def test_eval_fp64_small(small):
    s, (Eref, Fref) = small
    say("eval fp64 small")
    with ctx_for(s) as c:
        E, F = c.eval(s.pos)
    _check_fp64(E, F, Eref, Fref)


def test_eval_fp64_medium_batched_and_plain(medium):
    import paper_2212_03137_amd as q
    s, (Eref, Fref) = medium
    say("eval fp64 medium")
    with ctx_for(s) as c:
        E, F = c.eval(s.pos)
    _check_fp64(E, F, Eref, Fref)
    with ctx_for(s, exec_mode=q.PLAIN) as c:
        E2, F2 = c.eval(s.pos)
    _check_fp64(E2, F2, Eref, Fref)


def test_eval_fp32_pairs_medium(medium):
    import paper_2212_03137_amd as q
    s, (Eref, Fref) = medium
    say("eval fp32 medium")
    with ctx_for(s, precision=q.FP32_PAIRS) as c:
        E, F = c.eval(s.pos)
    assert rel_rms(F, Fref) <= 1e-5, rel_rms(F, Fref)
    # everything but the real-space pair terms is still FP64
    for t in (0, 1, 4, 5, 6):
        assert np.abs(E[:, t] - Eref[:, t]).max() <= 1e-11 * np.abs(Eref[:, t]).max()
    for t in (2, 3):
        assert np.abs(E[:, t] - Eref[:, t]).max() <= 1e-5 * np.abs(Eref[:, t]).max()


# ---------------------------------------------------------------------------- dynamics
def _oracle_rpmd(s):
    from oracle import rpmd
    R = rpmd.RPMD(s.n_beads, s.mass, s.kT, s.hbar, s.dt, s.gamma_centroid, s.trpmd_c, s.seed,
                  oracle_grad_fn(s))
    R.set_state(s.pos, s.vel)
    return R


def test_state_round_trip(small):
    s, _ = small
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 17)
        x, v, st = c.get_state()
    assert st == 17
    assert np.abs(x - s.pos).max() < 1e-12 * np.abs(s.pos).max()
    assert np.abs(v - s.vel).max() < 1e-12 * np.abs(s.vel).max()


@pytest.mark.parametrize("nsteps", [1, 100])
def test_rpmd_trajectory_small(small, nsteps):
    s, _ = small
    say("rpmd trajectory", nsteps)
    R = _oracle_rpmd(s)
    R.step(nsteps)
    xr, vr, _ = R.get_state()
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 0)
        E = c.step(nsteps, energy=True)
        x, v, st = c.get_state()
        kin, spr = c.mode_energies()
    assert st == nsteps
    tol = 1e-11 if nsteps == 1 else 1e-8
    assert np.abs(x - xr).max() / np.abs(xr).max() < tol
    assert np.abs(v - vr).max() / np.abs(vr).max() < tol * 100
    assert np.abs(E - R.E).max() / np.abs(R.E).max() < tol * 100
    assert math.isclose(kin, R.kinetic(), rel_tol=tol * 100)
    assert math.isclose(spr, R.spring(), rel_tol=tol * 100)


@pytest.mark.parametrize("nsteps", [1, 60])
def test_bcocb_trajectory_small(small, nsteps):
    """The Cayley (BCOCB) free ring-polymer step against the oracle's implicit-midpoint form."""
    import paper_2212_03137_amd as q
    from oracle import rpmd
    s, _ = small
    say("bcocb trajectory", nsteps)
    R = rpmd.RPMD(s.n_beads, s.mass, s.kT, s.hbar, s.dt, s.gamma_centroid, s.trpmd_c, s.seed,
                  oracle_grad_fn(s), integrator="BCOCB")
    R.set_state(s.pos, s.vel)
    R.step(nsteps)
    xr, vr, _ = R.get_state()
    with ctx_for(s, integrator=q.BCOCB) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(nsteps)
        x, v, st = c.get_state()
    assert st == nsteps
    tol = 1e-11 if nsteps == 1 else 1e-8
    assert np.abs(x - xr).max() / np.abs(xr).max() < tol
    assert np.abs(v - vr).max() / np.abs(vr).max() < tol * 100
    # and it is a different integrator from BAOAB
    R2 = _oracle_rpmd(s)
    R2.step(nsteps)
    assert np.abs(R2.get_state()[0] - xr).max() > 1e3 * tol * np.abs(xr).max()


def test_rpmd_trajectory_plain_fp64_equals_batched(small):
    import paper_2212_03137_amd as q
    s, _ = small
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(20)
        x1, v1, _ = c.get_state()
    with ctx_for(s, exec_mode=q.PLAIN) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(20)
        x2, v2, _ = c.get_state()
    assert np.abs(x1 - x2).max() / np.abs(x1).max() < 1e-11


# ---------------------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def large():
    return synth.large_rpmd()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_large_box_forces_on_sampled_beads(large, precision):
    """4,096 waters, P = 32, in the launch configuration the benchmark times; the oracle
    evaluates beads 0, 13 and 31 in full."""
    import paper_2212_03137_amd as q
    s = large
    say("large eval", precision)
    prec = q.FP64 if precision == "fp64" else q.FP32_PAIRS
    with ctx_for(s, precision=prec) as c:
        E, F = c.eval(s.pos)
        pairs_gpu = c.nlist()
    pairs = ofo.pair_list(ofo.centroids_of(s.pos), s.box, s.cutoff + s.skin)
    assert np.array_equal(pairs_gpu, pairs)
    for b in (0, 13, 31):
        Eb, g = ofo.bead_potential(s.pos[b], s, pairs)
        if precision == "fp64":
            assert rel_max(F[b], -g) <= 1e-11
            assert np.abs(E[b] - Eb).max() <= 1e-11 * np.abs(Eb).max()
        else:
            assert rel_rms(F[b], -g) <= 1e-5


def test_large_box_timed_path_step_matches_the_oracle(large):
    """One step of the path the benchmark times (FP32 pairs, autotuned launch shapes, the
    step captured as a graph with the SPME spread and transforms on the second stream)
    against one step of the FP64 oracle's integrator with the same Philox noise. The FP32
    pair forces (<= 1e-5 relative RMS) enter through the two half kicks: positions move by
    dt^2/2m of the force error, velocities by dt/m."""
    import paper_2212_03137_amd as q
    from oracle import rpmd
    s = large
    say("large timed-path step: oracle")
    R = rpmd.RPMD(s.n_beads, s.mass, s.kT, s.hbar, s.dt, s.gamma_centroid, s.trpmd_c, s.seed,
                  oracle_grad_fn(s))
    R.set_state(s.pos, s.vel)
    R.step(1)
    xr, vr, _ = R.get_state()
    say("large timed-path step: GPU")
    with ctx_for(s, precision=q.FP32_PAIRS) as c:
        c.set_state(s.pos, s.vel, 0)
        shapes = c.autotune(3)
        c.step(1)
        x, v, st = c.get_state()
    say("autotuned", shapes)
    assert st == 1
    assert np.abs(x - xr).max() <= 1e-7 * np.abs(xr).max()
    assert rel_rms(v, vr) <= 1e-5
    assert rel_max(v, vr) <= 1e-4


def test_large_box_step_stays_finite_and_rebuilds(large):
    import paper_2212_03137_amd as q
    s = large
    with ctx_for(s, precision=q.FP32_PAIRS) as c:
        c.set_state(s.pos, s.vel, 0)
        E = c.step(20, energy=True)
        x, v, st = c.get_state()
    assert st == 20 and np.all(np.isfinite(x)) and np.all(np.isfinite(E))


def test_rebuild_rule_holds_over_a_trajectory(large):
    """The list is rebuilt only when the skin is used up: count the builds, then check the
    energies of the last step (evaluated with the list kept from the last skin-triggered
    build) and the forces of a fresh evaluation against the oracle's definition (every
    pair within the cutoff) on one bead."""
    import paper_2212_03137_amd as q
    from helpers import oracle_forces_on
    s = large
    with ctx_for(s, precision=q.FP64) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(199)
        E_step = c.step(1, energy=True)
        st = c.nlist_stats()
        x, _, _ = c.get_state()
        E, F = c.eval(x)
    say("nlist stats after 200 steps", st)
    assert 1 < st["builds"] < 120
    assert st["max_count"] <= st["capacity"]
    b = 7
    pairs = ofo.pair_list(ofo.centroids_of(x), s.box, s.cutoff + s.skin)
    Eb, g = ofo.bead_potential(x[b], s, pairs)
    assert np.abs(E_step[b] - Eb).max() <= 1e-11 * np.abs(Eb).max()
    assert np.abs(E[b] - Eb).max() <= 1e-11 * np.abs(Eb).max()
    assert rel_max(F[b], -g) <= 1e-11
    sample = np.arange(0, s.n_atoms, 97)
    Fs, _ = oracle_forces_on(s, x[b], sample)
    assert np.abs(F[b][sample] - Fs).max() <= 1e-11 * np.sqrt(np.mean(g * g))


def test_trajectory_through_skin_rebuilds_matches_the_oracle():
    """343 waters (21.7 A) at P = 4 with rc + skin below L/2: the centroid list with its
    image shifts is built on the device and kept until the skin rule fires. The oracle
    finds every pair within the cutoff at every step, so a list kept too long or a wrong
    stored image shift shows as a trajectory difference."""
    import dataclasses
    import paper_2212_03137_amd as q
    s = dataclasses.replace(medium_box(P=4), skin=1.4)
    say("skin-rebuild trajectory")
    R = _oracle_rpmd(s)
    R.step(80)
    xr, vr, _ = R.get_state()
    with ctx_for(s, precision=q.FP64) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(80)
        x, v, st = c.get_state()
        stats = c.nlist_stats()
    say("builds", stats)
    assert st == 80
    assert stats["builds"] >= 4          # the build at set-up and at least three from the rule
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-8
    assert np.abs(v - vr).max() / np.abs(vr).max() < 1e-6


def test_rows_grow_when_a_build_finds_more_neighbours():
    """Rows that are too short for the list grow by themselves, in the stateless
    evaluation (host and device memory) and in a trajectory: the propagation restarts from
    the state the call began with. The trajectory's rows are sized to the largest count of
    the first build, which a later build of the same seeded run exceeds."""
    import dataclasses
    import torch
    import paper_2212_03137_amd as q
    s = dataclasses.replace(medium_box(P=4), skin=1.4)
    say("list growth")
    with ctx_for(s, precision=q.FP64) as c:
        c.set_state(s.pos, s.vel, 0)
        m0 = c.nlist_stats()["max_count"]
        mt = m0
        for _ in range(60):
            c.step(1)
            mt = max(mt, c.nlist_stats()["max_count"])
    say("largest counts", m0, mt)
    assert mt > m0
    R = _oracle_rpmd(s)
    R.step(60)
    xr, vr, _ = R.get_state()
    with ctx_for(s, precision=q.FP64, nbr_capacity=m0) as c:
        c.set_state(s.pos, s.vel, 0)
        assert c.nlist_stats()["capacity"] == m0
        c.step(60)
        x, v, st = c.get_state()
        grown = c.nlist_stats()["capacity"]
    assert st == 60 and grown > m0
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-8
    assert np.abs(v - vr).max() / np.abs(vr).max() < 1e-6
    Eref, Fref = ofo.evaluate(s.pos, s)
    with ctx_for(s, precision=q.FP64, nbr_capacity=8) as c:
        E, F = c.eval(s.pos, box=s.box)
        _check_fp64(E, F, Eref, Fref)
        assert c.nlist_stats()["capacity"] > 8
    with ctx_for(s, precision=q.FP64, nbr_capacity=8) as c:
        pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
        Et = torch.zeros((s.n_beads, q.NTERMS), dtype=torch.float64, device="cuda")
        Ft = torch.zeros_like(pos)
        c.eval_device(pos, Et, Ft)
        c.sync()
        _check_fp64(Et.cpu().numpy(), Ft.cpu().numpy(), Eref, Fref)
        with pytest.raises(q.QhpError):
            c.eval(s.pos, box=s.box * 1.01)


@pytest.mark.parametrize("P", [3, 6])
def test_bead_counts_that_are_not_powers_of_two(P):
    """P = 3 and 6 run in the lanes of 4 and 8: forces, energies and a trajectory against
    the oracle's P-bead ring polymer."""
    import paper_2212_03137_amd as q
    s = synth.water_box(64, P, 12.42, synth.SEED_BASE + 40 + P, cutoff=6.0, ewald_alpha=0.35,
                        pme_grid=16, pme_order=4)
    say("non-power-of-two P", P)
    Eref, Fref = ofo.evaluate(s.pos, s)
    R = _oracle_rpmd(s)
    R.step(40)
    xr, vr, _ = R.get_state()
    for mode in (q.BATCHED, q.PLAIN):
        with ctx_for(s, exec_mode=mode) as c:
            E, F = c.eval(s.pos)
            _check_fp64(E, F, Eref, Fref)
            c.set_state(s.pos, s.vel, 0)
            E = c.step(40, energy=True)
            x, v, st = c.get_state()
            kin, spr = c.mode_energies()
            noise = c.noise(5, 3)
        assert st == 40 and x.shape == (P, s.n_atoms, 3)
        assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-8
        assert np.abs(v - vr).max() / np.abs(vr).max() < 1e-6
        assert np.abs(E - R.E).max() / np.abs(R.E).max() < 1e-6
        assert math.isclose(kin, R.kinetic(), rel_tol=1e-6)
        assert math.isclose(spr, R.spring(), rel_tol=1e-6)
        assert noise.shape == (P, s.n_atoms, 3)


def test_fp32_pairs_with_six_beads():
    import paper_2212_03137_amd as q
    s = medium_box(P=6)
    say("fp32 P=6")
    Eref, Fref = ofo.evaluate(s.pos, s)
    with ctx_for(s, precision=q.FP32_PAIRS) as c:
        E, F = c.eval(s.pos)
    assert rel_rms(F, Fref) <= 1e-5, rel_rms(F, Fref)
    for t in (0, 1, 4, 5, 6):
        assert np.abs(E[:, t] - Eref[:, t]).max() <= 1e-11 * np.abs(Eref[:, t]).max()


def test_graph_replay_equals_eager_launches(small):
    """The captured-graph step and the launched step are the same kernels in the same
    order: trajectories agree to rounding (SPME accumulation order aside)."""
    s, _ = small
    out = []
    for g in (True, False):
        with ctx_for(s, use_graph=g) as c:
            c.set_state(s.pos, s.vel, 0)
            c.step(30)
            out.append(c.get_state())
    assert out[0][2] == out[1][2] == 30
    assert np.abs(out[0][0] - out[1][0]).max() / np.abs(out[1][0]).max() < 1e-12
