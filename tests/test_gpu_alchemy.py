"""Alchemical windows on the HIP path (scaled solute charges, soft-core solute-solvent LJ)
against the FP64 oracle, qhp_eval_lambda, and groups of contexts stepped as one graph."""
import dataclasses
import sys

import numpy as np
import pytest

import synth
from helpers import has_gpu, oracle_grad_fn, rel_max, rel_rms
from oracle import forces

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]

LAMBDAS = [(1.0, 1.0), (0.5, 1.0), (0.0, 0.6), (0.0, 0.15), (0.0, 0.0)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ctx_for(s, **kw):
    import paper_2212_03137_amd as q
    return q.Context.from_system(s, **kw)


@pytest.fixture(scope="module")
def medium():
    # 512 waters + the 12-atom solute (1,548 atoms), 24.8 A box: FP32 pairs apply
    return synth.alchemical_window(1, n_beads=4)


@pytest.fixture(scope="module")
def small():
    return synth.water_box(27, 2, 10.5, seed=41, cutoff=5.0, ewald_alpha=0.4, pme_grid=16,
                           pme_order=5, solute=4, name="alchem_small")


@pytest.mark.parametrize("le,lv", LAMBDAS)
def test_alchemical_forces_match_the_oracle(medium, le, lv):
    import paper_2212_03137_amd as q
    s = dataclasses.replace(medium, lambda_elec=le, lambda_vdw=lv)
    say("alchemical forces", le, lv, s.n_atoms, s.n_beads)
    E_r, F_r = forces.evaluate(s.pos, s)
    for prec in (q.FP64, q.FP32_PAIRS):
        # couplings set three ways: at creation, by qhp_set_lambda, by qhp_eval_lambda
        with ctx_for(s, precision=prec) as c:
            E1, F1 = c.eval(s.pos)
        with ctx_for(medium, precision=prec) as c:
            c.set_lambda(le, lv)
            E2, F2 = c.eval(s.pos)
            E3, F3 = c.eval_lambda(s.pos, le, lv)
        for E, F in ((E1, F1), (E2, F2), (E3, F3)):
            if prec == q.FP64:
                assert rel_max(F, F_r) <= 1e-11, (le, lv)
                assert np.allclose(E, E_r, rtol=1e-11, atol=1e-9)
            else:
                assert rel_rms(F, F_r) <= 1e-5, (le, lv)
                assert np.allclose(E, E_r, rtol=1e-5, atol=1e-4 * np.abs(E_r).max())


def test_soft_core_term_changes_with_lambda(medium):
    # the LJ energy moves with lambda_vdw, the electrostatic ones with lambda_elec only
    with ctx_for(medium) as c:
        Ea, _ = c.eval_lambda(medium.pos, 0.0, 1.0)
        Eb, _ = c.eval_lambda(medium.pos, 0.0, 0.5)
        Ec, _ = c.eval_lambda(medium.pos, 0.7, 0.5)
    assert np.all(Ea[:, 3] != Eb[:, 3])
    assert np.allclose(Ea[:, [2, 4, 5, 6]], Eb[:, [2, 4, 5, 6]], rtol=1e-12)
    assert np.allclose(Eb[:, 3], Ec[:, 3], rtol=1e-12)
    assert np.all(Eb[:, 6] != Ec[:, 6])


def test_eval_lambda_leaves_the_propagated_system_alone(medium):
    s = dataclasses.replace(medium, lambda_elec=0.0, lambda_vdw=0.5)
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(3)
        x1, v1, _ = c.get_state()
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(1)
        x, _, _ = c.get_state()
        c.eval_lambda(x, 1.0, 1.0)
        c.step(2)
        x2, v2, _ = c.get_state()
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x1).max()
    assert np.abs(v1 - v2).max() <= 1e-10 * np.abs(v1).max()


@pytest.mark.parametrize("le,lv", [(0.0, 0.3), (0.6, 1.0)])
def test_alchemical_trajectory_small(small, le, lv):
    from oracle import rpmd
    s = dataclasses.replace(small, lambda_elec=le, lambda_vdw=lv)
    say("alchemical trajectory", le, lv)
    R = rpmd.RPMD(s.n_beads, s.mass, s.kT, s.hbar, s.dt, s.gamma_centroid, s.trpmd_c, s.seed,
                  oracle_grad_fn(s))
    R.set_state(s.pos, s.vel)
    R.step(5)
    xr, vr, _ = R.get_state()
    with ctx_for(s) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(5)
        x, v, _ = c.get_state()
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-8
    assert np.abs(v - vr).max() / np.abs(vr).max() < 1e-6


def test_derivatives_of_alchemical_systems_are_rejected(small):
    import paper_2212_03137_amd as q
    with ctx_for(small) as c:
        with pytest.raises(q.QhpError) as e:
            c.param_grad(small.pos)
        assert e.value.code == q.EUNSUPPORTED
        with pytest.raises(q.QhpError) as e:
            c.hvp(small.pos, small.pos)
        assert e.value.code == q.EUNSUPPORTED
    plain = dataclasses.replace(small, type_soft=None)
    with ctx_for(plain) as c:
        with pytest.raises(q.QhpError) as e:
            c.set_lambda(0.5, 0.5)
        assert e.value.code == q.EINVAL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_group_steps_equal_separate_steps(prec):
    # uneven members (sizes, bead counts, couplings) in one graph per step; FP32 pairs round
    # differently once the FP64 sums differ in their last bits (their order of atomic
    # additions is not fixed), hence the looser bound there
    import paper_2212_03137_amd as q
    prec, tol = (q.FP64, 1e-10) if prec == "fp64" else (q.FP32_PAIRS, 1e-6)
    systems = [synth.water_box(27, 2, 10.5, seed=51, cutoff=5.0, ewald_alpha=0.4, pme_grid=16,
                               pme_order=5, solute=4),
               synth.alchemical_window(1, n_beads=4),
               synth.alchemical_window(6, n_beads=8)]
    systems[0].lambda_vdw = 0.4
    say("group", [s.n_atoms for s in systems], [s.n_beads for s in systems])
    ref = []
    for s in systems:
        with ctx_for(s, precision=prec) as c:
            c.set_state(s.pos, s.vel, 0)
            c.step(6)
            ref.append(c.get_state())
    ctxs = [ctx_for(s, precision=prec) for s in systems]
    try:
        for c, s in zip(ctxs, systems):
            c.set_state(s.pos, s.vel, 0)
        with q.Group(ctxs) as g:
            g.step(2)
            g.step(4)
        got = [c.get_state() for c in ctxs]
    finally:
        for c in ctxs:
            c.close()
    for (x, v, st), (xr, vr, sr) in zip(got, ref):
        assert st == sr == 6
        assert np.abs(x - xr).max() <= tol * np.abs(xr).max()
        assert np.abs(v - vr).max() <= 100 * tol * np.abs(vr).max()


def test_group_picks_up_a_change_of_coupling():
    import paper_2212_03137_amd as q
    s = synth.alchemical_window(2, n_beads=4)
    with ctx_for(s) as a, ctx_for(s) as b:
        a.set_state(s.pos, s.vel, 0)
        b.set_state(s.pos, s.vel, 0)
        with q.Group([a]) as g:
            g.step(2)
            a.set_lambda(0.2, 0.9)
            g.step(2)
        b.step(2)
        b.set_lambda(0.2, 0.9)
        b.step(2)
        xa, _, _ = a.get_state()
        xb, _, _ = b.get_state()
    assert np.abs(xa - xb).max() <= 1e-12 * np.abs(xb).max()


def test_full_size_window_on_sampled_beads():
    # the largest window of the workload (2,048 waters + solute, 6,156 atoms), P = 16, at an
    # intermediate coupling, in the precision the benchmark uses; the oracle on two beads
    import paper_2212_03137_amd as q
    s = synth.alchemical_window(7)
    say("full-size window", s.n_atoms, s.n_beads, s.lambda_elec, s.lambda_vdw)
    with ctx_for(s, precision=q.FP32_PAIRS) as c:
        E, F = c.eval(s.pos)
    for b in (0, s.n_beads - 1):
        Er, Fr = forces.evaluate(s.pos[b:b + 1], s)
        assert rel_rms(F[b], Fr[0]) <= 1e-5
        assert np.allclose(E[b], Er[0], rtol=1e-5, atol=1e-4 * np.abs(Er).max())


def test_autotune_keeps_results_and_the_state(medium):
    # the chosen spreading tile changes only the order of FP64 additions; the propagated
    # state is untouched by the timing runs
    with ctx_for(medium) as c:
        c.set_state(medium.pos, medium.vel, 0)
        E0, F0 = c.eval(medium.pos)
        x0, v0, _ = c.get_state()
        gb, zt, nb, w = c.autotune(3)
        x1, v1, _ = c.get_state()
        E1, F1 = c.eval(medium.pos)
        c.step(2)
    say("autotuned spread block", gb, zt, "fft slots", nb, "pair atoms", w)
    assert w in (0, 2, 4, 8)
    assert nb in (-1, 1, 2)                            # 4 beads: two complex slots
    assert gb in (1, 2, 4) and gb <= medium.n_beads
    assert zt in (1, 2, 4) and gb * zt <= 16          # 32^3 grid: four 8^3 tiles along z
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    assert rel_max(F1, F0) <= 1e-13
    assert np.allclose(E1, E0, rtol=1e-13, atol=1e-10)


def test_bar_inputs_and_estimate_match_the_oracle(small):
    # two neighbouring windows of the small box: configurations sampled by the HIP path,
    # the energy differences U_B - U_A (bead-averaged for PI-BAR, bead 0 for the single-bead
    # estimator) from qhp_eval_lambda against the oracle's on the same configurations, and
    # the library's BAR against the oracle's on them
    import paper_2212_03137_amd as q
    from oracle import bar as obar
    lam_a, lam_b = (0.0, 0.6), (0.0, 0.8)
    samples = {}
    for lam in (lam_a, lam_b):
        s = dataclasses.replace(small, lambda_elec=lam[0], lambda_vdw=lam[1])
        xs = []
        with ctx_for(s) as c:
            c.set_state(s.pos, s.vel, 0)
            for _ in range(4):
                c.step(5)
                xs.append(c.get_state()[0])
            E = {k: [c.eval_lambda(x, *l, forces=False)[0].sum(axis=1) for x in xs]
                 for k, l in (("a", lam_a), ("b", lam_b))}
        samples[lam] = (xs, E)
    beta = 1.0 / small.kT
    for est in ("pi", "single"):
        du = []
        du_ref = []
        for lam in (lam_a, lam_b):
            xs, E = samples[lam]
            Ea, Eb = np.array(E["a"]), np.array(E["b"])       # [samples][P]
            sa = dataclasses.replace(small, lambda_elec=lam_a[0], lambda_vdw=lam_a[1])
            sb = dataclasses.replace(small, lambda_elec=lam_b[0], lambda_vdw=lam_b[1])
            Era = np.array([forces.evaluate(x, sa)[0].sum(axis=1) for x in xs])
            Erb = np.array([forces.evaluate(x, sb)[0].sum(axis=1) for x in xs])
            pick = (lambda E: E.mean(axis=1)) if est == "pi" else (lambda E: E[:, 0])
            du.append(pick(Eb) - pick(Ea))
            du_ref.append(pick(Erb) - pick(Era))
        scale = max(1.0, float(np.abs(du_ref[0]).max()))
        assert np.abs(du[0] - du_ref[0]).max() <= 1e-9 * scale
        assert np.abs(du[1] - du_ref[1]).max() <= 1e-9 * scale
        dF, _ = q.bar(du[0], du[1], beta)
        dF_ref, _ = obar.bar(du_ref[0], du_ref[1], beta)
        say("BAR", est, dF, dF_ref)
        assert dF == pytest.approx(dF_ref, abs=1e-8 * max(1.0, abs(dF_ref)))
