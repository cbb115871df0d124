"""Parity of the HIP path's parameter gradients (and Hessian-vector products) with the FP64
oracle's, through the C ABI."""
import sys

import numpy as np
import pytest

import synth
from helpers import has_gpu, medium_box
from oracle import derivs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ctx_for(s, **kw):
    import paper_2212_03137_amd as q
    return q.Context.from_system(s, **kw)


def _small():
    return synth.water_box(27, 2, 10.5, seed=21, cutoff=5.0, ewald_alpha=0.4, pme_grid=16,
                           pme_order=5)


@pytest.mark.parametrize("which", ["small", "medium"])
def test_parameter_gradients_match_the_oracle(which):
    import paper_2212_03137_amd as q
    s = _small() if which == "small" else medium_box(P=4)
    say("param grad", which, s.n_atoms, s.n_beads)
    dq_r, de_r, ds_r = derivs.param_gradients(s.pos, s)
    # FP32 pairs: r, 1/r, erfc and the exponential of each pair term are FP32 values
    # (relative error ~1e-7 each), summed in FP64 over terms of both signs
    for prec, tol in ((q.FP64, 1e-10), (q.FP32_PAIRS, 1e-5)):
        with ctx_for(s, precision=prec) as c:
            c.set_state(s.pos, s.vel, 0)
            dq, de, ds = c.param_grad(s.pos)
            x, _, _ = c.get_state()
        say("param grad", prec, np.abs(dq - dq_r).max() / np.abs(dq_r).max())
        assert np.abs(dq - dq_r).max() <= tol * np.abs(dq_r).max(), prec
        assert np.allclose(de, de_r, rtol=tol, atol=tol * np.abs(de_r).max())
        assert np.allclose(ds, ds_r, rtol=tol, atol=tol * np.abs(ds_r).max())
        # the propagated state is left alone
        assert np.abs(x - s.pos).max() <= 1e-12 * np.abs(s.pos).max()


@pytest.mark.parametrize("which", ["small", "medium"])
def test_hessian_vector_products_match_the_oracle(which):
    import paper_2212_03137_amd as q
    s = _small() if which == "small" else medium_box(P=4)
    say("hvp", which, s.n_atoms, s.n_beads)
    rng = np.random.default_rng(11)
    u = rng.standard_normal(s.pos.shape)
    ref = derivs.hvp(s.pos, s, u)
    for prec, tol in ((q.FP64, 1e-6), (q.FP32_PAIRS, 1e-5)):
        with ctx_for(s, precision=prec) as c:
            c.set_state(s.pos, s.vel, 0)
            got = c.hvp(s.pos, u)
            x, _, _ = c.get_state()
        # the oracle's central difference carries O(h^2) and rounding errors of ~1e-8
        err = np.abs(got - ref).max() / np.sqrt(np.mean(ref ** 2))
        say("hvp", prec, err)
        assert err <= tol, (prec, err)
        assert np.abs(x - s.pos).max() <= 1e-12 * np.abs(s.pos).max()


def test_hessian_vector_products_are_linear_and_symmetric_at_full_size():
    # properties that hold exactly for the analytic operator at any size
    s = synth.large_rpmd()
    say("hvp large", s.n_atoms, s.n_beads)
    rng = np.random.default_rng(12)
    u = rng.standard_normal(s.pos.shape) * 0.01
    v = rng.standard_normal(s.pos.shape) * 0.01
    with ctx_for(s) as c:
        Hu = c.hvp(s.pos, u)
        Hv = c.hvp(s.pos, v)
        Huv = c.hvp(s.pos, 2.0 * u - 3.0 * v)
    assert np.all(np.isfinite(Hu))
    scale = np.abs(Huv).max()
    assert np.abs(Huv - (2.0 * Hu - 3.0 * Hv)).max() <= 1e-10 * scale
    a, b = float(np.sum(v * Hu)), float(np.sum(u * Hv))
    assert abs(a - b) <= 1e-9 * max(abs(a), abs(b))


def test_hessian_vector_product_on_one_bead_of_the_large_box():
    # the oracle's central difference on one bead of the 4,096-water box
    s = synth.large_rpmd()
    rng = np.random.default_rng(13)
    u = rng.standard_normal(s.pos.shape)
    with ctx_for(s) as c:
        got = c.hvp(s.pos, u)
    b = 7
    ref = derivs.hvp(s.pos, s, u, beads=[b])[b]
    err = np.abs(got[b] - ref).max() / np.sqrt(np.mean(ref ** 2))
    say("hvp large bead", b, err)
    assert err <= 1e-6


def test_torch_autograd_gradients_and_double_backward():
    import torch
    from paper_2212_03137_amd.autograd import bead_energy
    s = _small()
    dev = torch.device("cuda")
    rng = np.random.default_rng(14)
    v = rng.standard_normal(s.pos.shape)
    dq_r, de_r, ds_r = derivs.param_gradients(s.pos, s)
    hv_r = derivs.hvp(s.pos, s, v)
    with ctx_for(s) as c:
        _, F = c.eval(s.pos)
        pos = torch.tensor(s.pos, dtype=torch.float64, device=dev, requires_grad=True)
        q = torch.tensor(s.charge, dtype=torch.float64, device=dev, requires_grad=True)
        eps = torch.tensor(s.lj_epsilon, dtype=torch.float64, device=dev, requires_grad=True)
        sig = torch.tensor(s.lj_sigma, dtype=torch.float64, device=dev, requires_grad=True)
        E = bead_energy(c, pos, q, eps, sig)
        g, gq, ge, gs = torch.autograd.grad(E, (pos, q, eps, sig), create_graph=True)
        hv = torch.autograd.grad((g * torch.tensor(v, device=dev)).sum(), pos)[0]
    assert np.abs(g.detach().cpu().numpy() + F).max() <= 1e-12 * np.abs(F).max()
    assert np.abs(gq.detach().cpu().numpy() - dq_r).max() <= 1e-10 * np.abs(dq_r).max()
    assert np.allclose(ge.detach().cpu().numpy(), de_r, rtol=1e-10, atol=1e-12)
    assert np.allclose(gs.detach().cpu().numpy(), ds_r, rtol=1e-10, atol=1e-12)
    err = np.abs(hv.cpu().numpy() - hv_r).max() / np.sqrt(np.mean(hv_r ** 2))
    assert err <= 1e-6, err


def test_parameter_gradient_of_a_force_loss():
    # loss = mean (F(theta) - F_ref)^2 with F_ref from perturbed charges (the workload's
    # fitting objective): d loss / d theta = -2/n sum r . d(grad E)/d theta, the mixed
    # derivatives along the residual r, against central differences of the oracle's loss
    import dataclasses
    import torch
    from paper_2212_03137_amd.autograd import forces as tforces
    from oracle import forces as ofo
    s = _small()
    rng = np.random.default_rng(15)
    pert = dataclasses.replace(s, charge=s.charge * (1.0 + 0.05 * rng.uniform(-1, 1, s.n_atoms)))
    pert = dataclasses.replace(pert, charge=pert.charge - pert.charge.mean())
    _, F_ref = ofo.evaluate(s.pos, pert)
    dev = torch.device("cuda")
    with ctx_for(s) as c:
        pos = torch.tensor(s.pos, dtype=torch.float64, device=dev, requires_grad=True)
        q = torch.tensor(s.charge, dtype=torch.float64, device=dev, requires_grad=True)
        eps = torch.tensor(s.lj_epsilon, dtype=torch.float64, device=dev, requires_grad=True)
        sig = torch.tensor(s.lj_sigma, dtype=torch.float64, device=dev, requires_grad=True)
        F = tforces(c, pos, q, eps, sig)
        loss = ((F - torch.tensor(F_ref, device=dev)) ** 2).mean()
        gq, ge, gs = torch.autograd.grad(loss, (q, eps, sig))

    def oracle_loss(sys):
        _, Fo = ofo.evaluate(s.pos, sys)
        return float(((Fo - F_ref) ** 2).mean())

    h = 1e-6
    for a in (0, 4, 50):
        qp, qm = s.charge.copy(), s.charge.copy()
        qp[a] += h
        qm[a] -= h
        fd = (oracle_loss(dataclasses.replace(s, charge=qp))
              - oracle_loss(dataclasses.replace(s, charge=qm))) / (2 * h)
        assert fd == pytest.approx(float(gq[a]), rel=1e-5, abs=1e-7)
    for name, g in (("lj_epsilon", ge), ("lj_sigma", gs)):
        base = getattr(s, name).astype(float)
        p, m = base.copy(), base.copy()
        p[0] += h
        m[0] -= h
        fd = (oracle_loss(dataclasses.replace(s, **{name: p}))
              - oracle_loss(dataclasses.replace(s, **{name: m}))) / (2 * h)
        assert fd == pytest.approx(float(g[0]), rel=1e-5, abs=1e-7)


def test_mixed_derivatives_match_the_oracle():
    s = medium_box(P=4)
    rng = np.random.default_rng(16)
    u = rng.standard_normal(s.pos.shape)
    dq_r, de_r, ds_r = derivs.mixed(s.pos, s, u)
    import paper_2212_03137_amd as q
    for prec, tol in ((q.FP64, 1e-6), (q.FP32_PAIRS, 1e-5)):
        with ctx_for(s, precision=prec) as c:
            _, dq, de, ds = c.hvp(s.pos, u, mixed=True)
        say("mixed", prec, np.abs(dq - dq_r).max() / np.abs(dq_r).max())
        assert np.abs(dq - dq_r).max() <= tol * np.abs(dq_r).max(), prec
        assert np.allclose(de, de_r, rtol=tol, atol=1e-2 * tol * np.abs(de_r).max())
        assert np.allclose(ds, ds_r, rtol=tol, atol=1e-2 * tol * np.abs(ds_r).max())
