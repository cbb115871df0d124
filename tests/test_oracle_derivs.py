"""Pins for the oracle's parameter gradients and Hessian-vector products."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import derivs, forces


@pytest.fixture(scope="module")
def small():
    s = synth.water_box(27, 2, 10.5, seed=21, cutoff=5.0, ewald_alpha=0.4, pme_grid=16,
                        pme_order=5)
    return s


def total_energy(s, pos=None):
    E, _ = forces.evaluate(s.pos if pos is None else pos, s)
    return E.sum(axis=0)          # per term, summed over beads


COUL = [2, 4, 5, 6]               # real, exclusion, self, reciprocal


def test_charge_gradient_by_central_differences(small):
    s = small
    dq, _, _ = derivs.param_gradients(s.pos, s)
    h = 1e-6
    for a in (0, 1, 2, 40, 80):
        qp, qm = s.charge.copy(), s.charge.copy()
        qp[a] += h
        qm[a] -= h
        ep = total_energy(dataclasses.replace(s, charge=qp)).sum()
        em = total_energy(dataclasses.replace(s, charge=qm)).sum()
        fd = (ep - em) / (2 * h)
        assert fd == pytest.approx(dq[a], rel=1e-6, abs=1e-6)


def test_coulomb_is_homogeneous_of_degree_two_in_the_charges(small):
    # Euler: sum_i q_i dE/dq_i = 2 E_coulomb (every electrostatic term is bilinear in q)
    s = small
    dq, _, _ = derivs.param_gradients(s.pos, s)
    E = total_energy(s)
    assert float(np.dot(s.charge, dq)) == pytest.approx(2.0 * E[COUL].sum(), rel=1e-11)


def test_lj_gradients_by_central_differences_and_euler(small):
    s = small
    _, de, ds = derivs.param_gradients(s.pos, s)
    h = 1e-6
    for arr, g in (("lj_epsilon", de), ("lj_sigma", ds)):
        base = getattr(s, arr)
        for t in range(len(base)):
            if arr == "lj_epsilon" and base[t] == 0.0:
                assert g[t] == 0.0            # unbounded there: reported as 0
                continue
            p, m = base.astype(float).copy(), base.astype(float).copy()
            p[t] += h
            m[t] -= h
            ep = total_energy(dataclasses.replace(s, **{arr: p}))[3]
            em = total_energy(dataclasses.replace(s, **{arr: m}))[3]
            assert (ep - em) / (2 * h) == pytest.approx(g[t], rel=1e-6, abs=1e-8)
    # LJ is homogeneous of degree one in the epsilons
    E = total_energy(s)
    assert float(np.dot(s.lj_epsilon, de)) == pytest.approx(E[3], rel=1e-11)


def test_hvp_of_harmonic_bonds_has_the_closed_form(small):
    # with no charges, no LJ and no angle term, V = sum k/2 (r - r0)^2 over the O-H bonds and
    # the bond Hessian is k [rr^T + (1 - r0/r)(I - rr^T)] acting on u_H - u_O
    s = dataclasses.replace(small, charge=np.zeros_like(small.charge),
                            lj_epsilon=np.zeros_like(small.lj_epsilon), angle_k=0.0)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(s.pos.shape)
    got = derivs.hvp(s.pos, s, u)
    want = np.zeros_like(got)
    for b in range(s.n_beads):
        x = s.pos[b]
        for k in (1, 2):
            d = forces.min_image(x[k::3] - x[0::3], s.box)
            r = np.linalg.norm(d, axis=1)
            rh = d / r[:, None]
            du = u[b][k::3] - u[b][0::3]
            par = np.einsum("ij,ij->i", rh, du)[:, None] * rh
            hu = s.bond_k * (par + (1.0 - s.bond_r0 / r)[:, None] * (du - par))
            want[b][k::3] += hu
            want[b][0::3] -= hu
    assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()


def test_hvp_is_symmetric(small):
    s = small
    rng = np.random.default_rng(6)
    u = rng.standard_normal(s.pos.shape) * 0.1
    v = rng.standard_normal(s.pos.shape) * 0.1
    Hu, Hv = derivs.hvp(s.pos, s, u), derivs.hvp(s.pos, s, v)
    a, b = float(np.sum(v * Hu)), float(np.sum(u * Hv))
    assert a == pytest.approx(b, rel=1e-6)


def test_mixed_derivatives_are_the_directional_derivative_of_the_parameter_gradient(small):
    # d(u . grad E)/d theta: check against the parameter-gradient of u . grad E by central
    # differences in the parameters (the other order of the mixed derivative)
    s = small
    rng = np.random.default_rng(8)
    u = rng.standard_normal(s.pos.shape)
    dq, de, ds = derivs.mixed(s.pos, s, u)

    def u_dot_grad(sys):
        _, F = forces.evaluate(s.pos, sys)
        return -float(np.sum(u * F))

    h = 1e-6
    for a in (0, 5, 41):
        qp, qm = s.charge.copy(), s.charge.copy()
        qp[a] += h
        qm[a] -= h
        fd = (u_dot_grad(dataclasses.replace(s, charge=qp))
              - u_dot_grad(dataclasses.replace(s, charge=qm))) / (2 * h)
        assert fd == pytest.approx(dq[a], rel=1e-5, abs=1e-5)
    for arr, g in (("lj_epsilon", de), ("lj_sigma", ds)):
        base = getattr(s, arr).astype(float)
        p, m = base.copy(), base.copy()
        p[0] += h
        m[0] -= h
        fd = (u_dot_grad(dataclasses.replace(s, **{arr: p}))
              - u_dot_grad(dataclasses.replace(s, **{arr: m}))) / (2 * h)
        assert fd == pytest.approx(g[0], rel=1e-5, abs=1e-6)
