"""Pins of the oracle ground state: constraints, Euler-Lagrange residual, SMA and
two-component structure (Section 2.3 lemmas), chem-formula, uniform state."""
import numpy as np
import pytest

import workloads as W
from oracle import groundstate as gs, spin, spectral
from tests import _cases


def test_normalization_factors_meet_three_conditions():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a1, a0, am = rng.uniform(0.05, 1.0, 3)
        M = rng.uniform(-0.6, 0.6)
        s1, s0, sm = gs.normalization_factors(a1, a0, am, M)
        assert abs(s1 ** 2 * a1 + s0 ** 2 * a0 + sm ** 2 * am - 1) < 1e-13
        assert abs(s1 ** 2 * a1 - sm ** 2 * am - M) < 1e-13
        assert abs(s1 * sm - s0 ** 2) < 1e-13


def test_normalization_is_identity_at_sma_masses():
    for M in (-0.3, 0.0, 0.2, 0.7):
        a = np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2]) ** 2
        assert np.allclose(gs.normalization_factors(*a, M), 1.0, atol=1e-14)


def test_c1_ground_state_constraints_and_residual():
    w, V, r, _ = _cases.ground(_cases.C1)
    h = w.h
    assert r.residual <= 1e-12
    assert abs(spin.mass(r.phi, h) - 1) < 1e-13
    assert abs(spin.magnetization(r.phi, h) - w.magnetization) < 1e-13
    # independent residual: explicit GPE minus Lambda Phi
    hphi = np.real(spin.gpe_rhs_compact(r.phi.astype(complex), V, w.beta_n, w.beta_s, w.n, w.L))
    res = hphi - r.mu[:, None] * r.phi
    assert spectral.norm(res, h) < 2e-12


def test_fm_ground_state_is_single_mode():
    """SMA lemma: Phi = a phi_g with phi_g the scalar ground state of coupling
    beta_n + beta_s, and mu_1 = mu_0 = mu_-1."""
    w, V, r, _ = _cases.ground(_cases.C1)
    M = w.magnetization
    a = np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2])
    phi, mu, res, _ = gs.scalar_ground_state(V, w.beta_n + w.beta_s, w.n, w.L,
                                             phi0=np.exp(-0.5 * W.coordinates(w)[0] ** 2))
    assert res < 1e-12
    assert np.abs(r.phi - a[:, None] * phi[None]).max() < 1e-10
    assert np.allclose(r.mu, mu, atol=1e-10)


def test_polar_ground_state_is_two_component():
    """Two-component lemma at M = 0: Phi = (phi, 0, phi)/sqrt(2), phi the scalar ground
    state of coupling beta_n."""
    w, V, r, _ = _cases.ground(_cases.POLAR_1D)
    phi, mu, res, _ = gs.scalar_ground_state(V, w.beta_n, w.n, w.L,
                                             phi0=np.exp(-0.5 * W.coordinates(w)[0] ** 2))
    assert np.abs(r.phi[1]).max() == 0.0
    assert np.abs(r.phi[0] - phi / np.sqrt(2)).max() < 1e-10
    assert np.abs(r.phi[2] - phi / np.sqrt(2)).max() < 1e-10
    assert np.allclose(r.mu, mu, atol=1e-10)


def test_chem_formula_agrees_with_multipliers():
    for case in (_cases.C1, _cases.AFM_1D):
        w, V, r, _ = _cases.ground(case)
        q = gs.chemical_potentials_quotient(r.phi, V, w.beta_n, w.beta_s, w.n, w.L, w.h)
        ok = ~np.isnan(q)
        assert np.allclose(q[ok], r.mu[ok], atol=1e-10)
        assert abs(r.mu[0] + r.mu[2] - 2 * r.mu[1]) < 1e-12


def test_afm_magnetized_ground_state_two_components_distinct_mu():
    w, V, r, _ = _cases.ground(_cases.AFM_1D)
    assert np.abs(r.phi[1]).max() == 0.0
    assert abs(spin.magnetization(r.phi, w.h) - 0.3) < 1e-13
    assert r.mu[0] != pytest.approx(r.mu[2], abs=1e-6)


def test_uniform_box_flows_to_constant_state():
    w = W.Workload("u", 1, (32,), (4.0,), "zero", 5.0, -1.0, 0.2)
    V = W.potential(w)
    x = W.coordinates(w)[0]
    start = W.initial_spinor_weights(w)[:, None] * (1 + 0.3 * np.cos(np.pi * (x + 4) / 4))[None]
    r = gs.ground_state(V, w.beta_n, w.beta_s, 1.0, w.magnetization, w.n, w.L, start, tol=1e-12)
    nbar = 1 / 8.0
    a = W.initial_spinor_weights(w)
    assert np.abs(r.phi - a[:, None] * np.sqrt(nbar)).max() < 1e-11
    assert np.allclose(r.mu, (w.beta_n + w.beta_s) * nbar, atol=1e-11)
