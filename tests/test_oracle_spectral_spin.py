"""Pins of the oracle's discretization and spin-1 algebra against independent facts."""
import numpy as np
import pytest

import workloads as W
from oracle import spectral, spin


@pytest.mark.parametrize("n,L", [((16,), (3.0,)), ((8, 6), (2.0, 3.0)), ((4, 4, 6), (1.0, 2.0, 1.5))])
def test_fft_kinetic_equals_cosine_sum_matrix(n, L):
    rng = np.random.default_rng(3)
    shape = tuple(reversed(n))
    F = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    T = spectral.kinetic_matrix(n, L)
    assert np.allclose(T, T.T, atol=1e-13)
    got = spectral.kinetic_apply(F, n, L).ravel()
    assert np.allclose(got, T @ F.ravel(), rtol=0, atol=1e-12 * np.abs(got).max())


def test_kinetic_exact_on_band_limited_functions():
    # -1/2 d^2/dx^2 of cos(pi m (x+L)/L) is (pi m/L)^2/2 times itself, |m| < N/2
    n, L = 64, 5.0
    x = W.axis_points(n, L)
    for m in (1, 3, 17, 31):
        f = np.cos(np.pi * m * (x + L) / L) + 0.3 * np.sin(np.pi * m * (x + L) / L)
        got = np.real(spectral.kinetic_apply(f, (n,), (L,)))
        assert np.allclose(got, 0.5 * (np.pi * m / L) ** 2 * f, atol=1e-11)
    # the Nyquist mode (-1)^j is an eigenvector with eigenvalue (pi N/(2L))^2/2
    f = (-1.0) ** np.arange(n)
    got = np.real(spectral.kinetic_apply(f, (n,), (L,)))
    assert np.allclose(got, 0.5 * (np.pi * n / (2 * L)) ** 2 * f, atol=1e-10)


def test_wavenumber_order_matches_fft():
    mu = spectral.wavenumbers(8, np.pi)
    assert np.allclose(mu, [0, 1, 2, 3, -4, -3, -2, -1])


def test_spin_matrices_commutation():
    Sx, Sy, Sz = spin.SPIN
    assert np.allclose(Sx @ Sy - Sy @ Sx, 1j * Sz)
    assert np.allclose(Sy @ Sz - Sz @ Sy, 1j * Sx)
    assert np.allclose(Sz @ Sx - Sx @ Sz, 1j * Sy)
    # spin-1 Casimir S^2 = s(s+1) I = 2 I
    assert np.allclose(Sx @ Sx + Sy @ Sy + Sz @ Sz, 2 * np.eye(3))


def test_gpe_compact_equals_explicit_components():
    rng = np.random.default_rng(5)
    n, L = (12, 10), (3.0, 2.5)
    shape = tuple(reversed(n))
    Psi = rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)
    V = rng.standard_normal(shape)
    a = spin.gpe_rhs_explicit(Psi, V, 3.0, -0.7, n, L)
    b = spin.gpe_rhs_compact(Psi, V, 3.0, -0.7, n, L)
    assert np.allclose(a, b, atol=1e-12)


def test_spin_vector_real_ground_state_has_no_y_component():
    rng = np.random.default_rng(6)
    Phi = rng.standard_normal((3, 20))
    sx, sy, sz = spin.spin_vector(Phi.astype(complex))
    assert np.allclose(sy, 0)
    assert np.allclose(sz, Phi[0] ** 2 - Phi[2] ** 2)
    assert np.allclose(sx, np.sqrt(2) * Phi[1] * (Phi[0] + Phi[2]))
