"""Complex ground states for the general BdG form (Section 2.1, the matrix form
[[A, B], [-conj(B), -conj(A)]] with complex Hermitian A and complex symmetric B).

TEST INFRASTRUCTURE (CPU oracle).

The paper's experiments use real ground states; the general form of Section 2.1 covers
complex ones (vortex or moving states).  Two families of exact complex stationary states
serve as inputs with known spectra:

  * a real ground state turned by a global phase and a spin rotation about z,
    Phi_c = e^{i theta} e^{-i alpha S_z} Phi.  The energy and the constraints are invariant
    and Lambda = mu + lambda S_z commutes with S_z, so the BdG spectrum equals that of Phi;
  * the uniform polar state moving with momentum q along x on the periodic box,
    Phi = e^{i q x} (1, 0, 1) sqrt(nbar / 2).  Its chemical potential grows by q^2 / 2 and,
    by Galilean invariance, every Bogoliubov branch is Doppler shifted:
    omega(k) = omega_0(k) + q k_x with omega_0 the branches of the state at rest
    (sqrt(eps (eps + 2 beta_n nbar)) and twice sqrt(eps (eps + 2 beta_s nbar)),
    eps = |k|^2 / 2).  Below the smaller sound speed sqrt(beta_s nbar) every shifted
    frequency stays positive.

Pins (tests): the rotated state's dense spectrum equals the real state's; the moving state
satisfies the stationary equation and its dense spectrum equals the Doppler closed form.
"""
from __future__ import annotations

import numpy as np

from . import branch, spectral


def rotate(phi, alpha, theta):
    """e^{i theta} e^{-i alpha S_z} Phi for a (3, *grid) spinor (S_z = diag(1, 0, -1))."""
    phi = np.asarray(phi, dtype=np.complex128)
    m = np.array([1.0, 0.0, -1.0]).reshape((3,) + (1,) * (phi.ndim - 1))
    return np.exp(1j * theta) * np.exp(-1j * alpha * m) * phi


def moving_polar_state(n, L, beta_n, q_index):
    """Uniform polar state (mass 1, M = 0) moving with q = pi q_index / L_x along x; returns
    (Phi complex (3, *grid), mu (3,), q)."""
    phi0, mu0 = branch.uniform_ground_state(n, L, beta_n, 1.0, 0.0, "polar")
    q = np.pi * q_index / L[0]
    x = -L[0] + np.arange(n[0]) * (2.0 * L[0] / n[0])
    shape = [1] * len(n)
    shape[len(n) - 1] = n[0]
    phase = np.exp(1j * q * x).reshape(shape)
    return phi0 * phase[None], mu0 + 0.5 * q * q, q


def moving_polar_spectrum(n, L, beta_n, beta_s, q, k):
    """k smallest positive frequencies of the moving polar state: the branches at rest,
    Doppler shifted by q k_x on every grid wavevector k != 0."""
    vol = float(np.prod([2.0 * Li for Li in L]))
    nbar = 1.0 / vol
    mus = [spectral.wavenumbers(ni, Li) for ni, Li in zip(n, L)]
    grids = np.meshgrid(*reversed(mus), indexing="ij")        # (z, y, x) order
    kx = np.ravel(grids[-1])
    eps = np.ravel(spectral.kinetic_symbol(n, L))
    nz = eps > 0
    kx, eps = kx[nz], eps[nz]
    dens = np.sqrt(eps * (eps + 2 * beta_n * nbar)) + q * kx
    spin = np.sqrt(eps * (eps + 2 * beta_s * nbar)) + q * kx
    vals = np.sort(np.concatenate([dens, spin, spin]))
    vals = vals[vals > 0]
    return vals[:k]
