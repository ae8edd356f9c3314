"""Analytical Kohn eigenpairs of the harmonic trap and the accuracy measures of Section 4.1.

TEST INFRASTRUCTURE (CPU oracle).

For the harmonic trap of eq. (Vpoten), V = sum_a gamma_a^2 x_a^2 / 2, and any real ground
state Phi, the theorem "Analytical eigenpairs" (Section 2.3) gives for every axis a
    omega_a = gamma_a,
    u_a = (gamma_a^{-1/2} d_a Phi - gamma_a^{1/2} x_a Phi) / sqrt 2,
    v_a = (gamma_a^{-1/2} d_a Phi + gamma_a^{1/2} x_a Phi) / sqrt 2,
equivalently f = gamma^{-1/2} d_a Phi / sqrt 2, g = -gamma^{1/2} x_a Phi / sqrt 2 with
<f, g> = 1/4 when |Phi|^2 integrates to one.  On the grid d_a is the Fourier spectral
derivative; the Nyquist mode of a first derivative is dropped so a real field stays real.

Section 4.1 measures a computed pair (omega_N, u_N, v_N) against it by
    e_omega = |omega_N - omega| / |omega|,
    e_uv = |u_N - P_u u_N| / |u_N| + |v_N - P_v v_N| / |v_N|,
where P_u, P_v are the l2-orthogonal projections onto the span of the analytical u (resp. v)
of every axis sharing the eigenvalue (the multiplicity of omega).  The computed pair for
axis a is the not-yet-used computed mode nearest to gamma_a (reading: the paper does not
say how computed modes are matched to axes).

Pins (tests): the analytical pair is an eigenpair of the discrete operator to the
discretization error; <f, g> = 1/4; the 1-D errors reproduce the paper's Table Err_1D.
"""
from __future__ import annotations

import numpy as np

from . import spectral


def derivative(F: np.ndarray, n, L, axis: int) -> np.ndarray:
    """Spectral d/dx_axis of real grid fields F (last len(n) axes are the grid, x last),
    Nyquist mode dropped."""
    ax = F.ndim - 1 - axis
    mu = spectral.wavenumbers(n[axis], L[axis]).copy()
    mu[n[axis] // 2] = 0.0
    shape = [1] * F.ndim
    shape[ax] = n[axis]
    return np.real(np.fft.ifft(1j * mu.reshape(shape) * np.fft.fft(F, axis=ax), axis=ax))


def coordinate(n, L, axis: int) -> np.ndarray:
    """x_axis on the grid x_j = -L + j h, shaped to broadcast against (3, *grid)."""
    x = -L[axis] + np.arange(n[axis]) * (2.0 * L[axis] / n[axis])
    shape = [1] * len(n)
    shape[len(n) - 1 - axis] = n[axis]
    return x.reshape(shape)


def kohn_pair(phi: np.ndarray, n, L, gammas, axis: int):
    """(omega, u, v) of the theorem "Analytical eigenpairs" for one axis; u, v shaped like phi."""
    g = float(gammas[axis])
    dphi = derivative(phi, n, L, axis)
    xphi = coordinate(n, L, axis)[None] * phi
    u = (g ** -0.5 * dphi - g ** 0.5 * xphi) / np.sqrt(2.0)
    v = (g ** -0.5 * dphi + g ** 0.5 * xphi) / np.sqrt(2.0)
    return g, u, v


def _orth(vectors):
    q, _ = np.linalg.qr(np.array([x.ravel() for x in vectors]).T)
    return q


def accuracy_errors(omega, uv, phi, n, L, gammas):
    """e_omega and e_uv of Section 4.1 for every axis.  omega: computed eigenvalues; uv: computed
    (u, v) vectors, shape (k, 6, *grid).  Returns a list of dicts, one per axis."""
    omega = np.asarray(omega, dtype=float)
    used, out = set(), []
    for a, g in enumerate(gammas):
        axes = [b for b, gb in enumerate(gammas) if gb == g]
        pairs = [kohn_pair(phi, n, L, gammas, b) for b in axes]
        Qu = _orth([p[1] for p in pairs])
        Qv = _orth([p[2] for p in pairs])
        j = next(int(i) for i in np.argsort(np.abs(omega - g), kind="stable") if int(i) not in used)
        used.add(j)
        u, v = uv[j, :3].ravel(), uv[j, 3:].ravel()
        eu = np.linalg.norm(u - Qu @ (Qu.T @ u)) / np.linalg.norm(u)
        ev = np.linalg.norm(v - Qv @ (Qv.T @ v)) / np.linalg.norm(v)
        out.append({"axis": "xyz"[a], "omega": float(omega[j]), "e_omega": abs(omega[j] - g) / abs(g),
                    "e_uv": float(eu + ev)})
    return out
