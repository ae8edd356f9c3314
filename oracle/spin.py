"""Spin-1 Gross-Pitaevskii model (Section 1: GPE, spin matrices, conserved quantities).

TEST INFRASTRUCTURE (CPU oracle).

A spinor Psi = (psi_1, psi_0, psi_-1) is an array of shape (3, *grid).  Two independent
writings of the GPE right-hand side are kept: the explicit component form of eq. (GPE)
and the compact form ((L + beta_n rho) I + beta_s S.s(Psi)) Psi of eq. (GPEs); the
tests pin one against the other.
"""
from __future__ import annotations

import numpy as np

from . import spectral

SQ2 = np.sqrt(2.0)
S_x = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=np.complex128) / SQ2
S_y = 1j * np.array([[0, -1, 0], [1, 0, -1], [0, 1, 0]], dtype=np.complex128) / SQ2
S_z = np.diag([1.0, 0.0, -1.0]).astype(np.complex128)
SPIN = (S_x, S_y, S_z)


def mat3(Mx: np.ndarray, Psi: np.ndarray) -> np.ndarray:
    """Apply a constant 3x3 matrix to a spinor field."""
    return np.einsum("ab,b...->a...", Mx, Psi)


def spin_vector(Psi: np.ndarray):
    """s_j(Psi) = Psi^H S_j Psi, j = x, y, z (pointwise; real for any Psi)."""
    return tuple(np.real(np.einsum("a...,ab,b...->...", Psi.conj(), S, Psi)) for S in SPIN)


def density(Psi):
    return np.sum(np.abs(Psi) ** 2, axis=0)


def gpe_rhs_explicit(Psi, V, beta_n, beta_s, n, L):
    """Right-hand side of eq. (GPE), component by component."""
    p1, p0, pm = Psi
    rho = density(Psi)
    rhoz = np.abs(p1) ** 2 - np.abs(pm) ** 2
    kin = spectral.kinetic_apply(Psi, n, L)
    out = np.empty_like(Psi, dtype=np.complex128)
    out[0] = kin[0] + (V + beta_n * rho + beta_s * (np.abs(p0) ** 2 + rhoz)) * p1 \
        + beta_s * p0 * p0 * np.conj(pm)
    out[1] = kin[1] + (V + beta_n * rho + beta_s * (np.abs(p1) ** 2 + np.abs(pm) ** 2)) * p0 \
        + 2.0 * beta_s * pm * np.conj(p0) * p1
    out[2] = kin[2] + (V + beta_n * rho + beta_s * (np.abs(p0) ** 2 - rhoz)) * pm \
        + beta_s * np.conj(p1) * p0 * p0
    return out


def gpe_rhs_compact(Psi, V, beta_n, beta_s, n, L):
    """Right-hand side of eq. (GPEs): ((L + beta_n rho) I_3 + beta_s S.s(Psi)) Psi."""
    rho = density(Psi)
    s = spin_vector(Psi)
    out = spectral.kinetic_apply(Psi, n, L) + (V + beta_n * rho) * Psi
    for S, sj in zip(SPIN, s):
        out = out + beta_s * sj * mat3(S, Psi)
    return out


def mass(Psi, h) -> float:
    return float(np.prod(h) * np.sum(np.abs(Psi) ** 2))


def magnetization(Psi, h) -> float:
    return float(np.prod(h) * (np.sum(np.abs(Psi[0]) ** 2) - np.sum(np.abs(Psi[2]) ** 2)))


def energy(Psi, V, beta_n, beta_s, n, L, h) -> float:
    """Energy functional E(Psi) of Section 1 (kinetic term via <Psi, -1/2 Lap Psi>)."""
    kin = spectral.kinetic_apply(Psi, n, L)
    rho = density(Psi)
    s = spin_vector(Psi)
    s2 = sum(sj * sj for sj in s)
    dens = np.real(np.sum(np.conj(Psi) * kin, axis=0)) + V * rho \
        + 0.5 * beta_n * rho * rho + 0.5 * beta_s * s2
    return float(np.prod(h) * np.sum(dens))
