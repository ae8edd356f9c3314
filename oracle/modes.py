"""Perturbed densities of normal modes (Section 4.2, Applications).

TEST INFRASTRUCTURE (CPU oracle).

For an eigenpair (omega_l; u^l, v^l) around the ground state Phi and an amplitude eps,
    n_j^l(x, t) = | phi_j(x) + eps (u_j^l(x) e^{-i omega_l t} + conj(v_j^l(x)) e^{i omega_l t}) |^2,
j = 1, 0, -1: the density of the condensate displaced along the mode (the perturbation ansatz
of Section 2.1 evaluated at time t).

Pins (tests): eps = 0 gives |phi_j|^2; for real u, v, phi the closed form
(phi + eps (u + v) cos wt)^2 + (eps (u - v) sin wt)^2; period 2 pi / omega.
"""
from __future__ import annotations

import numpy as np


def perturbed_density(phi, uv, omega, eps, t):
    """phi (3, *grid) real or complex; uv (nmodes, 6, *grid) complex (u then v); omega (nmodes,);
    t (nt,).  Returns (nmodes, nt, 3, *grid) float64."""
    phi = np.asarray(phi)
    uv = np.asarray(uv, dtype=np.complex128)
    omega = np.asarray(omega, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    out = np.empty((len(omega), len(t)) + phi.shape, dtype=np.float64)
    for l, w in enumerate(omega):
        u, v = uv[l, :3], uv[l, 3:]
        for s, ts in enumerate(t):
            field = phi + eps * (u * np.exp(-1j * w * ts) + np.conj(v) * np.exp(1j * w * ts))
            out[l, s] = np.abs(field) ** 2
    return out
