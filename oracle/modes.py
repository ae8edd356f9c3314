"""Perturbed densities and Bogoliubov-amplitude summaries of normal modes (Section 4.2,
Applications).

TEST INFRASTRUCTURE (CPU oracle).

For an eigenpair (omega_l; u^l, v^l) around the ground state Phi and an amplitude eps,
    n_j^l(x, t) = | phi_j(x) + eps (u_j^l(x) e^{-i omega_l t} + conj(v_j^l(x)) e^{i omega_l t}) |^2,
j = 1, 0, -1: the density of the condensate displaced along the mode (the perturbation ansatz
of Section 2.1 evaluated at time t).

Pins (tests): eps = 0 gives |phi_j|^2; for real u, v, phi the closed form
(phi + eps (u + v) cos wt)^2 + (eps (u - v) sin wt)^2; period 2 pi / omega.

The paper's 3-D example shows isosurfaces of the amplitudes u_j^l, v_j^l of selected modes and
remarks on their symmetry (even or odd under reflections of a symmetric trap) and their
compression along the stiffer trap axis; ``mode_amplitudes`` reduces each amplitude field to
the numbers behind those remarks: its norm and maximum, its second moments along the axes and
its parity under each axis reflection.  Pins (tests): Gaussian-times-polynomial fields whose
norms, moments and parities are known in closed form; invariance under a global phase; the even
and odd parts of a random field.
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


AMPLITUDE_ENTRIES = 8


def mode_amplitudes(uv, n, L):
    """Summaries of every amplitude field w in (u_1, u_0, u_-1, v_1, v_0, v_-1) of each mode;
    uv (nmodes, 6, *grid) complex, grid (Nz, Ny, Nx)[-d:] with x fastest on the points
    x_m = -L + m h.  Returns (nmodes, 6, 8) float64:
      [0]      N = h^d sum |w|^2
      [1]      max |w|
      [2 + a]  h^d sum x_a^2 |w|^2 / N   (a = x, y, z; 0 for axes beyond the dimension)
      [5 + a]  Re h^d sum w(x) conj(w(R_a x)) / N, with R_a the reflection x_a -> -x_a, on the
               grid the index map m -> (N_a - m) mod N_a: +1 for an even field, -1 for an odd
               one (0 for axes beyond the dimension)
    Entries 2..7 are 0 for a field with N = 0."""
    uv = np.asarray(uv, dtype=np.complex128)
    d = len(n)
    h = [2.0 * Li / ni for Li, ni in zip(L, n)]
    hd = float(np.prod(h))
    nm = uv.shape[0]
    out = np.zeros((nm, 6, AMPLITUDE_ENTRIES))
    coords = []
    for a in range(d):
        x = -L[a] + h[a] * np.arange(n[a])
        shape = [1] * d
        shape[d - 1 - a] = n[a]          # coordinate a runs along array axis d - 1 - a
        coords.append(x.reshape(shape))
    for l in range(nm):
        for f in range(6):
            w = uv[l, f]
            a2 = np.abs(w) ** 2
            N = hd * a2.sum()
            out[l, f, 0] = N
            out[l, f, 1] = np.abs(w).max()
            if N == 0.0:
                continue
            for a in range(d):
                out[l, f, 2 + a] = hd * (coords[a] ** 2 * a2).sum() / N
                ax = d - 1 - a
                refl = np.roll(np.flip(w, axis=ax), 1, axis=ax)     # w(R_a x): index m -> (N - m) mod N
                out[l, f, 5 + a] = hd * np.real(w * np.conj(refl)).sum() / N
    return out
