"""Exact scalar branch decompositions of the BdG spectrum and the uniform-state dispersion.

TEST INFRASTRUCTURE (CPU oracle).  These are closed forms derived from the structure
results of Section 2.3; they use only scalar operators, so they are an independent
formulation of the same spectrum as the six-component operator of ``bdg``.

Ferromagnetic, single-mode ground state (SMA lemma; beta_s < 0, beta_n + beta_s >= 0):
Phi = a phi with phi the scalar ground state of coupling g = beta_n + beta_s and
mu_1 = mu_0 = mu_-1 = mu.  With h_0 = L - mu + g phi^2 (h_0 phi = 0),
h_2 = L - mu + (beta_n - beta_s) phi^2 and h_3 = L - mu + 3 g phi^2, the spin basis
W = [a, b, c] of the nullspace theorem turns H_- into diag(h_0, h_0, h_2) (the
paper's K) and H_+ into diag(h_3, h_0, h_2), so the positive spectrum is
    sqrt(eig(h_0 h_3))  U  eig(h_0) minus {0}  U  eig(h_2).

Polar ground state at M = 0 (two-component lemma; beta_s > 0): Phi = (phi, 0, phi)/sqrt 2
with phi the scalar ground state of coupling beta_n.  With h_0 = L - mu + beta_n phi^2,
h_s = h_0 + 2 beta_s phi^2 and h_3 = h_0 + 2 beta_n phi^2, in the basis
e_+ = (1,0,1)/sqrt2, e_0, e_- = (1,0,-1)/sqrt2:  H_- = diag(h_0, h_0, h_0) and
H_+ = diag(h_3, h_s, h_s), so the positive spectrum is
    sqrt(eig(h_0 h_3))  U  sqrt(eig(h_0 h_s)) (twice).

Uniform state (V = 0, periodic box of volume |D|, nbar = 1/|D|, eps = |k|^2/2 on the DFT
grid): FM  {sqrt(eps (eps + 2 g nbar)), eps, eps - 2 beta_s nbar};
polar  {sqrt(eps (eps + 2 beta_n nbar)), sqrt(eps (eps + 2 beta_s nbar)) twice}.
"""
from __future__ import annotations

import numpy as np

from . import spectral


def _scalar_dense(pot, n, L):
    """Dense scalar operator -Lap/2 + diag(pot)."""
    return spectral.kinetic_matrix(n, L) + np.diag(np.ravel(pot))


def _sqrt_psd(M):
    w, Q = np.linalg.eigh(M)
    return (Q * np.sqrt(np.clip(w, 0.0, None))) @ Q.T


def _lrep_scalar_dense(h0, h3, zero_tol=1e-9):
    """Positive square roots of eig(h0 h3) for symmetric h0 (PSD) and h3 (SPD); the
    zero modes (omega^2 <= zero_tol * max omega^2) are returned as exact zeros."""
    S = _sqrt_psd(h3)
    w = np.linalg.eigvalsh(S @ h0 @ S)
    w = np.where(w > zero_tol * np.max(np.abs(w)), w, 0.0)
    return np.sqrt(w)


def fm_branches_dense(phi, mu, V, beta_n, beta_s, n, L):
    """Three branch spectra (each sorted) of the FM-SMA decomposition, dense."""
    g = beta_n + beta_s
    p2 = np.ravel(phi) ** 2
    base = np.ravel(V) - mu
    h0 = _scalar_dense(base + g * p2, n, L)
    h2 = _scalar_dense(base + (beta_n - beta_s) * p2, n, L)
    h3 = _scalar_dense(base + 3.0 * g * p2, n, L)
    density_branch = np.sort(_lrep_scalar_dense(h0, h3))
    magnon = np.sort(np.linalg.eigvalsh(h0))
    gapped = np.sort(np.linalg.eigvalsh(h2))
    return density_branch, magnon, gapped


def polar_branches_dense(phi, mu, V, beta_n, beta_s, n, L):
    """Density branch and (doubly counted) spin branch of the polar M = 0 decomposition."""
    p2 = np.ravel(phi) ** 2
    base = np.ravel(V) - mu
    h0 = _scalar_dense(base + beta_n * p2, n, L)
    hs = _scalar_dense(base + (beta_n + 2.0 * beta_s) * p2, n, L)
    h3 = _scalar_dense(base + 3.0 * beta_n * p2, n, L)
    return np.sort(_lrep_scalar_dense(h0, h3)), np.sort(_lrep_scalar_dense(h0, hs))


def lowest_positive(values_with_mult, k, zero_tol=1e-7):
    """Merge branch spectra (list of (values, multiplicity)) and return the k smallest
    strictly positive values."""
    allv = []
    for vals, mult in values_with_mult:
        v = np.asarray(vals)
        v = v[v > zero_tol]
        allv.extend(list(v) * mult)
    return np.sort(np.array(allv))[:k]


def fm_spectrum_dense(phi, mu, V, beta_n, beta_s, n, L, k):
    dens, mag, gap = fm_branches_dense(phi, mu, V, beta_n, beta_s, n, L)
    return lowest_positive([(dens, 1), (mag, 1), (gap, 1)], k)


def polar_spectrum_dense(phi, mu, V, beta_n, beta_s, n, L, k):
    dens, spin = polar_branches_dense(phi, mu, V, beta_n, beta_s, n, L)
    return lowest_positive([(dens, 1), (spin, 2)], k)


def uniform_spectrum(n, L, beta_n, beta_s, kind, k):
    """k smallest positive BdG frequencies of the uniform state (V = 0), mass 1."""
    vol = float(np.prod([2.0 * Li for Li in L]))
    nbar = 1.0 / vol
    eps = np.ravel(spectral.kinetic_symbol(n, L))
    eps = eps[eps > 0]
    if kind == "fm":
        g = beta_n + beta_s
        vals = [(np.sqrt(eps * (eps + 2 * g * nbar)), 1), (eps, 1), (eps - 2 * beta_s * nbar, 1)]
        # the k = 0 gapped mode of the transverse spin branch is -2 beta_s nbar > 0
        vals.append((np.array([-2 * beta_s * nbar]), 1))
    elif kind == "polar":
        vals = [(np.sqrt(eps * (eps + 2 * beta_n * nbar)), 1),
                (np.sqrt(eps * (eps + 2 * beta_s * nbar)), 2)]
    else:
        raise ValueError(kind)
    return lowest_positive(vals, k, zero_tol=0.0)


def uniform_ground_state(n, L, beta_n, beta_s, M, kind):
    """Uniform ground state of mass 1 with (mu_1, mu_0, mu_-1): FM a*sqrt(nbar), polar
    (sqrt((1+M)/2), 0, sqrt((1-M)/2)) sqrt(nbar)."""
    vol = float(np.prod([2.0 * Li for Li in L]))
    nbar = 1.0 / vol
    shape = tuple(reversed(n))
    one = np.ones(shape)
    if kind == "fm":
        a = np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2])
        mu = (beta_n + beta_s) * nbar
        return np.stack([ai * np.sqrt(nbar) * one for ai in a]), np.array([mu, mu, mu])
    if kind == "polar":
        if M != 0.0:
            raise ValueError("uniform polar state is tabulated for M = 0 only")
        a = np.array([np.sqrt(0.5), 0.0, np.sqrt(0.5)])
        mu = beta_n * nbar
        return np.stack([ai * np.sqrt(nbar) * one for ai in a]), np.array([mu, mu, mu])
    raise ValueError(kind)
