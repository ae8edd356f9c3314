"""Ground state of the spin-1 condensate (Section 1: eqs. groundDef, NLEP, chem-formula).

TEST INFRASTRUCTURE (CPU oracle).

The ground state is the constrained energy minimiser on
    S_M = { ||Phi||^2 = mass, ||phi_1||^2 - ||phi_-1||^2 = M * mass }.
The paper precomputes it with an external PCG method whose steps it does not give;
this oracle uses a normalized gradient flow whose fixed point satisfies the
Euler-Lagrange problem H(Phi) Phi = Lambda Phi exactly:

  1. r = H(Phi) Phi - mu Phi - lambda S_z Phi, with (mu, lambda) the least-squares
     multipliers (r orthogonal to Phi and to S_z Phi), so Lambda = diag(mu+lambda, mu,
     mu-lambda) and mu_1 + mu_-1 = 2 mu_0 (the relation stated after chem-formula);
  2. Phi <- Phi - tau * P r, with P = (|k|^2/2 + alpha)^-1 applied in Fourier space;
  3. rescale the three components by sigma_1, sigma_0, sigma_-1 so that the mass and the
     magnetization are met and sigma_1 sigma_-1 = sigma_0^2 (normalization step of the
     normalized-gradient-flow literature the paper cites; closed form derived below);
  4. stop when ||r|| <= tol * mass^(1/2).

Real fields throughout (the paper takes the ground state real).  When phi_0 == 0
initially (polar / antiferromagnetic start) the flow keeps it zero and mu_0 is
defined as (mu_1 + mu_-1)/2.

Pins (tests): for beta_s < 0 the result equals a * phi with phi the scalar ground state
of coupling beta_n + beta_s (SMA lemma) and mu_1 = mu_0 = mu_-1; for beta_s > 0 and
M = 0 it equals (phi, 0, phi)/sqrt(2) with phi the scalar ground state of coupling
beta_n; the scalar ground state of a uniform box is the constant state; the residual,
mass and magnetization are checked directly; the chem-formula quotients agree with
mu +- lambda.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import spectral, spin


@dataclasses.dataclass
class GroundState:
    phi: np.ndarray          # (3, *grid) real
    mu: np.ndarray           # (mu_1, mu_0, mu_-1)
    residual: float
    iters: int
    energy: float


def normalization_factors(a1, a0, am, M):
    """sigma_1, sigma_0, sigma_-1 solving
         s1^2 a1 + s0^2 a0 + sm^2 am = 1,  s1^2 a1 - sm^2 am = M,  s1 sm = s0^2.
    With s = s0^2 the conditions reduce to (a0^2 - 4 a1 am) s^2 - 2 a0 s + (1 - M^2) = 0;
    the positive root is s = (1 - M^2) / (a0 + sqrt(a0^2 M^2 + 4 a1 am (1 - M^2))).
    """
    s = (1.0 - M * M) / (a0 + np.sqrt(a0 * a0 * M * M + 4.0 * a1 * am * (1.0 - M * M)))
    s1 = np.sqrt((1.0 - s * a0 + M) / (2.0 * a1))
    sm = np.sqrt((1.0 - s * a0 - M) / (2.0 * am))
    return s1, np.sqrt(s), sm


def _normalize(phi, h, mass, M):
    hd = np.prod(h)
    a = hd * np.sum(phi * phi, axis=tuple(range(1, phi.ndim))) / mass
    s1, s0, sm = normalization_factors(a[0], a[1], a[2], M)
    out = phi.copy()
    out[0] *= s1
    out[1] *= s0
    out[2] *= sm
    return out


def _rhs(phi, V, beta_n, beta_s, n, L):
    return np.real(spin.gpe_rhs_explicit(phi.astype(np.complex128), V, beta_n, beta_s, n, L))


def multipliers(phi, hphi, h):
    """Least-squares (mu, lambda) with r = H Phi - mu Phi - lambda S_z Phi orthogonal to
    Phi and S_z Phi."""
    hd = np.prod(h)
    szphi = np.stack([phi[0], np.zeros_like(phi[1]), -phi[2]])
    basis = [phi, szphi]
    G = np.array([[hd * np.sum(p * q) for q in basis] for p in basis])
    rhs = np.array([hd * np.sum(p * hphi) for p in basis])
    coef, *_ = np.linalg.lstsq(G, rhs, rcond=1e-14)
    return coef[0], coef[1], szphi


def ground_state(V, beta_n, beta_s, mass, M, n, L, phi0, tol=1e-12, max_iter=400000,
                 tau=None, alpha=None) -> GroundState:
    """Normalized gradient flow of the module header; phi0 is the (3, *grid) start."""
    h = tuple(2.0 * Li / ni for ni, Li in zip(n, L))
    d = len(n)
    axes = tuple(range(-d, 0))
    sym = spectral.kinetic_symbol(n, L)
    if alpha is None:
        alpha = float(np.max(V)) + 1.0
    if tau is None:
        tau = 1.0
    P = 1.0 / (sym + alpha)
    phi = _normalize(np.asarray(phi0, dtype=np.float64), h, mass, M)
    res = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        hphi = _rhs(phi, V, beta_n, beta_s, n, L)
        mu, lam, szphi = multipliers(phi, hphi, h)
        r = hphi - mu * phi - lam * szphi
        res = spectral.norm(r, h) / np.sqrt(mass)
        if res <= tol:
            break
        step = np.real(spectral.ifftn(P * spectral.fftn(r, axes=axes), axes=axes))
        phi = _normalize(phi - tau * step, h, mass, M)
    mus = np.array([mu + lam, mu, mu - lam])
    E = spin.energy(phi, V, beta_n, beta_s, n, L, h)
    return GroundState(phi=phi, mu=mus, residual=float(res), iters=it, energy=E)


def scalar_ground_state(V, g, n, L, phi0=None, tol=1e-12, max_iter=400000, tau=1.0,
                        alpha=None):
    """Scalar GP ground state: -1/2 Lap phi + V phi + g phi^3 = mu phi, ||phi|| = 1,
    by the same preconditioned normalized flow (one component, plain rescaling).
    Returns (phi, mu, residual, iters)."""
    h = tuple(2.0 * Li / ni for ni, Li in zip(n, L))
    d = len(n)
    axes = tuple(range(-d, 0))
    hd = np.prod(h)
    sym = spectral.kinetic_symbol(n, L)
    if alpha is None:
        alpha = float(np.max(V)) + 1.0
    P = 1.0 / (sym + alpha)
    phi = np.ones(V.shape) if phi0 is None else np.asarray(phi0, dtype=np.float64).copy()
    phi /= np.sqrt(hd * np.sum(phi * phi))
    res = np.inf
    it = 0
    mu = 0.0
    for it in range(1, max_iter + 1):
        hphi = np.real(spectral.kinetic_apply(phi, n, L)) + (V + g * phi * phi) * phi
        mu = hd * np.sum(phi * hphi)
        r = hphi - mu * phi
        res = np.sqrt(hd * np.sum(r * r))
        if res <= tol:
            break
        phi = phi - tau * np.real(spectral.ifftn(P * spectral.fftn(r, axes=axes), axes=axes))
        phi /= np.sqrt(hd * np.sum(phi * phi))
    return phi, float(mu), float(res), it


def chemical_potentials_quotient(phi, V, beta_n, beta_s, n, L, h):
    """mu_j = <phi_j, (H Phi)_j> / ||phi_j||^2 (eq. chem-formula); NaN where phi_j == 0."""
    hphi = _rhs(phi, V, beta_n, beta_s, n, L)
    out = []
    for j in range(3):
        nj = np.sum(phi[j] * phi[j])
        out.append(np.sum(phi[j] * hphi[j]) / nj if nj > 0 else np.nan)
    return np.array(out)
