"""The BdG operator around a ground state (Sections 2.1 and 3.1).

TEST INFRASTRUCTURE (CPU oracle).

Pointwise 3x3 coefficient matrices are written out literally from eqs. (def_A)-(def_D),
with complex spin matrices and Phi Phi^H products, so the same code covers complex
ground states.  The operators are
    A = (L I_3 - Lambda) + beta_n (rho I_3 + Phi Phi^H)
        + beta_s (S.s(Phi) + sum_j S_j Phi Phi^H S_j^H),
    B = beta_n Phi Phi^T + beta_s sum_j S_j Phi Phi^T S_j^T,
    C = -[beta_n conj(Phi) Phi^H + beta_s sum_j conj(S_j) conj(Phi) Phi^H S_j^H],
    D = -[(L I_3 - Lambda) + beta_n (rho I_3 + conj(Phi) Phi^T)
          + beta_s (conj(S).s(Phi) + sum_j conj(S_j) conj(Phi) Phi^T S_j^T)],
with L = -Lap/2 + V.  In the discrete setting (eqs. def_bfA, def_bfB) every pointwise
factor becomes a diagonal matrix and L uses the Fourier pseudo-spectral Laplacian.

Trial vectors: arrays (6, *grid) or blocks (b, 6, *grid) holding (u_1,u_0,u_-1,v_1,v_0,v_-1)
in the (u, v) form of eq. (BdG-d), or (f_1,f_0,f_-1,g_1,g_0,g_-1) in the linear-response
form of eq. (lrep-d):  [[0, H_-], [H_+, 0]] [f; g] = omega [f; g],  H_+- = A +- B,
u = f + g, v = f - g.

Pins (tests): the FFT apply equals the dense matrix product on tiny grids; A and D are
Hermitian, B symmetric, C = -conj(B), D = -conj(A); for a real ground state the dense
spectrum pairs +-omega, the Kohn modes omega = gamma_alpha appear, the zero-mode count
matches the generalized nullspace theorems, and the FM / polar spectra equal the scalar
branch decompositions of ``branch``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import spectral, spin


@dataclasses.dataclass
class Coefficients:
    """Pointwise 3x3 blocks (excluding the kinetic term), arrays of shape (3, 3, *grid)."""
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    D: np.ndarray


def _outer(p, q):
    return np.einsum("a...,b...->ab...", p, q)


def _sandwich(S, M, T):
    """S M T for constant 3x3 S, T and a field of 3x3 matrices M."""
    return np.einsum("ab,bc...,cd->ad...", S, M, T)


def coefficients(phi, mu, V, beta_n, beta_s) -> Coefficients:
    """Literal eqs. (def_A)-(def_D) without the -Lap/2 part; phi: (3, *grid), mu: (3,)."""
    phi = np.asarray(phi, dtype=np.complex128)
    grid = phi.shape[1:]
    eye = np.zeros((3, 3) + grid, dtype=np.complex128)
    for a in range(3):
        eye[a, a] = 1.0
    rho = spin.density(phi)
    s = spin.spin_vector(phi)
    PPh = _outer(phi, phi.conj())            # Phi Phi^H
    PPt = _outer(phi, phi)                   # Phi Phi^T
    cPPh = _outer(phi.conj(), phi.conj())    # conj(Phi) Phi^H
    cPPt = _outer(phi.conj(), phi)           # conj(Phi) Phi^T
    Ldiag = np.zeros((3, 3) + grid, dtype=np.complex128)
    for a in range(3):
        Ldiag[a, a] = V - mu[a]
    Sdots = sum(sj * S[:, :, None].reshape((3, 3) + (1,) * len(grid)) for S, sj in zip(spin.SPIN, s))
    cSdots = sum(sj * S.conj()[:, :, None].reshape((3, 3) + (1,) * len(grid))
                 for S, sj in zip(spin.SPIN, s))
    A = Ldiag + beta_n * (rho * eye + PPh) + beta_s * (
        Sdots + sum(_sandwich(S, PPh, S.conj().T) for S in spin.SPIN))
    B = beta_n * PPt + beta_s * sum(_sandwich(S, PPt, S.T) for S in spin.SPIN)
    C = -(beta_n * cPPh + beta_s * sum(_sandwich(S.conj(), cPPh, S.conj().T) for S in spin.SPIN))
    D = -(Ldiag + beta_n * (rho * eye + cPPt) + beta_s * (
        cSdots + sum(_sandwich(S.conj(), cPPt, S.T) for S in spin.SPIN)))
    return Coefficients(A=A, B=B, C=C, D=D)


def _pw(Mx, x):
    """Pointwise 3x3 product for a batch x of shape (nb, 3, *grid)."""
    out = np.zeros(np.broadcast_shapes(x.shape, x.shape), dtype=np.result_type(Mx, x))
    for a in range(3):
        for b in range(3):
            out[:, a] += Mx[a, b] * x[:, b]
    return out


def apply_uv(coef: Coefficients, X, n, L):
    """[[A, B], [C, D]] [u; v] for a block X of shape (b, 6, *grid) (or (6, *grid))."""
    X = np.asarray(X, dtype=np.complex128)
    single = X.ndim == len(n) + 1
    if single:
        X = X[None]
    u, v = X[:, :3], X[:, 3:]
    Tu = spectral.kinetic_apply(u, n, L)
    Tv = spectral.kinetic_apply(v, n, L)
    yu = Tu + _pw(coef.A, u) + _pw(coef.B, v)
    yv = _pw(coef.C, u) - Tv + _pw(coef.D, v)
    Y = np.concatenate([yu, yv], axis=1)
    return Y[0] if single else Y


def hpm(coef: Coefficients):
    """Pointwise parts of H_+ = A + B and H_- = A - B (real ground state)."""
    return coef.A + coef.B, coef.A - coef.B


def apply_fg(coef: Coefficients, X, n, L):
    """[[0, H_-], [H_+, 0]] [f; g] = [H_- g; H_+ f] for a block (b, 6, *grid)."""
    X = np.asarray(X, dtype=np.complex128)
    single = X.ndim == len(n) + 1
    if single:
        X = X[None]
    Hp, Hm = hpm(coef)
    f, g = X[:, :3], X[:, 3:]
    out_f = spectral.kinetic_apply(g, n, L) + _pw(Hm, g)
    out_g = spectral.kinetic_apply(f, n, L) + _pw(Hp, f)
    Y = np.concatenate([out_f, out_g], axis=1)
    return Y[0] if single else Y


def apply_hplus(coef, f, n, L, Hp=None):
    """H_+ f for f of shape (nb, 3, *grid); Hp: precomputed pointwise part (optional)."""
    Hp = hpm(coef)[0] if Hp is None else Hp
    return spectral.kinetic_apply(f, n, L) + _pw(Hp, f)


def apply_hminus(coef, g, n, L, Hm=None):
    """H_- g for g of shape (nb, 3, *grid); Hm: precomputed pointwise part (optional)."""
    Hm = hpm(coef)[1] if Hm is None else Hm
    return spectral.kinetic_apply(g, n, L) + _pw(Hm, g)


# ------------------------------------------------------------------------------------
# Dense matrices (tiny grids only)
# ------------------------------------------------------------------------------------
def _block_dense(Mx, T=None, sign_T=1.0):
    """3 npts x 3 npts matrix with blocks diag(M_ab) (+ sign_T * T on the diagonal)."""
    npts = int(np.prod(Mx.shape[2:]))
    out = np.zeros((3 * npts, 3 * npts), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            blk = np.diag(Mx[a, b].ravel())
            if a == b and T is not None:
                blk = blk + sign_T * T
            out[a * npts:(a + 1) * npts, b * npts:(b + 1) * npts] = blk
    return out


def dense_uv(coef: Coefficients, n, L):
    """Dense [[A, B], [C, D]] of eq. (BdG-d), 6 npts square (complex128)."""
    T = spectral.kinetic_matrix(n, L)
    A = _block_dense(coef.A, T, 1.0)
    B = _block_dense(coef.B)
    C = _block_dense(coef.C)
    D = _block_dense(coef.D, T, -1.0)
    return np.block([[A, B], [C, D]])


def dense_hpm(coef: Coefficients, n, L):
    """Dense H_+ and H_- (3 npts square)."""
    T = spectral.kinetic_matrix(n, L)
    Hp, Hm = hpm(coef)
    return _block_dense(Hp, T, 1.0), _block_dense(Hm, T, 1.0)


def positive_eigs_dense(Hd, k, imag_tol=1e-8, zero_tol=1e-7):
    """k smallest strictly positive real eigenvalues of a dense BdG matrix, with
    eigenvectors (columns).  Eigenvalues with |Im| > imag_tol*max(1,|Re|) or
    |omega| <= zero_tol are excluded."""
    import scipy.linalg
    w, vr = scipy.linalg.eig(Hd)
    keep = (np.abs(w.imag) <= imag_tol * np.maximum(1.0, np.abs(w.real))) & (w.real > zero_tol)
    idx = np.where(keep)[0]
    idx = idx[np.argsort(w.real[idx])][:k]
    return w.real[idx], vr[:, idx]


# ------------------------------------------------------------------------------------
# Normalization, residuals, conversions
# ------------------------------------------------------------------------------------
def uv_to_fg(X, grid_ndim):
    """f = (u + v)/2, g = (u - v)/2 (eq. c-o-v-h); X: (..., 6, *grid)."""
    u, v = split_fg(X, grid_ndim)
    ax = X.ndim - grid_ndim - 1
    return np.concatenate([(u + v) / 2, (u - v) / 2], axis=ax)


def fg_to_uv(X, grid_ndim):
    """u = f + g, v = f - g (eq. c-o-v); X: (..., 6, *grid)."""
    f, g = split_fg(X, grid_ndim)
    ax = X.ndim - grid_ndim - 1
    return np.concatenate([f + g, f - g], axis=ax)


def split_fg(X, grid_ndim):
    """Return (f, g) halves of a block (..., 6, *grid)."""
    ax = X.ndim - grid_ndim - 1
    f = np.take(X, [0, 1, 2], axis=ax)
    g = np.take(X, [3, 4, 5], axis=ax)
    return f, g


def normalize_fg(X, h, grid_ndim):
    """Scale each (f, g) pair by one common real factor so that <f, g> = 1/4 (the
    normalization remark of Section 3.1).  Returns (X_scaled, <f,g> before scaling)."""
    hd = np.prod(h)
    X = np.asarray(X, dtype=np.complex128)
    single = X.ndim == grid_ndim + 1
    if single:
        X = X[None]
    f, g = X[:, :3], X[:, 3:]
    fg = hd * np.sum((f * g.conj()).reshape(X.shape[0], -1), axis=1)
    scale = 1.0 / np.sqrt(4.0 * fg.real)
    Xs = X * scale[(slice(None),) + (None,) * (X.ndim - 1)]
    return (Xs[0], fg[0]) if single else (Xs, fg)


def lrep_residuals(coef, X, omega, n, L):
    """res_j = ||(H_- g - w f, H_+ f - w g)|| / (|w| ||(f, g)||) for X (b, 6, *grid)."""
    Y = apply_fg(coef, X, n, L)
    R = Y - np.asarray(omega).reshape((-1,) + (1,) * (X.ndim - 1)) * X
    num = np.linalg.norm(R.reshape(X.shape[0], -1), axis=1)
    den = np.abs(omega) * np.linalg.norm(X.reshape(X.shape[0], -1), axis=1)
    return num / den


def rayleigh_omega(coef, X, n, L, h):
    """omega_j = (<H_+ f, f> + <H_- g, g>) / (2 Re <f, g>) (minimization principle quotient)."""
    hd = np.prod(h)
    Y = apply_fg(coef, X, n, L)
    f, g = X[:, :3], X[:, 3:]
    Hm_g, Hp_f = Y[:, :3], Y[:, 3:]
    b = X.shape[0]
    num = hd * (np.sum((Hp_f * f.conj()).reshape(b, -1), axis=1)
                + np.sum((Hm_g * g.conj()).reshape(b, -1), axis=1))
    den = 2.0 * hd * np.sum((f * g.conj()).reshape(b, -1), axis=1).real
    return num.real / den
