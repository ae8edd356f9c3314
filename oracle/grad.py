"""Eigenvalue gradients with respect to V(x), beta_n and beta_s.

TEST INFRASTRUCTURE (CPU oracle).

For an eigenpair of [[0, H_-], [H_+, 0]] with right eigenvector (f, g), the left
eigenvector is (g, f) (J H = diag(H_+, H_-) is Hermitian), so a perturbation of H_+- changes
omega by  d omega = (<dH_+ f, f> + <dH_- g, g>) / (2 Re <f, g>)  (first-order perturbation).
H_+- = A +- B depend on theta in (V, beta_n, beta_s) directly and through the ground state
Phi and its multipliers Lambda = mu + lambda S_z (Euler-Lagrange problem, Section 1).  The
ground-state sensitivity solves the linearized Euler-Lagrange problem with its two
constraints; its real-direction Jacobian is H_+ = A + B.  The oracle writes this as one
symmetric bordered system and solves its adjoint with MINRES:
    [[H_+, Phi, S_z Phi], [Phi^T, 0, 0], [(S_z Phi)^T, 0, 0]] (y, e1, e2) = (q, -a_mu, -a_lambda)
where q, a_mu, a_lambda are the derivatives of omega with respect to Phi, mu and lambda at
fixed (f, g).  The derivative of the pointwise coefficient matrices with respect to Phi is
taken by central differences of the literal def_A / def_B matrices (exact: they are
quadratic in Phi).  Then  d omega / d theta = explicit - <y, d_theta (H(Phi) Phi)>.

Pins (tests): central finite differences of the whole pipeline (ground state re-solved,
dense eigensolve) along random directions, and of the frozen-ground-state operator for the
explicit part.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import bdg, spectral, spin


def _pw_form(Mx, F):
    """Re sum_ab conj(F_a) M_ab F_b pointwise for M (3, 3, *grid), F (3, *grid)."""
    return np.real(np.einsum("a...,ab...,b...->...", F.conj(), Mx, F))


def _hpm_parts(phi, beta_n, beta_s):
    """Pointwise H_+ and H_- parts without V - mu (literal coefficients with V = mu = 0)."""
    zero = np.zeros(phi.shape[1:])
    c = bdg.coefficients(phi, np.zeros(3), zero, beta_n, beta_s)
    return bdg.hpm(c)


def eigen_gradient(phi, mu, V, beta_n, beta_s, n, L, X, tol=1e-12, maxiter=200000):
    """Gradients for one eigenvector X = (f, g) (shape (6, *grid)).

    Returns (dV, dbeta_n, dbeta_s) with dV the functional derivative d omega / d V(x) / h^d.
    """
    h = tuple(2.0 * Li / ni for ni, Li in zip(n, L))
    hd = float(np.prod(h))
    phi = np.asarray(phi, dtype=np.float64)
    f, g = X[:3], X[3:]
    s = 1.0 / (2.0 * hd * np.real(np.vdot(g, f)))
    # explicit parts
    dens = np.sum(np.abs(f) ** 2 + np.abs(g) ** 2, axis=0)
    Pn, Mn = _hpm_parts(phi, 1.0, 0.0)
    Ps, Ms = _hpm_parts(phi, 0.0, 1.0)
    e_bn = s * hd * np.sum(_pw_form(Pn, f) + _pw_form(Mn, g))
    e_bs = s * hd * np.sum(_pw_form(Ps, f) + _pw_form(Ms, g))
    # derivatives with respect to Phi (central differences, exact for quadratic coefficients)
    step = 1e-2 * np.max(np.abs(phi))
    q = np.zeros_like(phi)
    for cidx in range(3):
        e = np.zeros_like(phi)
        e[cidx] = step
        Pp, Mp = _hpm_parts(phi + e, beta_n, beta_s)
        Pm, Mm = _hpm_parts(phi - e, beta_n, beta_s)
        q[cidx] = s * (_pw_form(Pp - Pm, f) + _pw_form(Mp - Mm, g)) / (2.0 * step)
    szphi = np.stack([phi[0], np.zeros_like(phi[1]), -phi[2]])
    a_mu = -s * hd * np.sum(dens)
    a_lam = -s * hd * np.sum(np.abs(f[0]) ** 2 - np.abs(f[2]) ** 2 + np.abs(g[0]) ** 2 - np.abs(g[2]) ** 2)
    # bordered adjoint system (scaled by h^d so that it is symmetric in the Euclidean product)
    Hp, _ = bdg.hpm(bdg.coefficients(phi, mu, V, beta_n, beta_s))
    Hp = Hp.real
    N = phi.size
    shape = phi.shape

    def matvec(z):
        z = np.asarray(z).ravel()
        y = z[:N].reshape(shape)
        e1, e2 = z[N], z[N + 1]
        hy = np.real(spectral.kinetic_apply(y, n, L)) + np.einsum("ab...,b...->a...", Hp, y)
        top = hd * (hy + e1 * phi + e2 * szphi)
        return np.concatenate([top.ravel(), [hd * np.sum(phi * y), hd * np.sum(szphi * y)]])

    op = spla.LinearOperator((N + 2, N + 2), matvec=matvec, dtype=np.float64)
    rhs = np.concatenate([(hd * q).ravel(), [-a_mu, -a_lam]])
    sol, info = spla.minres(op, rhs, rtol=tol, maxiter=maxiter)
    if info != 0:
        raise RuntimeError(f"MINRES did not converge (info={info})")
    y = sol[:N].reshape(shape)
    # d_theta (H(Phi) Phi) at fixed Phi
    rho = spin.density(phi)
    sx, sy, sz = spin.spin_vector(phi.astype(np.complex128))
    sphi = np.real(sx * spin.mat3(spin.S_x, phi.astype(complex)) + sy * spin.mat3(spin.S_y, phi.astype(complex))
                   + sz * spin.mat3(spin.S_z, phi.astype(complex)))
    dV = s * dens - np.sum(y * phi, axis=0)
    dbn = e_bn - hd * np.sum(y * rho * phi)
    dbs = e_bs - hd * np.sum(y * sphi)
    return dV, float(dbn), float(dbs)


def directional(dV, dbn, dbs, direction, h):
    """<grad, direction> with the grid weight h^d for the V field."""
    dVd, dbnd, dbsd = direction
    return float(np.prod(h) * np.sum(dV * dVd) + dbn * dbnd + dbs * dbsd)
