"""Block subspace iteration for the discrete linear-response problem (Section 3.2).

TEST INFRASTRUCTURE (CPU oracle).

    [[0, H_-], [H_+, 0]] [f; g] = omega [f; g],   H_+ = A + B,  H_- = A - B   (eq. lrep-d)

The paper solves it with its bi-orthogonal structure-preserving (BOSP) subspace
iteration, whose internal steps it does not print; it states that the method relies on
a modified Gram-Schmidt bi-orthogonalization, on the bi-orthogonality of eigenspaces
(Biorthogonality theorem) and on the generalized nullspace (Section 2.3).  This oracle
takes that as a locally optimal block iteration of the Bai-Li family, with the
following steps, each in plain numpy:

  deflation   f is kept orthogonal to N_- = ns(H_-), g to Q_g = ns(H_+) + span{Phi_hat}
              where H_+ Phi_hat = n for n in N_- (Jordan partners): the eigenvectors with
              omega != 0 are J-orthogonal to the generalized nullspace;
  residual    R_f = H_- G - F Theta, R_g = H_+ F - G Theta;
  correction  W_f = T R_g, W_g = T R_f (the gradient of the minimization-principle
              quotient with respect to f is H_+ f - omega g).  The paper prints no
              preconditioner; T is the symmetric kinetic-potential product
              T = D (|k|^2/2 + sigma)^-1 D,  D(x)^2 = sigma / (sigma + max(V(x) - mu, 0)),
              sigma = max(mu / 2, 1/2), the combination used by the preconditioned
              ground-state solvers the paper cites (Section 1): the Fourier factor
              handles the kinetic part, D the trap far outside the condensate where
              V - mu dominates.  Without V (a bare coefficient set) D = 1, sigma = 20;
  bi-orth     B_r = S_g^H S_f = U Sigma V^H, C_f = V Sigma^-1/2, C_g = U Sigma^-1/2
              (rank drop when sigma_i < 1e-8 sigma_1), so (S_g C_g)^H (S_f C_f) = I;
  Rayleigh-Ritz  M~ = C_f^H S_f^H H_+ S_f C_f = L_M L_M^H, K~ = C_g^H S_g^H H_- S_g C_g
              = L_K L_K^H; the projected problem K~ b = omega a, M~ a = omega b is
              solved by the SVD L_K^H L_M = U_G diag(omega) V_G^H: a = L_K u, b = L_M v;
  update      F <- S_f C_f a, G <- S_g C_g b (and their images), P from the W and P rows;
              the images of F and G are recomputed from F and G every 20 iterations; a
              projected problem that is not numerically definite is solved again with every
              image recomputed, then without P;
  stop        when res_j <= tol for the k wanted columns, with
              res_j = ||(H_- g_j - w_j f_j, H_+ f_j - w_j g_j)|| / (|w_j| ||(f_j, g_j)||).

The result (the k smallest positive omega and their eigenvectors, normalized to
<f, g> = 1/4) does not depend on the path; pins compare it with the dense
eigensolve, the branch decompositions and the uniform closed form.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg

from . import bdg, spectral, spin


@dataclasses.dataclass
class LrepResult:
    omega: np.ndarray        # (k,)
    X: np.ndarray            # (k, 6, *grid), (f, g) form, <f, g> = 1/4
    residual: np.ndarray     # (k,)
    iters: int
    history: list


def _gram(A, B, hd):
    """h^d A^H B for column blocks A (n x p), B (n x q)."""
    return hd * (A.conj().T @ B)


def orthonormal(vecs, hd, rtol=1e-10):
    """Orthonormal basis (columns, <.,.> with weight h^d) of the span of the given columns,
    with rank detection by the eigenvalues of their Gram matrix."""
    if vecs.shape[1] == 0:
        return vecs
    G = _gram(vecs, vecs, hd)
    w, Q = np.linalg.eigh(G)
    keep = w > rtol * max(w.max(), 1e-300)
    return vecs @ (Q[:, keep] / np.sqrt(w[keep]))


def _col_norms(X):
    nrm = np.linalg.norm(X, axis=0)
    return np.where(nrm > 0, nrm, 1.0)


def _unit_columns(X):
    """Scale every column to unit Euclidean norm (the span is unchanged); keeps the
    Gram matrices of the mixed block [X, W, P] well scaled as the residual shrinks."""
    return X / _col_norms(X)


def project_out(Q, X, hd):
    if Q is None or Q.shape[1] == 0:
        return X
    return X - Q @ _gram(Q, X, hd)


def _k_apply(op_symbol, X3, grid_shape):
    """Apply a Fourier multiplier to columns holding 3 stacked grid fields."""
    ncol = X3.shape[1]
    arr = X3.T.reshape((ncol, 3) + grid_shape)
    d = len(grid_shape)
    axes = tuple(range(-d, 0))
    out = spectral.ifftn(op_symbol * spectral.fftn(arr, axes=axes), axes=axes)
    return out.reshape(ncol, -1).T


def preconditioner_parameters(V, mu):
    """(sigma, D) of the kinetic-potential preconditioner: sigma = max(mu_0 / 2, 1/2) with
    mu_0 the middle chemical potential, D = sqrt(sigma / (sigma + max(V - mu_0, 0)))."""
    mu0 = float(np.asarray(mu, dtype=np.float64)[1])
    sigma = max(0.5 * mu0, 0.5)
    U = np.maximum(np.asarray(V, dtype=np.float64) - mu0, 0.0)
    return sigma, np.sqrt(sigma / (sigma + U))


class LrepProblem:
    """Operator access on column blocks: columns of F / G are flattened 3-component fields.
    weight: optional pointwise factor D of the preconditioner (grid shape)."""

    def __init__(self, coef: bdg.Coefficients, n, L, weight=None):
        self.coef, self.n, self.L = coef, tuple(n), tuple(L)
        self.weight = None if weight is None else np.tile(np.asarray(weight, dtype=np.float64).ravel(), 3)[:, None]
        self.grid_shape = tuple(reversed(n))
        self.h = tuple(2.0 * Li / ni for ni, Li in zip(n, L))
        self.hd = float(np.prod(self.h))
        self.sym = spectral.kinetic_symbol(n, L)
        Hp, Hm = bdg.hpm(coef)
        # a real ground state gives real pointwise parts; keep them real for speed
        self.Hp = Hp.real if np.abs(Hp.imag).max() == 0 else Hp
        self.Hm = Hm.real if np.abs(Hm.imag).max() == 0 else Hm
        self.napply = 0

    def _cols_to_fields(self, C):
        return C.T.reshape((C.shape[1], 3) + self.grid_shape)

    def _fields_to_cols(self, Fd):
        return Fd.reshape(Fd.shape[0], -1).T

    def hplus(self, F):
        self.napply += F.shape[1]
        return self._fields_to_cols(bdg.apply_hplus(self.coef, self._cols_to_fields(F), self.n, self.L, self.Hp))

    def hminus(self, G):
        self.napply += G.shape[1]
        return self._fields_to_cols(bdg.apply_hminus(self.coef, self._cols_to_fields(G), self.n, self.L, self.Hm))

    def precond(self, R, sigma):
        """D (|k|^2/2 + sigma)^-1 D on every column (D = 1 without a weight)."""
        if self.weight is None:
            return _k_apply(1.0 / (self.sym + sigma), R, self.grid_shape)
        return self.weight * _k_apply(1.0 / (self.sym + sigma), self.weight * R, self.grid_shape)


def null_candidates(phi):
    """Candidate generators (Section 2.3): for ns(H_-) the phase and the z- and x-spin
    rotations Phi, S_z Phi, S_x Phi; for ns(H_+) the y-rotation K Phi, K = -i S_y."""
    phi = np.asarray(phi, dtype=np.complex128)
    K = np.real(-1j * spin.S_y)
    cm = [phi, spin.mat3(spin.S_z, phi), spin.mat3(spin.S_x, phi)]
    cp = [spin.mat3(K.astype(np.complex128), phi)]
    return cm, cp


def projected_cg(apply_A, b, project, precond, tol, max_iter=5000):
    """Preconditioned CG for A x = b on the subspace selected by ``project``."""
    x = np.zeros_like(b)
    r = project(b.copy())
    z = project(precond(r))
    p = z.copy()
    rz = np.vdot(r, z)
    bnorm = np.linalg.norm(r)
    it = 0
    for it in range(1, max_iter + 1):
        Ap = project(apply_A(p))
        alpha = rz / np.vdot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        if np.linalg.norm(r) <= tol * bnorm:
            break
        z = project(precond(r))
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it


def deflation_sets(prob: LrepProblem, phi, null_tol=1e-6, cg_tol=1e-13, sigma=20.0):
    """(N_-, Q_g): orthonormal column bases for the f- and g-deflation (generalized
    nullspace of the Section 2.3 theorems).  Candidates are kept when
    ||H c|| <= null_tol ||c||; Jordan partners solve H_+ x = n on ns(H_+)^perp."""
    hd = prob.hd
    cm, cp = null_candidates(phi)
    to_col = lambda c: c.reshape(-1, 1)
    keep_m, keep_p = [], []
    for c in cm:
        col = to_col(c)
        nc = np.sqrt(hd) * np.linalg.norm(col)
        if nc > 0 and np.sqrt(hd) * np.linalg.norm(prob.hminus(col)) <= null_tol * nc:
            keep_m.append(col)
    for c in cp:
        col = to_col(c)
        nc = np.sqrt(hd) * np.linalg.norm(col)
        if nc > 1e-12 and np.sqrt(hd) * np.linalg.norm(prob.hplus(col)) <= null_tol * nc:
            keep_p.append(col)
    Nm = orthonormal(np.hstack(keep_m), hd) if keep_m else np.zeros((phi.size, 0), complex)
    Np = orthonormal(np.hstack(keep_p), hd) if keep_p else np.zeros((phi.size, 0), complex)
    # Jordan partners: H_+ x = n for n in the part of N_- orthogonal to N_+
    src = orthonormal(project_out(Np, Nm, hd), hd, rtol=1e-8)
    proj = lambda v: project_out(Np, v, hd)
    partners = []
    for j in range(src.shape[1]):
        x, _ = projected_cg(prob.hplus, src[:, j:j + 1], proj,
                            lambda r: prob.precond(r, sigma), cg_tol)
        partners.append(x)
    Qg = orthonormal(np.hstack([Np] + partners), hd) if (partners or Np.shape[1]) else Np
    return Nm, Qg


def _orth_factor(S, hd, rtol):
    """R with S R orthonormal (<.,.> weight h^d): eigen-decomposition of the Gram matrix
    S^H S = Q diag(d) Q^H, R = Q diag(d)^-1/2 over the eigenvalues d > rtol * max(d)."""
    Gm = _gram(S, S, hd)
    Gm = 0.5 * (Gm + Gm.conj().T)
    d, Q = np.linalg.eigh(Gm)
    keep = d > rtol * d.max()
    return Q[:, keep] / np.sqrt(d[keep])


def rayleigh_ritz(Sf, Sg, HSf, HSg, nkeep, hd, eps=1e-10, rtol=1e-14):
    """``_rayleigh_ritz_once`` with escalating cut-offs: rounding in the projected matrices can
    make them indefinite along nearly dependent directions of the basis (the Cholesky factor
    then does not exist); the step is repeated with both cut-offs raised 100x, at most twice.
    Dropping those directions leaves the part of the span that carries the wanted pairs."""
    for attempt in range(3):
        try:
            return _rayleigh_ritz_once(Sf, Sg, HSf, HSg, nkeep, hd, eps * 100.0 ** attempt, rtol * 100.0 ** attempt)
        except np.linalg.LinAlgError:
            if attempt == 2:
                raise


def _rayleigh_ritz_once(Sf, Sg, HSf, HSg, nkeep, hd, eps, rtol):
    """Bi-orthogonalize, project, solve; returns (omega, a, b) with F = Sf a, G = Sg b.

    Each basis is first made orthonormal on its own (dropping numerically dependent
    directions, eigenvalues of its Gram matrix below rtol of the largest); the pairing
    matrix of the orthonormal bases, B = Q_g^H Q_f = U Sigma V^H, then holds the cosines
    of the angles between the f- and g-spaces, and directions with sigma_i < eps are
    dropped.  C_f = R_f V Sigma^-1/2 and C_g = R_g U Sigma^-1/2 make the two bases
    bi-orthonormal."""
    Rf, Rg = _orth_factor(Sf, hd, rtol), _orth_factor(Sg, hd, rtol)
    Br = Rg.conj().T @ _gram(Sg, Sf, hd) @ Rf
    U, s, Vh = np.linalg.svd(Br)
    Mr = Rf.conj().T @ _gram(Sf, HSf, hd) @ Rf
    Kr = Rg.conj().T @ _gram(Sg, HSg, hd) @ Rg
    r = int(np.sum(s > eps))
    Cf = Vh.conj().T[:, :r] / np.sqrt(s[:r])
    Cg = U[:, :r] / np.sqrt(s[:r])
    Mt = Cf.conj().T @ Mr @ Cf
    Kt = Cg.conj().T @ Kr @ Cg
    Mt = 0.5 * (Mt + Mt.conj().T)
    Kt = 0.5 * (Kt + Kt.conj().T)
    LM = scipy.linalg.cholesky(Mt, lower=True)
    LK = scipy.linalg.cholesky(Kt, lower=True)
    Ug, sg, Vgh = np.linalg.svd(LK.conj().T @ LM)
    idx = np.argsort(sg)[:nkeep]
    om = sg[idx]
    a = Rf @ (Cf @ (LK @ Ug[:, idx]))
    b = Rg @ (Cg @ (LM @ Vgh.conj().T[:, idx]))
    # scale so that <f, g> = 1/4 (b^H a = omega in the bi-orthogonal basis)
    sc = 1.0 / np.sqrt(4.0 * om)
    return om, a * sc, b * sc


def lrep_eigs(prob: LrepProblem, k: int, X0: np.ndarray, tol: float, max_iter: int = 1000,
              Nm=None, Qg=None, sigma: float = 20.0, verbose: bool = False) -> LrepResult:
    """k smallest positive omega of eq. (lrep-d); X0: (block, 6, *grid) start block."""
    hd = prob.hd
    b = X0.shape[0]
    npts = int(np.prod(prob.grid_shape))
    X0 = np.asarray(X0, dtype=np.complex128).reshape(b, 6 * npts)
    F = X0[:, :3 * npts].T.copy()
    G = X0[:, 3 * npts:].T.copy()
    F = project_out(Nm, F, hd)
    G = project_out(Qg, G, hd)
    HF, HG = prob.hplus(F), prob.hminus(G)
    om, a, bb = rayleigh_ritz(F, G, HF, HG, b, hd)
    F, G, HF, HG = F @ a, G @ bb, HF @ a, HG @ bb
    Pf = Pg = HPf = HPg = None
    history = []
    it = 0
    res = np.full(b, np.inf)
    for it in range(1, max_iter + 1):
        if it % 20 == 0:
            # images by recurrence drift from H applied to the basis; recompute them
            HF, HG = prob.hplus(F), prob.hminus(G)
        Rf = HG - F * om          # H_- g - omega f
        Rg = HF - G * om          # H_+ f - omega g
        num = np.sqrt(np.sum(np.abs(Rf) ** 2, axis=0) + np.sum(np.abs(Rg) ** 2, axis=0))
        den = np.abs(om) * np.sqrt(np.sum(np.abs(F) ** 2, axis=0) + np.sum(np.abs(G) ** 2, axis=0))
        res = num / den
        history.append(res.copy())
        if verbose:
            print(it, om[:4], res[:k].max())
        if np.all(res[:k] <= tol):
            break
        Wf = _unit_columns(project_out(Nm, prob.precond(Rg, sigma), hd))
        Wg = _unit_columns(project_out(Qg, prob.precond(Rf, sigma), hd))
        HWf, HWg = prob.hplus(Wf), prob.hminus(Wg)
        parts_f = [F, Wf] + ([Pf] if Pf is not None else [])
        parts_g = [G, Wg] + ([Pg] if Pg is not None else [])
        hparts_f = [HF, HWf] + ([HPf] if HPf is not None else [])
        hparts_g = [HG, HWg] + ([HPg] if HPg is not None else [])
        Sf, Sg = np.hstack(parts_f), np.hstack(parts_g)
        HSf, HSg = np.hstack(hparts_f), np.hstack(hparts_g)
        try:
            om, a, bb = rayleigh_ritz(Sf, Sg, HSf, HSg, b, hd)
        except np.linalg.LinAlgError:
            # the projected problem lost definiteness along nearly dependent directions of
            # [F, W, P]: recompute every image from its vector, and if that is not enough
            # restart the step from [F, W] (the eigenpairs do not depend on the path)
            hparts_f = [prob.hplus(x) for x in parts_f]
            hparts_g = [prob.hminus(x) for x in parts_g]
            HSf, HSg = np.hstack(hparts_f), np.hstack(hparts_g)
            try:
                om, a, bb = rayleigh_ritz(Sf, Sg, HSf, HSg, b, hd)
            except np.linalg.LinAlgError:
                if Pf is None:
                    raise
                Sf, Sg = np.hstack(parts_f[:2]), np.hstack(parts_g[:2])
                HSf, HSg = np.hstack(hparts_f[:2]), np.hstack(hparts_g[:2])
                om, a, bb = rayleigh_ritz(Sf, Sg, HSf, HSg, b, hd)
        Pf, Pg = Sf[:, b:] @ a[b:], Sg[:, b:] @ bb[b:]
        HPf, HPg = HSf[:, b:] @ a[b:], HSg[:, b:] @ bb[b:]
        # unit columns for P as well; the images scale with them
        sf, sg = _col_norms(Pf), _col_norms(Pg)
        Pf, HPf, Pg, HPg = Pf / sf, HPf / sf, Pg / sg, HPg / sg
        F, G, HF, HG = Sf @ a, Sg @ bb, HSf @ a, HSg @ bb
    X = np.concatenate([F.T, G.T], axis=1).reshape((b, 6) + prob.grid_shape)
    return LrepResult(omega=om[:k], X=X[:k], residual=res[:k], iters=it, history=history)


def solve(coef, phi, n, L, k, X0, tol, max_iter=1000, sigma=None, verbose=False, V=None, mu=None):
    """Deflation sets + subspace iteration in one call.  With V and mu the
    kinetic-potential preconditioner is used (sigma from preconditioner_parameters unless
    given), otherwise the kinetic one with sigma = 20."""
    weight = None
    if V is not None and mu is not None:
        s0, weight = preconditioner_parameters(V, mu)
        sigma = s0 if sigma is None else sigma
    elif sigma is None:
        sigma = 20.0
    prob = LrepProblem(coef, n, L, weight)
    Nm, Qg = deflation_sets(prob, phi, sigma=sigma)
    out = lrep_eigs(prob, k, X0, tol, max_iter=max_iter, Nm=Nm, Qg=Qg, sigma=sigma,
                    verbose=verbose)
    return out, prob, Nm, Qg
