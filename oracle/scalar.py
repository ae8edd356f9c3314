"""Matrix-free scalar branch spectra of the BdG problem at full grid size (Section 2.3).

TEST INFRASTRUCTURE (CPU oracle).

For the two ground-state classes with a single spatial profile the six-component BdG
spectrum splits into spectra of real scalar operators (the derivations are in the header
of ``branch``, which forms the same operators as dense matrices on small grids):

  ferromagnetic single-mode state (SMA lemma; beta_s < 0), Phi = a phi, coupling
  g = beta_n + beta_s:
      h_0 = L - mu + g phi^2,  h_2 = L - mu + (beta_n - beta_s) phi^2,  h_3 = L - mu + 3 g phi^2,
      omega in  sqrt(eig(h_0 h_3))  U  eig(h_0) minus {0}  U  eig(h_2);
  polar state at M = 0 (two-component lemma; beta_s > 0), Phi = (phi, 0, phi)/sqrt 2:
      h_0 = L - mu + beta_n phi^2,  h_s = h_0 + 2 beta_s phi^2,  h_3 = h_0 + 2 beta_n phi^2,
      omega in  sqrt(eig(h_0 h_3))  U  sqrt(eig(h_0 h_s)) (twice),

with L = -Lap/2 + V the Fourier pseudo-spectral operator (Section 3.1) and phi, mu the
scalar Gross-Pitaevskii ground state of coupling g (FM) or beta_n (polar).

This module evaluates those spectra without forming any matrix, so that it runs on the
full 3-D grids:

  * every scalar operator h = L + U(x) is applied to real fields with a real FFT
    (pocketfft, ``spectral.WORKERS`` threads), kinetic symbol |k|^2/2 including the Nyquist mode;
  * eig(h) (h symmetric) is the standard symmetric problem h z = lambda z;
  * sqrt(eig(h_0 h_x)) (h_0 positive semidefinite with h_0 phi = 0, h_x positive definite)
    is the spectrum of the scalar linear-response problem [[0, h_0], [h_x, 0]], solved by
    the block iteration of ``product_branch`` with phi and h_x^-1 phi deflated (a scalar
    problem of the structure of eq. lrep-d; its Rayleigh-Ritz step is ``lrep``'s);
  * the symmetric problems are solved by the locally optimal block preconditioned
    conjugate gradient method (Knyazev's LOBPCG) written out below: basis [X, W, P],
    B-orthonormalization with rank detection, Rayleigh-Ritz by a dense symmetric
    eigensolve, soft locking of converged columns, images of W and P computed from W and P
    themselves, and a final explicit re-evaluation of the residuals.  The preconditioner T = D (|k|^2/2 + s)^-1 D, D^2 = s / (s + max(U, 0)),
    uses the operator's own pointwise part U; it changes the iteration count, never the
    eigenpairs.

This is an independent formulation of the spectrum: real scalar problems on one grid
field instead of one six-component linear-response problem, with their own deflation
(phi, h_x^-1 phi) and preconditioners; the magnon and gapped branches use a symmetric
eigensolver instead of the bi-orthogonal iteration.  (The generalized symmetric pencil
(h_x h_0 h_x, h_x) has the same eigenvalues omega^2, but its third-order operator leaves
LOBPCG with a preconditioned condition number near 1e5 even on 1-D grids; the
linear-response form keeps two second-order operators.)

Pins (tests): the scalar apply equals the dense matrix of ``branch`` on small grids; the
LOBPCG eigenvalues equal numpy's dense symmetric eigensolver; the branch spectra equal
``branch``'s dense decompositions and the dense six-component BdG eigensolve on small
1-D, 2-D and 3-D grids; on a 2-D grid they equal the six-component subspace iteration of
``lrep``.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional, Sequence

import numpy as np
import scipy.fft

from . import spectral


# --------------------------------------------------------------------------------------
# Scalar operators on real grid fields
# --------------------------------------------------------------------------------------
class ScalarGrid:
    """Real grid fields of shape (..., Nz, Ny, Nx)[-d:] (x fastest) and the real-FFT
    kinetic operator -Lap/2 on them."""

    def __init__(self, n: Sequence[int], L: Sequence[float]):
        self.n, self.L = tuple(n), tuple(L)
        self.d = len(self.n)
        self.shape = tuple(reversed(self.n))
        self.axes = tuple(range(-self.d, 0))
        self.npts = int(np.prod(self.n))
        self.hd = float(np.prod([2.0 * Li / ni for ni, Li in zip(self.n, self.L)]))
        full = spectral.kinetic_symbol(self.n, self.L)
        # the real transform keeps x-frequencies 0..N/2; the symbol is even, so the first
        # N/2 + 1 entries of the full (FFT-ordered) symbol are the right ones
        self.sym = np.ascontiguousarray(full[..., : self.n[0] // 2 + 1])

    def fourier(self, F: np.ndarray, symbol: np.ndarray) -> np.ndarray:
        """Real field(s) F times a real even Fourier multiplier."""
        Fh = scipy.fft.rfftn(F, axes=self.axes, workers=spectral.WORKERS)
        Fh *= symbol
        return scipy.fft.irfftn(Fh, s=self.shape, axes=self.axes, workers=spectral.WORKERS)

    def kinetic(self, F: np.ndarray) -> np.ndarray:
        return self.fourier(F, self.sym)


class ScalarOp:
    """h = -Lap/2 + U(x) on real fields (U: grid-shaped, real)."""

    def __init__(self, grid: ScalarGrid, U: np.ndarray):
        self.grid = grid
        self.U = np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(grid.shape))

    def __call__(self, F: np.ndarray) -> np.ndarray:
        return self.grid.kinetic(F) + self.U * F

    def preconditioner(self, s: float = 1.0) -> Callable[[np.ndarray], np.ndarray]:
        """T = D (|k|^2/2 + s)^-1 D with D^2 = s / (s + max(U, 0)): close to (h + s)^-1 where
        either the kinetic part or the pointwise part dominates."""
        Up = np.maximum(self.U, 0.0)
        D = np.sqrt(s / (s + Up))
        inv = 1.0 / (self.grid.sym + s)
        return lambda R: D * self.grid.fourier(D * R, inv)


# --------------------------------------------------------------------------------------
# LOBPCG for the symmetric-definite pencil A z = lambda B z (rows of 2-D arrays are vectors)
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class EigResult:
    values: np.ndarray        # ascending eigenvalues lambda
    vectors: np.ndarray       # (k, *grid), B-orthonormal (Euclidean sums, no h^d weight)
    residual: np.ndarray      # ||A z - lambda B z|| / (|lambda| ||B z||), explicitly re-evaluated
    iters: int


def _rows(F):
    return F.reshape(F.shape[0], -1)


def _b_orthonormal_coefficients(S, BS, rtol):
    """C with (C^T S)(B)(S^T C) = I over the numerically independent directions of S:
    eigen-decomposition of the Gram matrix S B S^T with rank detection."""
    G = _rows(S) @ _rows(BS).T
    G = 0.5 * (G + G.T)
    d, Q = np.linalg.eigh(G)
    keep = d > rtol * d.max()
    return Q[:, keep] / np.sqrt(d[keep])


def lobpcg(apply_ab: Callable[[np.ndarray], tuple], precond: Callable[[np.ndarray], np.ndarray],
           X0: np.ndarray, k: int, tol: float, max_iter: int = 2000, project=None,
           rtol: float = 1e-14, verbose: bool = False) -> EigResult:
    """The k smallest eigenpairs of A z = lambda B z (A symmetric, B symmetric positive
    definite), block size X0.shape[0] >= k.

    apply_ab(Z) -> (A Z, B Z) for a stack of fields Z (leading axis: vectors);
    precond(R) -> T R, T symmetric positive definite;
    project(Z) -> Z with the constrained directions removed (an orthogonal projector that
    commutes with the pencil's invariant subspaces), or None.
    """
    proj = (lambda Z: Z) if project is None else project
    X = proj(np.array(X0, dtype=np.float64))
    nb = X.shape[0]
    AX, BX = apply_ab(X)
    C = _b_orthonormal_coefficients(X, BX, rtol)
    X, AX, BX = (np.tensordot(C.T, Z, axes=1) for Z in (X, AX, BX))
    theta, Z = np.linalg.eigh(_rows(X) @ _rows(AX).T)
    X, AX, BX = (np.tensordot(Z.T, Y, axes=1) for Y in (X, AX, BX))
    P = AP = BP = None
    res = np.full(nb, np.inf)
    it = 0
    explicit = False
    for it in range(1, max_iter + 1):
        R = AX - theta.reshape((-1,) + (1,) * (X.ndim - 1)) * BX
        res = np.linalg.norm(_rows(R), axis=1) / (np.abs(theta) * np.linalg.norm(_rows(BX), axis=1))
        if verbose:
            print(f"  lobpcg {it}: lambda[:3] {theta[:3]}, max res (k) {res[:k].max():.2e}", flush=True)
        if np.all(res[:k] <= tol):
            if explicit:
                break
            # accept only after the images of X have been recomputed from X itself
            AX, BX = apply_ab(X)
            explicit = True
            continue
        explicit = False
        active = np.nonzero(res > tol)[0]
        W = proj(precond(R[active]))
        # W against X (B-orthonormal), then unit B-norm columns: keeps the Gram well scaled
        W = W - np.tensordot(_rows(W) @ _rows(BX).T, X, axes=1)
        AW, BW = apply_ab(W)
        nw = np.sqrt(np.einsum("ij,ij->i", _rows(W), _rows(BW)))
        nw = np.where(nw > 0, nw, 1.0).reshape((-1,) + (1,) * (X.ndim - 1))
        W, AW, BW = W / nw, AW / nw, BW / nw
        parts = [(X, AX, BX), (W, AW, BW)] + ([(P, AP, BP)] if P is not None else [])
        S = np.concatenate([p[0] for p in parts])
        AS = np.concatenate([p[1] for p in parts])
        BS = np.concatenate([p[2] for p in parts])
        C = _b_orthonormal_coefficients(S, BS, rtol)
        At = C.T @ (_rows(S) @ _rows(AS).T) @ C
        At = 0.5 * (At + At.T)
        theta_all, Z = np.linalg.eigh(At)
        Q = C @ Z[:, :nb]
        theta = theta_all[:nb]
        Xn, AXn, BXn = (np.tensordot(Q.T, Y, axes=1) for Y in (S, AS, BS))
        # P: the step taken inside span[W, P], scaled to unit B-norm with images computed from
        # P itself (a combination that shrinks as X converges carries the rounding of the
        # images it is built from; rescaled, that rounding would enter the next basis)
        P = np.tensordot(Q[nb:].T, S[nb:], axes=1)
        AP, BP = apply_ab(P)
        npn = np.sqrt(np.maximum(np.einsum("ij,ij->i", _rows(P), _rows(BP)), 0.0))
        npn = np.where(npn > 0, npn, 1.0).reshape((-1,) + (1,) * (X.ndim - 1))
        P, AP, BP = P / npn, AP / npn, BP / npn
        X, AX, BX = Xn, AXn, BXn
    order = np.argsort(theta)
    return EigResult(values=theta[order][:k], vectors=X[order][:k], residual=res[order][:k], iters=it)


# --------------------------------------------------------------------------------------
# Branches
# --------------------------------------------------------------------------------------
def _orth_projector(phi):
    """Z -> Z - phi (phi^T Z) / (phi^T phi) on every row of Z."""
    p = np.asarray(phi, dtype=np.float64)
    pn = p / np.linalg.norm(p)

    def proj(Z):
        c = _rows(Z) @ pn.ravel()
        return Z - c.reshape((-1,) + (1,) * p.ndim) * pn
    return proj


def _start(grid: ScalarGrid, nb: int, seed: int):
    return np.random.default_rng(seed).standard_normal((nb,) + grid.shape)


def symmetric_branch(h: ScalarOp, k: int, tol: float, nb: Optional[int] = None, phi=None, seed: int = 0,
                     max_iter: int = 2000, verbose: bool = False) -> EigResult:
    """The k smallest eigenvalues of h (restricted to phi's orthogonal complement if phi
    is given)."""
    nb = nb or k + max(4, k // 4)
    proj = None if phi is None else _orth_projector(phi)
    return lobpcg(lambda Z: (h(Z), Z), h.preconditioner(), _start(h.grid, nb, seed), k, tol,
                  max_iter=max_iter, project=proj, verbose=verbose)


def product_branch(h0: ScalarOp, hx: ScalarOp, phi, k: int, tol: float, nb: Optional[int] = None,
                   seed: int = 0, max_iter: int = 2000, verbose: bool = False):
    """The k smallest positive omega = sqrt(eig(h_0 h_x)), h_0 positive semidefinite with
    h_0 phi = 0 and h_x positive definite, as the scalar linear-response problem
        [[0, h_0], [h_x, 0]] [x; y] = omega [x; y]   (h_0 y = omega x, h_x x = omega y),
    whose x-part solves h_0 h_x x = omega^2 x.  For omega != 0, x = h_0 y / omega lies in
    phi's orthogonal complement and y = h_x x / omega in the complement of
    phi_hat = h_x^-1 phi (one preconditioned CG solve); both constraints are imposed on the
    search spaces.  Block iteration with basis [X, W, P] per half, corrections
    W_x = T_x (h_x x - omega y), W_y = T_0 (h_0 y - omega x) with each operator's own
    preconditioner, and the bi-orthogonal Rayleigh-Ritz step of ``lrep`` (pinned there
    against the dense eigensolve).  Returns (omega ascending, EigResult with
    values = omega^2, residual ||(h_0 y - w x, h_x x - w y)|| / (|w| ||(x, y)||))."""
    from . import lrep
    grid = h0.grid
    nb = nb or k + max(4, k // 4)
    hd = grid.hd
    cols = lambda Z: Z.reshape(Z.shape[0], -1).T            # stack of fields -> columns
    fields = lambda C: C.T.reshape((C.shape[1],) + grid.shape)
    T0, Tx = h0.preconditioner(), hx.preconditioner()
    opK = lambda C: cols(h0(fields(C)))
    opM = lambda C: cols(hx(fields(C)))
    pK = lambda C: cols(T0(fields(C)))
    pM = lambda C: cols(Tx(fields(C)))
    ph = np.asarray(phi, dtype=np.float64).reshape(-1, 1)
    Nx = ph / np.sqrt(hd * float((ph.T @ ph)[0, 0]))
    proj_x = lambda C: C - Nx @ (hd * (Nx.T @ C))
    phat, _ = lrep.projected_cg(opM, Nx.copy(), lambda v: v, pM, 1e-14)
    Ny = phat / np.sqrt(hd * float((phat.T @ phat)[0, 0]))
    proj_y = lambda C: C - Ny @ (hd * (Ny.T @ C))
    rng = np.random.default_rng(seed)
    X = proj_x(rng.standard_normal((grid.npts, nb)))
    Y = proj_y(rng.standard_normal((grid.npts, nb)))
    MX, KY = opM(X), opK(Y)
    om, a, b = lrep.rayleigh_ritz(X, Y, MX, KY, nb, hd)
    X, Y, MX, KY = X @ a, Y @ b, MX @ a, KY @ b
    Px = Py = MPx = KPy = None
    res = np.full(nb, np.inf)
    it = 0
    explicit = False
    for it in range(1, max_iter + 1):
        Rx = KY - X * om                 # h_0 y - omega x
        Ry = MX - Y * om                 # h_x x - omega y
        num = np.sqrt(np.sum(Rx * Rx, axis=0) + np.sum(Ry * Ry, axis=0))
        res = num / (np.abs(om) * np.sqrt(np.sum(X * X, axis=0) + np.sum(Y * Y, axis=0)))
        if verbose:
            print(f"  lrep {it}: omega[:3] {om[:3]}, max res (k) {res[:k].max():.2e}", flush=True)
        if np.all(res[:k] <= tol):
            if explicit:
                break
            MX, KY = opM(X), opK(Y)
            explicit = True
            continue
        explicit = False
        act = np.nonzero(res > tol)[0]
        Wx = lrep._unit_columns(proj_x(pM(Ry[:, act])))
        Wy = lrep._unit_columns(proj_y(pK(Rx[:, act])))
        MWx, KWy = opM(Wx), opK(Wy)
        Sx = np.hstack([X, Wx] + ([Px] if Px is not None else []))
        Sy = np.hstack([Y, Wy] + ([Py] if Py is not None else []))
        MSx = np.hstack([MX, MWx] + ([MPx] if MPx is not None else []))
        KSy = np.hstack([KY, KWy] + ([KPy] if KPy is not None else []))
        om, a, b = lrep.rayleigh_ritz(Sx, Sy, MSx, KSy, nb, hd)
        # P: the step inside [W, P] with images computed from P itself, unit columns
        Px = lrep._unit_columns(Sx[:, nb:] @ a[nb:])
        Py = lrep._unit_columns(Sy[:, nb:] @ b[nb:])
        MPx, KPy = opM(Px), opK(Py)
        X, Y, MX, KY = Sx @ a, Sy @ b, MSx @ a, KSy @ b
    order = np.argsort(om)
    r = EigResult(values=(om[order] ** 2)[:k], vectors=fields(X[:, order[:k]]), residual=res[order][:k], iters=it)
    return om[order][:k], r


@dataclasses.dataclass
class BranchSpectrum:
    omega: np.ndarray                 # the k smallest positive frequencies, merged
    branches: dict                    # name -> (omega ascending, multiplicity, EigResult)
    complete_below: float             # every branch eigenvalue below this was computed


def _merge(branches, k):
    allv = []
    for vals, mult, _ in branches.values():
        allv.extend(list(vals) * mult)
    allv = np.sort(np.array(allv))
    ceiling = min(vals[-1] for vals, _, _ in branches.values())
    return allv, ceiling


def fm_branches(phi, mu, V, beta_n, beta_s, n, L, counts: dict, tol: float = 1e-9, k_total: Optional[int] = None,
                verbose: bool = False) -> BranchSpectrum:
    """FM single-mode decomposition; counts = {"density": k_d, "magnon": k_m, "gapped": k_g}
    eigenvalues per branch.  With k_total, checks that the k_total smallest merged values lie
    strictly below every branch's largest computed value (so none is missing)."""
    grid = ScalarGrid(n, L)
    g = beta_n + beta_s
    p2 = np.asarray(phi, dtype=np.float64).reshape(grid.shape) ** 2
    base = np.asarray(V, dtype=np.float64).reshape(grid.shape) - mu
    h0 = ScalarOp(grid, base + g * p2)
    h2 = ScalarOp(grid, base + (beta_n - beta_s) * p2)
    h3 = ScalarOp(grid, base + 3.0 * g * p2)
    ph = np.asarray(phi, dtype=np.float64).reshape(grid.shape)
    out = {}
    om_d, rd = product_branch(h0, h3, ph, counts["density"], tol, verbose=verbose)
    out["density"] = (om_d, 1, rd)
    rm = symmetric_branch(h0, counts["magnon"], tol, phi=ph, verbose=verbose)
    out["magnon"] = (rm.values, 1, rm)
    rg = symmetric_branch(h2, counts["gapped"], tol, verbose=verbose)
    out["gapped"] = (rg.values, 1, rg)
    return _finish(out, k_total)


def polar_branches(phi, mu, V, beta_n, beta_s, n, L, counts: dict, tol: float = 1e-9,
                   k_total: Optional[int] = None, verbose: bool = False) -> BranchSpectrum:
    """Polar M = 0 decomposition; counts = {"density": k_d, "spin": k_s} (the spin branch
    counts twice in the spectrum)."""
    grid = ScalarGrid(n, L)
    p2 = np.asarray(phi, dtype=np.float64).reshape(grid.shape) ** 2
    base = np.asarray(V, dtype=np.float64).reshape(grid.shape) - mu
    h0 = ScalarOp(grid, base + beta_n * p2)
    hs = ScalarOp(grid, base + (beta_n + 2.0 * beta_s) * p2)
    h3 = ScalarOp(grid, base + 3.0 * beta_n * p2)
    ph = np.asarray(phi, dtype=np.float64).reshape(grid.shape)
    out = {}
    om_d, rd = product_branch(h0, h3, ph, counts["density"], tol, verbose=verbose)
    out["density"] = (om_d, 1, rd)
    om_s, rs = product_branch(h0, hs, ph, counts["spin"], tol, verbose=verbose)
    out["spin"] = (om_s, 2, rs)
    return _finish(out, k_total)


def _finish(out, k_total):
    allv, ceiling = _merge(out, k_total)
    if k_total is not None:
        if len(allv) < k_total or not allv[k_total - 1] < ceiling:
            raise ValueError(f"branch counts too small: the {k_total}-th value {allv[min(k_total, len(allv)) - 1]} "
                             f"is not below the smallest branch ceiling {ceiling}")
        allv = allv[:k_total]
    return BranchSpectrum(omega=allv, branches=out, complete_below=ceiling)
