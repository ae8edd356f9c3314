"""Pins of the oracle subspace iteration: it must reach the plain dense result (the
k smallest positive eigenvalues of the BdG matrix), the branch and uniform closed forms,
with the eigenvector structure of Section 2.2 (bi-orthogonality, <f, g> = 1/4)."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import bdg, branch, lrep
from tests import _cases


def _solve(case, tol=1e-10):
    w, V, r, c = _cases.ground(case)
    X0 = W.start_block(w)
    out, prob, Nm, Qg = lrep.solve(c, r.phi, w.n, w.L, w.k, X0, tol, V=V, mu=r.mu)
    return w, V, r, c, out, prob, Nm, Qg


def test_c1_subspace_iteration_matches_dense():
    w, V, r, c, out, prob, Nm, Qg = _solve(_cases.C1)
    om_d, _ = bdg.positive_eigs_dense(bdg.dense_uv(c, w.n, w.L), w.k)
    assert np.allclose(out.omega, om_d, rtol=1e-11)
    assert out.residual.max() <= 1e-10
    # independent residual through the (u, v) operator of eq. (BdG-d)
    uv = bdg.fg_to_uv(out.X, w.dim)
    Y = bdg.apply_uv(c, uv, w.n, w.L)
    R = Y - out.omega[:, None, None] * uv
    assert np.linalg.norm(R.reshape(w.k, -1), axis=1).max() < 1e-8 * np.linalg.norm(uv.reshape(w.k, -1), axis=1).min()
    assert (Nm.shape[1], Qg.shape[1]) == (2, 2)


def test_eigenvector_structure():
    w, V, r, c, out, prob, Nm, Qg = _solve(_cases.C1)
    hd = prob.hd
    f = out.X[:, :3].reshape(w.k, -1)
    g = out.X[:, 3:].reshape(w.k, -1)
    FG = hd * (f @ g.conj().T)          # <f_i, g_j>
    # normalization <f, g> = 1/4, i.e. int |u|^2 - |v|^2 = 1
    assert np.allclose(np.diag(FG), 0.25, atol=1e-12)
    uv = bdg.fg_to_uv(out.X, w.dim)
    norm_uv = hd * (np.sum(np.abs(uv[:, :3]) ** 2, axis=(1, 2)) - np.sum(np.abs(uv[:, 3:]) ** 2, axis=(1, 2)))
    assert np.allclose(norm_uv, 1.0, atol=1e-11)
    # bi-orthogonality for |omega_i| != |omega_j|
    off = FG - np.diag(np.diag(FG))
    assert np.abs(off).max() < 1e-9
    # Rayleigh quotient equals omega
    assert np.allclose(bdg.rayleigh_omega(c, out.X, w.n, w.L, w.h), out.omega, rtol=1e-12)


def test_fm_2d_matches_dense_and_branch():
    w, V, r, c, out, *_ = _solve(_cases.FM_2D)
    ev = scipy.linalg.eigvals(bdg.dense_uv(c, w.n, w.L))
    pos = np.sort(ev.real[(ev.real > 1e-5) & (np.abs(ev.imag) < 1e-7)])[:w.k]
    assert np.allclose(out.omega, pos, rtol=1e-10)
    M = w.magnetization
    phi = np.tensordot(np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2]), r.phi, axes=1)
    ref = branch.fm_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, w.k)
    assert np.allclose(out.omega, ref, rtol=1e-9)


def test_polar_2d_matches_branch():
    w, V, r, c, out, prob, Nm, Qg = _solve(_cases.POLAR_2D)
    phi = r.phi[0] * np.sqrt(2)
    ref = branch.polar_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, w.k)
    assert np.allclose(out.omega, ref, rtol=1e-9)
    assert (Nm.shape[1], Qg.shape[1]) == (3, 3)


def test_3d_matches_dense_with_kohn_modes():
    w, V, r, c, out, *_ = _solve(_cases.FM_3D)
    ev = scipy.linalg.eigvals(bdg.dense_uv(c, w.n, w.L))
    pos = np.sort(ev.real[(ev.real > 1e-5) & (np.abs(ev.imag) < 1e-7)])[:w.k]
    assert np.allclose(out.omega, pos, rtol=1e-10)


@pytest.mark.parametrize("kind,bs", [("fm", -1.0), ("polar", 1.0)])
def test_uniform_2d_matches_dispersion(kind, bs):
    n, L = (16, 16), (4.0, 4.0)
    phi, mu = branch.uniform_ground_state(n, L, 20.0, bs, 0.0, kind)
    V = np.zeros((16, 16))
    c = bdg.coefficients(phi, mu, V, 20.0, bs)
    w = W.Workload("u", 2, n, L, "zero", 20.0, bs, 0.0)
    X0 = W.start_block(w, nvec=12)
    out, *_ = lrep.solve(c, phi, n, L, 8, X0, 1e-10, V=V, mu=mu)
    ref = branch.uniform_spectrum(n, L, 20.0, bs, kind, 8)
    assert np.allclose(out.omega, ref, rtol=1e-12)


def test_preconditioner_is_symmetric_positive_and_path_independent():
    """The kinetic-potential preconditioner is Hermitian positive definite (so it cannot
    change the fixed points of the iteration), D = 1 where V <= mu, and the kinetic-only
    preconditioner reaches the same eigenvalues."""
    w, V, r, c = _cases.ground(_cases.C1)
    sigma, D = lrep.preconditioner_parameters(V, r.mu)
    assert sigma == max(0.5 * r.mu[1], 0.5)
    assert np.all(D <= 1.0) and np.all(D > 0.0)
    assert np.all(D[V <= r.mu[1]] == 1.0)
    prob = lrep.LrepProblem(c, w.n, w.L, D)
    n3 = 3 * V.size
    T = prob.precond(np.eye(n3, dtype=np.complex128), sigma)
    assert np.abs(T - T.conj().T).max() < 1e-14 * np.abs(T).max()
    assert np.linalg.eigvalsh(0.5 * (T + T.conj().T)).min() > 0
    X0 = W.start_block(w)
    a, *_ = lrep.solve(c, r.phi, w.n, w.L, w.k, X0, 1e-10, V=V, mu=r.mu)
    b, *_ = lrep.solve(c, r.phi, w.n, w.L, w.k, X0, 1e-10)
    assert np.allclose(a.omega, b.omega, rtol=1e-11)
    assert a.iters < b.iters
