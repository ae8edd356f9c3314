"""Pins of the oracle eigenvalue gradient: central finite differences of the whole pipeline
(ground state re-solved, dense eigensolve) and of the frozen-ground-state operator."""
import numpy as np

import workloads as W
from oracle import bdg, grad, groundstate as gs

CASE = W.Workload("1d_64_fm", 1, (64,), (8.0,), "harmonic1", 10.0, -0.5, 0.2)


def _solve(w, V, bn, bs, k=6):
    r = gs.ground_state(V, bn, bs, 1.0, w.magnetization, w.n, w.L, W.initial_spinor(w), tol=1e-13)
    c = bdg.coefficients(r.phi, r.mu, V, bn, bs)
    om, vec = bdg.positive_eigs_dense(bdg.dense_uv(c, w.n, w.L), k)
    X = bdg.uv_to_fg(vec.T.reshape((k, 6) + w.shape), w.dim)
    Xn, _ = bdg.normalize_fg(X, w.h, w.dim)
    return r, c, om, Xn


def test_gradient_matches_finite_differences_of_the_pipeline():
    w = CASE
    V0 = W.potential(w)
    r, c, om, X = _solve(w, V0, w.beta_n, w.beta_s)
    rng = np.random.default_rng(0)
    dV = rng.standard_normal(w.shape) * np.exp(-W.coordinates(w)[0] ** 2 / 8)
    dbn, dbs = rng.standard_normal(2)
    eps = 1e-5
    op = _solve(w, V0 + eps * dV, w.beta_n + eps * dbn, w.beta_s + eps * dbs)[2]
    om_ = _solve(w, V0 - eps * dV, w.beta_n - eps * dbn, w.beta_s - eps * dbs)[2]
    fd = (op - om_) / (2 * eps)
    for j in range(len(om)):
        gV, gbn, gbs = grad.eigen_gradient(r.phi, r.mu, V0, w.beta_n, w.beta_s, w.n, w.L, X[j])
        d = grad.directional(gV, gbn, gbs, (dV, dbn, dbs), w.h)
        assert abs(d - fd[j]) <= 1e-6 * abs(fd[j]), (j, d, fd[j])


def test_explicit_part_matches_frozen_ground_state_differences():
    """With Phi and Lambda frozen, d omega is the Hellmann-Feynman term alone; the oracle's
    explicit beta_n derivative must match the finite difference of the dense spectrum."""
    w = CASE
    V0 = W.potential(w)
    r, c, om, X = _solve(w, V0, w.beta_n, w.beta_s)
    eps = 1e-6
    # a frozen Phi is no longer a ground state of the perturbed problem, so the former zero
    # modes move off zero: match every eigenvalue to its nearest perturbed neighbour
    om_p, _ = bdg.positive_eigs_dense(bdg.dense_uv(bdg.coefficients(r.phi, r.mu, V0, w.beta_n + eps, w.beta_s),
                                                   w.n, w.L), 12, zero_tol=0.0)
    om_m, _ = bdg.positive_eigs_dense(bdg.dense_uv(bdg.coefficients(r.phi, r.mu, V0, w.beta_n - eps, w.beta_s),
                                                   w.n, w.L), 12, zero_tol=0.0)
    near = lambda arr, v: arr[np.argmin(np.abs(arr - v))]
    fd = np.array([(near(om_p, v) - near(om_m, v)) / (2 * eps) for v in om])
    hd = np.prod(w.h)
    Pn, Mn = grad._hpm_parts(r.phi, 1.0, 0.0)
    for j in range(6):
        f, g = X[j, :3], X[j, 3:]
        s = 1.0 / (2 * hd * np.real(np.vdot(g, f)))
        hf = s * hd * np.sum(grad._pw_form(Pn, f) + grad._pw_form(Mn, g))
        assert abs(hf - fd[j]) <= 1e-6 * max(1.0, abs(fd[j]))
