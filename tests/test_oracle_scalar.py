"""Pins of the matrix-free scalar branch oracle (Section 2.3 structure results).

The scalar operators are checked against the explicit cosine-sum matrices of ``branch``,
the LOBPCG against LAPACK's dense symmetric(-definite) eigensolvers, and the merged branch
spectra against both the dense branch decompositions and the dense six-component BdG
eigensolve (which is itself pinned to the zero-mode counts, the +-omega pairing and the
Kohn modes in test_oracle_bdg.py).
"""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import bdg, branch, scalar
from tests import _cases

FM_WEIGHTS = lambda M: np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2])


def _fm_profile(case):
    w, V, r, c = _cases.ground(case)
    phi = np.tensordot(FM_WEIGHTS(w.magnetization), r.phi, axes=1)
    return w, V, r, c, phi


@pytest.mark.parametrize("case", ["C1", "FM_2D", "FM_3D"])
def test_scalar_apply_equals_dense_matrix(case):
    w, V, r, c, phi = _fm_profile(getattr(_cases, case))
    U = V - r.mu[0] + (w.beta_n + w.beta_s) * phi ** 2
    h = scalar.ScalarOp(scalar.ScalarGrid(w.n, w.L), U)
    X = np.random.default_rng(3).standard_normal((3,) + w.shape)
    Hd = branch._scalar_dense(U, w.n, w.L)
    ref = (Hd @ X.reshape(3, -1).T).T.reshape(X.shape)
    assert np.abs(h(X) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_lobpcg_standard_and_generalized_match_lapack():
    rng = np.random.default_rng(5)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * np.linspace(0.5, 40.0, n)) @ Q.T
    G = rng.standard_normal((n, n))
    B = G @ G.T / n + np.eye(n)
    mat = lambda M: (lambda Z: (M @ Z.T).T)
    Tinv = np.linalg.inv(A + np.eye(n))
    X0 = rng.standard_normal((8, n))
    r1 = scalar.lobpcg(lambda Z: (mat(A)(Z), Z), mat(Tinv), X0, 6, 1e-11)
    assert np.allclose(r1.values, np.linalg.eigvalsh(A)[:6], rtol=1e-12)
    r2 = scalar.lobpcg(lambda Z: (mat(A)(Z), mat(B)(Z)), mat(Tinv), X0, 6, 1e-11)
    ref = scipy.linalg.eigh(A, B, eigvals_only=True)[:6]
    assert np.allclose(r2.values, ref, rtol=1e-12)
    # B-orthonormal eigenvectors with A z = lambda B z
    Z = r2.vectors
    assert np.allclose(Z @ B @ Z.T, np.eye(6), atol=1e-10)
    assert np.abs(Z @ A - r2.values[:, None] * (Z @ B)).max() < 1e-8


@pytest.mark.parametrize("case", ["C1", "FM_2D", "FM_3D"])
def test_fm_branches_match_dense_decomposition(case):
    w, V, r, c, phi = _fm_profile(getattr(_cases, case))
    dens, mag, gap = branch.fm_branches_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L)
    bs = scalar.fm_branches(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L,
                            {"density": 8, "magnon": 8, "gapped": 8}, tol=1e-10, k_total=12)
    for name, ref in (("density", dens[dens > 1e-6][:8]), ("magnon", mag[mag > 1e-6][:8]), ("gapped", gap[:8])):
        assert np.allclose(bs.branches[name][0], ref, rtol=1e-11), name
    ref = branch.fm_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, 12)
    assert np.allclose(bs.omega, ref, rtol=1e-11)


def test_fm_branches_match_six_component_dense_eigensolve():
    """3-D grid: the merged scalar spectra equal the 6-component BdG operator's eigenvalues."""
    w, V, r, c, phi = _fm_profile(_cases.FM_3D)
    bs = scalar.fm_branches(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L,
                            {"density": 8, "magnon": 10, "gapped": 10}, tol=1e-10, k_total=16)
    om, _ = bdg.positive_eigs_dense(bdg.dense_uv(c, w.n, w.L), 16)
    assert np.allclose(bs.omega, om, rtol=1e-9)


@pytest.mark.parametrize("case", ["POLAR_1D", "POLAR_2D"])
def test_polar_branches_match_dense(case):
    w, V, r, c = _cases.ground(getattr(_cases, case))
    phi = r.phi[0] * np.sqrt(2)
    bs = scalar.polar_branches(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, {"density": 8, "spin": 8},
                               tol=1e-10, k_total=10)
    ref = branch.polar_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, 10)
    assert np.allclose(bs.omega, ref, rtol=1e-11)
    # the six-dimensional generalized nullspace (Jordan blocks) perturbs geev's zero modes and
    # the values near them at the 1e-8 level: exclude |omega| <= 1e-4 and compare to 1e-8
    om, _ = bdg.positive_eigs_dense(bdg.dense_uv(c, w.n, w.L), 10, zero_tol=1e-4)
    assert np.allclose(bs.omega, om, rtol=1e-8)


def test_branch_counts_that_miss_values_are_rejected():
    """Too few values of one branch: the merged k-th value would not be certified."""
    w, V, r, c, phi = _fm_profile(_cases.C1)
    with pytest.raises(ValueError):
        scalar.fm_branches(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L,
                           {"density": 2, "magnon": 2, "gapped": 2}, tol=1e-9, k_total=12)
