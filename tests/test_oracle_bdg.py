"""Pins of the oracle BdG operator and dense spectra (Sections 2.1-2.3, 3.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import bdg, branch, groundstate as gs, spectral
from tests import _cases


def _herm_field(M):
    return np.abs(M - np.conj(np.swapaxes(M, 0, 1))).max()


def test_operator_symmetries_for_complex_spinor():
    """A = A^H, D = D^H, B = B^T, C = -conj(B), D = -conj(A) hold pointwise for any Phi."""
    rng = np.random.default_rng(2)
    phi = rng.standard_normal((3, 7)) + 1j * rng.standard_normal((3, 7))
    V = rng.standard_normal(7)
    c = bdg.coefficients(phi, np.array([0.3, 0.2, 0.1]), V, 2.0, -0.7)
    assert _herm_field(c.A) < 1e-13
    assert _herm_field(c.D) < 1e-13
    assert np.abs(c.B - np.swapaxes(c.B, 0, 1)).max() < 1e-13
    assert np.abs(c.C + np.conj(c.B)).max() < 1e-13
    assert np.abs(c.D + np.conj(c.A)).max() < 1e-13


def test_real_ground_state_gives_real_operators():
    _, _, _, c = _cases.ground(_cases.C1)
    for M in (c.A, c.B, c.C, c.D):
        assert np.abs(M.imag).max() == 0.0
    assert np.abs(c.C + c.B).max() == 0.0 and np.abs(c.D + c.A).max() == 0.0


@pytest.mark.parametrize("case", ["C1", "FM_2D"])
def test_fft_apply_equals_dense_product(case):
    w, V, r, c = _cases.ground(getattr(_cases, case))
    Hd = bdg.dense_uv(c, w.n, w.L)
    X = W.random_block((3, 6) + w.shape, 11)
    Y = bdg.apply_uv(c, X, w.n, w.L)
    Yd = (Hd @ X.reshape(3, -1).T).T.reshape(Y.shape)
    assert np.abs(Y - Yd).max() <= 1e-12 * np.abs(Yd).max()
    # (f, g) form equals the change of variables applied to the (u, v) form
    Xfg = bdg.uv_to_fg(X, w.dim)
    Yfg = bdg.apply_fg(c, Xfg, w.n, w.L)
    Yu, Yv = Y[:, :3], Y[:, 3:]
    assert np.allclose(Yfg[:, :3], (Yu + Yv) / 2, atol=1e-11 * np.abs(Y).max())
    assert np.allclose(Yfg[:, 3:], (Yu - Yv) / 2, atol=1e-11 * np.abs(Y).max())


def _dense_spectrum(case):
    w, V, r, c = _cases.ground(case)
    import scipy.linalg
    ev = scipy.linalg.eigvals(bdg.dense_uv(c, w.n, w.L))
    return w, V, r, c, ev


def test_c1_dense_spectrum_structure():
    w, V, r, c, ev = _dense_spectrum(_cases.C1)
    # Symmetric distribution theorem: +-omega pairs (real ground state)
    pos = np.sort(ev.real[ev.real > 1e-5])
    neg = np.sort(-ev.real[ev.real < -1e-5])
    assert np.allclose(pos, neg, atol=1e-10)
    # generalized nullspace of the FM theorem: dimension 4 (3 null + 1 Jordan partner)
    assert np.sum(np.abs(ev) < 1e-5) == 4
    # analytic Kohn mode omega_x = gamma_x = 1
    assert np.min(np.abs(pos - 1.0)) < 1e-10


def test_polar_dense_zero_mode_count_is_six():
    """At M = 0 the polar H_- is diag(h0, h0, h0): ns(H_-) is 3-dimensional and the
    generalized nullspace of H has dimension 6."""
    w, V, r, c, ev = _dense_spectrum(_cases.POLAR_1D)
    assert np.sum(np.abs(ev) < 1e-4) == 6
    Hp, Hm = bdg.dense_hpm(c, w.n, w.L)
    assert np.sum(np.abs(np.linalg.eigvalsh(Hm.real)) < 1e-9) == 3
    assert np.linalg.eigvalsh(Hp.real).min() > 1e-3


def test_fm_dense_null_spaces():
    w, V, r, c = _cases.ground(_cases.C1)
    Hp, Hm = bdg.dense_hpm(c, w.n, w.L)
    ep, em = np.linalg.eigvalsh(Hp.real), np.linalg.eigvalsh(Hm.real)
    assert np.sum(np.abs(em) < 1e-9) == 2 and np.sum(np.abs(ep) < 1e-9) == 1
    assert em.min() > -1e-9 and ep.min() > -1e-9      # both positive semidefinite
    M = w.magnetization
    b = np.array([np.sqrt((1 - M * M) / 2), -M, -np.sqrt((1 - M * M) / 2)])
    phi_g = r.phi.T @ np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2])
    Phi2 = (b[:, None] * phi_g[None]).ravel()
    assert np.linalg.norm(Hp.real @ Phi2) < 1e-10 and np.linalg.norm(Hm.real @ Phi2) < 1e-10


def test_fm_dense_equals_branch_decomposition():
    w, V, r, c, ev = _dense_spectrum(_cases.C1)
    pos = np.sort(ev.real[(ev.real > 1e-5) & (np.abs(ev.imag) < 1e-8)])[:40]
    M = w.magnetization
    phi = r.phi.T @ np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2])
    ref = branch.fm_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, 40)
    assert np.allclose(pos, ref, rtol=1e-9, atol=1e-11)


def test_polar_dense_equals_branch_decomposition():
    w, V, r, c, ev = _dense_spectrum(_cases.POLAR_1D)
    pos = np.sort(ev.real[(ev.real > 1e-4) & (np.abs(ev.imag) < 1e-6)])[:30]
    phi = r.phi[0] * np.sqrt(2)
    ref = branch.polar_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, 30)
    assert np.allclose(pos, ref, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("kind,bs", [("fm", -1.0), ("polar", 1.5)])
def test_uniform_state_dense_equals_dispersion(kind, bs):
    n, L = (24,), (3.0,)
    phi, mu = branch.uniform_ground_state(n, L, 6.0, bs, 0.0, kind)
    V = np.zeros(24)
    c = bdg.coefficients(phi, mu, V, 6.0, bs)
    import scipy.linalg
    ev = scipy.linalg.eigvals(bdg.dense_uv(c, n, L))
    pos = np.sort(ev.real[ev.real > 1e-6])[:20]
    ref = branch.uniform_spectrum(n, L, 6.0, bs, kind, 20)
    assert np.allclose(pos, ref, rtol=1e-11, atol=1e-10)
