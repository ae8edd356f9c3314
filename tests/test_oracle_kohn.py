"""Pins of the analytical Kohn pairs and the accuracy measures of Section 4.1 (oracle.kohn).

The analytical pair is checked against the oracle's discrete operator (a closed form of the
theorem "Analytical eigenpairs" against the operator written from eqs. def_A-def_D), and the
1-D accuracy errors against the values the paper prints in Table Err_1D."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import bdg, groundstate as gs, kohn, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table_err_1d.json")


def _ground(w, phi0=None, tol=1e-13):
    V = W.potential(w)
    p0 = W.initial_spinor(w) if phi0 is None else phi0
    r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L, p0, tol=tol)
    return V, r, bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)


@pytest.mark.parametrize("w,bound", [
    (W.Workload("1d_n256_fm", 1, (256,), (16.0,), "harmonic1", 10.0, -0.5, 0.2), 1e-10),
    (W.Workload("2d_n80_aniso_polar", 2, (80, 80), (7.0, 7.0), "harmonic2_aniso", 20.0, 1.0, 0.0), 1e-6),
], ids=lambda x: getattr(x, "name", ""))
def test_analytic_pair_is_an_eigenpair_of_the_discrete_operator(w, bound):
    V, r, c = _ground(w, tol=1e-12)
    gammas = W.TRAP_GAMMAS[w.potential]
    for a in range(w.dim):
        om, u, v = kohn.kohn_pair(r.phi, w.n, w.L, gammas, a)
        X = np.concatenate([u, v])[None].astype(complex)
        res = bdg.apply_uv(c, X, w.n, w.L) - om * X
        assert np.linalg.norm(res) <= bound * np.linalg.norm(X)
        # the normalization of the theorem: <f, g> = 1/4 with f = (u + v)/2, g = (u - v)/2
        f, g = (u + v) / 2, (u - v) / 2
        assert abs(spectral.inner(f, g, w.h) - 0.25) <= 1e-10


def test_pair_sign_and_scale_are_fixed():
    """Swapping u and v, or dropping the gamma^{-+1/2} weights, leaves no eigenpair at +gamma:
    the 2-D anisotropic y-mode (gamma = 2) tells both apart."""
    w = W.Workload("2d_n80_aniso_polar", 2, (80, 80), (7.0, 7.0), "harmonic2_aniso", 20.0, 1.0, 0.0)
    V, r, c = _ground(w, tol=1e-12)
    om, u, v = kohn.kohn_pair(r.phi, w.n, w.L, (1.0, 2.0), 1)
    dphi = kohn.derivative(r.phi, w.n, w.L, 1)
    yphi = kohn.coordinate(w.n, w.L, 1)[None] * r.phi

    def rel(uu, vv):
        X = np.concatenate([uu, vv])[None].astype(complex)
        return np.linalg.norm(bdg.apply_uv(c, X, w.n, w.L) - om * X) / np.linalg.norm(X)

    assert rel(u, v) <= 1e-6
    assert rel(v, u) > 1e-1
    assert rel(dphi - yphi, dphi + yphi) > 1e-1


def _errors(w, phi0=None):
    V, r, c = _ground(w, phi0)
    om, X = bdg.positive_eigs_dense(bdg.dense_uv(c, w.n, w.L), 40)
    uv = np.asarray(X).T.reshape((-1, 6) + w.shape)
    return r, kohn.accuracy_errors(om, uv, r.phi, w.n, w.L, (1.0,))[0]


@pytest.mark.parametrize("kind", ["FM", "AFM"])
def test_1d_errors_reproduce_table_err_1d(kind):
    """Case I of Section 4.1 at h = 1, 1/2, 1/4 (N = 32, 64, 128 on [-16, 16], M = 0).

    FM e_omega at N = 64 and 128 agrees with the printed values to their 4 digits; the other
    e_omega entries, and e_uv at N = 64 and 128, agree within a factor 5 (reading: the paper
    does not state the accuracy of its ground states, which sets the coarse-grid and AFM
    values at this level).  e_uv at h = 1 is not compared: the printed AFM value 0.91 says the
    paper's computed vector there was nearly orthogonal to the analytical one, i.e. another
    mode of the coarse spectrum was matched.  The coarse grids start from the N = 128 ground
    state sampled at their points (the same minimizer, reached in a few hundred steps
    instead of 10^5)."""
    with open(GOLDEN) as f:
        tab = json.load(f)
    bn, bs = tab["setup"][kind]
    ref = tab[kind]
    fine = None
    got = {}
    for n in (128, 64, 32):
        w = W.Workload(f"1d_n{n}_{kind}", 1, (n,), (16.0,), "harmonic1", bn, bs, 0.0)
        r, e = _errors(w, None if fine is None else fine[:, ::128 // n])
        if fine is None:
            fine = r.phi
        got[n] = e
    for i, n in enumerate(tab["N"][:3]):
        e, p_om, p_uv = got[n], ref["e_omega"][i], ref["e_uv"][i]
        assert p_om / 5 <= e["e_omega"] <= 5 * p_om, (n, e, p_om)
        if n > 32:
            assert p_uv / 5 <= e["e_uv"] <= 5 * p_uv, (n, e, p_uv)
        if kind == "FM" and n in (64, 128):
            assert e["e_omega"] == pytest.approx(p_om, rel=1e-3)
