"""Pins of the complex-ground-state inputs (oracle.complexgs) and of the oracle's general
BdG operator [[A, B], [-conj(B), -conj(A)]] on them (Section 2.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import bdg, complexgs, groundstate as gs, spin


@pytest.mark.parametrize("w", [
    W.Workload("1d_32_fm", 1, (32,), (8.0,), "harmonic1", 10.0, -0.5, 0.2),
    W.Workload("1d_32_afm", 1, (32,), (8.0,), "harmonic1", 10.0, 1.0, 0.3),
], ids=lambda w: w.name)
def test_rotated_state_keeps_the_spectrum(w):
    V = W.potential(w)
    r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L, W.initial_spinor(w), tol=1e-12)
    om_r, _ = bdg.positive_eigs_dense(bdg.dense_uv(bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s), w.n, w.L),
                                      12)
    phc = complexgs.rotate(r.phi, 0.7, 0.3)
    assert np.abs(phc.imag).max() > 0.1
    c = bdg.coefficients(phc, r.mu, V, w.beta_n, w.beta_s)
    assert np.abs(c.A.imag).max() > 1e-3 or np.abs(c.B.imag).max() > 1e-3
    om_c, _ = bdg.positive_eigs_dense(bdg.dense_uv(c, w.n, w.L), 12)
    assert np.allclose(om_c, om_r, rtol=1e-9)


def test_moving_polar_state_is_stationary_and_doppler_shifted():
    n, L, bn, bs = (16, 8), (4.0, 3.0), 100.0, 40.0
    phi, mu, q = complexgs.moving_polar_state(n, L, bn, 1)
    V = np.zeros(tuple(reversed(n)))
    # H(Phi) Phi = Lambda Phi with Lambda = mu (M = 0, no multiplier on S_z)
    rhs = spin.gpe_rhs_compact(phi, V, bn, bs, n, L)
    assert np.abs(rhs - mu[0] * phi).max() <= 1e-12 * np.abs(rhs).max()
    om, _ = bdg.positive_eigs_dense(bdg.dense_uv(bdg.coefficients(phi, mu, V, bn, bs), n, L), 16)
    ref = complexgs.moving_polar_spectrum(n, L, bn, bs, q, 16)
    assert np.allclose(om, ref, rtol=1e-9, atol=1e-10)
    # the shift is visible: the spectrum at rest differs
    rest = complexgs.moving_polar_spectrum(n, L, bn, bs, 0.0, 16)
    assert np.abs(rest - ref).max() > 1e-2
