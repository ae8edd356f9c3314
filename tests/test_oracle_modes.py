"""Pins of the perturbed-density formula of Section 4.2 (oracle.modes)."""
import numpy as np

from oracle import modes


def _data(seed=0, n=17):
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((3, n))
    uv = rng.standard_normal((2, 6, n)) + 1j * rng.standard_normal((2, 6, n))
    return phi, uv, np.array([0.7, 2.3]), np.array([0.0, 0.4, 10.6])


def test_zero_amplitude_is_the_ground_state_density():
    phi, uv, om, t = _data()
    n = modes.perturbed_density(phi, uv, om, 0.0, t)
    assert np.array_equal(n, np.broadcast_to(phi ** 2, n.shape))


def test_real_modes_match_the_closed_form():
    """u, v, phi real: u e^{-iwt} + v e^{iwt} = (u + v) cos wt - i (u - v) sin wt."""
    phi, uv, om, t = _data(1)
    uv = uv.real.astype(complex)
    eps = 0.1
    n = modes.perturbed_density(phi, uv, om, eps, t)
    for l, w in enumerate(om):
        u, v = uv[l, :3].real, uv[l, 3:].real
        for s, ts in enumerate(t):
            ref = (phi + eps * (u + v) * np.cos(w * ts)) ** 2 + (eps * (u - v) * np.sin(w * ts)) ** 2
            assert np.allclose(n[l, s], ref, rtol=1e-14, atol=1e-14)


def test_conjugation_of_v_and_period():
    """A purely imaginary v enters through conj(v); the density repeats after 2 pi / omega."""
    phi, uv, om, _ = _data(2)
    uv[:, 3:] = 1j * uv[:, 3:].imag
    eps = 0.3
    w = om[0]
    t = np.array([0.37, 0.37 + 2 * np.pi / w])
    n = modes.perturbed_density(phi, uv[:1], om[:1], eps, t)
    assert np.allclose(n[0, 0], n[0, 1], rtol=1e-12, atol=1e-12)
    # at t = 0: |phi + eps (u + conj(v))|^2 with conj(v) = -v for imaginary v
    n0 = modes.perturbed_density(phi, uv[:1], om[:1], eps, np.array([0.0]))
    ref = np.abs(phi + eps * (uv[0, :3] - uv[0, 3:])) ** 2
    assert np.allclose(n0[0, 0], ref, rtol=1e-14, atol=1e-14)
