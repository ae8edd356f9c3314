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


def _grid3(n=64, L=8.0):
    x = -L + (2 * L / n) * np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return (n, n, n), (L, L, L), X, Y, Z


def test_mode_amplitudes_of_gaussian_fields_match_closed_forms():
    """|w|^2 = x^2 exp(-r^2): N = pi^(3/2)/2, <x^2> = 3/2, <y^2> = <z^2> = 1/2, odd in x and
    even in y, z, max |w| = e^(-1/2) (at x = 1, on the grid); the trapezoid sums of these
    decaying fields equal the integrals to rounding.  Second field exp(-(x^2 + y^2 + 4 z^2)/2)
    y z: even in x, odd in y and z, and compressed along z (<z^2> = 3/8 against <y^2> = 3/2)."""
    n, L, X, Y, Z = _grid3()
    g = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 2)
    uv = np.zeros((2, 6) + n, dtype=complex)
    uv[0, 0] = X * g
    uv[0, 4] = (1 + 2j) * X * g          # a phase and a scale change nothing but N
    uv[1, 5] = np.exp(-(X ** 2 + Y ** 2 + 4 * Z ** 2) / 2) * Y * Z
    out = modes.mode_amplitudes(uv, n, L)
    r = out[0, 0]
    assert np.isclose(r[0], np.pi ** 1.5 / 2, rtol=1e-13)
    assert np.isclose(r[1], np.exp(-0.5), rtol=1e-13)
    assert np.allclose(r[2:5], [1.5, 0.5, 0.5], rtol=1e-12)
    assert np.allclose(r[5:8], [-1.0, 1.0, 1.0], atol=1e-13)
    q = out[0, 4]
    assert np.isclose(q[0], 5 * r[0], rtol=1e-13)
    assert np.allclose(q[2:], r[2:], atol=1e-13)
    # |w|^2 = y^2 z^2 exp(-(x^2 + y^2 + 4 z^2)): <x^2> = 1/2, <y^2> = 3/2, <z^2> = 3/8
    s = out[1, 5]
    assert np.allclose(s[2:5], [0.5, 1.5, 0.375], rtol=1e-12)
    assert np.allclose(s[5:8], [1.0, -1.0, -1.0], atol=1e-13)
    # empty fields report zeros
    assert np.all(out[0, 1] == 0.0) and np.all(out[1, 0] == 0.0)


def test_mode_amplitudes_parity_of_even_and_odd_parts():
    rng = np.random.default_rng(4)
    n, L = (8, 16), (3.0, 5.0)
    w = rng.standard_normal((16, 8)) + 1j * rng.standard_normal((16, 8))
    rx = np.roll(np.flip(w, axis=1), 1, axis=1)          # x runs along the last axis
    uv = np.zeros((1, 6, 16, 8), dtype=complex)
    uv[0, 0] = (w + rx) / 2
    uv[0, 1] = (w - rx) / 2
    out = modes.mode_amplitudes(uv, n, L)
    assert np.isclose(out[0, 0, 5], 1.0, atol=1e-14) and np.isclose(out[0, 1, 5], -1.0, atol=1e-14)
    assert out[0, 0, 7] == 0.0 and out[0, 0, 4] == 0.0     # no z axis in 2-D
