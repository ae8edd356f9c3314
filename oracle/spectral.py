"""Fourier pseudo-spectral discretization (Section 3.1, eqs. laplace_approx and FT_3).

TEST INFRASTRUCTURE (CPU oracle).

Grid: N points per axis on [-L, L), x_n = -L + n h, h = 2L/N, n = 0..N-1 (the paper's
index ranges are garbled; this reading keeps N points, periodic).  Plane waves
W_k(x) = exp(i mu_k (x + L)), mu_k = pi k / L, k = -N/2 .. N/2-1.  The discrete
Laplacian multiplies the k-th DFT coefficient by -mu_k^2 (Nyquist mode k = -N/2
included).  Arrays hold grid fields with x fastest: shape (..., Nz, Ny, Nx).

Pins: the FFT kinetic operator equals the explicit cosine-sum matrix (``kinetic_matrix``),
plane waves are its eigenvectors with eigenvalue mu_k^2/2, and it reproduces the exact
second derivative of band-limited trigonometric polynomials.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

# host threads for the FFTs: the OpenMP thread count when one is set, else every core
WORKERS = max(1, int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1))


def fftn(F: np.ndarray, axes) -> np.ndarray:
    """Unnormalized forward DFT over ``axes`` (pocketfft, WORKERS threads)."""
    return scipy.fft.fftn(F, axes=axes, workers=WORKERS)


def ifftn(F: np.ndarray, axes) -> np.ndarray:
    """Inverse DFT over ``axes`` with the 1/N factor (pocketfft, WORKERS threads)."""
    return scipy.fft.ifftn(F, axes=axes, workers=WORKERS)


def wavenumbers(n: int, L: float) -> np.ndarray:
    """mu_k = pi*k/L for k in FFT storage order 0..N/2-1, -N/2..-1."""
    k = np.fft.fftfreq(n, d=1.0 / n)          # exact integers, Nyquist stored as -N/2
    return np.pi * k / L


def kinetic_symbol(n, L) -> np.ndarray:
    """|mu|^2 / 2 on the DFT grid, shape (Nz, Ny, Nx)[-d:] (x fastest)."""
    mus = [wavenumbers(ni, Li) for ni, Li in zip(n, L)]
    grids = np.meshgrid(*reversed(mus), indexing="ij")     # (z, y, x) order
    return 0.5 * sum(g * g for g in grids)


def kinetic_apply(F: np.ndarray, n, L) -> np.ndarray:
    """-(1/2) Laplacian of grid fields F (last d axes are the grid), via numpy FFT."""
    d = len(n)
    axes = tuple(range(-d, 0))
    sym = kinetic_symbol(n, L)
    return ifftn(sym * fftn(F, axes=axes), axes=axes)


def kinetic_matrix_1d(n: int, L: float) -> np.ndarray:
    """Dense 1-D matrix of -(1/2) d^2/dx^2 in the Fourier pseudo-spectral basis.

    Written out from the definition: (T F)_p = sum_q T_pq F_q with
    T_pq = (1/N) sum_k (mu_k^2 / 2) exp(2 pi i k (p - q) / N); the sum is real
    because mu_k^2 is even in k and the Nyquist term is (-1)^(p-q).
    """
    ks = np.arange(-n // 2, n // 2)
    mu2 = (np.pi * ks / L) ** 2
    p = np.arange(n)
    diff = p[:, None] - p[None, :]
    T = np.zeros((n, n))
    for kk, m2 in zip(ks, mu2):
        T += 0.5 * m2 * np.cos(2.0 * np.pi * kk * diff / n)
    return T / n


def kinetic_matrix(n, L) -> np.ndarray:
    """Dense d-dimensional kinetic matrix (Kronecker sum of the 1-D ones), x fastest."""
    mats = [kinetic_matrix_1d(ni, Li) for ni, Li in zip(n, L)]
    sizes = list(n)
    total = int(np.prod(sizes))
    T = np.zeros((total, total))
    for axis, Ta in enumerate(mats):
        # index = x + Nx*(y + Ny*z): axis 0 (x) is the fastest
        left = int(np.prod(sizes[axis + 1:]))      # slower axes
        right = int(np.prod(sizes[:axis]))         # faster axes
        T += np.kron(np.kron(np.eye(left), Ta), np.eye(right))
    return T


def inner(a: np.ndarray, b: np.ndarray, h) -> complex:
    """Discrete inner product <a, b> = h^d sum a * conj(b) (inner product of Section 2.1 on the grid, as in Section 3.4)."""
    return complex(np.prod(h) * np.vdot(b, a))


def norm(a: np.ndarray, h) -> float:
    return float(np.sqrt(np.prod(h)) * np.linalg.norm(a.ravel()))
