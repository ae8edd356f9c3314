"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds no arithmetic of the method: it only describes the five
workloads (grid, box, trap, interaction strengths, magnetization, solver sizes)
and draws the seeded random inputs (start blocks, test blocks, finite-difference
directions).  Both the oracle and the GPU path receive these arrays as inputs.

Conventions (Section 3.1 of the paper, Fourier pseudo-spectral discretization):
  * box [-L, L] per axis, N points per axis, h = 2L/N, x_n = -L + n*h, n = 0..N-1;
  * a grid field is stored with x fastest: shape (Nz, Ny, Nx) in 3-D, (Ny, Nx) in 2-D;
  * a trial vector holds six complex grid fields, ordered
    (f_1, f_0, f_-1, g_1, g_0, g_-1) in the (f, g) form or
    (u_1, u_0, u_-1, v_1, v_0, v_-1) in the (u, v) form;
  * a block of b trial vectors is a C-contiguous array of shape (b, 6, *grid).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic trapped-condensate setup."""

    name: str
    dim: int
    n: Tuple[int, ...]          # points per axis, ordered (x, y, z)
    L: Tuple[float, ...]        # half box length per axis, ordered (x, y, z)
    potential: str              # key into POTENTIALS
    beta_n: float
    beta_s: float
    magnetization: float
    mass: float = 1.0
    k: int = 8                  # wanted eigenpairs
    block: int = 8              # block size of the subspace iteration
    tol: float = 1e-8           # relative residual target
    precision: str = "fp64"     # "fp64" or "fp32_apply"
    gs_tol: float = 1e-12       # ground-state residual target

    @property
    def shape(self) -> Tuple[int, ...]:
        """Array shape of one grid field (slowest axis first)."""
        return tuple(reversed(self.n))

    @property
    def npts(self) -> int:
        return int(np.prod(self.n))

    @property
    def h(self) -> Tuple[float, ...]:
        return tuple(2.0 * L / n for L, n in zip(self.L, self.n))

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def axis_points(n: int, L: float) -> np.ndarray:
    """Grid points x_j = -L + j*h, j = 0..n-1, h = 2L/n."""
    return -L + (2.0 * L / n) * np.arange(n, dtype=np.float64)


def coordinates(w: Workload):
    """Meshgrid of coordinates, each of shape w.shape, returned as (x, y, z)[:dim]."""
    axes = [axis_points(n, L) for n, L in zip(w.n, w.L)]
    # array axes are (z, y, x): build with reversed order then reverse back
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return tuple(reversed(mesh))


def _harmonic(gammas: Sequence[float]) -> Callable:
    def f(*xs):
        return 0.5 * sum((g * x) ** 2 for g, x in zip(gammas, xs))
    return f


def _harmonic_lattice_2d(*xs):
    x, y = xs
    return 0.5 * (x * x + y * y) + 0.5 * np.sin(x) ** 2 * np.sin(y) ** 2


def _harmonic_lattice_3d(*xs):
    x, y, z = xs
    return 0.5 * (x * x + y * y + z * z) + 5.0 * (
        np.sin(2 * x) ** 2 + np.sin(2 * y) ** 2 + np.sin(2 * z) ** 2)


POTENTIALS = {
    "harmonic1": _harmonic([1.0]),
    "harmonic2": _harmonic([1.0, 1.0]),
    "harmonic2_aniso": _harmonic([1.0, 2.0]),
    "harmonic3": _harmonic([1.0, 1.0, 1.0]),
    "harmonic3_z2": _harmonic([1.0, 1.0, 2.0]),
    "lattice2": _harmonic_lattice_2d,
    "lattice3": _harmonic_lattice_3d,
    "zero": lambda *xs: np.zeros_like(xs[0]),
}

# trap frequencies gamma_alpha of the harmonic potentials (for the analytic Kohn modes)
TRAP_GAMMAS = {
    "harmonic1": (1.0,),
    "harmonic2": (1.0, 1.0),
    "harmonic2_aniso": (1.0, 2.0),
    "harmonic3": (1.0, 1.0, 1.0),
    "harmonic3_z2": (1.0, 1.0, 2.0),
}


def potential(w: Workload) -> np.ndarray:
    """V(x) sampled on the grid, float64, shape w.shape."""
    return np.ascontiguousarray(POTENTIALS[w.potential](*coordinates(w)), dtype=np.float64)


# ----------------------------------------------------------------------------------------
# The five workloads (sizes of the paper's experiments: 1-D/2-D/3-D trapped condensates)
# ----------------------------------------------------------------------------------------
C1 = Workload("1d_n128_fm", 1, (128,), (16.0,), "harmonic1", 10.0, -0.5, 0.2,
              k=8, block=8, tol=1e-10, precision="fp64", gs_tol=1e-12)
C2_POLAR = Workload("2d_n256_polar", 2, (256, 256), (12.0, 12.0), "harmonic2", 100.0, 2.0, 0.0,
                    k=32, block=48, tol=1e-8, precision="fp64", gs_tol=1e-12)
C2_FM = C2_POLAR.with_(name="2d_n256_fm", beta_s=-2.0)
C3 = Workload("3d_n128_fm", 3, (128, 128, 128), (8.0, 8.0, 8.0), "harmonic3_z2", 400.0, -4.0, 0.1,
              k=64, block=80, tol=1e-8, precision="fp32_apply", gs_tol=1e-12)
C3_FP64 = C3.with_(name="3d_n128_fm_fp64", precision="fp64")
C4 = Workload("2d_n256_grad_fm", 2, (256, 256), (12.0, 12.0), "lattice2", 100.0, -2.0, 0.0,
              k=16, block=24, tol=1e-10, precision="fp64", gs_tol=1e-13)
C4_POLAR = C4.with_(name="2d_n256_grad_polar", beta_s=2.0)
C5 = Workload("3d_n256_lattice_fm", 3, (256, 256, 256), (10.0, 10.0, 10.0), "lattice3", 1000.0, -10.0, 0.0,
              k=64, block=64, tol=1e-6, precision="fp32_apply", gs_tol=1e-10)

ALL = {w.name: w for w in (C1, C2_POLAR, C2_FM, C3, C3_FP64, C4, C4_POLAR, C5)}


def scaled(w: Workload, n: int, name: Optional[str] = None) -> Workload:
    """The same physics on a coarser (or finer) grid with n points per axis."""
    return w.with_(n=tuple([n] * w.dim), name=name or f"{w.name}_n{n}")


# ----------------------------------------------------------------------------------------
# Seeded random inputs
# ----------------------------------------------------------------------------------------
def start_block(w: Workload, nvec: Optional[int] = None, seed: int = 0,
                dtype=np.complex128) -> np.ndarray:
    """Complex standard-normal start block, (re + i*im)/sqrt(2), shape (nvec, 6, *grid).

    Drawn with numpy.random.default_rng(seed): real parts first, then imaginary parts.
    """
    nvec = w.block if nvec is None else nvec
    rng = np.random.default_rng(seed)
    shp = (nvec, 6) + w.shape
    re = rng.standard_normal(shp)
    im = rng.standard_normal(shp)
    return ((re + 1j * im) / np.sqrt(2.0)).astype(dtype)


def random_block(shape: Sequence[int], seed: int, dtype=np.complex128, smooth: float = 0.0,
                 w: Optional[Workload] = None) -> np.ndarray:
    """Seeded random complex block of the given shape.

    With smooth > 0 and a workload, each field is multiplied by a Gaussian envelope
    exp(-|x|^2 / (2*smooth^2)) so that it decays toward the box edge like a trapped mode.
    """
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(tuple(shape))
    im = rng.standard_normal(tuple(shape))
    z = (re + 1j * im) / np.sqrt(2.0)
    if smooth > 0.0 and w is not None:
        r2 = sum(c * c for c in coordinates(w))
        z = z * np.exp(-r2 / (2.0 * smooth * smooth))
    return z.astype(dtype)


def fd_direction(w: Workload, seed: int):
    """Seeded finite-difference direction (dV field, d beta_n, d beta_s), all N(0, 1)."""
    rng = np.random.default_rng(seed)
    dV = rng.standard_normal(w.shape)
    dbn, dbs = rng.standard_normal(2)
    return dV, float(dbn), float(dbs)


def initial_spinor_weights(w: Workload) -> np.ndarray:
    """Spin weights of the ground-state flow's starting spinor (a Gaussian times these).

    Ferromagnetic (beta_s < 0): the single-mode vector ((1+M)/2, sqrt((1-M^2)/2), (1-M)/2)
    of the SMA lemma (Section 2.3).  Polar / antiferromagnetic (beta_s >= 0):
    (sqrt((1+M)/2), 0, sqrt((1-M)/2)), the two-component form of Section 2.3.
    """
    M = w.magnetization
    if w.beta_s < 0:
        return np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2])
    return np.array([np.sqrt((1 + M) / 2), 0.0, np.sqrt((1 - M) / 2)])


def initial_spinor(w: Workload) -> np.ndarray:
    """Starting spinor of the ground-state flow: Gaussian exp(-|x|^2/2) times the spin weights,
    shape (3, *grid), float64 (not normalized: the flow normalizes it)."""
    r2 = sum(c * c for c in coordinates(w))
    gauss = np.exp(-0.5 * r2)
    wts = initial_spinor_weights(w)
    return np.stack([wt * gauss for wt in wts]).astype(np.float64)
