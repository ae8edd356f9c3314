"""Small ground states and operators shared by the oracle tests (cached per session)."""
import functools

import numpy as np

import workloads as W
from oracle import bdg, groundstate as gs


@functools.lru_cache(maxsize=None)
def ground(name_or_w):
    w = W.ALL[name_or_w] if isinstance(name_or_w, str) else name_or_w
    V = W.potential(w)
    r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L,
                        W.initial_spinor(w), tol=1e-12)
    coef = bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)
    return w, V, r, coef


C1 = W.C1
POLAR_1D = W.Workload("1d_n64_polar", 1, (64,), (10.0,), "harmonic1", 30.0, 1.5, 0.0)
AFM_1D = W.Workload("1d_n64_afm", 1, (64,), (10.0,), "harmonic1", 30.0, 1.5, 0.3)
FM_2D = W.Workload("2d_n16_fm", 2, (16, 16), (6.0, 6.0), "harmonic2", 20.0, -1.0, 0.1, k=8, block=12)
POLAR_2D = W.Workload("2d_n16_polar", 2, (16, 16), (6.0, 6.0), "harmonic2", 20.0, 1.0, 0.0, k=8, block=12)
FM_3D = W.Workload("3d_n8_fm", 3, (8, 8, 8), (4.0, 4.0, 4.0), "harmonic3_z2", 10.0, -0.5, 0.1, k=6, block=8)
