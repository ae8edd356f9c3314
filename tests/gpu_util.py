"""Helpers for the GPU tests: device availability and oracle ground states as inputs."""
import functools
import sys

import numpy as np
import pytest

import workloads as W


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def oracle_ground(w: W.Workload, tol=1e-12):
    from oracle import bdg, groundstate as gs
    V = W.potential(w)
    r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L, W.initial_spinor(w), tol=tol)
    coef = bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)
    return V, r, coef


def make_ctx(w: W.Workload, precision=None, V=None):
    torch = torch_cuda()
    from paper_2506_08308_amd import BdgContext, Precision
    if V is None:
        V = W.potential(w)
    prec = precision if precision is not None else (
        Precision.FP32_APPLY if w.precision == "fp32_apply" else Precision.FP64)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).to("cuda")
    return BdgContext(w.dim, w.n, w.L, Vd, w.beta_n, w.beta_s, w.mass, w.magnetization, prec)
