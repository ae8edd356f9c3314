"""torch.autograd bindings of the library.

* :func:`apply` -- the BdG operator on a block of trial vectors (eqs. BdG-d / lrep-d, the
  matrix-free product of Section 3.2) with its hand-written adjoint: the backward pass is
  ``bdg_apply`` with ``transpose = 1`` (for the real operator of a real ground state the
  adjoint is the transpose: (H_+ g, H_- f) in the (f, g) form, [[A, -B], [B, -A]] in the
  (u, v) form).
* :func:`frequencies` -- the k lowest positive excitation frequencies as a function of
  (V, beta_n, beta_s): forward = ``bdg_ground_state`` + ``bdg_eigs``; backward =
  ``bdg_eigs_grad`` (left/right eigenvector form plus the ground-state sensitivity).

Both only marshal tensors: the operator, the solves and the gradient fields run in the HIP
library.  The backward of :func:`frequencies` contracts the per-eigenvalue gradient fields
with the incoming gradient (the chain rule), ``dL/dV_i = h^d sum_j dL/domega_j dV_j(x_i)``.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

from .api import BdgContext, Form, Precision


def _torch():
    import torch
    return torch


def _function_classes():
    torch = _torch()

    class _Apply(torch.autograd.Function):
        @staticmethod
        def forward(fctx, X, bdg, form):
            fctx.bdg, fctx.form = bdg, form
            return bdg.apply(X.contiguous(), form)

        @staticmethod
        def backward(fctx, gY):
            return fctx.bdg.apply(gY.contiguous(), fctx.form, transpose=True), None, None

    class _Frequencies(torch.autograd.Function):
        @staticmethod
        def forward(fctx, V, beta_n, beta_s, spec):
            bdg = BdgContext(spec["dim"], spec["n"], spec["L"], V.detach(), float(beta_n), float(beta_s),
                             spec.get("mass", 1.0), spec.get("magnetization", 0.0),
                             spec.get("precision", Precision.FP64))
            bdg.ground_state(tol=spec.get("gs_tol", 1e-12), max_iter=spec.get("gs_max_iter", 200000))
            out = bdg.eigs(spec["k"], spec["block"], tol=spec.get("tol", 1e-10),
                           max_iter=spec.get("max_iter", 3000), X0=spec.get("X0"), seed=spec.get("seed", 0))
            fctx.bdg, fctx.omega, fctx.uv = bdg, out["omega"], out["uv"]
            fctx.hd = math.prod(bdg.h)
            return torch.tensor(out["omega"], dtype=torch.float64, device=V.device)

        @staticmethod
        def backward(fctx, g):
            dV, dbn, dbs = fctx.bdg.eigs_grad(fctx.omega, fctx.uv)
            fctx.bdg.close()
            g = g.to(torch.float64)
            gV = fctx.hd * torch.tensordot(g, dV, dims=1)
            gbn = (g.cpu() * torch.tensor(dbn, dtype=torch.float64)).sum()
            gbs = (g.cpu() * torch.tensor(dbs, dtype=torch.float64)).sum()
            return gV, gbn.to(g.device), gbs.to(g.device), None

    return _Apply, _Frequencies


_CLASSES = None


def _classes():
    global _CLASSES
    if _CLASSES is None:
        _CLASSES = _function_classes()
    return _CLASSES


def apply(bdg: BdgContext, X, form: Form = Form.FG):
    """Y = H X with autograd support; X: (b, 6, *grid) complex (the context's vector dtype)."""
    return _classes()[0].apply(X, bdg, form)


def frequencies(V, beta_n, beta_s, *, dim: int, n: Sequence[int], L: Sequence[float], k: int, block: int,
                mass: float = 1.0, magnetization: float = 0.0, tol: float = 1e-10, gs_tol: float = 1e-12,
                max_iter: int = 3000, X0=None, seed: int = 0, precision: Precision = Precision.FP64):
    """k lowest positive BdG frequencies (ascending, float64 device tensor), differentiable in
    V (device float64, shape (Nz, Ny, Nx)[-dim:]), beta_n and beta_s (0-dim tensors).

    Eigenvalues within 1e-8 omega of each other form a cluster whose members receive the
    gradient of the cluster mean; choose k at a gap of the spectrum."""
    spec = dict(dim=dim, n=tuple(n), L=tuple(L), k=k, block=block, mass=mass, magnetization=magnetization,
                tol=tol, gs_tol=gs_tol, max_iter=max_iter, X0=X0, seed=seed, precision=precision)
    return _classes()[1].apply(V, beta_n, beta_s, spec)
