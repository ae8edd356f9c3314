"""Thin Python binding of the C ABI: torch tensors provide device memory and the stream.

Every call forwards to libbdg.so; no step of the method runs in Python or on the CPU.
"""
from __future__ import annotations

import ctypes
import enum
from typing import Optional, Sequence

from . import _lib


class BdgError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")


class Precision(enum.IntEnum):
    FP64 = _lib.BDG_FP64
    FP32_APPLY = _lib.BDG_FP32_APPLY


class Form(enum.IntEnum):
    UV = _lib.BDG_FORM_UV
    FG = _lib.BDG_FORM_FG


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


class BdgContext:
    """One problem (grid, box, V, beta_n, beta_s, mass, magnetization, precision) on the GPU.

    ``n`` and ``L`` are ordered (x, y, z); ``V`` is a float64 device tensor of shape
    ``(Nz, Ny, Nx)[-dim:]`` (x fastest).
    """

    def __init__(self, dim: int, n: Sequence[int], L: Sequence[float], V, beta_n: float, beta_s: float,
                 mass: float = 1.0, magnetization: float = 0.0, precision: Precision = Precision.FP64,
                 stream=None):
        torch = _torch()
        self._lib = _lib.load()
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)[:dim]
        self.L = tuple(float(v) for v in L)[:dim]
        self.npts = 1
        for v in self.n:
            self.npts *= v
        self.precision = Precision(precision)
        self.grid_shape = tuple(reversed(self.n))
        self.device = V.device
        if tuple(V.shape) != self.grid_shape:
            raise ValueError(f"V: expected shape {self.grid_shape}, got {tuple(V.shape)}")
        self._V = V.to(torch.float64).contiguous()
        pr = _lib.Problem()
        pr.dim = self.dim
        for a in range(3):
            pr.n[a] = self.n[a] if a < dim else 1
            pr.L[a] = self.L[a] if a < dim else 1.0
        pr.beta_n, pr.beta_s = float(beta_n), float(beta_s)
        pr.mass, pr.magnetization = float(mass), float(magnetization)
        pr.precision = int(self.precision)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self._lib.bdg_create(ctypes.byref(pr), ctypes.c_void_p(_ptr(self._V)),
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != _lib.BDG_OK:
            raise BdgError(st, "bdg_create failed")
        self._h = h
        self.h = tuple(2.0 * Li / ni for Li, ni in zip(self.L, self.n))

    # ------------------------------------------------------------------ helpers
    def _check(self, st: int, what: str):
        if st != _lib.BDG_OK:
            msg = self._lib.bdg_last_error(self._h)
            raise BdgError(st, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def vector_dtype(self):
        torch = _torch()
        return torch.complex64 if self.precision == Precision.FP32_APPLY else torch.complex128

    # ------------------------------------------------------------------ API
    def ground_state(self, phi0=None, tol: float = 1e-12, max_iter: int = 200000, check: bool = True):
        """Normalized gradient flow on the device; returns (phi, mu, residual, iters)."""
        torch = _torch()
        phi = torch.empty((3,) + self.grid_shape, dtype=torch.float64, device=self.device)
        mu = (ctypes.c_double * 3)()
        res = ctypes.c_double()
        its = ctypes.c_int()
        p0 = None
        if phi0 is not None:
            self._check_field(phi0, "phi0", 3)
            p0 = phi0.to(device=self.device, dtype=torch.float64).contiguous()
        st = self._lib.bdg_ground_state(self._h, ctypes.c_void_p(_ptr(p0)), tol, max_iter,
                                        ctypes.c_void_p(_ptr(phi)), mu, ctypes.byref(res), ctypes.byref(its))
        if check:
            self._check(st, "bdg_ground_state")
        return phi, [mu[0], mu[1], mu[2]], res.value, its.value

    def _check_field(self, t, name, lead):
        want = (lead,) + self.grid_shape
        if tuple(t.shape) != want:
            raise ValueError(f"{name}: expected shape {want}, got {tuple(t.shape)}")

    def set_ground_state(self, phi, mu):
        torch = _torch()
        self._check_field(phi, "phi", 3)
        self._phi = phi.to(device=self.device, dtype=torch.float64).contiguous()
        m = (ctypes.c_double * 3)(*[float(v) for v in mu])
        self._check(self._lib.bdg_set_ground_state(self._h, ctypes.c_void_p(_ptr(self._phi)), m),
                    "bdg_set_ground_state")

    def set_ground_state_complex(self, phi, mu):
        """Install a complex ground state (3, *grid) complex128 with chemical potentials mu."""
        torch = _torch()
        self._check_field(phi, "phi", 3)
        self._phic = phi.to(device=self.device, dtype=torch.complex128).contiguous()
        m = (ctypes.c_double * 3)(*[float(v) for v in mu])
        self._check(self._lib.bdg_set_ground_state_complex(self._h, ctypes.c_void_p(_ptr(self._phic)), m),
                    "bdg_set_ground_state_complex")

    def _check_block(self, X, name, dtype, rows=None, comps=6):
        """X must be a contiguous device tensor of `dtype` with shape (rows, comps, *grid)
        (rows: any count when None).  Checked before any pointer reaches the library."""
        if X.dtype != dtype:
            raise ValueError(f"{name}: expected {dtype}, got {X.dtype}")
        want = ((X.shape[0] if rows is None else rows), comps) + self.grid_shape
        if X.dim() != 2 + self.dim or tuple(X.shape) != want:
            raise ValueError(f"{name}: expected shape {want}, got {tuple(X.shape)}")
        if X.device != self.device:
            raise ValueError(f"{name}: expected a tensor on {self.device}")

    def apply(self, X, form: Form = Form.FG, transpose: bool = False, out=None):
        """Y = H X for a block X of shape (b, 6, *grid) (complex128, or complex64 in FP32_APPLY)."""
        torch = _torch()
        self._check_block(X, "X", self.vector_dtype())
        nvec = X.shape[0]
        if out is not None:
            self._check_block(out, "out", self.vector_dtype(), rows=nvec)
        Y = torch.empty_like(X) if out is None else out
        self._check(self._lib.bdg_apply(self._h, int(form), int(bool(transpose)), nvec,
                                        ctypes.c_void_p(_ptr(X)), ctypes.c_void_p(_ptr(Y))), "bdg_apply")
        return Y

    def biortho(self, F, G):
        """In-place bi-orthogonalization of F, G (nvec, 3, *grid) complex128; returns (sigma, rank)."""
        torch = _torch()
        nvec = F.shape[0]
        self._check_block(F, "F", torch.complex128, comps=3)
        self._check_block(G, "G", torch.complex128, rows=nvec, comps=3)
        sig = (ctypes.c_double * nvec)()
        rank = ctypes.c_int()
        self._check(self._lib.bdg_biortho(self._h, nvec, ctypes.c_void_p(_ptr(F)), ctypes.c_void_p(_ptr(G)),
                                          sig, ctypes.byref(rank)), "bdg_biortho")
        return list(sig), rank.value

    def biortho_noalloc(self, F, G, F_out=None, G_out=None):
        """bdg_biortho_noalloc: F_out = F C_f, G_out = G C_g (F, G unchanged) with the library's
        static workspace (nvec <= 64); returns (F_out, G_out, sigma, rank)."""
        torch = _torch()
        nvec = F.shape[0]
        self._check_block(F, "F", torch.complex128, comps=3)
        self._check_block(G, "G", torch.complex128, rows=nvec, comps=3)
        F_out = torch.empty_like(F) if F_out is None else F_out
        G_out = torch.empty_like(G) if G_out is None else G_out
        self._check_block(F_out, "F_out", torch.complex128, rows=nvec, comps=3)
        self._check_block(G_out, "G_out", torch.complex128, rows=nvec, comps=3)
        sig = (ctypes.c_double * max(nvec, 1))()
        rank = ctypes.c_int()
        self._check(self._lib.bdg_biortho_noalloc(self._h, nvec, ctypes.c_void_p(_ptr(F)), ctypes.c_void_p(_ptr(G)),
                                                  ctypes.c_void_p(_ptr(F_out)), ctypes.c_void_p(_ptr(G_out)), sig,
                                                  ctypes.byref(rank)), "bdg_biortho_noalloc")
        return F_out, G_out, list(sig)[:nvec], rank.value

    def eigs(self, k: int, block: int, tol: float = 1e-8, max_iter: int = 2000, X0=None, seed: int = 0,
             want_vectors: bool = True, check: bool = True):
        """k smallest positive omega; returns dict(omega, uv, residual, iters, status)."""
        torch = _torch()
        om = (ctypes.c_double * k)()
        res = (ctypes.c_double * k)()
        its = ctypes.c_int()
        uv = torch.empty((k, 6) + self.grid_shape, dtype=torch.complex128, device=self.device) \
            if want_vectors else None
        x0 = None
        if X0 is not None:
            x0 = X0.to(device=self.device, dtype=torch.complex128).contiguous()
            self._check_block(x0, "X0", torch.complex128, rows=block)
        st = self._lib.bdg_eigs(self._h, k, block, tol, max_iter, ctypes.c_void_p(_ptr(x0)), seed, om,
                                ctypes.c_void_p(_ptr(uv)), res, ctypes.byref(its))
        if check:
            self._check(st, "bdg_eigs")
        return {"omega": list(om), "uv": uv, "residual": list(res), "iters": its.value, "status": st}

    def eigs_grad(self, omega, uv):
        """d omega_j / d V(x) (k, *grid), d omega_j / d beta_n, d omega_j / d beta_s."""
        torch = _torch()
        k = len(omega)
        if uv.shape[0] < k:
            raise ValueError(f"uv: {uv.shape[0]} rows for {k} eigenvalues")
        uv = uv[:k].contiguous()
        self._check_block(uv, "uv", torch.complex128, rows=k)
        om = (ctypes.c_double * k)(*omega)
        dV = torch.empty((k,) + self.grid_shape, dtype=torch.float64, device=self.device)
        dbn = (ctypes.c_double * k)()
        dbs = (ctypes.c_double * k)()
        self._check(self._lib.bdg_eigs_grad(self._h, k, om, ctypes.c_void_p(_ptr(uv)),
                                            ctypes.c_void_p(_ptr(dV)), dbn, dbs), "bdg_eigs_grad")
        return dV, list(dbn), list(dbs)

    def perturbed_density(self, omega, uv, eps, t):
        """n_j^l(x, t_s) = |phi_j + eps (u_j^l e^{-i w_l t_s} + conj(v_j^l) e^{i w_l t_s})|^2 for the
        modes (omega, uv as eigs returns them) and times t; shape (nmodes, nt, 3, *grid)."""
        torch = _torch()
        nm, nt = len(omega), len(t)
        out = torch.empty((nm, nt, 3) + self.grid_shape, dtype=torch.float64, device=self.device)
        om = (ctypes.c_double * max(nm, 1))(*[float(v) for v in omega])
        ts = (ctypes.c_double * max(nt, 1))(*[float(v) for v in t])
        u = None
        if nm:
            if uv.shape[0] < nm:
                raise ValueError(f"uv: {uv.shape[0]} rows for {nm} modes")
            u = uv[:nm].to(dtype=torch.complex128).contiguous()
            self._check_block(u, "uv", torch.complex128, rows=nm)
        self._check(self._lib.bdg_perturbed_density(self._h, nm, om, ctypes.c_void_p(_ptr(u)), float(eps), nt, ts,
                                                    ctypes.c_void_p(_ptr(out))), "bdg_perturbed_density")
        return out

    def mode_amplitudes(self, uv):
        """bdg_mode_amplitudes: per mode and field of (u_1, u_0, u_-1, v_1, v_0, v_-1) the norm,
        max |w|, second moments along x, y, z and reflection parities; (nmodes, 6, 8) list."""
        torch = _torch()
        nm = uv.shape[0]
        if nm == 0:
            return []
        u = uv.to(dtype=torch.complex128).contiguous()
        self._check_block(u, "uv", torch.complex128, rows=nm)
        out = (ctypes.c_double * (nm * 6 * 8))()
        self._check(self._lib.bdg_mode_amplitudes(self._h, nm, ctypes.c_void_p(_ptr(u)), out), "bdg_mode_amplitudes")
        vals = list(out)
        return [[vals[(l * 6 + f) * 8:(l * 6 + f + 1) * 8] for f in range(6)] for l in range(nm)]

    def stats(self):
        out = (ctypes.c_double * 10)()
        self._check(self._lib.bdg_stats(self._h, out, 10), "bdg_stats")
        keys = ["total_ms", "apply_ms", "precond_ms", "gram_ms", "small_ms", "update_ms", "setup_ms",
                "iters", "applies_fp64", "applies_fp32"]
        return dict(zip(keys, list(out)))
