"""bdg_biortho_noalloc (the allocation-free bi-orthogonalization) against bdg_biortho.

Two calls in a row on one context, the second with fewer vectors, on a grid large enough
that the static workspace caps the Gram matrix's split-K partials (1024 x 1024 points,
3 Mi complex rows per half vector): singular values agree with the in-place entry point to
rounding, the output columns agree once each (f, g) column pair is aligned by the one unit
phase that singular vectors leave free, the pairing matrix of the outputs is the identity,
and the inputs are left unchanged.  Argument errors (too many vectors, overlapping buffers) are rejected
before any kernel runs.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import make_ctx, say, torch_cuda

pytestmark = pytest.mark.gpu


def _blocks(torch, nvec, shape, seed):
    """F complex normal; G_j = d_j F_j + 0.05 N_j with d_j = 1 + j/8, so the pairing matrix
    G^H F is close to a diagonal with well separated entries (distinct singular values)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    full = (nvec, 3) + shape
    F = torch.randn(full, dtype=torch.complex128, device="cuda", generator=g)
    N = torch.randn(full, dtype=torch.complex128, device="cuda", generator=g)
    d = (1.0 + torch.arange(nvec, dtype=torch.float64, device="cuda") / 8.0).reshape((nvec,) + (1,) * (len(shape) + 1))
    return F, (d * F + 0.05 * N).contiguous()


def _phase_aligned_error(Fo, Go, Fr, Gr):
    """Singular vectors are unique up to one unit phase per singular triplet, shared by the
    f and g columns: align each column pair of (Fo, Go) to (Fr, Gr) with the phase of
    <Fr_j, Fo_j> and return the largest relative column difference."""
    nvec = Fo.shape[0]
    fo, go = Fo.reshape(nvec, -1), Go.reshape(nvec, -1)
    fr, gr = Fr.reshape(nvec, -1), Gr.reshape(nvec, -1)
    ip = (fr.conj() * fo).sum(dim=1)
    ph = (ip / ip.abs()).conj().unsqueeze(1)
    ef = ((fo * ph - fr).abs().amax(dim=1) / fr.abs().amax(dim=1)).max()
    eg = ((go * ph - gr).abs().amax(dim=1) / gr.abs().amax(dim=1)).max()
    return float(max(ef, eg))


def test_noalloc_biortho_matches_biortho_twice():
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    w = W.Workload("2d_1024_fm", 2, (1024, 1024), (16.0, 16.0), "harmonic2", 100.0, -2.0, 0.0)
    ctx = make_ctx(w, Precision.FP64)
    hd = float(np.prod(w.h))
    for nvec, seed in ((64, 11), (24, 12)):
        say(f"noalloc biortho {w.name} nvec={nvec}")
        F, G = _blocks(torch, nvec, w.shape, seed)
        F0, G0 = F.clone(), G.clone()
        Fo, Go, sig, rank = ctx.biortho_noalloc(F, G)
        torch.cuda.synchronize()
        assert torch.equal(F, F0) and torch.equal(G, G0)
        Fr, Gr = F.clone(), G.clone()
        sig_r, rank_r = ctx.biortho(Fr, Gr)
        assert rank == rank_r == nvec
        assert np.allclose(sig, sig_r, rtol=1e-12)
        err = _phase_aligned_error(Fo, Go, Fr, Gr)
        say(f"   phase-aligned max rel column difference {err:.2e}")
        assert err <= 1e-10, err
        pair = hd * (Go.reshape(nvec, -1).conj() @ Fo.reshape(nvec, -1).T.contiguous())
        eye = torch.eye(nvec, dtype=torch.complex128, device="cuda")
        assert float((pair - eye).abs().max()) <= 1e-10
        del F, G, F0, G0, Fo, Go, Fr, Gr
        torch.cuda.empty_cache()
    ctx.close()


def test_noalloc_biortho_rejects_bad_arguments():
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision, _lib
    w = W.Workload("2d_32_fm", 2, (32, 32), (6.0, 6.0), "harmonic2", 20.0, -1.0, 0.0)
    ctx = make_ctx(w, Precision.FP64)
    lib = ctx._lib
    F, G = _blocks(torch, 4, w.shape, 3)
    Fo, Go = torch.empty_like(F), torch.empty_like(G)
    sig = (ctypes.c_double * 128)()
    rank = ctypes.c_int()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    # more vectors than the static workspace allows: rejected before any device access
    assert lib.bdg_biortho_noalloc(ctx._h, _lib.BDG_NOALLOC_MAX_VEC + 1, p(F), p(G), p(Fo), p(Go), sig,
                                   ctypes.byref(rank)) == _lib.BDG_EINVAL
    assert b"nvec" in lib.bdg_last_error(ctx._h)
    # an output overlapping an input, and the two outputs overlapping
    assert lib.bdg_biortho_noalloc(ctx._h, 4, p(F), p(G), p(F), p(Go), sig, ctypes.byref(rank)) == _lib.BDG_EINVAL
    assert lib.bdg_biortho_noalloc(ctx._h, 4, p(F), p(G), p(Fo), p(Fo), sig, ctypes.byref(rank)) == _lib.BDG_EINVAL
    # valid call after the rejections
    assert lib.bdg_biortho_noalloc(ctx._h, 4, p(F), p(G), p(Fo), p(Go), sig, ctypes.byref(rank)) == _lib.BDG_OK
    assert rank.value == 4
    ctx.close()
