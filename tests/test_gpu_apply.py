"""Parity of the HIP BdG operator (bdg_apply) with the oracle's literal def_A/def_B operator."""
import numpy as np
import pytest

import workloads as W
from oracle import bdg
from tests.gpu_util import make_ctx, oracle_ground, say, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [
    W.C1,
    W.Workload("2d_16x32_fm", 2, (16, 32), (6.0, 8.0), "harmonic2_aniso", 20.0, -1.0, 0.1),
    W.Workload("2d_64_polar", 2, (64, 64), (8.0, 8.0), "harmonic2", 50.0, 1.0, 0.0),
    W.Workload("3d_16x8x32_fm", 3, (16, 8, 32), (4.0, 3.0, 5.0), "harmonic3_z2", 10.0, -0.5, 0.2),
    W.Workload("3d_32_afm", 3, (32, 32, 32), (5.0, 5.0, 5.0), "harmonic3", 30.0, 1.5, 0.3),
    W.Workload("1d_512_fm", 1, (512,), (16.0,), "harmonic1", 10.0, -0.5, 0.2),
    W.Workload("2d_8x256_fm", 2, (8, 256), (3.0, 12.0), "harmonic2", 10.0, -0.5, 0.0),
    # 1024-point axes: the final x pass runs each thread over two of the six fields
    W.Workload("1d_1024_fm", 1, (1024,), (32.0,), "harmonic1", 10.0, -0.5, 0.2),
    W.Workload("2d_1024x8_fm", 2, (1024, 8), (24.0, 3.0), "harmonic2", 10.0, -0.5, 0.1),
    W.Workload("2d_8x1024_polar", 2, (8, 1024), (3.0, 24.0), "harmonic2", 10.0, 1.0, 0.0),
]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
@pytest.mark.parametrize("form", ["fg", "uv"])
@pytest.mark.parametrize("transpose", [0, 1])
def test_apply_fp64_matches_oracle(w, form, transpose):
    torch = torch_cuda()
    from paper_2506_08308_amd import Form, Precision
    say(f"apply fp64 {w.name} {form} T={transpose}")
    V, r, coef = oracle_ground(w)
    ctx = make_ctx(w, Precision.FP64, V)
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    X = W.random_block((3, 6) + w.shape, seed=7, smooth=0.0)
    Xd = torch.from_numpy(X).to("cuda")
    Y = ctx.apply(Xd, Form.FG if form == "fg" else Form.UV, bool(transpose)).cpu().numpy()
    if form == "fg":
        ref = bdg.apply_fg(coef, X, w.n, w.L)
        if transpose:   # adjoint: (H_+ g, H_- f)
            Hp, Hm = bdg.hpm(coef)
            from oracle import spectral
            f, g = X[:, :3], X[:, 3:]
            ref = np.concatenate([spectral.kinetic_apply(g, w.n, w.L) + bdg._pw(Hp, g),
                                  spectral.kinetic_apply(f, w.n, w.L) + bdg._pw(Hm, f)], axis=1)
    else:
        if transpose:   # [[A, B], [C, D]]^T with the oracle blocks: [[A^T, C^T], [B^T, D^T]]
            tr = lambda M: np.swapaxes(M, 0, 1)
            c2 = bdg.Coefficients(A=tr(coef.A), B=tr(coef.C), C=tr(coef.B), D=tr(coef.D))
            ref = bdg.apply_uv(c2, X, w.n, w.L)
        else:
            ref = bdg.apply_uv(coef, X, w.n, w.L)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}")
    assert err < 1e-13
    ctx.close()


@pytest.mark.parametrize("w", CASES[:5] + CASES[7:], ids=lambda w: w.name)
def test_apply_fp32_matches_oracle(w):
    torch = torch_cuda()
    from paper_2506_08308_amd import Form, Precision
    say(f"apply fp32 {w.name}")
    V, r, coef = oracle_ground(w)
    ctx = make_ctx(w, Precision.FP32_APPLY, V)
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    X = W.random_block((2, 6) + w.shape, seed=8)
    X32 = X.astype(np.complex64)
    Y = ctx.apply(torch.from_numpy(X32).to("cuda"), Form.FG).cpu().numpy().astype(np.complex128)
    ref = bdg.apply_fg(coef, X32.astype(np.complex128), w.n, w.L)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}")
    assert err < 2e-6
    ctx.close()


def _p(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


PLANE_CASE = W.Workload("3d_128x128x8_fm", 3, (128, 128, 8), (8.0, 8.0, 2.0), "harmonic3_z2", 40.0, -0.5, 0.1)


@pytest.mark.parametrize("transpose", [0, 1])
def test_apply_fp32_plane_passes_match_oracle(transpose, monkeypatch):
    """complex64 (f, g) operator on a 128 x 128 x nz grid: the three-pass form (xy planes in
    LDS) against the oracle, and against the five-pass form of the same context settings."""
    torch = torch_cuda()
    from paper_2506_08308_amd import Form, Precision
    w = PLANE_CASE
    say(f"apply fp32 planes {w.name} T={transpose}")
    # the operator alone is under test: the initial spinor of the flow serves as ground state
    V = W.potential(w)
    phi, mu = W.initial_spinor(w), np.array([1.0, 0.9, 1.1])
    coef = bdg.coefficients(phi, mu, V, w.beta_n, w.beta_s)
    X = W.random_block((5, 6) + w.shape, seed=9)
    X32 = X.astype(np.complex64)
    outs = []
    for planes in ("1", "0"):
        monkeypatch.setenv("BDG_APPLY_PLANES", planes)
        ctx = make_ctx(w, Precision.FP32_APPLY, V)
        ctx.set_ground_state(torch.from_numpy(phi), mu)
        outs.append(ctx.apply(torch.from_numpy(X32).to("cuda"), Form.FG, bool(transpose)).cpu().numpy()
                     .astype(np.complex128))
        ctx.close()
    Xr = X32.astype(np.complex128)
    if transpose:
        Hp, Hm = bdg.hpm(coef)
        from oracle import spectral
        f, g = Xr[:, :3], Xr[:, 3:]
        ref = np.concatenate([spectral.kinetic_apply(g, w.n, w.L) + bdg._pw(Hp, g),
                              spectral.kinetic_apply(f, w.n, w.L) + bdg._pw(Hm, f)], axis=1)
    else:
        ref = bdg.apply_fg(coef, Xr, w.n, w.L)
    scale = np.abs(ref).max()
    err = np.abs(outs[0] - ref).max() / scale
    cross = np.abs(outs[0] - outs[1]).max() / scale
    say(f"   rel err {err:.2e} (oracle), {cross:.2e} (five-pass form)")
    assert err < 2e-6
    assert cross < 2e-6
    monkeypatch.delenv("BDG_APPLY_PLANES")


@pytest.mark.parametrize("transpose", [0, 1])
def test_apply_fp64_half_plane_passes_match_oracle(transpose, monkeypatch):
    """complex128 (f, g) operator on a 128 x 128 x nz grid: the three-pass form (each xy plane
    as two half-planes in LDS) against the oracle, and against the five-pass form."""
    torch = torch_cuda()
    from paper_2506_08308_amd import Form, Precision
    w = PLANE_CASE
    say(f"apply fp64 half-planes {w.name} T={transpose}")
    V = W.potential(w)
    phi, mu = W.initial_spinor(w), np.array([1.0, 0.9, 1.1])
    coef = bdg.coefficients(phi, mu, V, w.beta_n, w.beta_s)
    X = W.random_block((3, 6) + w.shape, seed=19)
    outs = []
    for planes in ("1", "0"):
        monkeypatch.setenv("BDG_APPLY_PLANES64", planes)
        ctx = make_ctx(w, Precision.FP64, V)
        ctx.set_ground_state(torch.from_numpy(phi), mu)
        outs.append(ctx.apply(torch.from_numpy(X).to("cuda"), Form.FG, bool(transpose)).cpu().numpy())
        ctx.close()
    if transpose:
        Hp, Hm = bdg.hpm(coef)
        from oracle import spectral
        f, g = X[:, :3], X[:, 3:]
        ref = np.concatenate([spectral.kinetic_apply(g, w.n, w.L) + bdg._pw(Hp, g),
                              spectral.kinetic_apply(f, w.n, w.L) + bdg._pw(Hm, f)], axis=1)
    else:
        ref = bdg.apply_fg(coef, X, w.n, w.L)
    scale = np.abs(ref).max()
    err = np.abs(outs[0] - ref).max() / scale
    cross = np.abs(outs[0] - outs[1]).max() / scale
    say(f"   rel err {err:.2e} (oracle), {cross:.2e} (five-pass form)")
    assert err < 1e-13
    assert cross < 1e-13
    monkeypatch.delenv("BDG_APPLY_PLANES64")


@pytest.mark.parametrize("planes", ["1", "0"])
def test_precond_mixed_matches_oracle(planes, monkeypatch):
    """The mixed solve's preconditioner D (|k|^2/2 + sigma)^-1 D in float32 on a 128 x 128 x nz
    grid: the three-pass plane form (planes = 1) and the five-pass form against the oracle."""
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision, _lib
    from oracle import lrep
    w = PLANE_CASE
    say(f"precond mixed {w.name} planes={planes}")
    V = W.potential(w)
    phi, mu = W.initial_spinor(w), np.array([1.0, 0.9, 1.1])
    coef = bdg.coefficients(phi, mu, V, w.beta_n, w.beta_s)
    X = W.random_block((3, 6) + w.shape, seed=23).astype(np.complex64)
    monkeypatch.setenv("BDG_APPLY_PLANES", planes)
    ctx = make_ctx(w, Precision.FP32_APPLY, V)
    ctx.set_ground_state(torch.from_numpy(phi), mu)
    Xd = torch.from_numpy(X.copy()).to("cuda")
    Yd = torch.zeros(X.shape, dtype=torch.complex128, device="cuda")
    assert ctx._lib.bdg_test_precond_mixed(ctx._h, X.shape[0], _p(Xd), _p(Yd)) == _lib.BDG_OK
    got = Yd.cpu().numpy()
    ctx.close()
    monkeypatch.delenv("BDG_APPLY_PLANES")
    sigma, D = lrep.preconditioner_parameters(V, mu)
    prob = lrep.LrepProblem(coef, w.n, w.L, D)
    npts = int(np.prod(w.shape))
    cols = X.astype(np.complex128).reshape(X.shape[0] * 2, 3 * npts).T     # one column per half
    ref = prob.precond(cols, sigma).T.reshape(X.shape)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}")
    assert err < 2e-6


def test_apply_rejects_bad_arguments():
    torch = torch_cuda()
    from paper_2506_08308_amd import BdgError, Form, Precision
    w = CASES[1]
    V, r, coef = oracle_ground(w)
    ctx = make_ctx(w, Precision.FP64, V)
    X = torch.zeros((1, 6) + w.shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(BdgError) as e:           # no ground state yet
        ctx.apply(X, Form.FG)
    assert "BDG_ESTATE" in str(e.value)
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    with pytest.raises(BdgError):                # X and Y overlap
        ctx.apply(X, Form.FG, out=X)
    ctx.close()
