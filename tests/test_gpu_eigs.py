"""Parity of the HIP eigensolver (bdg_eigs, bdg_biortho, bdg_ground_state) with the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import bdg, branch, lrep, scalar
from tests.gpu_util import make_ctx, oracle_ground, say, torch_cuda

pytestmark = pytest.mark.gpu


def test_biortho_gives_identity_pairing():
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    w = W.Workload("2d_32_fm", 2, (32, 32), (6.0, 6.0), "harmonic2", 20.0, -1.0, 0.1)
    say("biortho 2d_32 nvec=40")
    V, r, coef = oracle_ground(w)
    ctx = make_ctx(w, Precision.FP64, V)
    nv = 40
    F0 = W.random_block((nv, 3) + w.shape, seed=3)
    G0 = W.random_block((nv, 3) + w.shape, seed=4)
    F = torch.from_numpy(F0.copy()).to("cuda")
    G = torch.from_numpy(G0.copy()).to("cuda")
    sig, rank = ctx.biortho(F, G)
    assert rank == nv
    hd = np.prod(w.h)
    Fh = F.cpu().numpy().reshape(nv, -1)
    Gh = G.cpu().numpy().reshape(nv, -1)
    pair = hd * (Gh.conj() @ Fh.T)        # (G^H F)_{ij} = <f_j, g_i>
    assert np.abs(pair - np.eye(nv)).max() < 1e-10
    # singular values of the pairing matrix (independent numpy SVD)
    B = hd * (G0.reshape(nv, -1).conj() @ F0.reshape(nv, -1).T)
    s_ref = np.linalg.svd(B, compute_uv=False)
    assert np.allclose(sig, s_ref, rtol=1e-10)
    # spans are preserved
    for X0, X in ((F0, Fh), (G0, Gh)):
        Q, _ = np.linalg.qr(X0.reshape(nv, -1).T)
        resid = X.T - Q @ (Q.conj().T @ X.T)
        assert np.abs(resid).max() < 1e-9 * np.abs(X).max()
    ctx.close()


def test_c1_eigs_match_dense_oracle():
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    w = W.C1
    say("eigs C1")
    V, r, coef = oracle_ground(w)
    om_d, _ = bdg.positive_eigs_dense(bdg.dense_uv(coef, w.n, w.L), w.k)
    ctx = make_ctx(w, Precision.FP64, V)
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    X0 = torch.from_numpy(W.start_block(w)).to("cuda")
    out = ctx.eigs(w.k, w.block, tol=1e-10, max_iter=2000, X0=X0)
    say("   iters", out["iters"], "omega", np.array(out["omega"]))
    assert np.allclose(out["omega"], om_d, rtol=1e-9)
    assert max(out["residual"]) <= 1e-10
    # eigenvectors: independent residual through the oracle (u, v) operator and normalization
    uv = out["uv"].cpu().numpy()
    Y = bdg.apply_uv(coef, uv, w.n, w.L)
    R = Y - np.array(out["omega"])[:, None, None] * uv
    assert (np.linalg.norm(R.reshape(w.k, -1), axis=1) / np.linalg.norm(uv.reshape(w.k, -1), axis=1)).max() < 1e-8
    hd = np.prod(w.h)
    nrm = hd * (np.sum(np.abs(uv[:, :3]) ** 2, axis=(1, 2)) - np.sum(np.abs(uv[:, 3:]) ** 2, axis=(1, 2)))
    assert np.allclose(nrm, 1.0, atol=1e-10)
    ctx.close()


@pytest.mark.parametrize("kind", ["fm", "polar"])
def test_2d_eigs_match_oracle_and_branch(kind):
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    bs = -1.0 if kind == "fm" else 1.0
    w = W.Workload(f"2d_32_{kind}", 2, (32, 32), (6.0, 6.0), "harmonic2", 20.0, bs, 0.0, k=12, block=16)
    say("eigs", w.name)
    V, r, coef = oracle_ground(w)
    if kind == "fm":
        M = w.magnetization
        phi = np.tensordot(np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2]), r.phi, axes=1)
        ref = branch.fm_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, w.k)
    else:
        ref = branch.polar_spectrum_dense(r.phi[0] * np.sqrt(2), r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, w.k)
    ctx = make_ctx(w, Precision.FP64, V)
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    out = ctx.eigs(w.k, w.block, tol=1e-9, max_iter=3000, X0=torch.from_numpy(W.start_block(w)).to("cuda"))
    say("   iters", out["iters"], "stats", ctx.stats())
    assert np.allclose(out["omega"], ref, rtol=1e-9)
    ctx.close()


def test_mixed_precision_eigs_agree_with_fp64_and_oracles():
    """3-D 16^3 trap: the FP64 solve within 1e-9 and the float32-apply solve within 1e-6 of
    the six-component oracle iteration and of the scalar branch oracle; the two GPU forms
    agree with each other."""
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    w = W.Workload("3d_16_fm", 3, (16, 16, 16), (5.0, 5.0, 5.0), "harmonic3_z2", 40.0, -1.0, 0.1, k=8, block=12)
    say("eigs mixed", w.name)
    V, r, coef = oracle_ground(w)
    out_o, _, _, _ = lrep.solve(coef, r.phi, w.n, w.L, w.k, W.start_block(w), 1e-10, V=V, mu=r.mu)
    M = w.magnetization
    phi = np.tensordot(np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2]), r.phi, axes=1)
    bs = scalar.fm_branches(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, {"density": 6, "magnon": 8, "gapped": 8},
                            tol=1e-10, k_total=w.k)
    res = {}
    for prec in (Precision.FP64, Precision.FP32_APPLY):
        ctx = make_ctx(w, prec, V)
        ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
        out = ctx.eigs(w.k, w.block, tol=1e-8, max_iter=3000, X0=torch.from_numpy(W.start_block(w)).to("cuda"))
        say("   ", prec.name, out["iters"], ctx.stats())
        res[prec] = out
        ctx.close()
    a, b = np.array(res[Precision.FP64]["omega"]), np.array(res[Precision.FP32_APPLY]["omega"])
    for ref in (out_o.omega, bs.omega):
        say("   rel err fp64", np.abs(a / ref - 1).max(), "mixed", np.abs(b / ref - 1).max())
        assert np.allclose(a, ref, rtol=1e-9)
        assert np.allclose(b, ref, rtol=1e-6)
    assert np.allclose(a, b, rtol=1e-6)
    assert max(res[Precision.FP32_APPLY]["residual"]) <= 1e-8
    # the x and y Kohn modes omega = gamma = 1 of the (1, 1, 2) trap (Analytical eigenpairs
    # theorem) are among the lowest eight, up to the 16^3 grid's discretization error
    assert np.sum(np.abs(a - 1.0) < 1e-4) == 2


def test_ground_state_matches_oracle():
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    for w in (W.C1, W.Workload("2d_32_polar", 2, (32, 32), (6.0, 6.0), "harmonic2", 20.0, 1.0, 0.0)):
        say("ground state", w.name)
        V, r, coef = oracle_ground(w)
        ctx = make_ctx(w, Precision.FP64, V)
        phi, mu, res, its = ctx.ground_state(tol=1e-12, max_iter=100000)
        say("   iters", its, "res", res, "mu", mu)
        assert res <= 1e-12
        assert np.abs(phi.cpu().numpy() - r.phi).max() < 1e-10
        assert np.allclose(mu, r.mu, atol=1e-10)
        ctx.close()


def test_1024_point_axis_eigs_match_branch_decomposition():
    """1-D FM trap on 1024 points (the largest axis): the spectrum equals the oracle's scalar
    branch decomposition, and the GPU ground state equals the oracle flow."""
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    w = W.Workload("1d_1024_fm", 1, (1024,), (32.0,), "harmonic1", 10.0, -0.5, 0.2, k=16, block=24)
    say("eigs", w.name)
    V, r, coef = oracle_ground(w)
    M = w.magnetization
    phi = np.tensordot(np.array([(1 + M) / 2, np.sqrt((1 - M * M) / 2), (1 - M) / 2]), r.phi, axes=1)
    ref = branch.fm_spectrum_dense(phi, r.mu[0], V, w.beta_n, w.beta_s, w.n, w.L, w.k)
    ctx = make_ctx(w, Precision.FP64, V)
    g_phi, g_mu, g_res, g_its = ctx.ground_state(tol=1e-12, max_iter=200000)
    say("   ground state iters", g_its, "res", g_res)
    assert np.abs(g_phi.cpu().numpy() - r.phi).max() < 1e-9
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    out = ctx.eigs(w.k, w.block, tol=1e-10, max_iter=3000, seed=3)
    say("   iters", out["iters"])
    assert np.allclose(out["omega"], ref, rtol=1e-9)
    ctx.close()
