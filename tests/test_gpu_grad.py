"""Parity of the HIP eigenvalue gradients (bdg_eigs_grad) with the oracle gradient and with
central finite differences of the GPU's own pipeline (ground state + eigensolve)."""
import numpy as np
import pytest

import workloads as W
from oracle import bdg, grad, groundstate as gs, lrep
from tests.gpu_util import make_ctx, say, torch_cuda

pytestmark = pytest.mark.gpu


def _cluster_mean(vals, omega, tol=1e-8):
    vals = np.array(vals, dtype=float)
    out = vals.copy()
    j0 = 0
    while j0 < len(omega):
        j1 = j0 + 1
        while j1 < len(omega) and abs(omega[j1] - omega[j0]) <= tol * abs(omega[j0]):
            j1 += 1
        out[j0:j1] = vals[j0:j1].mean(axis=0)
        j0 = j1
    return out


@pytest.mark.parametrize("case", ["1d", "2d", "2d64"])
def test_gradient_matches_oracle(case):
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    if case == "1d":
        w = W.Workload("1d_64_fm", 1, (64,), (8.0,), "harmonic1", 10.0, -0.5, 0.2, k=6, block=8)
    elif case == "2d64":
        # the gradient configuration's lattice trap and interactions on the 64^2 grid; k = 6
        # ends at a gap (omega_7 / omega_6 = 1.09)
        w = W.Workload("2d_64_grad_fm", 2, (64, 64), (12.0, 12.0), "lattice2", 100.0, -2.0, 0.0, k=6, block=10)
    else:
        # k = 7 keeps the degenerate pair omega_6 = omega_7 whole (x <-> y symmetry); a cut
        # through a degenerate eigenspace makes the gradient of its members basis dependent
        w = W.Workload("2d_32_grad_fm", 2, (32, 32), (6.0, 6.0), "lattice2", 20.0, -1.0, 0.0, k=7, block=10)
    say("grad vs oracle", w.name)
    V = W.potential(w)
    r = gs.ground_state(V, w.beta_n, w.beta_s, 1.0, w.magnetization, w.n, w.L, W.initial_spinor(w), tol=1e-13)
    coef = bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)
    # oracle eigenpairs and gradients
    out_o, prob, Nm, Qg = lrep.solve(coef, r.phi, w.n, w.L, w.k, W.start_block(w), 1e-11, V=V, mu=r.mu)
    og = [grad.eigen_gradient(r.phi, r.mu, V, w.beta_n, w.beta_s, w.n, w.L, out_o.X[j]) for j in range(w.k)]
    o_dV = _cluster_mean([g[0] for g in og], out_o.omega)
    o_bn = _cluster_mean([g[1] for g in og], out_o.omega)
    o_bs = _cluster_mean([g[2] for g in og], out_o.omega)
    # GPU on the same ground state
    ctx = make_ctx(w, Precision.FP64, V)
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    out = ctx.eigs(w.k, w.block, tol=1e-11, max_iter=3000, X0=torch.from_numpy(W.start_block(w)).to("cuda"))
    assert np.allclose(out["omega"], out_o.omega, rtol=1e-10)
    dV, dbn, dbs = ctx.eigs_grad(out["omega"], out["uv"])
    dV = dV.cpu().numpy()
    say("   dbeta_n", dbn, o_bn)
    assert np.allclose(dbn, o_bn, rtol=1e-7, atol=1e-9)
    assert np.allclose(dbs, o_bs, rtol=1e-7, atol=1e-9)
    scale = np.abs(o_dV).max()
    assert np.abs(dV - o_dV).max() <= 1e-7 * scale
    ctx.close()


def test_gradient_matches_gpu_finite_differences():
    """Central differences h = 1e-6 of the GPU pipeline along seeded random directions
    (dV ~ N(0,1) per point, d beta_n, d beta_s ~ N(0,1)); relative error <= 1e-5."""
    torch = torch_cuda()
    from paper_2506_08308_amd import Precision
    w = W.Workload("2d_64_grad_fm", 2, (64, 64), (12.0, 12.0), "lattice2", 100.0, -2.0, 0.0, k=6, block=10)
    say("grad vs FD", w.name)
    V = W.potential(w)
    X0 = torch.from_numpy(W.start_block(w)).to("cuda")

    def pipeline(Vx, bn, bs, want_grad=False):
        ww = w.with_(beta_n=bn, beta_s=bs)
        ctx = make_ctx(ww, Precision.FP64, Vx)
        ctx.ground_state(tol=1e-13, max_iter=400000)
        out = ctx.eigs(w.k, w.block, tol=1e-11, max_iter=4000, X0=X0)
        g = ctx.eigs_grad(out["omega"], out["uv"]) if want_grad else None
        ctx.close()
        return np.array(out["omega"]), g

    om, (dV, dbn, dbs) = pipeline(V, w.beta_n, w.beta_s, True)
    dV = dV.cpu().numpy()
    hd = np.prod(w.h)
    eps = 1e-6
    for seed in range(2):
        dVd, dbnd, dbsd = W.fd_direction(w, seed)
        op, _ = pipeline(V + eps * dVd, w.beta_n + eps * dbnd, w.beta_s + eps * dbsd)
        omm, _ = pipeline(V - eps * dVd, w.beta_n - eps * dbnd, w.beta_s - eps * dbsd)
        fd = _cluster_mean((op - omm) / (2 * eps), om)
        ad = np.array([hd * np.sum(dV[j] * dVd) + dbn[j] * dbnd + dbs[j] * dbsd for j in range(w.k)])
        gnorm = np.array([np.sqrt(hd * np.sum(dV[j] ** 2) + dbn[j] ** 2 + dbs[j] ** 2) for j in range(w.k)])
        dnorm = np.sqrt(hd * np.sum(dVd ** 2) + dbnd ** 2 + dbsd ** 2)
        err = np.where(np.abs(fd) >= 1e-3 * gnorm * dnorm, np.abs(fd - ad) / np.abs(fd),
                       np.abs(fd - ad) / (gnorm * dnorm))
        say("   seed", seed, "max rel err", err.max())
        assert err.max() <= 1e-5
