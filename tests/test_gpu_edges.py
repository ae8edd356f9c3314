"""Edge cases of the GPU path: call order and argument errors, the iteration limit, the
smallest grid with the largest admissible block, ragged (non-square) grids, mass != 1 and a
magnetization near its limit, each against the oracle's dense eigensolve where a result is
produced."""
import numpy as np
import pytest

import workloads as W
from oracle import bdg, groundstate as gs
from tests.gpu_util import make_ctx, oracle_ground, say, torch_cuda

pytestmark = pytest.mark.gpu


def _status(fn):
    from paper_2506_08308_amd import BdgError
    try:
        fn()
    except BdgError as e:
        return e.status
    return 0


def test_call_order_and_argument_errors():
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib, Form
    w = W.Workload("1d_8", 1, (8,), (4.0,), "harmonic1", 5.0, -0.5, 0.2, k=4, block=8)
    say("errors", w.name)
    ctx = make_ctx(w)
    X = torch.zeros((1, 6, 8), dtype=torch.complex128, device="cuda")
    # no ground state yet
    assert _status(lambda: ctx.eigs(4, 8)) == _lib.BDG_ESTATE
    assert _status(lambda: ctx.apply(X, Form.FG)) == _lib.BDG_ESTATE
    uv = torch.zeros((1, 6, 8), dtype=torch.complex128, device="cuda")
    assert _status(lambda: ctx.eigs_grad([0.5], uv)) == _lib.BDG_ESTATE
    ctx.ground_state(tol=1e-12)
    # block limits: 1 <= k <= block <= min(160, 3 npts - 4) = 20
    assert _status(lambda: ctx.eigs(0, 8)) == _lib.BDG_EINVAL
    assert _status(lambda: ctx.eigs(9, 8)) == _lib.BDG_EINVAL
    assert _status(lambda: ctx.eigs(4, 21)) == _lib.BDG_EINVAL
    assert _status(lambda: ctx.eigs(4, 8, tol=0.0)) == _lib.BDG_EINVAL
    assert _status(lambda: ctx.eigs(4, 8, max_iter=0)) == _lib.BDG_EINVAL
    # empty apply is a no-op; overlapping input and output are rejected
    E = torch.zeros((0, 6, 8), dtype=torch.complex128, device="cuda")
    assert _status(lambda: ctx.apply(E, Form.FG)) == 0
    assert _status(lambda: ctx.apply(X, Form.FG, out=X)) == _lib.BDG_EINVAL
    ctx.close()


def test_iteration_limit_returns_last_iterate():
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    w = W.C1
    say("iteration limit", w.name)
    ctx = make_ctx(w)
    ctx.ground_state(tol=1e-12)
    out = ctx.eigs(w.k, w.block, tol=1e-12, max_iter=3, check=False)
    assert out["status"] == _lib.BDG_ENOCONV
    assert out["iters"] == 3
    assert np.all(np.isfinite(out["omega"])) and max(out["residual"]) > 1e-12
    ctx.close()


def _dense_check(w, k, block, tol=1e-10, rtol=1e-9):
    torch = torch_cuda()
    V, r, coef = oracle_ground(w)
    om_d, _ = bdg.positive_eigs_dense(bdg.dense_uv(coef, w.n, w.L), k)
    ctx = make_ctx(w, None, V)
    ctx.set_ground_state(torch.from_numpy(r.phi), r.mu)
    out = ctx.eigs(k, block, tol=tol, max_iter=2000, seed=5)
    rel = np.abs(np.array(out["omega"]) - om_d) / om_d
    say(f"   k={k} block={block}: {out['iters']} iterations, max rel err {rel.max():.2e}")
    assert rel.max() <= rtol
    ctx.close()


def test_smallest_grid_with_largest_block():
    """N = 8 points (48 unknowns): block = 3 N - 4 = 20, the largest the deflated halves admit."""
    w = W.Workload("1d_8", 1, (8,), (4.0,), "harmonic1", 5.0, -0.5, 0.2)
    say("largest block", w.name)
    _dense_check(w, 8, 20)
    _dense_check(w, 4, 6)


@pytest.mark.parametrize("w", [
    W.Workload("2d_8x32_fm", 2, (8, 32), (3.0, 8.0), "harmonic2_aniso", 20.0, -1.0, 0.3),
    W.Workload("2d_32x8_polar", 2, (32, 8), (8.0, 3.0), "harmonic2", 20.0, 1.0, 0.0),
], ids=lambda w: w.name)
def test_ragged_grids_match_dense(w):
    say("ragged", w.name)
    _dense_check(w, 10, 16)


def test_mass_and_magnetization_edges():
    """mass 2 with M = 0.9 (ferromagnetic): the GPU ground state against the oracle flow and the
    GPU spectrum against the dense eigensolve of the oracle's ground state."""
    torch = torch_cuda()
    w = W.Workload("1d_64_m09", 1, (64,), (8.0,), "harmonic1", 10.0, -0.5, 0.9, mass=2.0)
    say("mass and magnetization", w.name)
    V = W.potential(w)
    r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L, W.initial_spinor(w), tol=1e-12)
    ctx = make_ctx(w, None, V)
    phi, mu, res, _ = ctx.ground_state(tol=1e-12)
    assert np.allclose(mu, r.mu, rtol=1e-9)
    p = phi.cpu().numpy()
    hd = float(np.prod(w.h))
    assert abs(hd * np.sum(p ** 2) - 2.0) <= 1e-12
    assert abs(hd * (np.sum(p[0] ** 2) - np.sum(p[2] ** 2)) - 0.9 * 2.0) <= 1e-12
    assert np.abs(p - r.phi).max() <= 1e-8 * np.abs(r.phi).max()
    coef = bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)
    om_d, _ = bdg.positive_eigs_dense(bdg.dense_uv(coef, w.n, w.L), 8)
    out = ctx.eigs(8, 12, tol=1e-10)
    rel = np.abs(np.array(out["omega"]) - om_d) / om_d
    say(f"   max rel err {rel.max():.2e}")
    assert rel.max() <= 1e-9
    ctx.close()


def test_solves_are_bitwise_deterministic():
    """Fixed-order reductions everywhere: two solves from the same seed (device start block)
    and two applies give bit-identical results."""
    torch = torch_cuda()
    from paper_2506_08308_amd import Form
    w = W.Workload("2d_32_fm", 2, (32, 32), (6.0, 6.0), "harmonic2", 20.0, -1.0, 0.1)
    say("determinism", w.name)
    ctx = make_ctx(w)
    ctx.ground_state(tol=1e-12)
    a = ctx.eigs(8, 12, tol=1e-10, seed=11)
    b = ctx.eigs(8, 12, tol=1e-10, seed=11)
    assert a["omega"] == b["omega"] and a["iters"] == b["iters"]
    assert torch.equal(a["uv"], b["uv"])
    X = torch.from_numpy(W.random_block((3, 6) + w.shape, seed=2)).to("cuda")
    assert torch.equal(ctx.apply(X, Form.FG), ctx.apply(X, Form.FG))
    ctx.close()


def test_tolerance_below_the_rounding_floor():
    """tol = 1e-15 is below the float64 floor eps ||H|| / omega of the relative residual for
    the ferromagnetic spin modes (omega ~ 0.02): every column stops at
    max(tol, 100 eps ||H|| / omega_j) with status OK, and the spectrum equals the oracle's
    dense eigensolve of the same ground state."""
    torch = torch_cuda()
    w = W.Workload("1d_128_fm_m0", 1, (128,), (16.0,), "harmonic1", 885.4, -4.1, 0.0)
    say("rounding floor", w.name)
    V = W.potential(w)
    ctx = make_ctx(w, None, V)
    phi, mu, res, its = ctx.ground_state(tol=1e-12, max_iter=400000)
    out = ctx.eigs(12, 16, tol=1e-15, max_iter=1500, seed=2)
    coef = bdg.coefficients(phi.cpu().numpy(), np.array(mu), V, w.beta_n, w.beta_s)
    om_d, _ = bdg.positive_eigs_dense(bdg.dense_uv(coef, w.n, w.L), 12)
    # the operator bound the library uses: largest kinetic symbol + largest pointwise row sum
    kin = 0.5 * (np.pi * 128 / 32.0) ** 2
    Hp, Hm = bdg.hpm(coef)
    rows = max(np.abs(Hp).sum(axis=1).max(), np.abs(Hm).sum(axis=1).max())
    floor = 100 * np.finfo(float).eps * (kin + rows) / np.array(out["omega"])
    res = np.array(out["residual"])
    say(f"   iters {out['iters']}, residuals {res.min():.1e}..{res.max():.1e}, floors {floor.min():.1e}..{floor.max():.1e}")
    assert out["status"] == 0
    assert np.all(res <= floor * 1.01)
    assert np.any(res > 1e-15)
    assert np.allclose(out["omega"], om_d, rtol=1e-10)
    ctx.close()
