"""Parity of bdg_perturbed_density (Section 4.2) with the oracle's formula, and the O(eps^2)
change of the total density along a normal mode (a mode at omega != 0 is orthogonal to the
phase zero mode, so the linear term of the norm vanishes)."""
import numpy as np
import pytest

import workloads as W
from oracle import modes
from tests.gpu_util import make_ctx, say, torch_cuda

pytestmark = pytest.mark.gpu


def _solve(w, k, block):
    ctx = make_ctx(w)
    phi, mu, res, its = ctx.ground_state(tol=1e-12)
    out = ctx.eigs(k, block, tol=1e-10, seed=1)
    return ctx, phi, out


@pytest.mark.parametrize("w,k,block", [
    (W.C1, 8, 8),
    (W.Workload("2d_64x32_aniso_fm", 2, (64, 32), (8.0, 6.0), "harmonic2_aniso", 40.0, -1.0, 0.0), 10, 14),
], ids=lambda x: getattr(x, "name", str(x)))
def test_perturbed_density_matches_oracle(w, k, block):
    torch = torch_cuda()
    say("perturbed density", w.name)
    ctx, phi, out = _solve(w, k, block)
    t = [0.0, 1.3, 10.6]
    sel = [0, k // 2, k - 1]
    om = [out["omega"][j] for j in sel]
    uv = out["uv"][sel]
    n = ctx.perturbed_density(om, uv, 0.1, t).cpu().numpy()
    ref = modes.perturbed_density(phi.cpu().numpy(), uv.cpu().numpy(), om, 0.1, t)
    assert n.shape == ref.shape
    assert np.abs(n - ref).max() <= 1e-13 * np.abs(ref).max()
    # arbitrary (non-eigen) input vectors and a large amplitude take the same formula
    X = torch.from_numpy(W.random_block((2, 6) + w.shape, seed=4)).to("cuda")
    n2 = ctx.perturbed_density([0.5, 3.0], X, 2.5, [0.2, -7.0]).cpu().numpy()
    ref2 = modes.perturbed_density(phi.cpu().numpy(), X.cpu().numpy(), [0.5, 3.0], 2.5, [0.2, -7.0])
    assert np.abs(n2 - ref2).max() <= 1e-13 * np.abs(ref2).max()
    ctx.close()


def test_total_density_changes_at_second_order():
    torch = torch_cuda()
    w = W.Workload("2d_64x32_aniso_fm", 2, (64, 32), (8.0, 6.0), "harmonic2_aniso", 40.0, -1.0, 0.0)
    say("perturbed density norm", w.name)
    ctx, phi, out = _solve(w, 10, 14)
    hd = float(np.prod(w.h))
    n0 = hd * float((phi.cpu().numpy() ** 2).sum())
    for j in (0, 5, 9):
        dn = []
        for eps in (1e-3, 2e-3):
            n = ctx.perturbed_density([out["omega"][j]], out["uv"][j:j + 1], eps, [0.0, 0.7]).cpu().numpy()
            dn.append(hd * n.sum(axis=(2, 3, 4)) - n0)
        ratio = np.asarray(dn[1]) / np.asarray(dn[0])
        assert np.all(np.abs(ratio - 4.0) <= 0.02), ratio
    ctx.close()


def test_perturbed_density_edges():
    torch = torch_cuda()
    from paper_2506_08308_amd import BdgError, _lib
    w = W.Workload("1d_16", 1, (16,), (4.0,), "harmonic1", 5.0, -0.5, 0.2)
    ctx = make_ctx(w)
    uv = torch.zeros((1, 6, 16), dtype=torch.complex128, device="cuda")
    with pytest.raises(BdgError) as e:
        ctx.perturbed_density([1.0], uv, 0.1, [0.0])
    assert e.value.status == _lib.BDG_ESTATE
    ctx.ground_state(tol=1e-12)
    assert ctx.perturbed_density([], uv[:0], 0.1, [0.0]).shape[0] == 0
    assert ctx.perturbed_density([1.0], uv, 0.1, []).shape[1] == 0
    with pytest.raises(BdgError) as e:
        ctx.perturbed_density([1.0], uv, float("nan"), [0.0])
    assert e.value.status == _lib.BDG_EINVAL
    ctx.close()


@pytest.mark.parametrize("w,k,block", [
    (W.C1, 8, 8),
    (W.Workload("2d_64x32_aniso_fm", 2, (64, 32), (8.0, 6.0), "harmonic2_aniso", 40.0, -1.0, 0.0), 10, 14),
    (W.Workload("3d_32_z2_fm", 3, (32, 32, 32), (6.0, 6.0, 6.0), "harmonic3_z2", 40.0, -1.0, 0.1), 10, 16),
], ids=lambda x: getattr(x, "name", str(x)))
def test_mode_amplitudes_match_oracle(w, k, block):
    """bdg_mode_amplitudes on eigenvectors and on arbitrary fields against oracle.modes."""
    torch = torch_cuda()
    say("mode amplitudes", w.name)
    ctx, phi, out = _solve(w, k, block)
    X = torch.from_numpy(W.random_block((2, 6) + w.shape, seed=5)).to("cuda")
    for uv in (out["uv"], X):
        got = np.array(ctx.mode_amplitudes(uv))
        ref = modes.mode_amplitudes(uv.cpu().numpy(), w.n, w.L)
        assert got.shape == ref.shape
        assert np.allclose(got[..., :2], ref[..., :2], rtol=1e-13, atol=0)
        assert np.abs(got[..., 2:] - ref[..., 2:]).max() <= 1e-12 * max(1.0, np.abs(ref[..., 2:]).max())
    ctx.close()


def test_mode_amplitudes_closed_forms_on_device():
    """x exp(-r^2/2) on a 64^3 grid of [-8, 8]^3: N = pi^(3/2)/2, max e^(-1/2), moments (3/2, 1/2,
    1/2), parities (-1, +1, +1); a zero field gives zeros; no ground state is needed."""
    torch = torch_cuda()
    from paper_2506_08308_amd import BdgError, _lib
    w = W.Workload("3d_64_box", 3, (64, 64, 64), (8.0, 8.0, 8.0), "harmonic3", 10.0, -1.0, 0.0)
    ctx = make_ctx(w)
    X, Y, Z = W.coordinates(w)
    uv = np.zeros((1, 6) + w.shape, dtype=complex)
    uv[0, 2] = (0.3 - 1j) * X * np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 2)
    got = np.array(ctx.mode_amplitudes(torch.from_numpy(uv).to("cuda")))
    r = got[0, 2]
    assert np.isclose(r[0], 1.09 * np.pi ** 1.5 / 2, rtol=1e-13)
    assert np.isclose(r[1], np.sqrt(1.09) * np.exp(-0.5), rtol=1e-13)
    assert np.allclose(r[2:5], [1.5, 0.5, 0.5], rtol=1e-12)
    assert np.allclose(r[5:8], [-1.0, 1.0, 1.0], atol=1e-13)
    assert np.all(got[0, 0] == 0.0)
    assert ctx.mode_amplitudes(torch.zeros((0, 6) + w.shape, dtype=torch.complex128, device="cuda")) == []
    import ctypes
    assert ctx._lib.bdg_mode_amplitudes(ctx._h, -1, None, None) == _lib.BDG_EINVAL
    ctx.close()
