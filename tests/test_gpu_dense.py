"""Parity of the dense kernels (MFMA Gram and update, Jacobi SVD, Cholesky) with numpy."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import make_ctx, say, torch_cuda

pytestmark = pytest.mark.gpu

W2 = W.Workload("2d_8", 2, (8, 8), (2.0, 2.0), "harmonic2", 1.0, -0.1, 0.0)


def _ctx():
    from paper_2506_08308_amd import Precision
    return make_ctx(W2, Precision.FP64)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


# herm: 0 general A^H B; 1 Hermitian with B = A; 2 Hermitian with a distinct operand
# B = D A (D real diagonal), the case of the Rayleigh-Ritz Grams S^H (H S).  The shapes reach
# the three forms (64-tiles; 80-tiles for 70..80 columns and 80 x 240; the thin form for
# m1 <= 16, single dot products included), diagonal and off-diagonal tiles, one and several
# K-splits, and ragged row and column tails.
@pytest.mark.parametrize("K,m1,m2,herm", [(37, 5, 7, 0), (1000, 40, 40, 0), (3072, 64, 64, 1), (5000, 80, 120, 0),
                                          (100000, 240, 240, 1), (70001, 16, 3, 0), (12, 130, 130, 1),
                                          (20000, 144, 144, 2), (4099, 70, 70, 2), (50000, 160, 160, 1),
                                          (20000, 80, 80, 1), (7001, 80, 80, 0), (30000, 80, 240, 0),
                                          (100003, 75, 75, 2), (1000003, 1, 1, 0), (200000, 8, 80, 0),
                                          (9000, 12, 12, 1)])
def test_gram_matches_numpy(K, m1, m2, herm):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"gram K={K} {m1}x{m2} herm={herm}")
    ctx = _ctx()
    A = W.random_block((m1, K), seed=1)
    if herm == 1:
        B = A
    elif herm == 2:
        B = A * np.random.default_rng(3).uniform(0.5, 2.0, K)[None, :]
    else:
        B = W.random_block((m2, K), seed=2)
    Ad = torch.from_numpy(A).cuda()
    Bd = Ad if herm == 1 else torch.from_numpy(np.ascontiguousarray(B)).cuda()
    C = torch.zeros((m2, m1), dtype=torch.complex128, device="cuda")   # column-major m1 x m2
    st = ctx._lib.bdg_test_gram(ctx._h, K, m1, m2, _p(Ad), K, _p(Bd), K, 0.5, _p(C), m1, 1 if herm else 0)
    assert st == _lib.BDG_OK
    got = C.cpu().numpy().T
    ref = 0.5 * (A.conj() @ B.T)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}")
    assert err < 1e-13
    ctx.close()


@pytest.mark.parametrize("K,m,nb,beta", [(37, 5, 3, 0.0), (1000, 40, 16, 0.0), (5000, 240, 80, 1.0),
                                         (129, 7, 33, -0.5), (100000, 24, 8, 0.0), (100003, 1, 1, 1.0),
                                         (4099, 8, 16, -0.5)])
def test_update_matches_numpy(K, m, nb, beta):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"update K={K} m={m} nb={nb}")
    ctx = _ctx()
    S = W.random_block((m, K), seed=3)
    Cm = W.random_block((nb, m), seed=4)      # column-major m x nb
    Y0 = W.random_block((nb, K), seed=5)
    Sd, Cd, Yd = (torch.from_numpy(a).cuda() for a in (S, Cm, Y0))
    st = ctx._lib.bdg_test_update(ctx._h, K, m, _p(Sd), K, _p(Cd), m, nb, beta, _p(Yd), K)
    assert st == _lib.BDG_OK
    got = Yd.cpu().numpy()
    ref = (S.T @ Cm.T).T + beta * Y0
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}")
    assert err < 1e-13
    ctx.close()


@pytest.mark.parametrize("rows,m", [(6, 6), (40, 40), (37, 24), (240, 240), (17, 33)])
def test_jacobi_svd_matches_numpy(rows, m):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"svd {rows}x{m}")
    ctx = _ctx()
    G = W.random_block((m, rows), seed=6)     # column-major rows x m
    Gd = torch.from_numpy(G.copy()).cuda()
    V = torch.zeros((m, m), dtype=torch.complex128, device="cuda")
    s = torch.zeros(m, dtype=torch.float64, device="cuda")
    st = ctx._lib.bdg_test_svd(ctx._h, rows, m, _p(Gd), rows, _p(V), m, _p(s))
    assert st == _lib.BDG_OK
    Gm = G.T                                   # rows x m
    s_ref = np.linalg.svd(Gm, compute_uv=False)
    sh = s.cpu().numpy()
    kk = min(rows, m)
    assert np.allclose(sh[:kk], s_ref[:kk], rtol=1e-12, atol=1e-12 * s_ref[0])
    assert np.all(sh[kk:] < 1e-12 * s_ref[0])
    Vm = V.cpu().numpy().T
    US = Gd.cpu().numpy().T
    assert np.abs(Gm @ Vm - US).max() < 1e-12 * s_ref[0]
    assert np.abs(Vm.conj().T @ Vm - np.eye(m)).max() < 1e-12
    ctx.close()


@pytest.mark.parametrize("rows,m,spread", [(6, 6, 1.0), (40, 40, 3.0), (37, 24, 2.0), (240, 240, 3.6),
                                           (17, 33, 1.0), (161, 161, 3.6)])
def test_jacobi_svd_real_matches_numpy(rows, m, spread):
    """Real variant (paired real form): singular values spread over `spread` decades, as the
    projected frequencies are; U S = G V, V orthogonal, all parts real."""
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"svd real {rows}x{m}")
    ctx = _ctx()
    rng = np.random.default_rng(11)
    kk = min(rows, m)
    Ua, _ = np.linalg.qr(rng.standard_normal((rows, kk)))
    Va, _ = np.linalg.qr(rng.standard_normal((m, kk)))
    Gm = (Ua * np.logspace(0.0, -spread, kk)) @ Va.T          # rows x m
    Gd = torch.from_numpy(Gm.T.astype(np.complex128).copy()).cuda()
    V = torch.zeros((m, m), dtype=torch.complex128, device="cuda")
    s = torch.zeros(m, dtype=torch.float64, device="cuda")
    st = ctx._lib.bdg_test_svd_real(ctx._h, rows, m, _p(Gd), rows, _p(V), m, _p(s))
    assert st == _lib.BDG_OK
    s_ref = np.linalg.svd(Gm, compute_uv=False)
    sh = s.cpu().numpy()
    assert np.allclose(sh[:kk], s_ref[:kk], rtol=1e-12, atol=1e-14 * s_ref[0])
    assert np.all(sh[kk:] < 1e-12 * s_ref[0])
    Vm = V.cpu().numpy().T
    US = Gd.cpu().numpy().T
    assert np.abs(Vm.imag).max() == 0 and np.abs(US.imag).max() == 0
    assert np.abs(Gm @ Vm.real - US.real).max() < 1e-12 * s_ref[0]
    assert np.abs(Vm.real.T @ Vm.real - np.eye(m)).max() < 1e-12
    ctx.close()


# A real Jacobi round shares each column-block pair among BDG_JACOBI_SPLIT workgroups (8 by
# default), each computing the pair's rotation and rotating a share of the rows, the rounds
# alternating between two buffers; with 1 the pair's workgroup works in place.  Same
# rotations and the same arithmetic per row: the two must agree bit for bit (odd and even
# numbers of rounds, ragged blocks, more rows than columns and fewer).
@pytest.mark.parametrize("rows,m", [(240, 240), (161, 161), (37, 24), (17, 33)])
def test_jacobi_svd_real_split_matches_single(rows, m, monkeypatch):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"svd real split vs single {rows}x{m}")
    rng = np.random.default_rng(12)
    kk = min(rows, m)
    Ua, _ = np.linalg.qr(rng.standard_normal((rows, kk)))
    Va, _ = np.linalg.qr(rng.standard_normal((m, kk)))
    Gm = (Ua * np.logspace(0.0, -3.6, kk)) @ Va.T
    out = {}
    for split in ("1", "8"):
        monkeypatch.setenv("BDG_JACOBI_SPLIT", split)
        ctx = _ctx()
        Gd = torch.from_numpy(Gm.T.astype(np.complex128).copy()).cuda()
        V = torch.zeros((m, m), dtype=torch.complex128, device="cuda")
        s = torch.zeros(m, dtype=torch.float64, device="cuda")
        assert ctx._lib.bdg_test_svd_real(ctx._h, rows, m, _p(Gd), rows, _p(V), m, _p(s)) == _lib.BDG_OK
        out[split] = (Gd.cpu().numpy(), V.cpu().numpy(), s.cpu().numpy())
        ctx.close()
    for a, b in zip(out["1"], out["8"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("m", [1, 5, 64, 240])
def test_cholesky_matches_numpy(m):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"cholesky {m}")
    ctx = _ctx()
    X = W.random_block((m, m), seed=7)
    A = X @ X.conj().T + m * np.eye(m)
    Ad = torch.from_numpy(A.T.copy()).cuda()   # column-major
    st = ctx._lib.bdg_test_cholesky(ctx._h, m, _p(Ad), m)
    assert st == _lib.BDG_OK
    Lg = Ad.cpu().numpy().T
    assert np.allclose(Lg, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12 * np.sqrt(m))
    # an indefinite matrix is reported
    B = -np.eye(m)
    Bd = torch.from_numpy(B.astype(np.complex128)).cuda()
    assert ctx._lib.bdg_test_cholesky(ctx._h, m, _p(Bd), m) == _lib.BDG_EBREAKDOWN
    ctx.close()


@pytest.mark.parametrize("m,rank", [(12, 12), (48, 40), (144, 144), (240, 200)])
def test_pivoted_cholesky_orthonormalizes(m, rank):
    """R^H A R = I on the numerical range; dependent columns are detected."""
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"pchol m={m} rank={rank}")
    ctx = _ctx()
    K = 3 * m
    S = W.random_block((rank, K), seed=9).T @ W.random_block((rank, m), seed=10)   # K x m, rank `rank`
    S = S * np.exp(np.linspace(-3, 3, m))[None, :]                                  # uneven column norms
    A = S.conj().T @ S
    Ad = torch.from_numpy(A.T.copy()).cuda()
    R = torch.zeros((m, m), dtype=torch.complex128, device="cuda")
    r = ctypes.c_int()
    st = ctx._lib.bdg_test_pchol(ctx._h, m, _p(Ad), m, 1e-12, _p(R), ctypes.byref(r))
    assert st == _lib.BDG_OK and r.value == rank
    Rm = R.cpu().numpy().T[:, :rank]
    Q = S @ Rm
    assert np.abs(Q.conj().T @ Q - np.eye(rank)).max() < 1e-6
    # the span of S is kept
    U, s, _ = np.linalg.svd(S, full_matrices=False)
    U = U[:, :rank]
    assert np.abs(Q - U @ (U.conj().T @ Q)).max() < 1e-8
    ctx.close()


@pytest.mark.parametrize("p,q,rank", [(10, 10, 10), (40, 36, 36), (144, 144, 130)])
def test_complete_pivoting_lu_biorthogonalizes(p, q, rank):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"plu {p}x{q} rank={rank}")
    ctx = _ctx()
    B = W.random_block((rank, p), seed=11).T @ W.random_block((rank, q), seed=12)   # p x q
    Bd = torch.from_numpy(B.T.copy()).cuda()
    Cf = torch.zeros((q, q), dtype=torch.complex128, device="cuda")
    Cg = torch.zeros((p, p), dtype=torch.complex128, device="cuda")
    r = ctypes.c_int()
    st = ctx._lib.bdg_test_plu(ctx._h, p, q, _p(Bd), p, 1e-10, _p(Cf), _p(Cg), ctypes.byref(r))
    assert st == _lib.BDG_OK and r.value == rank
    cf = Cf.cpu().numpy().reshape(-1)[:q * rank].reshape(rank, q).T
    cg = Cg.cpu().numpy().reshape(-1)[:p * rank].reshape(rank, p).T
    assert np.abs(cg.conj().T @ B @ cf - np.eye(rank)).max() < 1e-8
    ctx.close()


# Paired real form: A, B hold two real columns per complex column (real part, imaginary part);
# sym: 0 general, 1 B = A, 2 B = D A (the Rayleigh-Ritz shape S^T (H S) with symmetric H);
# shapes reach single and several tiles, K-splits and ragged tails; symmetric forms of 65..128
# complex columns take the whole-matrix kernel (one workgroup per K-split), 100 and 128 with
# ragged K included, and general ones of at most 40 block pairs (the F rows of the projected
# operators).
@pytest.mark.parametrize("K,m1,m2,sym", [(37, 5, 7, 0), (3072, 64, 64, 1), (20000, 120, 120, 2), (100000, 120, 120, 1),
                                         (5000, 40, 120, 0), (12, 65, 65, 1), (70001, 3, 16, 0), (9000, 36, 36, 2),
                                         (50003, 100, 100, 2), (4099, 128, 128, 2), (777, 97, 97, 1),
                                         (30011, 33, 100, 0), (2048, 80, 40, 0)])
def test_gram_pair_matches_numpy(K, m1, m2, sym):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"gram pair K={K} {m1}x{m2} sym={sym}")
    ctx = _ctx()
    A = W.random_block((m1, K), seed=1)
    if sym == 1:
        B = A
    elif sym == 2:
        B = A * np.random.default_rng(3).uniform(0.5, 2.0, K)[None, :]
    else:
        B = W.random_block((m2, K), seed=2)
    Ad = torch.from_numpy(A).cuda()
    Bd = Ad if sym == 1 else torch.from_numpy(np.ascontiguousarray(B)).cuda()
    C = torch.zeros((2 * m2, 2 * m1), dtype=torch.complex128, device="cuda")   # column-major 2 m1 x 2 m2
    st = ctx._lib.bdg_test_gram_pair(ctx._h, K, m1, m2, _p(Ad), K, _p(Bd), K, 0.5, _p(C), 2 * m1, 1 if sym else 0)
    assert st == _lib.BDG_OK
    got = C.cpu().numpy().T
    # real columns: 2 p + u is the real (u = 0) or imaginary (u = 1) part of complex column p
    Ar = np.stack([A.real, A.imag], axis=1).reshape(2 * m1, K)
    Br = np.stack([B.real, B.imag], axis=1).reshape(2 * m2, K)
    ref = 0.5 * (Ar @ Br.T)
    assert np.all(got.imag == 0.0)
    err = np.abs(got.real - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}")
    assert err < 1e-13
    ctx.close()


# The whole-matrix paired Gram in blocks of 8 complex columns loads its operands straight
# into LDS (BDG_GRAM_W8=2, the default) or stages them through registers (1): the same tiles
# and the same summation order, so the two must agree bit for bit (ragged tails included).
@pytest.mark.parametrize("K,m1,m2,sym", [(20000, 120, 120, 2), (4099, 128, 128, 1), (777, 97, 97, 2),
                                         (30011, 33, 100, 0), (50003, 100, 100, 2)])
def test_gram_pair_w8_direct_matches_staged(K, m1, m2, sym, monkeypatch):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"gram pair w8 direct vs staged K={K} {m1}x{m2} sym={sym}")
    A = W.random_block((m1, K), seed=1)
    B = A if sym == 1 else (A * np.random.default_rng(3).uniform(0.5, 2.0, K)[None, :] if sym == 2
                            else W.random_block((m2, K), seed=2))
    Ad = torch.from_numpy(A).cuda()
    Bd = Ad if sym == 1 else torch.from_numpy(np.ascontiguousarray(B)).cuda()
    out = {}
    for mode in ("1", "2"):
        monkeypatch.setenv("BDG_GRAM_W8", mode)
        ctx = _ctx()
        C = torch.zeros((2 * m2, 2 * m1), dtype=torch.complex128, device="cuda")
        st = ctx._lib.bdg_test_gram_pair(ctx._h, K, m1, m2, _p(Ad), K, _p(Bd), K, 1.0, _p(C), 2 * m1,
                                         1 if sym else 0)
        assert st == _lib.BDG_OK
        out[mode] = C.cpu().numpy()
        ctx.close()
    assert np.array_equal(out["1"], out["2"])


# Deeper staging of the loads (thin Grams of at most 16 x 16, the split-K reductions of every
# Gram) against the plain forms: the same K-splits, chunk order, matrix-core operands and
# order of additions, so the two agree bit for bit.  The solver's dot products over
# 3 x 128^3 rows, projections onto one or two vectors, the 64- and 80-tilings, Hermitian
# mirrors and ragged tails.
@pytest.mark.parametrize("K,m1,m2,herm", [(6291456, 1, 1, 0), (6291456, 1, 1, 1), (6291456, 2, 1, 0),
                                          (1000003, 1, 2, 0), (70001, 16, 3, 0), (9000, 12, 12, 1),
                                          (37, 5, 7, 0), (100003, 16, 16, 0), (4099, 3, 16, 0),
                                          (200000, 2, 40, 0), (100000, 240, 240, 1), (5000, 80, 120, 0),
                                          (20000, 144, 144, 1)])
def test_deep_loads_gram_matches_plain(K, m1, m2, herm, monkeypatch):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"gram deep loads vs plain K={K} {m1}x{m2} herm={herm}")
    Ad = torch.from_numpy(W.random_block((m1, K), seed=4)).cuda()
    Bd = Ad if herm else torch.from_numpy(W.random_block((m2, K), seed=5)).cuda()
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("BDG_DEEP_LOADS", mode)
        ctx = _ctx()
        C = torch.zeros((m2, m1), dtype=torch.complex128, device="cuda")
        st = ctx._lib.bdg_test_gram(ctx._h, K, m1, m2, _p(Ad), K, _p(Bd), K, 0.5, _p(C), m1, herm)
        assert st == _lib.BDG_OK
        out[mode] = C.cpu().numpy()
        ctx.close()
    assert np.array_equal(out["0"].view(np.uint64), out["1"].view(np.uint64))
    ref = 0.5 * (Ad.cpu().numpy().conj() @ Bd.cpu().numpy().T)
    assert np.abs(out["1"].T - ref).max() <= 1e-13 * np.abs(ref).max()


# The paired Grams' split-K reductions, staged and plain: the same bits (the 8-column, wide
# and 64-tile forms).
@pytest.mark.parametrize("K,m1,m2,sym", [(20000, 120, 120, 1), (30011, 33, 100, 0), (100003, 40, 40, 1),
                                         (4099, 128, 128, 1), (777, 97, 97, 0)])
def test_deep_loads_gram_pair_matches_plain(K, m1, m2, sym, monkeypatch):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"gram pair deep loads vs plain K={K} {m1}x{m2} sym={sym}")
    Ad = torch.from_numpy(W.random_block((m1, K), seed=1)).cuda()
    Bd = Ad if sym else torch.from_numpy(W.random_block((m2, K), seed=2)).cuda()
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("BDG_DEEP_LOADS", mode)
        ctx = _ctx()
        C = torch.zeros((2 * m2, 2 * m1), dtype=torch.complex128, device="cuda")
        st = ctx._lib.bdg_test_gram_pair(ctx._h, K, m1, m2, _p(Ad), K, _p(Bd), K, 1.0, _p(C), 2 * m1, sym)
        assert st == _lib.BDG_OK
        out[mode] = C.cpu().numpy()
        ctx.close()
    assert np.array_equal(out["0"].view(np.uint64), out["1"].view(np.uint64))


# Updates of at most 8 into 16 columns by a row loop per wave, and of at most 8 into more
# columns with Z loaded first: the MFMAs of the general form on the same operands, so the
# two agree bit for bit (projections of one vector, or of a block, onto one or two vectors
# over up to 3 x 128^3 rows, beta 0 and not, ragged row and column tails).
@pytest.mark.parametrize("K,m,nb,beta", [(6291456, 1, 1, 1.0), (6291456, 2, 1, 1.0), (1000003, 8, 16, 0.0),
                                         (37, 5, 3, 0.5), (100003, 3, 7, -1.0), (5, 1, 1, 1.0),
                                         (1000003, 2, 40, 1.0), (100003, 3, 33, -0.5), (4099, 8, 80, 0.5),
                                         (37, 5, 17, 1.0)])
def test_update_thin_matches_general(K, m, nb, beta, monkeypatch):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"update thin vs general K={K} m={m} nb={nb} beta={beta}")
    Sd = torch.from_numpy(W.random_block((m, K), seed=6)).cuda()
    Cd = torch.from_numpy(W.random_block((nb, m), seed=7)).cuda()
    Y0 = torch.from_numpy(W.random_block((nb, K), seed=8)).cuda()
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("BDG_DEEP_LOADS", mode)
        ctx = _ctx()
        Yd = Y0.clone()
        st = ctx._lib.bdg_test_update(ctx._h, K, m, _p(Sd), K, _p(Cd), m, nb, beta, _p(Yd), K)
        assert st == _lib.BDG_OK
        out[mode] = Yd.cpu().numpy()
        ctx.close()
    assert np.array_equal(out["0"].view(np.uint64), out["1"].view(np.uint64))


# One-pass update of the eigensolver (F columns first): the solve's shape, a ragged row tail,
# no F part, no [W, P] part, and the widest block it takes (96 real columns)
@pytest.mark.parametrize("K,m,mF,nb", [(5000, 120, 40, 80), (777, 24, 8, 16), (300, 16, 0, 10), (513, 16, 16, 6),
                                       (100003, 72, 24, 96)])
def test_update_pair_fused_matches_numpy(K, m, mF, nb):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"update pair fused K={K} m={m} mF={mF} nb={nb}")
    ctx = _ctx()
    S = W.random_block((m, K), seed=13)
    Cr = np.random.default_rng(14).standard_normal((nb, 2 * m))    # column-major 2 m x nb, real
    Sd = torch.from_numpy(S).cuda()
    Cd = torch.from_numpy((Cr + 0.0j).astype(np.complex128)).cuda()
    Yp = torch.full((nb // 2, K), 7.0 + 7.0j, dtype=torch.complex128, device="cuda")
    Yf = torch.full((nb // 2, K), 7.0 + 7.0j, dtype=torch.complex128, device="cuda")
    st = ctx._lib.bdg_test_update_pair_fused(ctx._h, K, m, mF, _p(Sd), K, _p(Cd), 2 * m, nb, _p(Yp), _p(Yf), K)
    assert st == _lib.BDG_OK
    Sr = np.stack([S.real, S.imag], axis=1).reshape(2 * m, K)
    ref_p = Cr[:, 2 * mF:] @ Sr[2 * mF:]
    ref_f = Cr[:, :2 * mF] @ Sr[:2 * mF] + ref_p
    scale = max(np.abs(ref_f).max(), np.abs(ref_p).max())
    for got, ref in ((Yp, ref_p), (Yf, ref_f)):
        g = got.cpu().numpy()
        g_r = np.stack([g.real, g.imag], axis=1).reshape(nb, K)
        err = np.abs(g_r - ref).max() / scale
        say(f"   rel err {err:.2e}")
        assert err < 1e-13
    # unsupported shapes are rejected (odd or too wide blocks, F not a multiple of 8)
    assert ctx._lib.bdg_test_update_pair_fused(ctx._h, K, m, mF, _p(Sd), K, _p(Cd), 2 * m, 98, _p(Yp), _p(Yf),
                                               K) == _lib.BDG_EINVAL
    assert ctx._lib.bdg_test_update_pair_fused(ctx._h, K, m, 3, _p(Sd), K, _p(Cd), 2 * m, nb, _p(Yp), _p(Yf),
                                               K) == _lib.BDG_EINVAL
    ctx.close()


@pytest.mark.parametrize("K,m,nb,beta", [(37, 5, 4, 0.0), (1000, 20, 16, 0.0), (5000, 120, 80, 1.0),
                                         (129, 7, 34, -0.5), (100000, 12, 8, 0.0)])
def test_update_pair_matches_numpy(K, m, nb, beta):
    torch = torch_cuda()
    from paper_2506_08308_amd import _lib
    say(f"update pair K={K} m={m} nb={nb}")
    ctx = _ctx()
    S = W.random_block((m, K), seed=3)
    Cr = np.random.default_rng(4).standard_normal((nb, 2 * m))     # column-major 2 m x nb, real
    Y0 = W.random_block((nb // 2, K), seed=5)
    Sd, Yd = torch.from_numpy(S).cuda(), torch.from_numpy(Y0).cuda()
    Cd = torch.from_numpy((Cr + 0.0j).astype(np.complex128)).cuda()
    st = ctx._lib.bdg_test_update_pair(ctx._h, K, m, _p(Sd), K, _p(Cd), 2 * m, nb, beta, _p(Yd), K)
    assert st == _lib.BDG_OK
    got = Yd.cpu().numpy()
    Sr = np.stack([S.real, S.imag], axis=1).reshape(2 * m, K)
    Yr0 = np.stack([Y0.real, Y0.imag], axis=1).reshape(nb, K)
    ref = Cr @ Sr + beta * Yr0                                   # rows: real output columns
    got_r = np.stack([got.real, got.imag], axis=1).reshape(nb, K)
    err = np.abs(got_r - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}")
    assert err < 1e-13
    ctx.close()
