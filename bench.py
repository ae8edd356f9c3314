"""Benchmark: time to the k lowest BdG eigenpairs on one MI355X, with kernel rooflines.

One step = one full bdg_eigs solve (deflation set-up, subspace iteration with the FFT apply,
bi-orthogonalization, Rayleigh-Ritz, updates, float64 certification) from the seed-0
complex-normal start block (for the real ground state of these workloads the library iterates
on real vectors, Re + Im of each start vector) to residual <= tol for all k wanted pairs.  The ground state is
computed on the GPU (bdg_ground_state) before the timed region; inputs are resident in HBM.

Default workload: the 3-D trap, 128^3 grid on [-8, 8]^3, V = (x^2 + y^2 + 4 z^2)/2,
beta_n = 400, beta_s = -4, M = 0.1, k = 64, block 80, residual 1e-8, float32-apply mixed
precision; the float64 solve of the same problem is timed beside it (--no-fp64 skips it).

Wall-clock budget (--budget-s, default 480 s from process start): at most one warmup solve
runs, and timed solves stop once another one would not leave room for the float64 solve,
the roofline launches and the CPU baseline; "steps" reports the solves actually timed
(config.steps_requested the number asked for).

Prints ONE JSON line.  ``roofline`` is the Gram kernel of the solve (k_gram_pair, the real
Gram matrices of the paired form) against the FP64 matrix peak; ``roofline_apply`` is the BdG
apply against the HBM peak (also reported for float64 vectors and at the 256^3 shape).  Both are timed live with HIP events on the context stream at the solve's own
shapes.  ``--kernels-only`` runs just those launches (plus a 1 GiB device copy as the
traffic reference) for counter collection under rocprofv3.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

T_START = time.time()
ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "time-to-k-eigenpairs @1e-8 (FP32-apply vs FP64); BdG apply GB/s vs HBM peak"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6

WORKLOADS = {
    "c3": (W.C3, W.C3_FP64),
    "c3_fp64": (W.C3_FP64, None),
    "c2_fm": (W.C2_FM, None),
    "c2_polar": (W.C2_POLAR, None),
    "c1": (W.C1, None),
}
CPU_BASELINE_RESERVE_S = 90.0
KERNEL_SOURCES = {"gram": "paper_2506_08308_amd/csrc/dense.hip", "apply": "paper_2506_08308_amd/csrc/fft_apply.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _prec(w):
    from paper_2506_08308_amd import Precision
    return Precision.FP32_APPLY if w.precision == "fp32_apply" else Precision.FP64


def _context(w):
    import torch
    from paper_2506_08308_amd import BdgContext
    V = torch.from_numpy(W.potential(w)).to("cuda")
    return BdgContext(w.dim, w.n, w.L, V, w.beta_n, w.beta_s, w.mass, w.magnetization, _prec(w))


def _event_ms(stream, fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _source_hash(key):
    with open(os.path.join(ROOT, KERNEL_SOURCES[key]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _traffic(key, workload_name):
    """HBM bytes per launch from the committed counter runs, or None when the kernel source
    or the workload differs from the one the counters were taken on."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != _source_hash(key) or rec.get("workload") != workload_name:
        return None
    return rec.get("bytes_per_launch")


def gram_launch(ctx, w, reps=5):
    """One Rayleigh-Ritz Gram of the solve in its paired real form: M_r = S^T (H S) with
    m = 3 block real columns (m / 2 complex columns, two real vectors each) over K = 3 npts
    rows (symmetric result, distinct operands).  Algorithmic flops: m (m + 1) / 2 real
    entries x 2 K."""
    import torch
    K, m = 3 * w.npts, 3 * w.block
    mc = m // 2
    g = torch.Generator(device="cuda").manual_seed(0)
    A = torch.randn((mc, K), dtype=torch.complex128, device="cuda", generator=g)
    d = torch.rand((K,), dtype=torch.float64, device="cuda", generator=g) + 0.5
    B = A * d
    C = torch.empty((m, m), dtype=torch.complex128, device="cuda")
    lib = ctx._lib

    def run():
        st = lib.bdg_test_gram_pair(ctx._h, K, mc, mc, ctypes.c_void_p(A.data_ptr()), K,
                                    ctypes.c_void_p(B.data_ptr()), K, 1.0, ctypes.c_void_p(C.data_ptr()), m, 1)
        if st != 0:
            raise RuntimeError(f"bdg_test_gram_pair failed with status {st}")

    ms = _event_ms(ctx.stream, run, reps)
    flops = 1.0 * K * m * (m + 1)
    del A, B, C, d
    torch.cuda.empty_cache()
    return ms, flops


def apply_launch(ctx, w, reps=10):
    """bdg_apply on the full block (the correction block's apply in the solve).  Algorithmic
    bytes: read X and write Y (6 complex fields per vector) plus one read of the 12
    coefficient fields."""
    import torch
    from paper_2506_08308_amd import Form
    dt = ctx.vector_dtype()
    X = torch.randn((w.block, 6) + w.shape, dtype=dt, device="cuda")
    Y = torch.empty_like(X)
    ms = _event_ms(ctx.stream, lambda: ctx.apply(X, Form.FG, out=Y), reps)
    csize = 8 if dt == torch.complex64 else 16
    nbytes = w.block * 2 * 6 * w.npts * csize + 12 * w.npts * (csize // 2)
    del X, Y
    torch.cuda.empty_cache()
    return ms, nbytes


def apply_launch_large(reps=3):
    """bdg_apply at the 256^3 lattice trap's shape (64 complex64 vectors, the block of the
    largest configuration: X and Y 51.5 GB each).  Only the operator is exercised, so any real
    ground state serves (the initial spinor of the flow)."""
    import torch
    from paper_2506_08308_amd import BdgContext, Precision
    w = W.C5
    V = torch.from_numpy(W.potential(w)).to("cuda")
    ctx = BdgContext(w.dim, w.n, w.L, V, w.beta_n, w.beta_s, w.mass, w.magnetization, Precision.FP32_APPLY)
    ctx.set_ground_state(torch.from_numpy(W.initial_spinor(w)).to("cuda"), [1.0, 1.0, 1.0])
    del V
    ms, nbytes = apply_launch(ctx, w, reps=reps)
    ctx.close()
    torch.cuda.empty_cache()
    return ms, nbytes


def _apply_roof(ms, nbytes, label):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "kernel": label, "ms_per_launch": round(ms, 3),
            "algorithmic_bytes": nbytes}


def copy_reference(reps=3):
    """A plain device copy of 1 GiB (the traffic-counter reference)."""
    import torch
    x = torch.empty((1 << 27,), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    ms = _event_ms(torch.cuda.current_stream(), lambda: y.copy_(x), reps)
    del x, y
    return ms


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, gpu_iters, iters=2):
    """The CPU oracle's subspace iteration (numpy/scipy FP64 on the host cores) on a bounded
    sample of the same problem: `iters` iterations at the largest grid of at most 64 points
    per axis whose basis fits in half the free host memory, same k, block and seed-0 start
    block.  The oracle's ground-state flow runs a bounded 50 steps (the per-iteration cost
    does not depend on how far it got) and the deflation set-up is left out (a few
    projections per iteration).  Per-iteration time is split into the FFT operator applies
    (timed around them) and the rest (Gram matrices, projected problem, updates); the FFT
    share is scaled by DOF log DOF and the rest by DOF to the full grid, then multiplied
    by the GPU's iteration count."""
    import psutil
    from oracle import bdg, groundstate as gs, lrep, spectral
    n_s = min(w.n[0], 64)
    # the oracle holds about 30 half-blocks of block x 3 npts complex128 at once
    free = psutil.virtual_memory().available
    while n_s > 8 and 30 * w.block * 3 * (n_s ** w.dim) * 16 > 0.5 * free:
        n_s //= 2
    ws = W.scaled(w, n_s) if n_s != w.n[0] else w
    V = W.potential(ws)
    r = gs.ground_state(V, ws.beta_n, ws.beta_s, ws.mass, ws.magnetization, ws.n, ws.L, W.initial_spinor(ws),
                        tol=1e-10, max_iter=50)
    coef = bdg.coefficients(r.phi, r.mu, V, ws.beta_n, ws.beta_s)
    sigma, D = lrep.preconditioner_parameters(V, r.mu)
    prob = lrep.LrepProblem(coef, ws.n, ws.L, D)
    fft_s = [0.0]

    def timed(fn):
        def run(*a, **kw):
            t = time.time()
            out = fn(*a, **kw)
            fft_s[0] += time.time() - t
            return out
        return run

    prob.hplus, prob.hminus, prob.precond = timed(prob.hplus), timed(prob.hminus), timed(prob.precond)
    X0 = W.start_block(ws)
    t0 = time.time()
    lrep.lrep_eigs(prob, ws.k, X0, 1e-30, max_iter=iters, sigma=sigma)
    wall = time.time() - t0
    per_it, fft_it = wall / iters, fft_s[0] / iters
    s_fft, s_dof = 1.0, 1.0
    if ws is not w:
        d_full, d_s = 6 * w.npts, 6 * ws.npts
        s_dof = d_full / d_s
        s_fft = (d_full * np.log2(d_full)) / (d_s * np.log2(d_s))
    full_it = fft_it * s_fft + (per_it - fft_it) * s_dof
    cores = spectral.WORKERS
    return {"value": round(full_it * gpu_iters, 1), "unit": "s", "cores": int(cores), "kind": "oracle",
            "sample": f"{iters} iterations (the start-up projection counted in) of the oracle subspace iteration "
                      f"(numpy/scipy FP64, FFT and BLAS on {cores} threads of {os.cpu_count()} cores, "
                      f"{_cpu_model()}) at grid {list(ws.n)}, k {ws.k}, block {ws.block}: {per_it:.2f} s per "
                      f"iteration, {fft_it:.2f} s of it in FFT applies; scaled to {list(w.n)} by DOF log DOF "
                      f"(x{s_fft:.2f}) for the FFT part and DOF (x{s_dof:.1f}) for the rest = {full_it:.1f} s "
                      f"per iteration, x {gpu_iters} GPU iterations"}


def solve(w, X0, steps, warmup, max_iter, deadline=None, reserve_s=0.0, reserve_fn=None):
    """Ground state (untimed), `warmup` untimed solves, then up to `steps` timed solves; a
    further timed solve starts only when it is expected to end `reserve_s` (or
    reserve_fn(longest step so far)) before `deadline` (time.time() scale), so the run fits
    the caller's wall-clock budget."""
    import torch
    ctx = _context(w)
    t = time.time()
    _, mu, gres, gits = ctx.ground_state(tol=w.gs_tol, max_iter=200000)
    torch.cuda.synchronize()
    gs_s = time.time() - t
    log(f"[{w.name}] ground state: {gits} iterations, residual {gres:.2e}, mu {mu}, {gs_s:.2f} s")
    for i in range(warmup):
        out = ctx.eigs(w.k, w.block, tol=w.tol, max_iter=max_iter, X0=X0, want_vectors=False)
        log(f"[{w.name}] warmup {i}: {out['iters']} iterations")
    times, out = [], None
    for i in range(steps):
        res_s = reserve_fn(max(times)) if (times and reserve_fn is not None) else (reserve_s or 0.0)
        if times and deadline is not None and time.time() + max(times) + res_s > deadline:
            log(f"[{w.name}] wall-clock budget reached after {len(times)} timed solves of {steps}")
            break
        torch.cuda.synchronize()
        t0 = time.time()
        out = ctx.eigs(w.k, w.block, tol=w.tol, max_iter=max_iter, X0=X0, want_vectors=False)
        torch.cuda.synchronize()
        times.append(time.time() - t0)
        log(f"[{w.name}] step {i}: {times[-1]:.3f} s, {out['iters']} iterations, stats {ctx.stats()}")
    return ctx, out, times, gs_s


def kernels_only(w):
    """Only the roofline launches and the copy reference (for rocprofv3 counter runs)."""
    import torch
    ctx = _context(w)
    ctx.set_ground_state(torch.from_numpy(W.initial_spinor(w)).to("cuda"), [1.0, 1.0, 1.0])
    c_ms = copy_reference()
    g_ms, _ = gram_launch(ctx, w, reps=2)
    a_ms, _ = apply_launch(ctx, w, reps=2)
    log(f"copy 1 GiB {c_ms:.3f} ms, gram {g_ms:.3f} ms, apply {a_ms:.3f} ms")
    ctx.close()


# ------------------------------------------------------------------------------------------
# The paper's own campaigns (Section 4.1): accuracy of the Kohn modes against the analytical
# eigenpairs of the harmonic trap (Theorem "Analytical eigenpairs") and time against DOF.
# Ferromagnetic (beta_n, beta_s) = (885.4, -4.1), anti-ferromagnetic (240.8, 7.5), M = 0
# (the paper does not state M), box [-16, 16]^d in 1-D/2-D and [-8, 8]^3 in 3-D.
# ------------------------------------------------------------------------------------------
CAMPAIGN_BETAS = {"FM": (885.4, -4.1), "AFM": (240.8, 7.5)}
ACCURACY_CASES = [("I", "harmonic1", 1, 16.0, (32, 64, 128, 256, 512)),
                  ("II", "harmonic2", 2, 16.0, (32, 64, 128, 256, 512)),
                  ("III", "harmonic2_aniso", 2, 16.0, (32, 64, 128, 256, 512)),
                  ("IV", "harmonic3", 3, 8.0, (16, 32, 64, 128))]


def _kohn_errors(w, phi, omega, uv, gammas):
    """e_omega and e_uv of the paper for each trap frequency gamma_a: the computed modes nearest
    gamma_a (as many as gamma_a occurs) against the analytical eigenspace spanned by
    (gamma^-1/2 d_a Phi -+ gamma^1/2 x_a Phi) / sqrt 2 for all axes with that frequency."""
    coords = W.coordinates(w)                      # per axis, grid shaped, x first
    phi = np.asarray(phi)
    out = []
    om = np.asarray(omega)
    used = set()
    for a, g in enumerate(gammas):
        same = [b for b, gb in enumerate(gammas) if gb == g]
        U, Vv = [], []
        for b in same:
            ax = phi.ndim - 1 - b                  # array axis of coordinate b (x is last)
            n = phi.shape[ax]
            kk = np.fft.fftfreq(n, d=1.0 / n) * np.pi / w.L[b]
            kk[n // 2] = 0.0                       # first derivative: Nyquist mode dropped
            shape = [1] * phi.ndim
            shape[ax] = n
            dphi = np.real(np.fft.ifft(1j * kk.reshape(shape) * np.fft.fft(phi, axis=ax), axis=ax))
            xphi = coords[b][None] * phi
            U.append(((g ** -0.5) * dphi - (g ** 0.5) * xphi).ravel() / np.sqrt(2))
            Vv.append(((g ** -0.5) * dphi + (g ** 0.5) * xphi).ravel() / np.sqrt(2))
        QU, _ = np.linalg.qr(np.array(U).T)
        QV, _ = np.linalg.qr(np.array(Vv).T)
        order = [j for j in np.argsort(np.abs(om - g)) if j not in used]
        j = int(order[0])
        used.add(j)
        u = uv[j, :3].ravel()
        v = uv[j, 3:].ravel()
        eu = np.linalg.norm(u - QU @ (QU.conj().T @ u)) / np.linalg.norm(u)
        ev = np.linalg.norm(v - QV @ (QV.conj().T @ v)) / np.linalg.norm(v)
        out.append({"axis": "xyz"[a], "gamma": g, "omega": float(om[j]), "e_omega": abs(om[j] - g) / g,
                    "e_uv": float(eu + ev)})
    return out


def _ground_state(ctx, tol=1e-12, max_iter=400000, chunk=20000):
    """bdg_ground_state in chunks of `chunk` steps, each continuing from the last iterate, with
    a progress line per chunk (a slow flow stays visibly alive)."""
    phi, its = None, 0
    while True:
        phi, mu, res, n = ctx.ground_state(phi0=phi, tol=tol, max_iter=chunk, check=False)
        its += n
        if res <= tol or its >= max_iter:
            return phi, mu, res, its
        log(f"  ground state: {its} steps, residual {res:.2e}")


def campaign_accuracy(k=40, block=48, dims=(1, 2, 3)):
    import torch
    for case, pot, d, L, ns in ACCURACY_CASES:
        if d not in dims:
            continue
        for kind, (bn, bs) in CAMPAIGN_BETAS.items():
            for n in ns:
                w = W.Workload(f"acc_{case}_{kind}_{n}", d, (n,) * d, (L,) * d, pot, bn, bs, 0.0, k=k,
                               block=block)
                log(f"accuracy {w.name}")
                ctx = _context(w)
                t0 = time.time()
                phi, mu, gres, gits = _ground_state(ctx)
                # the k lowest modes must reach the largest trap frequency (the Kohn modes sit at
                # omega = gamma_a); widen the solve while they do not
                kk, bb = k, block
                while True:
                    out = ctx.eigs(kk, bb, tol=1e-10, max_iter=1500, seed=0, check=False)
                    if max(out["omega"]) > 1.05 * max(W.TRAP_GAMMAS[pot]) or kk >= 148:
                        break
                    # basis memory: 4 arrays x 4 slots x block x 3 npts complex128 <= 160 GB
                    bb = min(min(2 * kk, 148) + 12, 3 * w.npts - 4, int(160e9 / (256 * 3 * w.npts)))
                    if bb <= kk:
                        break
                    kk = min(2 * kk, 148, bb - 8)
                torch.cuda.synchronize()
                errs = _kohn_errors(w, phi.cpu().numpy(), out["omega"], out["uv"].cpu().numpy(),
                                    W.TRAP_GAMMAS[pot])
                ctx.close()
                print(json.dumps({"campaign": "accuracy", "case": case, "kind": kind, "dim": d, "N": n,
                                  "h": 2 * L / n, "ground_state_iters": gits, "ground_state_residual": gres,
                                  "k": kk, "eig_status": out["status"], "eig_iters": out["iters"],
                                  "max_residual": max(out["residual"]),
                                  "seconds": round(time.time() - t0, 2), "kohn": errs}), flush=True)


def campaign_efficiency(k=40, block=48, tol=1e-8, dims=(2, 3)):
    import torch
    for d, L, ns in ((2, 16.0, (32, 64, 128, 256, 512, 1024)), (3, 8.0, (16, 32, 64, 128))):
        if d not in dims:
            continue
        for kind, (bn, bs) in CAMPAIGN_BETAS.items():
            for n in ns:
                w = W.Workload(f"eff_{d}d_{kind}_{n}", d, (n,) * d, (L,) * d, f"harmonic{d}", bn, bs, 0.0, k=k,
                               block=block)
                log(f"efficiency {w.name}")
                ctx = _context(w)
                _ground_state(ctx)
                torch.cuda.synchronize()
                t0 = time.time()
                out = ctx.eigs(k, block, tol=tol, max_iter=3000, seed=0, want_vectors=False)
                torch.cuda.synchronize()
                dt = time.time() - t0
                st = ctx.stats()
                ctx.close()
                print(json.dumps({"campaign": "efficiency", "dim": d, "kind": kind, "N": n, "DOF": 6 * n ** d,
                                  "nev": k, "block": block, "tol": tol, "seconds": round(dt, 3),
                                  "iters": out["iters"], "phase_ms": {kk: round(st[kk], 1) for kk in (
                                      "apply_ms", "precond_ms", "gram_ms", "small_ms", "update_ms", "setup_ms")}}),
                      flush=True)


# Section 4.2, Example "2D Case": perturbed densities n_j^l(x, t = 10.6) with eps = 0.1 at
# h = 1/8 on [-16, 16]^2; Case I antiferromagnetic isotropic (l = 20, 35), Case II
# ferromagnetic with gamma_y = 2 gamma_x (l = 30, 55); l counts the ascending eigenvalues from 1.
MODES_CASES = [("I", "harmonic2", "AFM", (20, 35)), ("II", "harmonic2_aniso", "FM", (30, 55))]


def campaign_modes(n=256, k=56, block=64, eps=0.1, t_snap=10.6):
    import torch
    for case, pot, kind, ells in MODES_CASES:
        bn, bs = CAMPAIGN_BETAS[kind]
        w = W.Workload(f"modes_{case}_{kind}_{n}", 2, (n, n), (16.0, 16.0), pot, bn, bs, 0.0, k=k, block=block)
        log(f"modes {w.name}")
        ctx = _context(w)
        phi, mu, gres, gits = _ground_state(ctx)
        out = ctx.eigs(k, block, tol=1e-9, max_iter=1500, seed=0, check=False)
        hd = float(np.prod(w.h))
        sel = [l - 1 for l in ells]
        dens = ctx.perturbed_density([out["omega"][j] for j in sel], out["uv"][sel], eps, [t_snap]).cpu().numpy()
        rho0 = hd * (phi.cpu().numpy() ** 2).sum(axis=(1, 2))
        snaps = []
        for i, l in enumerate(ells):
            nj = dens[i, 0]
            snaps.append({"l": l, "omega": out["omega"][l - 1], "norm_j": (hd * nj.sum(axis=(1, 2))).tolist(),
                          "max_j": nj.max(axis=(1, 2)).tolist()})
        # bandwidth of the density kernel: all k modes at 16 times
        times = list(np.linspace(0.0, t_snap, 16))
        ms = _event_ms(ctx.stream, lambda: ctx.perturbed_density(out["omega"], out["uv"], eps, times), 5)
        nbytes = k * (6 * w.npts * 16 + 3 * w.npts * 8) + k * len(times) * 3 * w.npts * 8
        ctx.close()
        print(json.dumps({"campaign": "modes", "case": case, "kind": kind, "N": n, "eps": eps, "t": t_snap,
                          "eig_status": out["status"], "eig_iters": out["iters"], "ground_norm_j": rho0.tolist(),
                          "snapshots": snaps,
                          "density_kernel": {"modes": k, "times": len(times), "ms": round(ms, 4),
                                             "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                                             "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}}),
              flush=True)


def campaign_complex(n=256, L=12.0, beta_n=200.0, beta_s=80.0, k=32, block=48, tol=1e-10):
    """A complex ground state (Section 2.1, general BdG form): the uniform polar state moving with
    one grid quantum of momentum along x on [-L, L]^2.  Its spectrum is the Doppler-shifted
    Bogoliubov branches (computed here in closed form from the dispersion relation, no oracle).
    Times the pencil solve and one complex (u, v) apply on the block."""
    import torch
    from paper_2506_08308_amd import BdgContext, Form, Precision
    nn, LL = (n, n), (L, L)
    nbar = 1.0 / (2 * L) ** 2
    q = np.pi / L
    x = -L + np.arange(n) * (2 * L / n)
    phi = np.zeros((3, n, n), dtype=np.complex128)
    amp = np.sqrt(nbar / 2) * np.exp(1j * q * x)[None, :]
    phi[0] = amp
    phi[2] = amp
    mu = [beta_n * nbar + 0.5 * q * q] * 3
    # closed form: sqrt(e (e + 2 b nbar)) + q k_x over the grid wavevectors (b = beta_n once, beta_s twice)
    kk = np.fft.fftfreq(n, d=1.0 / n) * np.pi / L
    KY, KX = np.meshgrid(kk, kk, indexing="ij")
    eps = 0.5 * (KX ** 2 + KY ** 2)
    nz = eps > 0
    vals = np.concatenate([np.sqrt(eps[nz] * (eps[nz] + 2 * beta_n * nbar)) + q * KX[nz],
                           np.repeat(np.sqrt(eps[nz] * (eps[nz] + 2 * beta_s * nbar)) + q * KX[nz], 2)])
    ref = np.sort(vals[vals > 0])[:k]
    V = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx = BdgContext(2, nn, LL, V, beta_n, beta_s, 1.0, 0.0, Precision.FP64)
    ctx.set_ground_state_complex(torch.from_numpy(phi).to("cuda"), mu)
    torch.cuda.synchronize()
    t0 = time.time()
    out = ctx.eigs(k, block, tol=tol, max_iter=2000, seed=0, want_vectors=False, check=False)
    torch.cuda.synchronize()
    dt = time.time() - t0
    st = ctx.stats()
    X = torch.randn((block, 6, n, n), dtype=torch.complex128, device="cuda")
    Y = torch.empty_like(X)
    ms = _event_ms(ctx.stream, lambda: ctx.apply(X, Form.UV, out=Y), 5)
    npts = n * n
    nbytes = block * 2 * 6 * npts * 16 + 21 * npts * 8
    ctx.close()
    rel = float(np.max(np.abs(np.array(out["omega"]) - ref) / ref))
    print(json.dumps({"campaign": "complex", "state": "moving uniform polar", "N": n, "L": L, "q": q,
                      "beta_n": beta_n, "beta_s": beta_s, "k": k, "block": block, "tol": tol,
                      "eig_status": out["status"], "iters": out["iters"], "seconds": round(dt, 3),
                      "max_residual": max(out["residual"]), "max_rel_err_vs_doppler": rel,
                      "setup_ms": round(st["setup_ms"], 1),
                      "apply": {"vectors": block, "ms": round(ms, 3), "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}}),
          flush=True)


# Section 4.2, Example "3D Case": Bogoliubov amplitudes of the l-th mode at h = 1/8 on [-8, 8]^3;
# Case I ferromagnetic isotropic (l = 25), II antiferromagnetic isotropic (26), III
# ferromagnetic with gamma_z = 2 gamma_x = 2 gamma_y (62), IV antiferromagnetic, same trap (42);
# l counts the ascending eigenvalues from 1, M = 0 (the paper does not state M).
AMPLITUDE_CASES = [("I", "harmonic3", "FM", 25), ("II", "harmonic3", "AFM", 26),
                   ("III", "harmonic3_z2", "FM", 62), ("IV", "harmonic3_z2", "AFM", 42)]
FIELD_NAMES = ("u_1", "u_0", "u_-1", "v_1", "v_0", "v_-1")


def campaign_amplitudes(n=128, L=8.0, tol=1e-9):
    """The paper's figures show isosurfaces of u_j^l and v_j^l; the campaign reports, for the
    l-th mode and every member of its degenerate cluster, the per-field norm, maximum, second
    moments along x, y, z (the compression along the stiffer axis) and reflection parities
    (bdg_mode_amplitudes), with the amplitude kernel's time over all computed modes."""
    import torch
    for case, pot, kind, ell in AMPLITUDE_CASES:
        bn, bs = CAMPAIGN_BETAS[kind]
        k = ell + 4
        w = W.Workload(f"amp_{case}_{kind}_{n}", 3, (n,) * 3, (L,) * 3, pot, bn, bs, 0.0, k=k, block=k + 16)
        log(f"amplitudes {w.name}")
        ctx = _context(w)
        t0 = time.time()
        _ground_state(ctx)
        out = ctx.eigs(k, w.block, tol=tol, max_iter=1500, seed=0, check=False)
        om = out["omega"]
        j = ell - 1
        members = [i for i in range(k) if abs(om[i] - om[j]) <= 1e-8 * om[j]]
        summ = ctx.mode_amplitudes(out["uv"][members])
        ms = _event_ms(ctx.stream, lambda: ctx.mode_amplitudes(out["uv"]), 3)
        nbytes = k * 6 * w.npts * 16
        modes_out = []
        for i, s_l in zip(members, summ):
            modes_out.append({"index": i + 1, "omega": om[i], "fields": {
                FIELD_NAMES[f]: {"norm": s_l[f][0], "max": s_l[f][1], "x2": s_l[f][2:5], "parity": s_l[f][5:8]}
                for f in range(6)}})
        ctx.close()
        print(json.dumps({"campaign": "amplitudes", "case": case, "kind": kind, "trap": pot, "N": n,
                          "h": 2 * L / n, "l": ell, "eig_status": out["status"], "eig_iters": out["iters"],
                          "max_residual": max(out["residual"]), "seconds": round(time.time() - t0, 1),
                          "cluster": modes_out,
                          "amplitude_kernel": {"modes": k, "ms": round(ms, 3),
                                               "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}}), flush=True)


def _cluster_means(vals, omega, tol=1e-8):
    """Each member of a cluster |omega_i - omega_j| <= tol omega gets the cluster mean (the
    derivative of a degenerate eigenvalue is defined for the cluster's mean only)."""
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


def campaign_grad(ndir=32, eps=1e-6):
    """Gradients of the 16 lowest frequencies of the 2-D 256^2 lattice trap (beta_s = -2
    primary, +2 secondary) with respect to V(x), beta_n and beta_s (bdg_eigs_grad: left/right
    eigenvector form plus the ground-state sensitivity), against central differences of the
    whole GPU pipeline (ground state to 1e-13, eigensolve to 1e-10) along `ndir` seeded
    directions dV ~ N(0, 1) per point, d beta_n, d beta_s ~ N(0, 1), step eps.  k is widened
    past a degenerate pair at 16; relative error |FD - adjoint| / |FD| (absolute over
    ||grad|| ||dir|| where |FD| < 1e-3 ||grad|| ||dir||)."""
    import torch
    for w in (W.C4, W.C4_POLAR):
        V = W.potential(w)
        X0 = torch.from_numpy(W.start_block(w)).to("cuda")
        kq = w.k + 2

        def pipeline(Vx, bn, bs, k_use=None):
            ww = w.with_(beta_n=bn, beta_s=bs)
            from paper_2506_08308_amd import BdgContext, Precision
            ctx = BdgContext(ww.dim, ww.n, ww.L, torch.from_numpy(np.ascontiguousarray(Vx)).to("cuda"), bn, bs,
                             ww.mass, ww.magnetization, Precision.FP64)
            ctx.ground_state(tol=ww.gs_tol, max_iter=400000)
            out = ctx.eigs(kq, ww.block, tol=ww.tol, max_iter=3000, X0=X0)
            om = np.array(out["omega"])
            g, g_ms = None, None
            if k_use is not None:
                torch.cuda.synchronize()
                t0 = time.time()
                g = ctx.eigs_grad(list(om[:k_use]), out["uv"][:k_use].contiguous())
                torch.cuda.synchronize()
                g_ms = 1000.0 * (time.time() - t0)
            ctx.close()
            return om, g, g_ms

        om, _, _ = pipeline(V, w.beta_n, w.beta_s)
        k_use = w.k
        while k_use < kq and abs(om[k_use] - om[k_use - 1]) <= 1e-8 * om[k_use - 1]:
            k_use += 1
        om, (dV, dbn, dbs), g_ms = pipeline(V, w.beta_n, w.beta_s, k_use)
        om = om[:k_use]
        dV = dV.cpu().numpy()
        hd = float(np.prod(w.h))
        gnorm = np.array([np.sqrt(hd * np.sum(dV[j] ** 2) + dbn[j] ** 2 + dbs[j] ** 2) for j in range(k_use)])
        worst, per_dir = 0.0, []
        t0 = time.time()
        for seed in range(ndir):
            dVd, dbnd, dbsd = W.fd_direction(w, seed)
            op, _, _ = pipeline(V + eps * dVd, w.beta_n + eps * dbnd, w.beta_s + eps * dbsd)
            omm, _, _ = pipeline(V - eps * dVd, w.beta_n - eps * dbnd, w.beta_s - eps * dbsd)
            fd = _cluster_means((op[:k_use] - omm[:k_use]) / (2 * eps), om)
            ad = np.array([hd * np.sum(dV[j] * dVd) + dbn[j] * dbnd + dbs[j] * dbsd for j in range(k_use)])
            dnorm = np.sqrt(hd * np.sum(dVd ** 2) + dbnd ** 2 + dbsd ** 2)
            err = np.where(np.abs(fd) >= 1e-3 * gnorm * dnorm, np.abs(fd - ad) / np.abs(fd),
                           np.abs(fd - ad) / (gnorm * dnorm))
            per_dir.append(float(err.max()))
            worst = max(worst, float(err.max()))
            log(f"grad {w.name} direction {seed}: max rel err {err.max():.2e}")
        print(json.dumps({"campaign": "grad", "workload": w.name, "grid": list(w.n), "beta_s": w.beta_s,
                          "k": k_use, "directions": ndir, "eps": eps, "max_rel_err": worst,
                          "per_direction_max_rel_err": per_dir, "bound": 1e-5, "pass": worst <= 1e-5,
                          "eigs_grad_ms": round(g_ms, 1), "fd_seconds": round(time.time() - t0, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-clock budget of the whole run from process start: at most one warmup solve, and "
                         "timed solves stop early (the JSON line reports how many ran) so the float64 solve, "
                         "rooflines and CPU baseline still fit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 solve timed beside the mixed one")
    ap.add_argument("--kernels-only", action="store_true")
    ap.add_argument("--campaign", choices=("accuracy", "efficiency", "modes", "complex", "grad", "amplitudes"),
                    help="the paper's accuracy (Kohn modes vs h) or efficiency (time vs DOF) campaign, or its "
                         "perturbed-density example")
    ap.add_argument("--campaign-dims", default="1,2,3", help="comma-separated dimensions to run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; the multi-GPU sharding is designed, not built. "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    w, w64 = WORKLOADS[args.workload]
    if args.no_fp64:
        w64 = None
    if args.kernels_only:
        kernels_only(w)
        return
    dims = tuple(int(x) for x in args.campaign_dims.split(","))
    if args.campaign == "accuracy":
        campaign_accuracy(dims=dims)
        return
    if args.campaign == "efficiency":
        campaign_efficiency(dims=dims)
        return
    if args.campaign == "modes":
        campaign_modes()
        return
    if args.campaign == "complex":
        campaign_complex()
        return
    if args.campaign == "grad":
        campaign_grad()
        return
    if args.campaign == "amplitudes":
        campaign_amplitudes()
        return
    deadline = T_START + args.budget_s
    line_extra = {}
    cpu_reserve = 0.0 if args.no_cpu_baseline else CPU_BASELINE_RESERVE_S
    warmup = min(args.warmup, 1)
    X0 = torch.from_numpy(W.start_block(w)).to("cuda")

    def reserve(step_s):
        # what must still fit after the last timed solve: the float64 solve beside it, the
        # roofline launches and the CPU baseline
        return (1.2 * step_s + 10.0 if w64 is not None else 0.0) + 35.0 + cpu_reserve

    # the reserve depends on the step time, known after the first solve; solve() checks
    # before each further timed solve
    ctx, out, times, gs_s = solve(w, X0, args.steps, warmup, args.max_iter, deadline=deadline,
                                  reserve_fn=reserve)
    st = ctx.stats()
    ms = 1000.0 * float(np.mean(times))
    g_ms, g_flops = gram_launch(ctx, w)
    a_ms, a_bytes = apply_launch(ctx, w)
    ctx.close()
    g_tfs = g_flops / (g_ms * 1e-3) / 1e12
    a_gbs = a_bytes / (a_ms * 1e-3) / 1e9
    roof = {"bound": "mfma", "achieved": round(g_tfs, 2), "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(g_tfs / FP64_MFMA_PEAK_TFS, 4), "traffic": _traffic("gram", w.name),
            "kernel": f"k_gram_pair_w8d + k_gram_reduce_real_st: Rayleigh-Ritz Gram S^T (H S) of {3 * w.block} real "
                      f"columns (paired, {3 * w.block // 2} complex) x {3 * w.npts} rows, FP64 MFMA",
            "ms_per_launch": round(g_ms, 3), "algorithmic_flops": g_flops}
    roof_apply = {"bound": "hbm", "achieved": round(a_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(a_gbs / HBM_PEAK_GBS, 4), "traffic": _traffic("apply", w.name),
                  "kernel": f"bdg_apply on {w.block} vectors ({'complex64' if _prec(w) == 1 else 'complex128'})",
                  "ms_per_launch": round(a_ms, 3), "algorithmic_bytes": a_bytes}
    config = {"workload": w.name, "grid": list(w.n), "box": [-w.L[0], w.L[0]], "potential": w.potential,
              "beta_n": w.beta_n, "beta_s": w.beta_s, "magnetization": w.magnetization, "k": w.k,
              "block": w.block, "tol": w.tol, "precision": w.precision, "iters": int(st["iters"]),
              "applies_fp64": int(st["applies_fp64"]), "applies_fp32": int(st["applies_fp32"]),
              "phase_ms": {k: round(st[k], 1) for k in ("apply_ms", "precond_ms", "gram_ms", "small_ms",
                                                       "update_ms", "setup_ms")},
              "ground_state_s": round(gs_s, 3), "omega_first": [round(v, 12) for v in out["omega"][:4]],
              "max_residual": max(out["residual"]), "step_times_s": [round(t, 3) for t in times],
              "steps_requested": args.steps, "warmup_requested": args.warmup,
              "budget_s": args.budget_s}
    if w64 is not None:
        if time.time() + 1.2 * max(times) + 10.0 + 15.0 + cpu_reserve <= deadline:
            ctx64, out64, t64, _ = solve(w64, X0, 1, 0, args.max_iter)
            st64 = ctx64.stats()
            a64_ms, a64_bytes = apply_launch(ctx64, w64, reps=5)
            line_extra["roofline_apply_fp64"] = _apply_roof(
                a64_ms, a64_bytes, f"bdg_apply on {w64.block} complex128 vectors, {list(w64.n)} grid")
            ctx64.close()
            rel = max(abs(a - b) / abs(b) for a, b in zip(out["omega"], out64["omega"]))
            config["fp64_solve"] = {"s": round(t64[0], 3), "iters": int(st64["iters"]),
                                    "applies_fp64": int(st64["applies_fp64"]),
                                    "phase_ms": {k: round(st64[k], 1) for k in (
                                        "apply_ms", "precond_ms", "gram_ms", "small_ms", "update_ms", "setup_ms")},
                                    "max_rel_omega_diff_vs_mixed": rel}
        else:
            config["fp64_solve"] = {"skipped": "wall-clock budget"}
    line = {
        "metric": METRIC,
        "value": round(ms / 1000.0, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": len(times),
        "warmup": warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "c64-apply/f64" if w.precision == "fp32_apply" else "f64",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "roofline_apply": roof_apply,
    }
    line.update(line_extra)
    if time.time() + 20.0 + cpu_reserve <= deadline + 30.0:
        try:
            c5_ms, c5_bytes = apply_launch_large()
            line["roofline_apply_256"] = _apply_roof(
                c5_ms, c5_bytes, f"bdg_apply on {W.C5.block} complex64 vectors, {list(W.C5.n)} grid")
        except Exception as e:  # report, do not hide
            line["roofline_apply_256"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        if time.time() + cpu_reserve <= deadline + 30.0:
            try:
                line["cpu_baseline"] = cpu_baseline(w, int(st["iters"]))
            except Exception as e:  # report, do not hide
                line["cpu_baseline"] = {"value": None, "error": repr(e)}
        else:
            line["cpu_baseline"] = {"value": None, "skipped": "wall-clock budget"}
    config["wall_s"] = round(time.time() - T_START, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
