"""Host-side pieces of bench.py: the multi-GPU refusal and the accuracy campaign's error
measure (its own numpy code) against the oracle's definition of Section 4.1."""
import os
import subprocess
import sys

import numpy as np

import bench
import workloads as W
from oracle import bdg, groundstate as gs, kohn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_campaign_errors_equal_the_oracle_definition():
    """2-D anisotropic polar trap on a small grid (x and y modes at gamma = 1 and 2) and the
    1-D trap: bench's e_omega / e_uv equal oracle.kohn's on the same dense eigenpairs."""
    for w in (W.Workload("2d_n16_aniso", 2, (16, 16), (5.0, 5.0), "harmonic2_aniso", 10.0, 1.0, 0.0),
              W.Workload("1d_n64_fm", 1, (64,), (10.0,), "harmonic1", 30.0, -1.0, 0.0)):
        V = W.potential(w)
        r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L, W.initial_spinor(w),
                            tol=1e-12)
        c = bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)
        om, X = bdg.positive_eigs_dense(bdg.dense_uv(c, w.n, w.L), 24)
        uv = np.asarray(X).T.reshape((-1, 6) + w.shape)
        gam = W.TRAP_GAMMAS[w.potential]
        ref = kohn.accuracy_errors(om, uv, r.phi, w.n, w.L, gam)
        got = bench._kohn_errors(w, r.phi, om, uv, gam)
        assert len(ref) == len(got) == w.dim
        for a, b in zip(ref, got):
            assert a["omega"] == b["omega"]
            assert abs(a["e_omega"] - b["e_omega"]) <= 1e-15
            assert abs(a["e_uv"] - b["e_uv"]) <= 1e-10 * max(a["e_uv"], 1e-6)
