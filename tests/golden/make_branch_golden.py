"""Writes the stored branch-oracle spectra of the full-size parity tests.

Every value comes from the CPU oracle (``oracle/``) alone: the scalar Gross-Pitaevskii
ground state by the normalized gradient flow (``groundstate.scalar_ground_state``) and the
matrix-free scalar branch spectra of ``oracle.scalar`` (the single-mode lemma and the
nullspace theorem of Section 2.3), which never form the six-component operator.

  3d_n128_fm   the 3-D trap, 128^3 grid on [-8, 8]^3, V = (x^2 + y^2 + 4 z^2)/2,
               beta_n = 400, beta_s = -4 (M = 0.1 does not enter the scalar branches):
               the 64 lowest frequencies;
  3d_n64_fm    the same physics on the 64^3 grid: the 64 lowest frequencies;
  2d_n256_fm   the 2-D trap, 256^2 grid on [-12, 12]^2, V = (x^2 + y^2)/2, beta_n = 100,
  2d_n256_polar  beta_s = -2 and +2 (M = 0): the 32 lowest frequencies.

The 64^3 six-component subspace iteration of ``oracle.lrep`` (16 lowest, block 24) is
written by ``lrep64``.

Run from the repository root:  python tests/golden/make_branch_golden.py [name ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import bdg, groundstate as gs, lrep, scalar  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-10
# eigenvalues computed per branch: more than each branch contributes to the k lowest, so
# that the k-th merged value lies below every branch's largest computed one (checked)
COUNTS = {
    "3d_n128_fm": (W.C3, 128, 64, {"density": 12, "magnon": 34, "gapped": 34}),
    "3d_n64_fm": (W.C3, 64, 64, {"density": 12, "magnon": 34, "gapped": 34}),
    "2d_n256_fm": (W.C2_FM, 256, 32, {"density": 12, "magnon": 18, "gapped": 16}),
    "2d_n256_polar": (W.C2_POLAR, 256, 32, {"density": 12, "spin": 16}),
}


def _gauss(w):
    return np.exp(-0.5 * sum(c * c for c in W.coordinates(w)))


def branch_golden(name):
    w0, n, k, counts = COUNTS[name]
    w = W.scaled(w0, n) if n != w0.n[0] else w0
    V = W.potential(w)
    t = time.time()
    g = w.beta_n + w.beta_s if w.beta_s < 0 else w.beta_n
    phi, mu, gres, gits = gs.scalar_ground_state(V, g, w.n, w.L, phi0=_gauss(w), tol=1e-12)
    print(f"{name}: scalar ground state {gits} steps, residual {gres:.2e}, mu {mu!r}, {time.time() - t:.0f} s",
          flush=True)
    t = time.time()
    if w.beta_s < 0:
        bs = scalar.fm_branches(phi, mu, V, w.beta_n, w.beta_s, w.n, w.L, counts, tol=TOL, k_total=k)
    else:
        bs = scalar.polar_branches(phi, mu, V, w.beta_n, w.beta_s, w.n, w.L, counts, tol=TOL, k_total=k)
    br = {}
    for key, (vals, mult, res) in bs.branches.items():
        br[key] = {"multiplicity": mult, "omega": [float(v) for v in vals], "iters": int(res.iters),
                   "max_residual": float(np.max(res.residual)),
                   "count_in_k": int(mult * np.sum(np.asarray(vals) <= bs.omega[-1]))}
    print(f"{name}: branches {time.time() - t:.0f} s, "
          + ", ".join(f"{kk} {v['count_in_k']} ({v['iters']} its)" for kk, v in br.items()), flush=True)
    rec = {"workload": name, "grid": list(w.n), "L": list(w.L), "potential": w.potential, "beta_n": w.beta_n,
           "beta_s": w.beta_s, "k": k, "oracle": "oracle.scalar branch decomposition", "oracle_tol": TOL,
           "ground_state_residual": gres, "ground_state_iters": gits, "mu": mu,
           "complete_below": float(bs.complete_below), "omega": [float(v) for v in bs.omega], "branches": br}
    with open(os.path.join(HERE, f"{name}_branch_omega.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def lrep64():
    """Six-component oracle iteration on the 64^3 grid of the 3-D trap: 16 lowest, block 24."""
    w = W.scaled(W.C3, 64).with_(k=16, block=24)
    V = W.potential(w)
    t = time.time()
    r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L, W.initial_spinor(w), tol=1e-12,
                        max_iter=100000)
    coef = bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)
    out, prob, Nm, Qg = lrep.solve(coef, r.phi, w.n, w.L, w.k, W.start_block(w), 1e-9, max_iter=800, V=V, mu=r.mu,
                                   verbose=True)
    print(f"lrep64: ground state {r.iters} its, eigensolve {out.iters} its, max residual {out.residual.max():.1e}, "
          f"{time.time() - t:.0f} s", flush=True)
    rec = {"workload": "3d_n64_fm", "grid": list(w.n), "L": list(w.L), "potential": w.potential,
           "beta_n": w.beta_n, "beta_s": w.beta_s, "magnetization": w.magnetization, "k": w.k, "block": w.block,
           "oracle": "oracle.lrep six-component subspace iteration", "oracle_tol": 1e-9,
           "oracle_iters": int(out.iters), "oracle_max_residual": float(out.residual.max()),
           "mu": [float(v) for v in r.mu], "omega": [float(v) for v in out.omega]}
    with open(os.path.join(HERE, "3d_n64_fm_lrep_omega.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def main(names):
    for name in names or list(COUNTS) + ["lrep64"]:
        if name == "lrep64":
            lrep64()
        else:
            branch_golden(name)


if __name__ == "__main__":
    main(sys.argv[1:])
