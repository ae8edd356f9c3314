"""Writes the stored expected values of the full-size parity tests.

Every value comes from the CPU oracle (``oracle/``) alone: the normalized-gradient-flow
ground state, the deflation sets and the oracle's own block subspace iteration on the
2-D 256 x 256 trap (box [-12, 12]^2, V = (x^2 + y^2)/2, beta_n = 100, M = 0, k = 32, block 48,
seed-0 start block), for beta_s = -2 (ferromagnetic) and +2 (polar), to residual 1e-9.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import bdg, groundstate as gs, lrep  # noqa: E402


def c2_omega(w, tol=1e-9):
    V = W.potential(w)
    t = time.time()
    r = gs.ground_state(V, w.beta_n, w.beta_s, w.mass, w.magnetization, w.n, w.L, W.initial_spinor(w), tol=1e-12,
                        max_iter=100000)
    coef = bdg.coefficients(r.phi, r.mu, V, w.beta_n, w.beta_s)
    out, prob, Nm, Qg = lrep.solve(coef, r.phi, w.n, w.L, w.k, W.start_block(w), tol, max_iter=600, V=V, mu=r.mu,
                                   verbose=True)
    print(f"{w.name}: ground state {r.iters} its, eigensolve {out.iters} its, max residual {out.residual.max():.1e}, "
          f"{time.time() - t:.0f} s", flush=True)
    return {"workload": w.name, "grid": list(w.n), "L": list(w.L), "potential": w.potential, "beta_n": w.beta_n,
            "beta_s": w.beta_s, "magnetization": w.magnetization, "k": w.k, "block": w.block,
            "oracle_tol": tol, "oracle_iters": int(out.iters), "oracle_max_residual": float(out.residual.max()),
            "mu": [float(v) for v in r.mu], "omega": [float(v) for v in out.omega]}


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    for w in (W.C2_FM, W.C2_POLAR):
        rec = c2_omega(w)
        with open(os.path.join(here, f"{w.name}_omega.json"), "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
