"""The stored full-size spectra of the two oracle formulations agree with each other.

tests/golden holds spectra written by two independent oracles (both scripts call only
oracle/): the six-component bi-orthogonal subspace iteration of ``oracle.lrep``
(make_golden.py, make_branch_golden.py lrep64) and the matrix-free scalar branch
decomposition of ``oracle.scalar`` (make_branch_golden.py), which solves real scalar problems
with their own ground state (the scalar Gross-Pitaevskii flow), deflation and eigensolvers.
Agreement pins both at sizes where no dense eigensolve is possible.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("six,branch", [("2d_n256_fm_omega.json", "2d_n256_fm_branch_omega.json"),
                                        ("2d_n256_polar_omega.json", "2d_n256_polar_branch_omega.json"),
                                        ("3d_n64_fm_lrep_omega.json", "3d_n64_fm_branch_omega.json")])
def test_six_component_and_branch_oracles_agree(six, branch):
    a, b = _load(six), _load(branch)
    assert a["grid"] == b["grid"] and a["beta_n"] == b["beta_n"] and a["beta_s"] == b["beta_s"]
    wa = np.array(a["omega"])
    wb = np.array(b["omega"])[:len(wa)]
    assert np.abs(wa / wb - 1.0).max() <= 1e-11
    # the chemical potentials of the two ground-state flows (three-component, scalar)
    assert np.allclose(a["mu"], b["mu"], rtol=1e-11)


def test_branch_golden_is_complete():
    """Every branch computed past the k-th merged value (none of the k lowest is missing)."""
    for name in sorted(os.listdir(GOLDEN)):
        if not name.endswith("_branch_omega.json"):
            continue
        g = _load(name)
        assert len(g["omega"]) == g["k"]
        assert g["omega"][-1] < g["complete_below"]
        # values <= omega_k, with multiplicity: k, or k + 1 when a doubly counted value of the
        # polar spin branch straddles the k-th place
        counted = sum(v["count_in_k"] for v in g["branches"].values())
        assert g["k"] <= counted <= g["k"] + 1, name


def test_3d_branch_spectra_converge_with_the_grid():
    """The 3-D trap's 64 branch frequencies on the 64^3 and 128^3 grids agree to 1e-8 relative
    (spectral accuracy of the Fourier discretization, Section 3.1: the smooth ground state is
    resolved at h = 1/4; stored values differ by 1.1e-9), and the Kohn modes at the trap
    frequencies 1 (x, y) and 2 (z) appear on the fine grid to 1e-9 (Section 2.3, analytical
    eigenpairs)."""
    a = np.array(_load("3d_n128_fm_branch_omega.json")["omega"])
    b = np.array(_load("3d_n64_fm_branch_omega.json")["omega"])
    assert np.abs(a / b - 1.0).max() <= 1e-8
    assert np.sum(np.abs(a - 1.0) <= 1e-9) >= 2
    assert np.sum(np.abs(a - 2.0) <= 2e-9) >= 1
