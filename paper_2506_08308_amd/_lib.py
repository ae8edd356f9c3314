"""ctypes declarations of the C ABI in include/bdg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbdg.so")

BDG_OK, BDG_EINVAL, BDG_ENOMEM, BDG_ENOCONV, BDG_EBREAKDOWN, BDG_EDEVICE, BDG_ESTATE = range(7)
STATUS_NAMES = {0: "BDG_OK", 1: "BDG_EINVAL", 2: "BDG_ENOMEM", 3: "BDG_ENOCONV", 4: "BDG_EBREAKDOWN",
                5: "BDG_EDEVICE", 6: "BDG_ESTATE"}
BDG_FP64, BDG_FP32_APPLY = 0, 1
BDG_FORM_UV, BDG_FORM_FG = 0, 1
BDG_NOALLOC_MAX_VEC = 64              # include/bdg.h

EXPORTS = ("bdg_create", "bdg_destroy", "bdg_last_error", "bdg_ground_state", "bdg_set_ground_state",
           "bdg_set_ground_state_complex", "bdg_apply", "bdg_biortho", "bdg_eigs", "bdg_eigs_grad",
           "bdg_perturbed_density", "bdg_stats", "bdg_biortho_noalloc",
           "bdg_mode_amplitudes",
           "bdg_test_gram", "bdg_test_update", "bdg_test_svd", "bdg_test_svd_real", "bdg_test_cholesky", "bdg_test_pchol",
           "bdg_test_plu", "bdg_test_gram_pair", "bdg_test_update_pair", "bdg_test_precond_mixed",
           "bdg_test_update_pair_fused")


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3),
                ("beta_n", ctypes.c_double), ("beta_s", ctypes.c_double), ("mass", ctypes.c_double),
                ("magnetization", ctypes.c_double), ("precision", ctypes.c_int)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libbdg.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2506_08308_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, d, i, st = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int
    pd, pi = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.bdg_create.argtypes = [ctypes.POINTER(Problem), vp, vp, ctypes.POINTER(vp)]
    lib.bdg_create.restype = st
    lib.bdg_destroy.argtypes = [vp]
    lib.bdg_destroy.restype = None
    lib.bdg_last_error.argtypes = [vp]
    lib.bdg_last_error.restype = ctypes.c_char_p
    lib.bdg_ground_state.argtypes = [vp, vp, d, i, vp, pd, pd, pi]
    lib.bdg_ground_state.restype = st
    lib.bdg_set_ground_state.argtypes = [vp, vp, pd]
    lib.bdg_set_ground_state.restype = st
    lib.bdg_apply.argtypes = [vp, i, i, i, vp, vp]
    lib.bdg_apply.restype = st
    lib.bdg_biortho.argtypes = [vp, i, vp, vp, pd, pi]
    lib.bdg_biortho.restype = st
    lib.bdg_biortho_noalloc.argtypes = [vp, i, vp, vp, vp, vp, pd, pi]
    lib.bdg_biortho_noalloc.restype = st
    lib.bdg_eigs.argtypes = [vp, i, i, d, i, vp, ctypes.c_ulonglong, pd, vp, pd, pi]
    lib.bdg_eigs.restype = st
    lib.bdg_eigs_grad.argtypes = [vp, i, pd, vp, vp, pd, pd]
    lib.bdg_eigs_grad.restype = st
    lib.bdg_set_ground_state_complex.argtypes = [vp, vp, pd]
    lib.bdg_set_ground_state_complex.restype = st
    lib.bdg_perturbed_density.argtypes = [vp, i, pd, vp, d, i, pd, vp]
    lib.bdg_perturbed_density.restype = st
    lib.bdg_mode_amplitudes.argtypes = [vp, i, vp, pd]
    lib.bdg_mode_amplitudes.restype = st
    lib.bdg_stats.argtypes = [vp, pd, i]
    lib.bdg_stats.restype = st
    ll = ctypes.c_longlong
    lib.bdg_test_gram.argtypes = [vp, ll, i, i, vp, ll, vp, ll, d, vp, i, i]
    lib.bdg_test_gram.restype = st
    lib.bdg_test_update.argtypes = [vp, ll, i, vp, ll, vp, i, i, d, vp, ll]
    lib.bdg_test_update.restype = st
    lib.bdg_test_gram_pair.argtypes = [vp, ll, i, i, vp, ll, vp, ll, d, vp, i, i]
    lib.bdg_test_gram_pair.restype = st
    lib.bdg_test_update_pair.argtypes = [vp, ll, i, vp, ll, vp, i, i, d, vp, ll]
    lib.bdg_test_precond_mixed.argtypes = [vp, i, vp, vp]
    lib.bdg_test_precond_mixed.restype = st
    lib.bdg_test_update_pair.restype = st
    lib.bdg_test_svd.argtypes = [vp, i, i, vp, i, vp, i, vp]
    lib.bdg_test_svd.restype = st
    lib.bdg_test_update_pair_fused.argtypes = [vp, ll, i, i, vp, ll, vp, i, i, vp, vp, ll]
    lib.bdg_test_update_pair_fused.restype = st
    lib.bdg_test_svd_real.argtypes = [vp, i, i, vp, i, vp, i, vp]
    lib.bdg_test_svd_real.restype = st
    lib.bdg_test_cholesky.argtypes = [vp, i, vp, i]
    lib.bdg_test_cholesky.restype = st
    lib.bdg_test_pchol.argtypes = [vp, i, vp, i, d, vp, pi]
    lib.bdg_test_pchol.restype = st
    lib.bdg_test_plu.argtypes = [vp, i, i, vp, i, d, vp, vp, pi]
    lib.bdg_test_plu.restype = st
    _lib = lib
    return lib
