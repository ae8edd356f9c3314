"""The Python binding rejects buffers of the wrong shape, dtype or row count before any
pointer reaches the library (a short buffer would otherwise be read or written past its
end on the device).  CPU only: the context is built without the library."""
import pytest
import torch

from paper_2506_08308_amd import api


def _ctx(grid=(4, 8), precision=api.Precision.FP64):
    c = object.__new__(api.BdgContext)
    c._h = None
    c.dim = len(grid)
    c.grid_shape = tuple(grid)
    c.n = tuple(reversed(grid))
    c.npts = 1
    for v in grid:
        c.npts *= v
    c.precision = precision
    c.device = torch.device("cpu")
    return c


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"{name} reached the library")


def test_apply_rejects_wrong_dtype_shape_and_out():
    c = _ctx()
    c._lib = _NoLib()
    ok = torch.zeros((2, 6, 4, 8), dtype=torch.complex128)
    with pytest.raises(ValueError, match="complex128"):
        c.apply(ok.to(torch.complex64))
    with pytest.raises(ValueError, match="shape"):
        c.apply(torch.zeros((2, 6, 4, 4), dtype=torch.complex128))
    with pytest.raises(ValueError, match="shape"):
        c.apply(torch.zeros((2, 3, 4, 8), dtype=torch.complex128))
    with pytest.raises(ValueError, match="shape"):
        c.apply(torch.zeros((2, 2, 6, 4, 8), dtype=torch.complex128))
    with pytest.raises(ValueError, match="out"):
        c.apply(ok, out=torch.zeros((1, 6, 4, 8), dtype=torch.complex128))
    with pytest.raises(ValueError, match="out"):
        c.apply(ok, out=torch.zeros((2, 6, 4, 8), dtype=torch.complex64))
    c32 = _ctx(precision=api.Precision.FP32_APPLY)
    c32._lib = _NoLib()
    with pytest.raises(ValueError, match="complex64"):
        c32.apply(ok)


def test_eigs_rejects_start_block_of_wrong_shape():
    c = _ctx()
    c._lib = _NoLib()
    with pytest.raises(ValueError, match="X0"):
        c.eigs(2, 4, X0=torch.zeros((3, 6, 4, 8), dtype=torch.complex128), want_vectors=False)
    with pytest.raises(ValueError, match="X0"):
        c.eigs(2, 4, X0=torch.zeros((4, 6, 8, 4), dtype=torch.complex128), want_vectors=False)


def test_grad_density_biortho_reject_short_or_mistyped_vectors():
    c = _ctx()
    c._lib = _NoLib()
    uv = torch.zeros((1, 6, 4, 8), dtype=torch.complex128)
    with pytest.raises(ValueError, match="rows"):
        c.eigs_grad([0.5, 0.7], uv)
    with pytest.raises(ValueError, match="uv"):
        c.eigs_grad([0.5], torch.zeros((1, 3, 4, 8), dtype=torch.complex128))
    with pytest.raises(ValueError, match="rows"):
        c.perturbed_density([0.5, 0.7], uv, 0.1, [0.0])
    with pytest.raises(ValueError, match="uv"):
        c.perturbed_density([0.5], torch.zeros((1, 6, 4, 4), dtype=torch.complex128), 0.1, [0.0])
    F = torch.zeros((2, 3, 4, 8), dtype=torch.complex128)
    with pytest.raises(ValueError, match="G"):
        c.biortho(F, torch.zeros((1, 3, 4, 8), dtype=torch.complex128))
    with pytest.raises(ValueError, match="F"):
        c.biortho(F.to(torch.complex64), F)


def test_ground_state_inputs_need_three_grid_fields():
    c = _ctx()
    c._lib = _NoLib()
    with pytest.raises(ValueError, match="phi"):
        c.set_ground_state(torch.zeros((2, 4, 8), dtype=torch.float64), [1.0, 1.0, 1.0])
    with pytest.raises(ValueError, match="phi0"):
        c.ground_state(phi0=torch.zeros((3, 8, 4), dtype=torch.float64))
    with pytest.raises(ValueError, match="phi"):
        c.set_ground_state_complex(torch.zeros((3, 4, 4), dtype=torch.complex128), [1.0, 1.0, 1.0])
