"""The torch binding rejects mismatched shapes before any pointer reaches
the library (a wrongly shaped buffer would be read or written out of
bounds by the kernels).  CPU tensors suffice: the shape checks run before
the device checks, so no GPU is needed."""
import pytest
import torch

import paper_2004_08962_amd as hicu
from paper_2004_08962_amd.autograd import hicu_objective

KD = (1, 5, 5)


def _x(shape=(1, 20, 24, 4)):
    return torch.zeros(shape, dtype=torch.complex64)


def test_objective_grad_filter_rows():
    # n = 25 taps x 4 coils = 100 rows
    with pytest.raises(ValueError, match="taps"):
        hicu.objective_grad(_x(), None, torch.zeros((99, 8), dtype=torch.complex64), KD)
    with pytest.raises(ValueError, match="2-D"):
        hicu.objective_grad(_x(), None, torch.zeros(100, dtype=torch.complex64), KD)


def test_objective_grad_mask_shape():
    with pytest.raises(ValueError, match="mask"):
        hicu.objective_grad(_x(), torch.zeros((1, 20, 23), dtype=torch.uint8),
                            torch.zeros((100, 8), dtype=torch.complex64), KD)


def test_kspace_rank():
    with pytest.raises(ValueError, match="D0, D1, D2, Nc"):
        hicu.objective_grad(torch.zeros((20, 24, 4), dtype=torch.complex64), None,
                            torch.zeros((100, 8), dtype=torch.complex64), KD)
    with pytest.raises(ValueError, match="D0, D1, D2, Nc"):
        hicu.gram(torch.zeros((20, 24, 4), dtype=torch.complex64), KD)


def test_line_search_and_update_shapes():
    F = torch.zeros((100, 8), dtype=torch.complex64)
    with pytest.raises(ValueError, match="taps"):
        hicu.line_search(_x(), torch.zeros((), dtype=torch.float64), F[:50], KD)
    with pytest.raises(ValueError, match="does not match"):
        hicu.update(_x(), _x((1, 20, 23, 4)), torch.zeros((), dtype=torch.float64))
    with pytest.raises(ValueError, match="one value"):
        hicu.update(_x(), _x(), torch.zeros(2, dtype=torch.float64))


def test_nullspace_shapes():
    with pytest.raises(ValueError, match="square"):
        hicu.nullspace(torch.zeros((10, 9), dtype=torch.complex128), 3)
    with pytest.raises(ValueError, match="V0"):
        hicu.nullspace(torch.zeros((10, 10), dtype=torch.complex128), 3,
                       V0=torch.zeros((9, 9), dtype=torch.complex128))
    with pytest.raises(ValueError, match="rank"):
        hicu.nullspace(torch.zeros((10, 10), dtype=torch.complex128), 10)


def test_solve_shapes():
    with pytest.raises(ValueError, match="mask"):
        hicu.solve(_x(), torch.zeros((1, 20, 25), dtype=torch.uint8), KD, 30, [((0, 0, 0), (1, 20, 24), 1)])
    with pytest.raises(ValueError, match="out"):
        hicu.solve(_x(), None, KD, 30, [((0, 0, 0), (1, 20, 24), 1)], out=_x((1, 20, 24, 3)))


def test_autograd_checks_shapes():
    with pytest.raises(ValueError, match="taps"):
        hicu_objective(_x(), torch.zeros((64, 8), dtype=torch.complex64), KD)


def test_right_shapes_on_cpu_are_refused_as_non_device():
    # with consistent shapes the next check is the device: CPU tensors are refused
    with pytest.raises(TypeError, match="CUDA"):
        hicu.objective_grad(_x(), None, torch.zeros((100, 8), dtype=torch.complex64), KD)
