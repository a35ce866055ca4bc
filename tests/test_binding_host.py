"""Host-side checks of the Python binding's argument marshalling: caller
outputs of the wrong dtype, shape, layout or device are refused before any
launch, and overlapping or transposed input views are copied to a plain
row-major layout first (no GPU needed: the checks run on CPU tensors)."""
import pytest
import torch

import paper_2603_20889_amd as q

CPU = torch.device("cpu")


def test_out_accepts_plain_and_padded_matrices():
    R = torch.empty((5, 5), dtype=torch.float64)
    assert q._out(R, 5, 5, CPU, "R") is R
    wide = torch.empty((5, 9), dtype=torch.float64)[:, :5]   # ldr = 9 >= n
    assert q._out(wide, 5, 5, CPU, "R") is wide


@pytest.mark.parametrize("make,exc", [
    (lambda: torch.empty((5, 5), dtype=torch.float32), TypeError),
    (lambda: torch.empty((4, 5), dtype=torch.float64), ValueError),
    (lambda: torch.empty((5, 4), dtype=torch.float64), ValueError),
    (lambda: torch.empty(25, dtype=torch.float64), ValueError),
    (lambda: torch.empty((5, 5), dtype=torch.float64).t(), ValueError),              # column-major view
    (lambda: torch.empty((1, 5), dtype=torch.float64).expand(5, 5), ValueError),     # overlapping rows
    (lambda: "not a tensor", TypeError),
])
def test_out_rejects_bad_matrices(make, exc):
    with pytest.raises(exc):
        q._out(make(), 5, 5, CPU, "R")


def test_out_vectors():
    assert q._out(torch.empty(3, dtype=torch.int32), 0, 1, CPU, "info", torch.int32) is not None
    with pytest.raises(TypeError):
        q._out(torch.empty(3, dtype=torch.int64), 0, 1, CPU, "info", torch.int32)
    with pytest.raises(ValueError):
        q._out(torch.empty(3, dtype=torch.float64), 0, 4, CPU, "x")
    with pytest.raises(ValueError):
        q._out(torch.empty(8, dtype=torch.float64)[::2], 0, 4, CPU, "x")   # strided vector


def test_out_rejects_another_device():
    with pytest.raises(ValueError):
        q._out(torch.empty((3, 3), dtype=torch.float64), 3, 3, torch.device("cuda:0"), "R")


def test_inputs_must_be_gpu_float64_matrices():
    with pytest.raises(TypeError):
        q._matrix(torch.zeros((10, 3), dtype=torch.float64))            # on the CPU
    with pytest.raises(TypeError):
        q._matrix(torch.zeros(10, dtype=torch.float64))
    with pytest.raises(TypeError):
        q._matrix(torch.zeros((10, 3), dtype=torch.float32))
