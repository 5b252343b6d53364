"""The binding's argument marshalling (host logic, no device calls): what a
tensor becomes at the C boundary, and the errors raised before any call."""
import pytest
import torch

import paper_1705_08743_amd as sr


def test_mat_rejects_non_matrices():
    with pytest.raises(ValueError, match="2-D"):
        sr._mat(torch.zeros(8, dtype=torch.uint16), "A")
    with pytest.raises(ValueError, match="2-D"):
        sr._mat(torch.zeros(2, 2, 2, dtype=torch.uint16), "A")


def test_mat_rejects_strided_columns_and_host_tensors():
    t = torch.zeros(8, 16, dtype=torch.uint16)
    with pytest.raises(ValueError, match="unit column stride"):
        sr._mat(t[:, ::2], "A")
    with pytest.raises(ValueError, match="device tensor"):
        sr._mat(t, "B")


def test_mat_empty_and_none():
    assert sr._mat(None, "C") == (None, 0, 0, 0)
    # an empty matrix needs no pointer and is not checked for its device
    p, ld, r, c = sr._mat(torch.zeros(0, 16, dtype=torch.uint16), "A")
    assert (p, r, c) == (None, 0, 16)
    p, ld, r, c = sr._mat(torch.zeros(4, 0, dtype=torch.uint16), "A")
    assert (p, r, c) == (None, 4, 0)


class FakeDeviceTensor:
    """What _mat reads of a device tensor: shape, strides, device, pointer."""

    def __init__(self, shape, stride, ptr=4096):
        self.shape, self._stride, self.is_cuda, self._ptr = tuple(shape), tuple(stride), True, ptr

    def stride(self):
        return self._stride

    def data_ptr(self):
        return self._ptr


def test_mat_row_stride():
    # a view of the first 10 columns of 64-column rows keeps the row stride
    assert sr._mat(FakeDeviceTensor((5, 10), (64, 1)), "A") == (4096, 64, 5, 10)
    # a single row reports at least its width as the stride
    assert sr._mat(FakeDeviceTensor((1, 10), (10, 1)), "A") == (4096, 10, 1, 10)
    assert sr._mat(FakeDeviceTensor((1, 10), (1, 1)), "A") == (4096, 10, 1, 10)
    with pytest.raises(ValueError, match="unit column stride"):
        sr._mat(FakeDeviceTensor((5, 10), (64, 2)), "A")


def test_stream_handles_pass_through():
    assert sr._stream(0) == 0
    assert sr._stream(12345) == 12345

    class S:
        cuda_stream = 777
    assert sr._stream(S()) == 777
