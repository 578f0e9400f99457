"""Argument checks of the Python binding, which reject a tensor before any
library call (no GPU needed): wrong device, wrong length, wrong rank, wrong
dtype."""
import pytest

torch = pytest.importorskip("torch")

from paper_2205_04194_amd import _check_vec  # noqa: E402

DEV = torch.device("cuda:0")


def test_host_tensor_is_rejected():
    with pytest.raises(ValueError, match="device"):
        _check_vec(torch.zeros(10, dtype=torch.float64), "u", 10, DEV)


@pytest.mark.parametrize("shape", [(9,), (11,), (2, 9), (1, 2, 10), (0, 10)])
def test_wrong_shape_is_rejected(shape, monkeypatch):
    t = torch.zeros(shape, dtype=torch.float64)
    # a tensor that claims to be on the tree's device, so the shape check is reached
    monkeypatch.setattr(torch.Tensor, "is_cuda", property(lambda self: True))
    monkeypatch.setattr(torch.Tensor, "device", property(lambda self: DEV))
    with pytest.raises(ValueError, match="shape"):
        _check_vec(t, "u", 10, DEV)


def test_two_dimensional_tensor_rejected_where_one_column_is_required(monkeypatch):
    monkeypatch.setattr(torch.Tensor, "is_cuda", property(lambda self: True))
    monkeypatch.setattr(torch.Tensor, "device", property(lambda self: DEV))
    _check_vec(torch.zeros((3, 10)), "u", 10, DEV)                 # accepted where columns are allowed
    with pytest.raises(ValueError, match="shape"):
        _check_vec(torch.zeros((3, 10)), "u", 10, DEV, allow_2d=False)


@pytest.mark.parametrize("dtype", [torch.int64, torch.float16, torch.bfloat16, torch.complex128])
def test_wrong_dtype_is_rejected(dtype, monkeypatch):
    monkeypatch.setattr(torch.Tensor, "is_cuda", property(lambda self: True))
    monkeypatch.setattr(torch.Tensor, "device", property(lambda self: DEV))
    with pytest.raises(ValueError, match="float64 or float32"):
        _check_vec(torch.zeros(10, dtype=dtype), "u", 10, DEV)


def test_not_a_tensor_is_rejected():
    with pytest.raises(TypeError):
        _check_vec([0.0] * 10, "u", 10, DEV)
