"""Argument checks of the binding that need no GPU: host tensors and
non-tensors are refused before any pointer is taken."""
import numpy as np
import pytest
import torch

from paper_2104_13755_amd.solver import _dev_f64


def test_dev_tensor_check_refuses_host_and_non_tensors():
    with pytest.raises(TypeError):
        _dev_f64(np.zeros(4))
    with pytest.raises(TypeError):
        _dev_f64(torch.zeros(4, dtype=torch.float64))          # host memory
    with pytest.raises(TypeError):
        _dev_f64([0.0, 1.0])
