"""CPU checks of the Python binding's argument validation (no GPU, no kernel).

The C ABI receives only pointers, so the binding checks every tensor's shape
against the plan before anything reaches the library: a short dh, a strided or
smaller `out`, or a batch item whose tensors differ from the plan's items would
otherwise mean out-of-bounds device reads or writes.  These checks run before
the device check, so they are exercised here with CPU tensors.
"""
import pytest
import torch

import paper_2608_14497_amd as hd


def t(*shape, dtype=torch.float32):
    return torch.zeros(shape, dtype=dtype)


def test_forward_batch_axes_and_kernel_extents():
    with pytest.raises(ValueError, match="batch axes"):
        hd.conv_forward(t(3, 16), t(2, 16), ndim=1)
    with pytest.raises(ValueError, match="batch axes"):
        hd.conv_forward(t(16, 16), t(16), ndim=1)
    with pytest.raises(ValueError, match="extents"):
        hd.conv_forward(t(16), t(17))


def test_backward_checks_dh_and_g():
    with pytest.raises(ValueError, match="dh"):
        hd.conv_backward(t(16), t(16), t(15))
    with pytest.raises(ValueError, match="dh"):
        hd.conv_backward(t(2, 16), t(2, 16), t(16), ndim=1)
    with pytest.raises(ValueError, match="batch axes"):
        hd.conv_backward(t(2, 16), t(3, 16), t(2, 16), ndim=1)


def test_batch_backward_list_lengths_and_shapes():
    with pytest.raises(ValueError, match="equal"):
        hd.conv_batch_backward([t(8), t(9)], [t(8), t(9)], [t(8)])
    with pytest.raises(ValueError, match="equal"):
        hd.conv_batch_backward([t(8)], [t(8), t(9)], [t(8)])
    with pytest.raises(ValueError, match=r"dh\[1\]"):
        hd.conv_batch_backward([t(8), t(9)], [t(8), t(9)], [t(8), t(8)])
    with pytest.raises(ValueError, match="extents"):
        hd.conv_batch_backward([t(8)], [t(9)], [t(8)])


class _FakePlan:
    def __init__(self, items):
        self.items = items


def test_batch_tensors_must_match_the_plan_items():
    plan = _FakePlan([{"shape": (8,)}, {"shape": (4, 5), "kernel_shape": (2, 5)}])
    hd._check_batch_items(plan, [t(8), t(4, 5)], [t(8), t(2, 5)])
    with pytest.raises(ValueError, match="items"):
        hd._check_batch_items(plan, [t(8)], [t(8)])
    with pytest.raises(ValueError, match=r"f\[1\]"):
        hd._check_batch_items(plan, [t(8), t(4, 6)], [t(8), t(2, 5)])
    with pytest.raises(ValueError, match=r"g\[1\]"):
        hd._check_batch_items(plan, [t(8), t(4, 5)], [t(8), t(4, 5)])
    with pytest.raises(ValueError, match=r"f\[0\]"):
        hd.conv_batch([t(9), t(4, 5)], [t(9), t(2, 5)], plan)


def test_output_tensor_checks():
    like = t(4, 16)
    hd._check_out(t(4, 16), like)
    with pytest.raises(ValueError, match="shape"):
        hd._check_out(t(4, 15), like)
    with pytest.raises(ValueError, match="float32"):
        hd._check_out(t(4, 16, dtype=torch.float64), like)
    with pytest.raises(ValueError, match="contiguous"):
        hd._check_out(t(16, 4).t(), like)
    with pytest.raises(ValueError, match="out needs"):
        hd.conv_batch([t(8)], [t(8)], out=[t(8), t(8)])
