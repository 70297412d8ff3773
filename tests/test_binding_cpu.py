"""Host-side argument checks of the Python binding (no GPU): the C ABI takes plain
pointers, so the binding must refuse buffers of the wrong size or type before a
call could read or write past their ends."""

import numpy as np
import pytest
import torch

from paper_1812_05264_amd import _rfo


def test_sizes_are_checked():
    _rfo._need(np.zeros(6), 6, "x")
    _rfo._need(None, 6, "x")
    _rfo._need(np.zeros(5), 0, "x")            # no Hamiltonian yet: the library decides
    with pytest.raises(ValueError, match="must hold 6 values"):
        _rfo._need(np.zeros(5), 6, "x")
    with pytest.raises(ValueError):
        _rfo._need(torch.zeros(2, 4), 6, "x")


def test_output_buffers_must_be_float64_of_the_right_size():
    assert _rfo._out_f64(None, 81, "out") is None
    a = np.zeros((1, 9, 9))
    assert _rfo._out_f64(a, 81, "out") is a
    t = torch.zeros(81, dtype=torch.float64)
    assert _rfo._out_f64(t, 81, "out") is t
    with pytest.raises(TypeError):
        _rfo._out_f64(np.zeros(81, dtype=np.float32), 81, "out")
    with pytest.raises(TypeError):
        _rfo._out_f64(torch.zeros(81, dtype=torch.float32), 81, "out")
    with pytest.raises(ValueError):
        _rfo._out_f64(np.zeros(80), 81, "out")


def test_input_blocks_become_contiguous_float64():
    a = _rfo._in_f64(np.arange(12, dtype=np.int32).reshape(3, 4).T, 12, "in")
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    assert np.array_equal(a, np.arange(12).reshape(3, 4).T)
    t = _rfo._in_f64(torch.arange(12, dtype=torch.float64).reshape(3, 4).t(), 12, "in")
    assert t.is_contiguous()
    with pytest.raises(TypeError):
        _rfo._in_f64(torch.zeros(12, dtype=torch.float32), 12, "in")
    with pytest.raises(ValueError):
        _rfo._in_f64(np.zeros(11), 12, "in")
