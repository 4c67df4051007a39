"""Host-side argument checks of the binding (no GPU needed): buffers the
kernels write or read are refused before any device call when they cannot
hold what the call needs."""
import numpy as np
import pytest
import torch

from paper_2601_19901_amd import lfdpr


def _bare(cls, **attrs):
    obj = object.__new__(cls)
    obj.h = None
    obj._torch = torch
    for k, v in attrs.items():
        setattr(obj, k, v)
    return obj


def test_backward_needs_a_forward_first():
    net = _bare(lfdpr.Net, _last_shape=None, loss_buf=None)
    with pytest.raises(ValueError, match="forward first"):
        net.backward(torch.zeros((1, 2, 2, 4), dtype=torch.int16))


def test_backward_refuses_a_host_target():
    net = _bare(lfdpr.Net, _last_shape=(48, 8, 8), loss_buf=None)
    with pytest.raises(ValueError, match="target must be a device tensor"):
        net.backward(torch.zeros((48, 8, 8, 4), dtype=torch.int16))


def test_check_dev_refuses_host_tensors_and_arrays():
    for bad in (np.zeros(16, np.uint8), torch.zeros(16, dtype=torch.uint8)):
        with pytest.raises(ValueError, match="device tensor"):
            lfdpr._check_dev(bad, torch.uint8, 16, "panels")


def test_batch_panels_need_a_lens(monkeypatch):
    R = _bare(lfdpr.Renderer, lens=None, device=0)
    b = _bare(lfdpr.Batch, R=R, n=2, shape=(2, 4, 8, 8))
    monkeypatch.setattr(lfdpr, "_check_dev", lambda *a, **k: None)
    with pytest.raises(ValueError, match="need a lens"):
        b.render(np.zeros((2, 12), np.float32), object(), panels=object())
