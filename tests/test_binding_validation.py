"""The binding refuses tensors the kernels would read or write out of
bounds (wrong size, element type, layout or device) before any pointer
crosses the ABI (runs without a GPU: a net object is set up by hand, no
library call is made)."""
import numpy as np
import pytest
import torch

from paper_0808_0487_amd import fdwt


def fake_net(p=2, m=4, s=3):
    net = fdwt.Net.__new__(fdwt.Net)
    net.h, net.p, net.m, net.s, net.N, net.device = None, p, m, s, p ** m, 0
    return net


def test_transform_buffers_checked():
    net = fake_net()
    with pytest.raises(ValueError, match="16 elements"):
        net.forward(torch.zeros(15))
    with pytest.raises(ValueError, match="must be"):
        net.forward(torch.zeros(16, dtype=torch.int64))
    with pytest.raises(ValueError, match="out must be"):
        net.forward(torch.zeros(16), out=torch.zeros(16, dtype=torch.int32))
    with pytest.raises(ValueError, match="device tensor"):
        net.forward(torch.zeros(16), out=torch.zeros(16))  # all checks passed: host memory refused last
    with pytest.raises(ValueError, match="16 elements"):
        net.inverse(torch.zeros(16), out=torch.zeros(32))
    odd = fake_net(3, 3, 2)
    with pytest.raises(ValueError, match="must be"):
        odd.inverse(torch.zeros(27))  # odd p takes complex coefficients
    with pytest.raises(ValueError, match="out must be"):
        odd.forward(torch.zeros(27), out=torch.zeros(27))  # complex output expected


def test_spline_and_effdim_buffers_checked():
    net = fake_net()
    kern = fdwt.Kernel(2.0, np.ones(3))
    with pytest.raises(ValueError, match="16 elements"):
        net.spline_coef(kern, torch.zeros(8), out=torch.zeros(16))
    with pytest.raises(ValueError, match="16 elements"):
        net.eff_dim(kern, torch.zeros(17))
    with pytest.raises(ValueError, match="shape"):
        net.spline_eval(kern, torch.zeros(16), torch.zeros((2, 5), dtype=torch.int32))
    with pytest.raises(ValueError, match="queries must be"):
        net.spline_eval(kern, torch.zeros(16), torch.zeros((3, 5)))
    with pytest.raises(ValueError, match="5 elements"):
        net.spline_eval(kern, torch.zeros(16), torch.zeros((3, 5), dtype=torch.int32), out=torch.zeros(4))
    with pytest.raises(ValueError, match="contiguous"):
        net.walsh_interp(kern, torch.zeros(32)[::2])
    with pytest.raises(ValueError, match="sf_out"):
        net.walsh_interp(kern, torch.zeros(16), torch.zeros((3, 5), dtype=torch.int32),
                         c_out=torch.zeros(16), sf_out=torch.zeros(6))


def test_sampling_and_net_buffers_checked():
    net = fake_net()
    with pytest.raises(ValueError, match="3 values"):
        net.sample("product", np.ones(2), out=torch.zeros(16))
    with pytest.raises(ValueError, match="5 values"):
        net.sample("asian", np.ones(3), out=torch.zeros(16))
    with pytest.raises(ValueError, match="48 elements"):
        net.digits(out=torch.zeros((3, 15), dtype=torch.int32))
    with pytest.raises(ValueError, match="must be float32"):
        net.points(out=torch.zeros((3, 16), dtype=torch.float64))
    with pytest.raises(ValueError, match="16 elements"):
        net.split_cost(torch.zeros(8), 2.0, 1.0, -2.0)
