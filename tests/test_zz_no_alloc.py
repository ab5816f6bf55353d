"""fdwt_dwt_inverse_noalloc (the no-allocation entry point) against
fdwt_dwt_inverse, through the C ABI: equal outputs bit for bit on two calls
in a row, the second on a smaller net (the shared scratch array keeps the
first call's contents), for complex-to-real and complex-to-complex inverses;
sizes beyond the fixed scratch array are refused before any work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_0808_0487_amd import fdwt, inputs
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


def call(name, net, it, x, ot, y):
    fn = getattr(fdwt.lib(), name)
    return fn(net.h, it, ctypes.c_void_p(x.data_ptr()), ot, ctypes.c_void_p(y.data_ptr()),
              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def coefficients(p, m, seed, dtype):
    g = np.random.default_rng(seed)
    N = p ** m
    return torch.from_numpy((g.standard_normal(N) + 1j * g.standard_normal(N)).astype(dtype)).cuda()


@pytest.mark.parametrize("sizes", [[(3, 13), (3, 9)], [(5, 9), (5, 6)], [(7, 8), (3, 10)], [(3, 14), (5, 2)]])
def test_noalloc_inverse_equals_inverse(sizes):
    for i, (p, m) in enumerate(sizes):
        announce("noalloc inverse", p, m, i)
        net = fdwt.Net(p, m, 1, inputs.upper_triangular_generators(p, m, 1, 7 + i))
        for cdt, it, rdt, rt in ((np.complex64, fdwt.CF32, torch.float32, fdwt.F32),
                                 (np.complex128, fdwt.CF64, torch.float64, fdwt.F64)):
            if p ** m * (8 if cdt == np.complex64 else 16) > (64 << 20):
                continue
            ct = coefficients(p, m, 100 * i + m, cdt)
            want = torch.empty(p ** m, dtype=rdt, device="cuda")
            got = torch.full_like(want, float("nan"))
            assert call("fdwt_dwt_inverse", net, it, ct, rt, want) == fdwt.OK
            assert call("fdwt_dwt_inverse_noalloc", net, it, ct, rt, got) == fdwt.OK
            torch.cuda.synchronize()
            assert torch.equal(got, want)
            wantc = torch.empty_like(ct)
            gotc = torch.empty_like(ct)
            assert call("fdwt_dwt_inverse", net, it, ct, it, wantc) == fdwt.OK
            assert call("fdwt_dwt_inverse_noalloc", net, it, ct, it, gotc) == fdwt.OK
            torch.cuda.synchronize()
            assert torch.equal(gotc, wantc)
        net.close()


def test_noalloc_inverse_p2_and_limits():
    announce("noalloc inverse p2 / limits")
    net = fdwt.Net(2, 20, 1, inputs.upper_triangular_generators(2, 20, 1, 3))
    x = torch.randn(2 ** 20, device="cuda")
    want, got = torch.empty_like(x), torch.empty_like(x)
    assert call("fdwt_dwt_inverse", net, fdwt.F32, x, fdwt.F32, want) == fdwt.OK
    assert call("fdwt_dwt_inverse_noalloc", net, fdwt.F32, x, fdwt.F32, got) == fdwt.OK
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    # p = 3, m = 16: 3^16 complex floats (344 MB) exceed the 64 MiB array
    big = fdwt.Net(3, 16, 1, inputs.upper_triangular_generators(3, 16, 1, 4))
    ct = torch.zeros(3 ** 16, dtype=torch.complex64, device="cuda")
    out = torch.zeros(3 ** 16, dtype=torch.float32, device="cuda")
    assert call("fdwt_dwt_inverse_noalloc", big, fdwt.CF32, ct, fdwt.F32, out) == fdwt.EBUDGET
    assert b"67108864" in fdwt.lib().fdwt_last_error()
    assert call("fdwt_dwt_inverse_noalloc", big, fdwt.F32, out, fdwt.F32, out) == fdwt.EINVAL
