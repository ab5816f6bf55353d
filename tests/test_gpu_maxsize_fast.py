"""Every output at the largest net of each prime (p^m <= 2^26), against the
fast CPU reference (oracle/fast, float64; pinned to the oracle's definitions
in tests/test_oracle_fast.py): p = 2, m = 26 (three passes; float and int32),
p = 3, m = 16, p = 5, m = 11, p = 7, m = 9 (complex float, forward of real
data and inverse of arbitrary complex data), and the float64 reference path
at p = 3, m = 16.  Tolerances as elsewhere: normwise and max-abs 1e-5 for
float32 data, 1e-12 for float64, exact for int32 (mod 2^32)."""
import numpy as np
import pytest
import torch

from oracle import fast
from paper_0808_0487_amd import fdwt, inputs
from tests.gpu_common import announce, nrel

pytestmark = pytest.mark.gpu


def close(got, ref, tol=1e-5):
    assert nrel(got, ref) <= tol, nrel(got, ref)
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.timeout(600)
def test_p2_m26_every_output():
    p, m = 2, 26
    N = p ** m
    announce("max size vs fast reference", p, m)
    net = fdwt.Net(p, m, 2, inputs.upper_triangular_generators(p, m, 2, 6))
    f = inputs.uniform_float(N, 126)
    ft = net.forward(torch.from_numpy(f).cuda())
    close(ft.cpu().numpy().astype(np.float64), fast.fwt(p, m, f.astype(np.float64)))
    back = net.inverse(ft).cpu().numpy().astype(np.float64)
    close(back, f.astype(np.float64))
    del ft
    fi = inputs.uniform_int32(N, -1000, 1000, 127)
    gi = net.forward(torch.from_numpy(fi).cuda()).cpu().numpy()
    exact = np.rint(fast.fwt(p, m, fi.astype(np.float64)) * N).astype(np.int64)
    assert np.array_equal(gi, (exact & 0xFFFFFFFF).astype(np.uint32).view(np.int32))
    net.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("p,m", [(3, 16), (5, 11), (7, 9)])
def test_odd_p_largest_net_every_output(p, m):
    N = p ** m
    announce("max size vs fast reference", p, m)
    net = fdwt.Net(p, m, 3, inputs.upper_triangular_generators(p, m, 3, 7))
    f = inputs.uniform_float(N, 200 + p)
    ft = net.forward(torch.from_numpy(f).cuda())
    close(ft.cpu().numpy().astype(np.complex128), fast.fwt(p, m, f.astype(np.float64)))
    del ft
    g = np.random.default_rng(300 + p)
    ct = (g.standard_normal(N) + 1j * g.standard_normal(N)).astype(np.complex64)
    back = net.inverse(torch.from_numpy(ct).cuda()).cpu().numpy().astype(np.complex128)
    close(back, fast.fwt(p, m, ct.astype(np.complex128), inverse=True))
    net.close()


@pytest.mark.timeout(600)
def test_double_precision_path_at_the_largest_p3_net():
    p, m = 3, 16
    N = p ** m
    announce("max size f64 vs fast reference", p, m)
    net = fdwt.Net(p, m, 1, inputs.identity_generators(p, m, 1))
    f = inputs.uniform_float(N, 316, dtype=np.float64)
    ft = net.forward(torch.from_numpy(f).cuda())
    close(ft.cpu().numpy(), fast.fwt(p, m, f), 1e-12)
    back = net.inverse(ft, real=True).cpu().numpy()
    close(back, f, 1e-12)
    net.close()
