"""Net generation and sampling on the GPU against the oracle (bit-exact
digits; float points and samples)."""
import numpy as np
import pytest
import torch

from oracle import families, net as onet, walsh
from paper_0808_0487_amd import fdwt, inputs
from tests.gpu_common import announce, correctly_rounded_points, nrel, sample_indices

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p,m,s,seed", [(2, 1, 1, 1), (2, 7, 3, 2), (2, 10, 4, 1), (2, 13, 8, 3),
                                        (2, 17, 5, 4), (2, 12, 64, 11), (3, 1, 2, 5), (3, 6, 4, 6),
                                        (3, 9, 3, 7), (3, 5, 64, 12), (5, 1, 1, 8), (5, 4, 3, 9),
                                        (5, 7, 2, 10), (7, 1, 2, 15), (7, 4, 3, 16), (7, 8, 5, 17),
                                        (7, 5, 64, 18)])
def test_net_digits_bit_exact(p, m, s, seed):
    announce("net_digits", p, m, s, seed)
    C = inputs.upper_triangular_generators(p, m, s, seed)
    net = fdwt.Net(p, m, s, C)
    X = net.digits().cpu().numpy().astype(np.int64)
    assert np.array_equal(X, onet.net_int(p, m, C))
    x = net.points().cpu().numpy()
    assert np.array_equal(x, correctly_rounded_points(p, m, onet.net_points(p, m, C)))


@pytest.mark.parametrize("p,m,s,seed", [(2, 6, 3, 21), (3, 4, 3, 22)])
def test_singular_generators_bit_exact(p, m, s, seed):
    announce("net_digits singular", p, m, s, seed)
    C = inputs.random_generators(p, m, s, seed)
    net = fdwt.Net(p, m, s, C)
    assert np.array_equal(net.digits().cpu().numpy().astype(np.int64), onet.net_int(p, m, C))


@pytest.mark.parametrize("p,m,s,seed", [(2, 24, 20, 2), (3, 14, 10, 3), (5, 11, 8, 4), (2, 26, 3, 5),
                                        (3, 16, 3, 6)])
def test_net_digits_full_size_sampled(p, m, s, seed):
    """Full-size nets: sampled digits bit-exact and sampled points
    correctly rounded (p = 3, m = 16 and p = 2, m = 26 have X > 2^24); every
    coordinate a permutation of 0..p^m-1 (non-singular generators)."""
    announce("net_digits full", p, m, s, seed)
    C = inputs.upper_triangular_generators(p, m, s, seed)
    net = fdwt.Net(p, m, s, C)
    Xd = net.digits()
    idx = sample_indices(p ** m, 20000, seed)
    it = torch.from_numpy(idx).cuda()
    got = Xd[:, it].cpu().numpy().astype(np.int64)
    Xo = onet.net_int(p, m, C, idx)
    assert np.array_equal(got, Xo)
    x = net.points()[:, it].cpu().numpy()
    assert np.array_equal(x, correctly_rounded_points(p, m, Xo.astype(np.float64) / float(p ** m)))
    ar = torch.arange(p ** m, dtype=torch.int32, device="cuda")
    for j in range(s):
        assert torch.equal(torch.sort(Xd[j])[0], ar)


@pytest.mark.parametrize("kind,p,m,s,seed", [("product", 2, 10, 4, 1), ("exp", 2, 12, 20, 2),
                                             ("product", 2, 9, 64, 7),
                                             ("wangfang", 2, 12, 10, 3), ("product", 3, 8, 10, 4),
                                             ("exp", 5, 6, 5, 5), ("wangfang", 3, 7, 6, 6)])
def test_sample_families(kind, p, m, s, seed):
    announce("sample", kind, p, m, s, seed)
    C = inputs.upper_triangular_generators(p, m, s, seed)
    a = {"product": inputs.family_params("product", s, seed=seed),
         "exp": inputs.family_params("exp", s),
         "wangfang": inputs.family_params("wangfang", s, a="k")}[kind]
    net = fdwt.Net(p, m, s, C)
    f = net.sample(kind, a).cpu().numpy().astype(np.float64)
    fo = families.evaluate(kind, onet.net_points(p, m, C), a)
    assert nrel(f, fo) <= 1e-6
    assert np.max(np.abs(f - fo) / np.maximum(np.abs(fo), 1e-30)) <= 1e-5


def test_sample_full_size_exp_family_sampled():
    """The C2 workload's sampler (p = 2, m = 24, s = 20, w_j = 0.1^j) at
    sampled points."""
    p, m, s = 2, 24, 20
    announce("sample full", p, m, s)
    C = inputs.upper_triangular_generators(p, m, s, 2)
    a = inputs.family_params("exp", s, ratio=0.1)
    net = fdwt.Net(p, m, s, C)
    f = net.sample("exp", a)
    idx = sample_indices(p ** m, 50000, 7)
    got = f[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    fo = families.exponential(onet.net_points(p, m, C, idx), a)
    assert np.max(np.abs(got - fo) / np.abs(fo)) <= 1e-6


# p = 2 with m >= 10 samples inside the first pass (first-pass tiles of 2^10
# .. 2^14 elements; m <= 14 is a single pass); m < 10 and odd p sample into
# memory first.
@pytest.mark.parametrize("p,m,s,family", [(2, 12, 5, "exp"), (2, 18, 8, "product"), (3, 8, 4, "wangfang"),
                                          (5, 6, 3, "product"), (2, 9, 4, "exp"), (2, 10, 3, "product"),
                                          (2, 11, 7, "wangfang"), (2, 13, 64, "exp"), (2, 14, 2, "product"),
                                          (2, 15, 6, "wangfang"), (2, 16, 33, "product"), (2, 21, 4, "asian"),
                                          (2, 14, 9, "asian"), (2, 22, 12, "exp"), (2, 26, 3, "product")])
def test_forward_of_sampled_family_equals_two_calls(p, m, s, family):
    """fdwt_dwt_forward_family equals fdwt_sample then fdwt_dwt_forward bit
    for bit, and the oracle's transform of the oracle's samples to 1e-5."""
    announce("forward family", p, m, s, family)
    C = inputs.upper_triangular_generators(p, m, s, 21)
    if family == "asian":
        a = np.array([100.0, 100.0, 0.2, 0.1, 1.0])
    elif family == "wangfang":
        a = inputs.family_params(family, s, a="k")
    else:
        a = inputs.family_params(family, s, seed=4)
    net = fdwt.Net(p, m, s, C)
    fused = net.forward_family(family, a).cpu().numpy()
    two = net.forward(net.sample(family, a)).cpu().numpy()
    assert np.array_equal(fused, two)
    hs = sample_indices(p ** m, 200, m)
    if p ** m <= 1 << 22:
        fo = families.evaluate(family, onet.net_points(p, m, C), a)
        ref = walsh.dwt_phase(p, m, fo, hs)
        assert nrel(fused[hs], ref.real if p == 2 else ref) <= 1e-5


@pytest.mark.parametrize("p,m,s", [(2, 14, 8), (2, 10, 32), (3, 8, 5), (5, 5, 3), (7, 4, 6)])
def test_asian_payoff_against_oracle(p, m, s):
    """Section 5.3 payoff sampled on the device (double, inverse normal by
    A&S 26.2.23 + Newton) against the oracle (scipy ndtri) at every point."""
    announce("asian", p, m, s)
    C = inputs.upper_triangular_generators(p, m, s, 31)
    prm = np.array([100.0, 100.0, 0.2, 0.1, 1.0])
    net = fdwt.Net(p, m, s, C)
    got = net.sample("asian", prm).cpu().numpy().astype(np.float64)
    ref = families.asian(onet.net_points(p, m, C), *prm)
    assert nrel(got, ref) <= 2e-7
    assert got[0] == 0.0  # the point 0 collapses the path
