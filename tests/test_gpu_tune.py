"""Kernel-parameter selection of Section 5.1 on the GPU against the oracle:
Sf on the second half and the cost at given parameters, the exact case of a
kernel section, and the Nelder-Mead result."""
import itertools

import numpy as np
import pytest
import torch

from oracle import families, kernel, net as onet, tuning
from paper_0808_0487_amd import fdwt, inputs
from tests.gpu_common import announce, nrel

pytestmark = pytest.mark.gpu


def setup(m2, s, seed, a="k"):
    C2 = inputs.upper_triangular_generators(2, m2, s, seed)
    x = onet.net_points(2, m2, C2)
    f2 = families.wangfang(x, inputs.family_params("wangfang", s, a=a))
    net = fdwt.Net(2, m2, s, C2)
    return C2, f2, net, torch.from_numpy(f2.astype(np.float32)).cuda()


@pytest.mark.parametrize("m2,s,seed,prm", [(6, 2, 1, (2.0, 1.0, -2.0)), (9, 4, 2, (1.6, 0.5, -1.0)),
                                           (12, 8, 3, (3.0, 2.0, -2.5)), (11, 5, 4, (2.2, 0.3, 0.0)),
                                           (10, 20, 6, (2.0, 1.0, -2.0)), (10, 40, 7, (1.8, 0.8, -1.5)),
                                           (10, 40, 8, (2.5, 1.5, -3.0))])
def test_second_half_and_cost_against_oracle(m2, s, seed, prm):
    announce("split cost", m2, s, seed, prm)
    C2, f2, net, fd = setup(m2, s, seed)
    cost, sf = net.split_cost(fd, *prm, want_sf=True)
    ref_sf = tuning.split_sf(m2, C2, f2.astype(np.float32).astype(np.float64), *prm)
    assert nrel(sf.cpu().numpy(), ref_sf) <= 1e-5
    N = 2 ** (m2 - 1)
    r = f2.astype(np.float32).astype(np.float64)[N:] - ref_sf
    ref_cost = float(np.dot(r, r))
    # the residual is small against f: compare it normwise against the size of f
    assert abs(np.sqrt(cost) - np.sqrt(ref_cost)) <= 1e-5 * np.linalg.norm(f2[N:])


def test_kernel_section_cost_vanishes():
    announce("split cost kernel section")
    m2, s, seed = 10, 3, 5
    C2 = inputs.upper_triangular_generators(2, m2, s, seed)
    X2 = onet.net_int(2, m2, C2)
    alpha, beta, q = 2.5, 0.7, -1.5
    f2 = kernel.kernel_K(2, alpha, tuning.weights(s, beta, q), m2, X2, X2[:, 7:8])
    net = fdwt.Net(2, m2, s, C2)
    cost = net.split_cost(torch.from_numpy(f2.astype(np.float32)).cuda(), alpha, beta, q)
    assert cost <= 1e-10 * float(np.dot(f2, f2))


def test_nelder_mead_selection():
    """The selected parameters, costed by the oracle, beat the start and a
    brute-force grid; the reported cost is the oracle's to 1e-4."""
    announce("kernel tune")
    m2, s, seed = 8, 3, 6
    C2, f2, net, fd = setup(m2, s, seed)
    f2r = f2.astype(np.float32).astype(np.float64)
    start = (2.0, 1.0, -2.0)
    fit = net.kernel_tune(fd, start=start, max_evals=300)
    got = tuning.split_cost(m2, C2, f2r, fit["alpha"], fit["beta"], fit["q"])
    assert got <= tuning.split_cost(m2, C2, f2r, *start)
    grid = min(tuning.split_cost(m2, C2, f2r, al, be, qq)
               for al, be, qq in itertools.product([1.5, 2.0, 3.0, 4.0], [0.25, 1.0, 4.0], [-3.0, -2.0, -1.0, 0.0]))
    assert got <= grid * (1 + 1e-3)
    assert abs(np.sqrt(fit["cost"]) - np.sqrt(got)) <= 1e-5 * np.linalg.norm(f2[2 ** (m2 - 1):])
    assert fit["evaluations"] <= 300 + 3


def test_tuning_rejects_other_nets():
    announce("kernel tune errors")
    net3 = fdwt.Net(3, 5, 2, inputs.upper_triangular_generators(3, 5, 2, 1))
    f = torch.zeros(3 ** 5, device="cuda")
    with pytest.raises(fdwt.FdwtError) as e:
        net3.split_cost(f, 2.0, 1.0, -2.0)
    assert e.value.code == fdwt.EUNSUPPORTED
    C = inputs.random_generators(2, 6, 2, 3)
    C[:, 5, 0] = 1  # last output digit depends on the first index digit
    net = fdwt.Net(2, 6, 2, C)
    with pytest.raises(fdwt.FdwtError) as e:
        net.split_cost(torch.zeros(64, device="cuda"), 2.0, 1.0, -2.0)
    assert e.value.code == fdwt.EINVAL
    netok = fdwt.Net(2, 6, 2, inputs.upper_triangular_generators(2, 6, 2, 3))
    with pytest.raises(fdwt.FdwtError):
        netok.split_cost(torch.zeros(64, device="cuda"), 0.9, 1.0, -2.0)
