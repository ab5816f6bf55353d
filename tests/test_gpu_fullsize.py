"""Parity at the full benchmark sizes through closed forms.

When the data are a kernel section f = K(., x_v), the interpolation system of
Section 3.2 has the solution c = e_v, so the interpolant is K(., x_v) itself:
Sf(q) = K(q, x_v) at every query q, and the ANOVA variances of Section 4 are
those of the kernel section, var_trc(d) = prod_{j<=d} (1 + gamma_j^2 R'(0)) - 1
and var_sup(d) = sum_{i<=d} e_i(gamma_1^2 R'(0), ..., gamma_s^2 R'(0)).  Both
sides come from the oracle's closed forms, so every query and every d of the
full-size runs is compared, not a sample.

Tolerances: f is rounded to float32 (relative 6e-8 per value) and the
transforms run in float32, so the interpolant and the variances carry errors
of a few float32 roundings, amplified by at most the spectral solve's
cancellation; 1e-5 (normwise for Sf, relative per d for the variances) is the
float bar used throughout.
"""
import numpy as np
import pytest
import torch

from oracle import anova, kernel, net as onet
from paper_0808_0487_amd import fdwt, inputs
from tests.gpu_common import announce, kernel_section_p2, net_int_p2_doubling, nrel

pytestmark = pytest.mark.gpu


def qdev(Q):
    return torch.from_numpy(np.ascontiguousarray(Q, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()


@pytest.mark.timeout(300)
def test_prime_three_full_size_kernel_section_at_every_query():
    """p = 3, m = 14 (4,782,969 points), s = 10, 65536 random 20-digit queries
    (the interpolation workload's shape; k_spline_eval for p odd with
    9 <= s <= 16): Sf(q) = K(q, x_v) at every query, and at net points."""
    p, m, s, v = 3, 14, 10, 12345
    announce("full p3 kernel section", p, m, s)
    C = inputs.upper_triangular_generators(p, m, s, 3)
    X = onet.net_int(p, m, C)
    gam = inputs.kernel_weights(s)
    f = kernel.kernel_K(p, 2.0, gam, m, X, X[:, v:v + 1])
    D = inputs.QUERY_DEPTH[p]
    Q = inputs.queries(p, s, 65536, 3).astype(np.int64)
    idx = np.array([0, v, 1, 77, p ** m - 1])
    Qall = np.concatenate([Q, kernel.to_depth(p, m, D, X[:, idx])], axis=1)
    ref = kernel.kernel_K(p, 2.0, gam, D, Qall, kernel.to_depth(p, m, D, X[:, v:v + 1]))
    net = fdwt.Net(p, m, s, C)
    c, sf = net.walsh_interp(fdwt.Kernel(2.0, gam), torch.from_numpy(f).float().cuda(), qdev(Qall))
    sf = sf.cpu().numpy().astype(np.float64)
    # (c itself is e_v only up to the float32 solve, whose rounding errors in
    # the bins where K~ is smallest are amplified by 1/K~; the evaluation
    # multiplies them by the same small K~ again, so Sf is accurate.)
    assert nrel(sf, ref) <= 1e-5
    assert np.max(np.abs(sf - ref)) <= 1e-5 * np.max(np.abs(ref))
    net.close()


def c2_kernel_section(s=20, v=7):
    p, m = 2, 24
    C = inputs.upper_triangular_generators(p, m, s, 9)
    X = net_int_p2_doubling(m, C)
    gam = inputs.kernel_weights(s, q=-1.0, beta=0.8)
    f = kernel_section_p2(2.0, gam, m, X, X[:, v])
    return p, m, C, X, gam, f


@pytest.mark.timeout(300)
def test_plain_at_scale_kernel_section_variances_every_d():
    """p = 2, m = 24, s = 20 (the benchmark's shape): eff_dim of a kernel
    section against the closed forms at every d = 1..20, for both the
    truncation (generated first pass) and the superposition (symmetric
    polynomial columns) variances."""
    s = 20
    announce("full p2 kernel section eff_dim", s)
    p, m, C, X, gam, f = c2_kernel_section(s)
    net = fdwt.Net(p, m, s, C)
    res = net.eff_dim(fdwt.Kernel(2.0, gam), net.forward(torch.from_numpy(f).float().cuda()))
    r0 = gam ** 2 * kernel.rprime_closed(p, 2.0, 0)
    e = anova.esp(list(r0))
    for d in range(1, s + 1):
        assert res["var_trc"][d] == pytest.approx(np.prod(1 + r0[:d]) - 1, rel=1e-5), d
        assert res["var_sup"][d] == pytest.approx(sum(e[1:d + 1]), rel=1e-5), d
    dt, ds = anova.effective_dims(res["var_trc"], res["var_sup"])
    assert (res["d_trc"], res["d_sup"]) == (dt, ds)
    net.close()


@pytest.mark.timeout(300)
def test_plain_at_scale_kernel_section_at_queries():
    """p = 2, m = 24, s = 20, 4096 random 32-digit queries (k_spline_eval for
    p = 2 with 17 <= s <= 32): Sf(q) = K(q, x_v) at every query."""
    s, v = 20, 7
    announce("full p2 kernel section queries", s)
    p, m, C, X, gam, f = c2_kernel_section(s, v)
    D = inputs.QUERY_DEPTH[p]
    Q = inputs.queries(p, s, 4096, 5).astype(np.int64)
    Qall = np.concatenate([Q, kernel.to_depth(p, m, D, X[:, [0, v, 3, 2 ** m - 1]])], axis=1)
    ref = kernel_section_p2(2.0, gam, D, Qall, kernel.to_depth(p, m, D, X[:, v]))
    net = fdwt.Net(p, m, s, C)
    _, sf = net.walsh_interp(fdwt.Kernel(2.0, gam), torch.from_numpy(f).float().cuda(), qdev(Qall))
    sf = sf.cpu().numpy().astype(np.float64)
    assert nrel(sf, ref) <= 1e-5
    assert np.max(np.abs(sf - ref)) <= 1e-5 * np.max(np.abs(ref))
    net.close()
