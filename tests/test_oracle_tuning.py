"""Pins of the oracle's kernel-parameter selection (Section 5.1): the
structure of the half split, an exact case (f a kernel section has cost 0),
the Walsh-transform route to Sf on the second half (numpy FFT over the digit
tensor), and the optimiser against a brute-force grid."""
import itertools

import numpy as np
import pytest

from oracle import kernel, net, tuning
from paper_0808_0487_amd import inputs
from tests._libdwt import lib_dwt, lib_idwt


def case(m2, s, seed):
    C2 = inputs.upper_triangular_generators(2, m2, s, seed)
    X2 = net.net_int(2, m2, C2)
    x = X2 / float(2 ** m2)
    f2 = np.prod(1.0 + (x - 0.5) / np.arange(1, s + 1)[:, None] ** 1.5, axis=0) + 0.3 * np.sin(7 * x[0])
    return C2, X2, f2


@pytest.mark.parametrize("m2,s,seed", [(5, 2, 1), (7, 3, 2), (8, 4, 3)])
def test_second_half_is_first_half_shifted_by_x_N(m2, s, seed):
    """Digital nets are groups: x_{N+n} = x_n (+) x_N, and the first half,
    read with one digit less, is the net of the leading m x m blocks."""
    C2, X2, _ = case(m2, s, seed)
    N = 2 ** (m2 - 1)
    first, second = tuning.halves(m2, C2)
    assert np.array_equal(second, (first * 2) ^ X2[:, N:N + 1])
    lead = np.ascontiguousarray(C2[:, :m2 - 1, :m2 - 1])
    assert np.array_equal(first, net.net_int(2, m2 - 1, lead))


@pytest.mark.parametrize("m2,s,seed", [(6, 2, 4), (7, 3, 5)])
def test_kernel_section_has_zero_cost(m2, s, seed):
    """f = K(., x_v) for a point v of the first half lies in the span of the
    spline, so Sf = f everywhere and the cost vanishes."""
    C2, X2, _ = case(m2, s, seed)
    alpha, beta, q = 2.5, 0.7, -1.5
    gam = tuning.weights(s, beta, q)
    v = 3
    f2 = kernel.kernel_K(2, alpha, gam, m2, X2, X2[:, v:v + 1])
    cost = tuning.split_cost(m2, C2, f2, alpha, beta, q)
    assert cost <= 1e-20 * float(np.dot(f2, f2))


@pytest.mark.parametrize("m2,s,seed", [(6, 2, 6), (8, 3, 7), (9, 4, 8)])
def test_second_half_by_walsh_transforms(m2, s, seed):
    """Sf(x_{N+n}) = sum_v c_v K(x_n (+) x_N (-) x_v) is a group convolution on
    the first half: with g(u) = K(x_u (+) x_N, 0) it equals the inverse
    transform of f~(h) G(h) / K_u(h) (G, K_u unnormalised transforms of g and
    of the kernel data).  Computed here with numpy's FFT over the digit tensor
    and compared with the dense solve plus direct sums."""
    C2, X2, f2 = case(m2, s, seed)
    m, N = m2 - 1, 2 ** (m2 - 1)
    alpha, beta, q = 2.0, 1.0, -2.0
    gam = tuning.weights(s, beta, q)
    first, _ = tuning.halves(m2, C2)
    k = kernel.kernel_K(2, alpha, gam, m2, first * 2, np.zeros_like(first))
    g = kernel.kernel_K(2, alpha, gam, m2, (first * 2) ^ X2[:, N:N + 1], np.zeros_like(first))
    Ku = (N * lib_dwt(2, m, k)).real
    G = (N * lib_dwt(2, m, g)).real
    ft = lib_dwt(2, m, f2[:N])
    spectral = lib_idwt(2, m, ft * G / Ku).real
    direct = tuning.split_sf(m2, C2, f2, alpha, beta, q)
    assert np.allclose(spectral, direct, rtol=0, atol=1e-10 * np.max(np.abs(direct)))


def test_nelder_mead_beats_a_grid():
    """The tuned cost is below the start's and below the best of a brute-force
    grid over (alpha, beta, q)."""
    m2, s, seed = 7, 3, 9
    C2, _, f2 = case(m2, s, seed)
    start = (2.0, 1.0, -2.0)
    a, b, q, cost, nfev = tuning.tune(m2, C2, f2, start=start, maxfev=300)
    assert a > 1.0 and b > 0.0 and nfev <= 301
    assert cost <= tuning.split_cost(m2, C2, f2, *start)
    grid = min(tuning.split_cost(m2, C2, f2, al, be, qq)
               for al, be, qq in itertools.product([1.5, 2.0, 3.0, 4.0], [0.25, 1.0, 4.0], [-3.0, -2.0, -1.0, 0.0]))
    assert cost <= grid * (1 + 1e-6)
    assert abs(tuning.split_cost(m2, C2, f2, a, b, q) - cost) <= 1e-12 * max(cost, 1e-300)
