"""Pins for oracle.kernel: the closed forms of K' and R' against their Walsh
series (Section 4), first-differing-digit indexing, the Gram system and the
spline interpolant (Section 3.2)."""
import numpy as np
import pytest

from oracle import kernel, net, walsh
from paper_0808_0487_amd import inputs
from tests._libdwt import lib_dwt, lib_idwt


@pytest.mark.parametrize("p", [2, 3, 5])
@pytest.mark.parametrize("alpha", [1.5, 2.0, 3.0])
def test_kprime_and_rprime_closed_forms_equal_their_series(p, alpha):
    """For z with first non-zero digit i <= a the series truncated at p^a is
    exact (every term of higher degree vanishes); at z = 0 the truncated
    series tends to 1 (K') and to the constant of R'."""
    a = {2: 9, 3: 6, 5: 4}[p]
    g = np.random.default_rng(int(alpha * 10) + p)
    for i in range(1, a + 1):
        for _ in range(2):
            z = [0] * (i - 1) + [int(g.integers(1, p))] + [int(v) for v in g.integers(0, p, a - i)]
            ks = kernel.kprime_series(p, alpha, z, p ** a)
            rs = kernel.rprime_series(p, alpha, z, p ** a)
            assert abs(ks.imag) < 1e-12 and abs(rs.imag) < 1e-12
            assert np.isclose(ks.real, kernel.kprime_closed(p, alpha, i), rtol=0, atol=1e-12)
            assert np.isclose(rs.real, kernel.rprime_closed(p, alpha, i), rtol=0, atol=1e-12)
    tail = p ** (a * (1 - alpha))
    assert abs(kernel.kprime_series(p, alpha, [0] * a, p ** a).real - 1.0) <= 2 * tail
    assert abs(kernel.rprime_series(p, alpha, [0] * a, p ** a).real
               - kernel.rprime_closed(p, alpha, 0)) <= 2 * tail


@pytest.mark.parametrize("p", [2, 3, 5])
def test_kprime_normalised_to_one_at_zero(p):
    """sum_k K'^(k) = K'(0,0) = 1 (Section 4 normalisation), summed over
    degrees analytically: (p-1) p^a terms of degree a."""
    alpha = 2.0
    total = sum((p - 1) * p ** a * kernel.kprime_coef(p, alpha, p ** a) for a in range(200))
    assert np.isclose(total, 1.0)
    assert kernel.kprime_closed(p, alpha, 0) == 1.0


@pytest.mark.parametrize("p,D", [(2, 12), (3, 7), (5, 5)])
def test_first_diff_digit_against_string_compare(p, D):
    g = np.random.default_rng(p)
    a = g.integers(0, p ** D, 300)
    b = a.copy()
    b[::3] = g.integers(0, p ** D, 100)
    got = kernel.first_diff_digit(p, D, a, b)
    for x, y, i in zip(a, b, got):
        sx = np.base_repr(int(x), p).rjust(D, "0")
        sy = np.base_repr(int(y), p).rjust(D, "0")
        want = next((t + 1 for t in range(D) if sx[t] != sy[t]), 0)
        assert i == want


CASES = [(2, 6, 3, 1), (2, 8, 4, 2), (3, 4, 3, 3), (5, 3, 2, 4)]


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_gram_is_symmetric_positive_definite(p, m, s, seed):
    C = inputs.upper_triangular_generators(p, m, s, seed)
    X = net.net_int(p, m, C)
    G = kernel.gram(p, m, 2.0, inputs.kernel_weights(s), X)
    assert np.allclose(G, G.T)
    np.linalg.cholesky(G)


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_spline_of_a_kernel_section_is_that_section(p, m, s, seed):
    """f = K(., x_v) sampled at the net interpolates with c = e_v."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    X = net.net_int(p, m, C)
    gam = inputs.kernel_weights(s)
    v = 5
    f = kernel.kernel_K(p, 2.0, gam, m, X, X[:, v:v + 1])
    c = kernel.spline_coef_dense(p, m, 2.0, gam, X, f)
    e = np.zeros(p ** m)
    e[v] = 1
    assert np.allclose(c, e, atol=1e-10)


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_dense_spline_equals_spectral_solution(p, m, s, seed):
    """Eq. (splinecoef): c~ = f~/(p^m K~) with K~ the DWT of the kernel data;
    the DWTs here are numpy FFTs over the digit tensor."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    X = net.net_int(p, m, C)
    x = X / N
    gam = inputs.kernel_weights(s)
    f = np.prod(1 + (x - 0.5) / np.arange(1, s + 1)[:, None] ** 2, axis=0)
    c = kernel.spline_coef_dense(p, m, 2.0, gam, X, f)
    Kt = lib_dwt(p, m, kernel.kernel_data(p, m, 2.0, gam, X))
    assert np.max(np.abs(Kt.imag)) < 1e-12 and np.min(Kt.real) > 0
    c_spec = lib_idwt(p, m, lib_dwt(p, m, f) / (N * Kt))
    assert np.max(np.abs(c_spec.imag)) < 1e-10
    assert np.allclose(c, c_spec.real, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_spline_interpolates_and_evaluates_at_depth(p, m, s, seed):
    """Sf(x_n) = f(x_n) when the queries are the net points lifted to the
    query depth D (Section 3.2)."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    X = net.net_int(p, m, C)
    gam = inputs.kernel_weights(s)
    f = np.random.default_rng(seed).standard_normal(N)
    c = kernel.spline_coef_dense(p, m, 2.0, gam, X, f)
    D = inputs.QUERY_DEPTH[p]
    idx = np.arange(0, N, max(1, N // 16))
    sf = kernel.spline_eval(p, m, 2.0, gam, X, c, kernel.to_depth(p, m, D, X[:, idx]), D)
    assert np.allclose(sf, f[idx], atol=1e-9)


def test_kernel_data_dwt_is_real_positive_and_bounded():
    """K~(h) = sum over the coset of K^ >= 0 (Section 3.2) and
    sum_h K~(h) = K(0,0) = prod (1 + gamma_j)."""
    p, m, s = 2, 8, 4
    C = inputs.upper_triangular_generators(p, m, s, 7)
    X = net.net_int(p, m, C)
    gam = inputs.kernel_weights(s)
    Kt = walsh.dwt_direct(p, m, C, kernel.kernel_data(p, m, 2.0, gam, X))
    assert np.all(Kt.real > 0) and np.allclose(Kt.imag, 0)
    assert np.isclose(np.sum(Kt.real), np.prod(1 + gam))
