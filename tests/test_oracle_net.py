"""Pins for oracle.net: digital nets (Definition and Eq. (defy)) and t-values."""
import itertools

import numpy as np
import pytest

from oracle import net
from paper_0808_0487_amd import inputs


def radical_inverse_digits_reversed(p, m, n):
    """van der Corput: the base-p digit string of n, written in reverse after
    the radix point, read as an m-digit integer (textbook construction via
    numpy's base representation, independent of any matrix product)."""
    s = np.base_repr(n, base=p).rjust(m, "0")
    return int(s[::-1], p)


@pytest.mark.parametrize("p,m", [(2, 6), (3, 4), (5, 3)])
def test_identity_generator_is_van_der_corput(p, m):
    C = inputs.identity_generators(p, m, 1)
    X = net.net_int(p, m, C)
    ref = [radical_inverse_digits_reversed(p, m, n) for n in range(p ** m)]
    assert X[0].tolist() == ref


@pytest.mark.parametrize("p,m", [(2, 5), (3, 3), (5, 2)])
def test_anti_identity_gives_hammersley_and_t0(p, m):
    """C_1 = I, C_2 = anti-identity: x_2 = n / p^m, the Hammersley set, a
    (0, m, 2)-net (textbook)."""
    C = np.stack([np.eye(m, dtype=np.uint8), np.eye(m, dtype=np.uint8)[::-1]])
    X = net.net_int(p, m, C)
    assert X[1].tolist() == list(range(p ** m))
    assert net.t_value(p, m, C) == 0
    assert net.t_value_geometric(p, m, X) == 0


@pytest.mark.parametrize("p,m,s,seed", [(2, 8, 3, 1), (3, 5, 3, 2), (5, 3, 4, 3)])
def test_nonsingular_coordinates_are_permutations(p, m, s, seed):
    C = inputs.upper_triangular_generators(p, m, s, seed)
    X = net.net_int(p, m, C)
    for j in range(s):
        assert sorted(X[j].tolist()) == list(range(p ** m))


@pytest.mark.parametrize("p,m,s,seed", [(2, 7, 2, 4), (3, 4, 3, 5)])
def test_net_is_a_group_under_digitwise_subtraction(p, m, s, seed):
    """x_n (-) x_v = x_{n (-) v}: the map n -> X is Z_p-linear (Section 3.3)."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    X = net.net_int(p, m, C)
    g = np.random.default_rng(seed)
    nd = lambda v: np.array([(v // p ** i) % p for i in range(m)])
    todigit = lambda d: int(sum(int(d[i]) * p ** i for i in range(m)))
    for _ in range(50):
        a, b = (int(t) for t in g.integers(0, p ** m, 2))
        diff = todigit((nd(a) - nd(b)) % p)
        for j in range(s):
            xa = nd(int(X[j, a]))
            xb = nd(int(X[j, b]))
            assert todigit((xa - xb) % p) == int(X[j, diff])


def test_output_digit_matvec_small_bruteforce():
    """y = C n over Z_p against a scalar triple loop."""
    p, m = 3, 4
    C = inputs.random_generators(p, m, 2, 11).astype(np.int64)
    y = net.output_digits(p, m, C, np.arange(p ** m))
    for n in range(p ** m):
        nd = [(n // p ** i) % p for i in range(m)]
        for j in range(2):
            for r in range(m):
                acc = 0
                for c in range(m):
                    acc += int(C[j, r, c]) * nd[c]
                assert y[j, n, r] == acc % p


@pytest.mark.parametrize("p,m,s", [(2, 3, 2), (2, 4, 3), (3, 2, 2), (3, 3, 2), (5, 2, 2)])
def test_rank_t_value_equals_geometric_t_value(p, m, s):
    """The rank condition after the Definition gives the same t as exhaustive
    counting of points in elementary intervals, for seeded random (also
    singular) generators."""
    for seed in range(6):
        C = inputs.random_generators(p, m, s, 100 + seed)
        X = net.net_int(p, m, C)
        assert net.t_value(p, m, C) == net.t_value_geometric(p, m, X)


def test_every_one_dimensional_binary_net_t_value():
    """s = 1, p = 2, m = 2: all 16 matrices; t = 0 exactly for non-singular
    ones, and t equals m - rank of the leading-row system otherwise."""
    for Cm in net.all_generators(2, 2):
        C = Cm[None]
        X = net.net_int(2, 2, C)
        t = net.t_value(2, 2, C)
        assert t == net.t_value_geometric(2, 2, X)
        if net.rank_mod_p(Cm, 2) == 2:
            assert t == 0


def test_asian_payoff_one_step_is_half_a_black_scholes_call():
    """With s = 1 the payoff is exp(-rT) max((S0 + S1)/2 - K, 0), half a
    European call on S1 with strike 2K - S0: the integral of the oracle's
    payoff over [0, 1] (midpoint rule, 2^18 cells) equals half the
    Black-Scholes price."""
    from math import erf, exp, log, sqrt
    from oracle import families
    S0, K, sigma, r, T = 100.0, 95.0, 0.2, 0.1, 1.0
    M = 1 << 18
    x = ((np.arange(M) + 0.5) / M)[None, :]
    price = float(np.mean(families.asian(x, S0, K, sigma, r, T)))
    Phi = lambda z: 0.5 * (1.0 + erf(z / sqrt(2.0)))
    K2 = 2 * K - S0
    d1 = (log(S0 / K2) + (r + 0.5 * sigma ** 2) * T) / (sigma * sqrt(T))
    bs = S0 * Phi(d1) - K2 * exp(-r * T) * Phi(d1 - sigma * sqrt(T))
    assert abs(price - 0.5 * bs) <= 2e-4 * bs


def test_asian_payoff_limits():
    """No volatility: a deterministic path, payoff (mean over j = 0..s of
    S0 e^{r t_j} - K)+ discounted; a zero coordinate collapses the rest of
    the path."""
    from oracle import families
    s, S0, K, r, T = 4, 100.0, 95.0, 0.05, 1.0
    x = np.full((s, 1), 0.3)
    v = families.asian(x, S0, K, 1e-12, r, T)[0]
    t = np.arange(0, s + 1) * T / s
    assert abs(v - np.exp(-r * T) * (np.mean(S0 * np.exp(r * t)) - K)) <= 1e-8
    x[0, 0] = 0.0
    assert families.asian(x, S0, K, 0.2, r, T)[0] == 0.0  # only S0 remains: (S0/(s+1) - K)+ = 0


@pytest.mark.parametrize("p,m", [(3, 16), (5, 11), (7, 9), (3, 9), (2, 26)])
def test_float_points_from_the_float64_quotient_are_correctly_rounded(p, m):
    """Definition of a digital net: x = X p^-m.  The float32 points the GPU
    tests expect (the float64 quotient cast to float32) equal the float32
    nearest to the exact rational X / p^m, found here with Fractions among
    the neighbours of the candidate.  For odd p no ties occur (X / p^m is
    never a float midpoint); for p = 2 at m > 24 they do, and go to the even
    mantissa, as the device's conversion of X to float rounds them."""
    from fractions import Fraction
    from tests.gpu_common import correctly_rounded_points
    N = p ** m
    X = np.unique(np.concatenate([np.arange(0, 200), N - 1 - np.arange(0, 200),
                                  np.random.default_rng(p * 100 + m).integers(0, N, 3000)]))
    got = correctly_rounded_points(p, m, X.astype(np.float64) / float(N))
    for Xi, g in zip(X.tolist(), got.tolist()):
        q = Fraction(Xi, N)
        c = np.float32(g)
        even = int(np.array(c).view(np.uint32)) & 1 == 0
        for nb in (np.nextafter(c, np.float32(-1)), np.nextafter(c, np.float32(2))):
            dc, dn = abs(Fraction(float(c)) - q), abs(Fraction(float(nb)) - q)
            assert dc < dn or (p == 2 and dc == dn and even), (p, m, Xi)


def test_p2_doubling_net_equals_the_oracle():
    """The tests' O(N) construction of p = 2 nets (XOR doubling) equals the
    oracle's matrix-vector definition: every point at m = 12, sampled points
    at m = 24."""
    from tests.gpu_common import net_int_p2_doubling
    for m, s, seed in ((12, 3, 1), (9, 5, 2)):
        C = inputs.random_generators(2, m, s, seed)
        assert np.array_equal(net_int_p2_doubling(m, C), net.net_int(2, m, C))
    C = inputs.upper_triangular_generators(2, 24, 2, 9)
    X = net_int_p2_doubling(24, C)
    idx = np.random.default_rng(3).integers(0, 1 << 24, 3000)
    assert np.array_equal(X[:, idx], net.net_int(2, 24, C, idx))


def test_p2_first_differing_digit_and_kernel_section_equal_the_oracle():
    """The bit-length form of the first differing digit equals the oracle's
    digit-by-digit one (D = 24 and 32), and the p = 2 kernel section built on
    it equals oracle.kernel.kernel_K."""
    from oracle import kernel
    from tests.gpu_common import first_diff_digit_p2, kernel_section_p2
    g = np.random.default_rng(4)
    for D in (24, 32):
        a = g.integers(0, 1 << D, 5000, dtype=np.int64)
        b = np.where(g.random(5000) < 0.3, a ^ (1 << g.integers(0, D, 5000)), g.integers(0, 1 << D, 5000))
        b[:10] = a[:10]
        assert np.array_equal(first_diff_digit_p2(D, a, b), kernel.first_diff_digit(2, D, a, b))
    X = g.integers(0, 1 << 24, (5, 4000), dtype=np.int64)
    gam = np.array([0.9, 0.5, 0.3, 0.2, 0.1])
    ref = kernel.kernel_K(2, 2.5, gam, 24, X, X[:, 17:18])
    assert np.allclose(kernel_section_p2(2.5, gam, 24, X, X[:, 17]), ref, rtol=1e-15, atol=0)
