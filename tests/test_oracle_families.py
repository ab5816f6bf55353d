"""Pins of the oracle's test functions (oracle/families.py) against what the
paper prints, without the GPU.

  * Section 5.2: f(x) = prod_k (|4 x_k - 2| + a_k)/(1 + a_k).  Each factor has
    mean 1 and variance 1/(3 (1 + a_k)^2); by quadrature of the oracle's own
    function, the product's variance reproduces Table 2's sigma^2(f) column.
  * Section 5.3: the Asian payoff.  The section prints the average
    (1/s) sum_{j=1..s} S_j, while its Table 4 variances are those of the mean
    of the s + 1 prices S_0..S_s (the reading the oracle takes).  A seeded
    Monte Carlo estimate of the oracle's payoff variance lies within three
    combined standard errors (the estimate's and the table's own, from its
    2^14 points) of Table 4's sigma^2_QMC column; the printed average does
    not.
"""
import json
import os

import numpy as np
import pytest
from scipy.special import ndtri

from oracle import families

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def gauss_on_halves(n=8):
    """Gauss-Legendre nodes and weights on [0, 1/2] and [1/2, 1]: exact for
    polynomials of degree < 2n on each half, so exact for the squares of the
    Section 5.2 factors (linear on each half)."""
    t, w = np.polynomial.legendre.leggauss(n)
    x = np.concatenate([0.25 * (t + 1.0), 0.5 + 0.25 * (t + 1.0)])
    return x, np.concatenate([0.25 * w, 0.25 * w])


@pytest.mark.parametrize("a", [0.0, 0.5, 1.0, 3.0, 17.0, 400.0])
def test_wangfang_factor_mean_one_and_variance(a):
    """Section 5.2: one coordinate of the oracle's function integrates to 1
    and has variance 1/(3 (1 + a)^2)."""
    x, w = gauss_on_halves()
    g = families.wangfang(x[None, :], [a])
    assert float(w @ g) == pytest.approx(1.0, abs=1e-14)
    assert float(w @ (g - 1.0) ** 2) == pytest.approx(1.0 / (3.0 * (1.0 + a) ** 2), rel=1e-12)


def test_wangfang_is_a_product_over_coordinates():
    """Two coordinates on a tensor grid: mean 1 and variance
    (1 + v_1)(1 + v_2) - 1, so the function is the product of its factors."""
    x, w = gauss_on_halves()
    a = [1.0, 4.0]
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w).ravel()
    f = families.wangfang(np.stack([X1.ravel(), X2.ravel()]), a)
    v = [1.0 / (3.0 * (1.0 + ai) ** 2) for ai in a]
    assert float(W @ f) == pytest.approx(1.0, abs=1e-14)
    assert float(W @ (f - 1.0) ** 2) == pytest.approx((1 + v[0]) * (1 + v[1]) - 1, rel=1e-12)


def test_wangfang_variance_reproduces_table_2():
    """Table 2's sigma^2(f) for a_k in {1, k, k^2} and s in {10, 20, 40}
    (printed to four decimals) from the quadrature of the oracle's factors."""
    rows = json.load(open(os.path.join(GOLDEN, "table1_table2_exact.json")))["rows"]
    x, w = gauss_on_halves()
    for row in rows:
        s = row["s"]
        k = np.arange(1, s + 1, dtype=np.float64)
        a = {"1": np.ones(s), "k": k, "k2": k ** 2}[row["a"]]
        var_k = [float(w @ (families.wangfang(x[None, :], [ak]) - 1.0) ** 2) for ak in a]
        total = float(np.prod(1.0 + np.array(var_k)) - 1.0)
        assert abs(total - row["var_f"]) <= 0.5e-4 * max(1.0, 10 ** np.floor(np.log10(row["var_f"]))), row


# Table 4 (Section 5.3): sigma^2_QMC for s = 8, 16, 32 at S0 = K = 100,
# sigma = 0.2, r = 0.1, T = 1 (N = 2^14 Sobol' points).
TABLE4_VAR_QMC = {8: 70.3669, 16: 71.6402, 32: 72.6395}
ASIAN = (100.0, 100.0, 0.2, 0.1, 1.0)


def printed_average_payoff(x, S0, K, sigma, r, T):
    """The payoff as the section prints it: the average (1/s) sum_{j=1..s} S_j
    of the prices after each step (S_0 left out)."""
    s = x.shape[0]
    dt = T / s
    logS = np.log(S0) + np.cumsum((r - 0.5 * sigma ** 2) * dt + sigma * np.sqrt(dt) * ndtri(x), axis=0)
    return np.exp(-r * T) * np.maximum(np.exp(logS).mean(axis=0) - K, 0.0)


def mc_variance(fn, s, paths, seed):
    """Sample variance of fn over `paths` seeded uniform points of [0,1)^s
    (zeros replaced by the smallest positive double) and the standard error
    of that estimate, sqrt((mu_4 - sigma^4)/n)."""
    rng = np.random.default_rng(seed)
    vals = []
    for _ in range(paths // (1 << 16)):
        x = rng.random((s, 1 << 16))
        x[x == 0.0] = np.finfo(np.float64).tiny
        vals.append(fn(x, *ASIAN))
    v = np.concatenate(vals)
    d = v - v.mean()
    var = float(np.mean(d ** 2))
    se = float(np.sqrt(max(np.mean(d ** 4) - var ** 2, 0.0) / len(v)))
    return var, se


def test_asian_payoff_variance_matches_table_4():
    """2^20 seeded paths per s.  Table 4's sigma^2_QMC is itself an estimate
    from 2^14 points; its error is taken as the Monte Carlo standard error at
    2^14 points (the standard error at 2^20 paths times 8), and the
    difference is measured in the combined standard error z.  The oracle's
    payoff (mean of S_0..S_s) lies within |z| <= 3 for every s; the printed
    average (1/s) sum_{j=1..s} S_j lies beyond z = 3 for every s and its
    sum of z^2 over the three rows exceeds 100."""
    chi2_printed = 0.0
    for s in (8, 16, 32):
        var, se = mc_variance(families.asian, s, 1 << 20, seed=1000 + s)
        z = (var - TABLE4_VAR_QMC[s]) / np.hypot(se, 8.0 * se)
        assert abs(z) <= 3.0, (s, var, se, z)
        var_p, se_p = mc_variance(printed_average_payoff, s, 1 << 20, seed=1000 + s)
        z_p = (var_p - TABLE4_VAR_QMC[s]) / np.hypot(se_p, 8.0 * se_p)
        assert abs(z_p) > 3.0, (s, var_p, se_p, z_p)
        chi2_printed += z_p ** 2
    assert chi2_printed > 100.0
