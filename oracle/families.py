"""Test functions sampled at the net, in float64.  Test infrastructure only;
see the package docstring.

  * product:  f(x) = prod_j (1 + a_j (x_j - 1/2))
  * exp:      f(x) = exp(-sum_j w_j x_j^2)
  * wangfang: f(x) = prod_j (|4 x_j - 2| + a_j)/(1 + a_j)   (Section 5.2)
  * asian:    discounted payoff of an arithmetic-average Asian call under
              geometric Brownian motion, standard construction (Section 5.3)
"""
import numpy as np
from scipy.special import ndtri


def product(x, a):
    a = np.asarray(a, dtype=np.float64)[:, None]
    return np.prod(1.0 + a * (np.asarray(x) - 0.5), axis=0)


def exponential(x, w):
    w = np.asarray(w, dtype=np.float64)[:, None]
    return np.exp(-np.sum(w * np.asarray(x) ** 2, axis=0))


def wangfang(x, a):
    a = np.asarray(a, dtype=np.float64)[:, None]
    return np.prod((np.abs(4.0 * np.asarray(x) - 2.0) + a) / (1.0 + a), axis=0)


def asian(x, S0, K, sigma, r, T):
    """Section 5.3: S_j = S_{j-1} exp((r - sigma^2/2) T/s + sigma sqrt(T/s) Z_j)
    with Z_j = Phi^-1(x_j) (coordinate j drives step j); the payoff is
    max(A - K, 0) discounted by exp(-rT), A the mean of the s + 1 prices
    S_0..S_s at t_j = jT/s, j = 0..s.  (The printed payoff averages S_1..S_s
    over s; the section's own variances, Table 4, are those of the mean over
    j = 0..s, which is the reading taken.)  x_j = 0 gives Z_j = -inf (the
    path collapses to 0 from step j on)."""
    x = np.asarray(x, dtype=np.float64)
    s = x.shape[0]
    dt = T / s
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        Z = ndtri(x)
        logS = np.log(S0) + np.cumsum((r - 0.5 * sigma ** 2) * dt + sigma * np.sqrt(dt) * Z, axis=0)
        S = np.exp(logS)
    S = np.where(np.isnan(S), 0.0, S)
    A = (S0 + S.sum(axis=0)) / (s + 1)
    return np.exp(-r * T) * np.maximum(A - K, 0.0)


def evaluate(kind, x, params):
    if kind == "product":
        return product(x, params)
    if kind == "exp":
        return exponential(x, params)
    if kind == "wangfang":
        return wangfang(x, params)
    if kind == "asian":
        return asian(x, *params)
    raise ValueError(kind)
