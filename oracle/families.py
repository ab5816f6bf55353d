"""Test functions sampled at the net, in float64.  Test infrastructure only;
see the package docstring.

  * product:  f(x) = prod_j (1 + a_j (x_j - 1/2))
  * exp:      f(x) = exp(-sum_j w_j x_j^2)
  * wangfang: f(x) = prod_j (|4 x_j - 2| + a_j)/(1 + a_j)   (Section 5.2)
"""
import numpy as np


def product(x, a):
    a = np.asarray(a, dtype=np.float64)[:, None]
    return np.prod(1.0 + a * (np.asarray(x) - 0.5), axis=0)


def exponential(x, w):
    w = np.asarray(w, dtype=np.float64)[:, None]
    return np.exp(-np.sum(w * np.asarray(x) ** 2, axis=0))


def wangfang(x, a):
    a = np.asarray(a, dtype=np.float64)[:, None]
    return np.prod((np.abs(4.0 * np.asarray(x) - 2.0) + a) / (1.0 + a), axis=0)


def evaluate(kind, x, params):
    if kind == "product":
        return product(x, params)
    if kind == "exp":
        return exponential(x, params)
    if kind == "wangfang":
        return wangfang(x, params)
    raise ValueError(kind)
