"""Selection of the kernel parameters (Section 5.1, "Optimization of the
Kernel Parameters").  Test infrastructure only; see the package docstring.

A base-2 digital net of 2N points (m + 1 digits) whose first N points form
an m-digit net carries the spline: the interpolant of f is fitted at
x_0..x_{N-1} and its error is measured by the cost
    sum_n (f(x_n) - Sf(x_n))^2 over the second N points,
with weights gamma_j = beta j^q, so that (alpha, beta, q) are the only
parameters; they are chosen by minimising the cost with the Nelder-Mead
simplex method (the method of the paper's fminsearch).

Reading taken: the printed lower summation limit N + 1 is read as N (the
paper evaluates Sf at n = N..2N-1 in the next sentence); every point of the
second half enters the cost.
"""
import numpy as np
from scipy.optimize import minimize

from .kernel import spline_coef_dense, spline_eval
from .net import net_int


def weights(s, beta, q):
    """gamma_j = beta j^q (Section 5.1)."""
    j = np.arange(1, s + 1, dtype=np.float64)
    return beta * j ** q


def halves(m2, C2):
    """Integer coordinates of the 2N-point net (m2 = m + 1 digits) split into
    the first half (as m-digit integers; its last digit must be 0, which holds
    when each C_j is upper triangular) and the second half (m2 digits)."""
    X2 = net_int(2, m2, C2)
    N = 2 ** (m2 - 1)
    first = X2[:, :N]
    if np.any(first % 2):
        raise ValueError("the first N points do not form an m-digit net")
    return first // 2, X2[:, N:]


def split_sf(m2, C2, f2, alpha, beta, q):
    """Sf at the second half, Sf fitted to f2[:N] at the first half by the
    dense solve of Section 3.2 and evaluated by the direct sum at depth m2."""
    m = m2 - 1
    N = 2 ** m
    Xtr, Xval = halves(m2, C2)
    s = Xtr.shape[0]
    gam = weights(s, beta, q)
    f2 = np.asarray(f2, dtype=np.float64)
    c = spline_coef_dense(2, m, alpha, gam, Xtr, f2[:N])
    return spline_eval(2, m, alpha, gam, Xtr, c, Xval, m2)


def split_cost(m2, C2, f2, alpha, beta, q):
    """The cost of Section 5.1: sum over the second half of (f - Sf)^2."""
    N = 2 ** (m2 - 1)
    sf = split_sf(m2, C2, f2, alpha, beta, q)
    r = np.asarray(f2, dtype=np.float64)[N:] - sf
    return float(np.dot(r, r))


def to_params(theta):
    """Unconstrained coordinates (log(alpha - 1), log beta, q) -> (alpha, beta, q)."""
    return 1.0 + float(np.exp(theta[0])), float(np.exp(theta[1])), float(theta[2])


def from_params(alpha, beta, q):
    return np.array([np.log(alpha - 1.0), np.log(beta), q], dtype=np.float64)


def tune(m2, C2, f2, start=(2.0, 1.0, -2.0), maxfev=200):
    """Nelder-Mead over (log(alpha - 1), log beta, q) from `start` (initial
    simplex: steps of 0.5 along each coordinate); returns (alpha, beta, q,
    cost, evaluations)."""
    th0 = from_params(*start)
    simplex = np.vstack([th0] + [th0 + 0.5 * e for e in np.eye(3)])  # steps of 0.5 per coordinate
    res = minimize(lambda th: split_cost(m2, C2, f2, *to_params(th)), th0, method="Nelder-Mead",
                   options={"maxfev": maxfev, "xatol": 1e-4, "fatol": 1e-12, "initial_simplex": simplex})
    a, b, q = to_params(res.x)
    return a, b, q, float(res.fun), int(res.nfev)
