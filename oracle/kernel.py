"""Walsh reproducing kernels and the spline interpolant (Sections 3.1-3.2 and
4).  Test infrastructure only; see the package docstring.

Points are handled as exact base-p digit strings of a fixed depth D: a value
x in [0,1) is the integer Xd = x p^D.  The first digit where x and y differ is
the index i of the first non-zero digit of x (-) y, which is all the closed
forms of K' and R' need (Section 4).
"""
import numpy as np

from .walsh import int_digits


# ---------------------------------------------------------------- univariate
def kprime_coef(p, alpha, k):
    """Walsh coefficient of K'(.,0) (Section 4):
        0 for k = 0, else (p^a - p)/(p^a (p-1)) p^(-alpha a), a = nu(k) - 1."""
    if k == 0:
        return 0.0
    a = -1
    q = k
    while q > 0:
        a += 1
        q //= p
    return (p ** alpha - p) / (p ** alpha * (p - 1)) * p ** (-alpha * a)


def kprime_closed(p, alpha, i):
    """K'(z, 0) for z whose first non-zero digit is z_i (Section 4 closed form):
        1 - p^(i (1 - alpha)) (p^alpha - 1)/(p - 1);   i = 0 encodes z = 0 -> 1."""
    i = np.asarray(i)
    val = 1.0 - np.power(float(p), i * (1.0 - alpha)) * (p ** alpha - 1.0) / (p - 1.0)
    return np.where(i == 0, 1.0, val)


def rprime_closed(p, alpha, i):
    """R'(z, 0) = int_0^1 K'(x, z) K'(x, 0) dx, closed form of Section 4:
        (p^a - p)^2 / ((p-1)(p^2a - p)) [1 - p^(i(1-2a)) (p^2a - 1)/(p-1)],
    i = 0 encoding z = 0 (the bracket is then 1)."""
    i = np.asarray(i)
    A = (p ** alpha - p) ** 2 / ((p - 1.0) * (p ** (2 * alpha) - p))
    val = A * (1.0 - np.power(float(p), i * (1.0 - 2 * alpha)) * (p ** (2 * alpha) - 1.0) / (p - 1.0))
    return np.where(i == 0, A, val)


def kprime_series(p, alpha, zdig, kmax):
    """sum_{1 <= k < kmax} K'^(k) wal_k(z) for z given by digits (z_1, z_2, ...):
    the Walsh series that defines K' (Section 4), truncated."""
    w = np.exp(2j * np.pi * np.arange(p) / p)
    zdig = list(zdig)
    total = 0.0 + 0.0j
    for k in range(1, kmax):
        kd = int_digits(p, k, len(zdig))
        e = sum(a * b for a, b in zip(kd, zdig)) % p
        total += kprime_coef(p, alpha, k) * w[e]
    return total


def rprime_series(p, alpha, zdig, kmax):
    """sum_{1 <= k < kmax} (K'^(k))^2 wal_k(z): the series defining R' (Section 4)."""
    w = np.exp(2j * np.pi * np.arange(p) / p)
    zdig = list(zdig)
    total = 0.0 + 0.0j
    for k in range(1, kmax):
        kd = int_digits(p, k, len(zdig))
        e = sum(a * b for a, b in zip(kd, zdig)) % p
        total += kprime_coef(p, alpha, k) ** 2 * w[e]
    return total


# ---------------------------------------------------------------- digits
def first_diff_digit(p, D, a, b):
    """Index i (1-based, most significant first) of the first base-p digit at
    which the D-digit integers a and b differ, 0 when a == b.  Arrays
    broadcast.  Written digit by digit."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    a, b = np.broadcast_arrays(a, b)
    out = np.zeros(a.shape, dtype=np.int64)
    found = np.zeros(a.shape, dtype=bool)
    for i in range(1, D + 1):
        da = (a // p ** (D - i)) % p
        db = (b // p ** (D - i)) % p
        hit = (~found) & (da != db)
        out[hit] = i
        found |= hit
    return out


def weights_vec(gamma, s):
    g = np.asarray(gamma, dtype=np.float64)
    if g.shape != (s,):
        raise ValueError("gamma must have one weight per coordinate")
    return g


# ---------------------------------------------------------------- kernels
def kernel_K(p, alpha, gamma, D, Xa, Xb):
    """K(x, y) = prod_j [1 + gamma_j K'(x_j (-) y_j, 0)] (Section 4) for points
    given as D-digit integers, Xa and Xb of shape (s, ...) broadcasting."""
    Xa = np.asarray(Xa, dtype=np.int64)
    Xb = np.asarray(Xb, dtype=np.int64)
    s = Xa.shape[0]
    g = weights_vec(gamma, s)
    out = 1.0
    for j in range(s):
        i = first_diff_digit(p, D, Xa[j], Xb[j])
        out = out * (1.0 + g[j] * kprime_closed(p, alpha, i))
    return out


def to_depth(p, m, D, X):
    """Net integers X (m digits) as D-digit integers."""
    return np.asarray(X, dtype=np.int64) * p ** (D - m)


def gram(p, m, alpha, gamma, X):
    """G[n, v] = K(x_n, x_v) over the net (Section 3.2 linear system)."""
    X = np.asarray(X, dtype=np.int64)
    return kernel_K(p, alpha, gamma, m, X[:, :, None], X[:, None, :])


def spline_coef_dense(p, m, alpha, gamma, X, f):
    """Solve sum_v c_v K(x_n, x_v) = f(x_n) for c (Section 3.2) by a dense
    float64 LU solve.  Only for N up to a few thousand."""
    G = gram(p, m, alpha, gamma, X)
    return np.linalg.solve(G, np.asarray(f, dtype=np.float64))


def spline_eval(p, m, alpha, gamma, X, c, Q, D):
    """Sf(q) = sum_n c_n K(q, x_n) (Section 3.2) for queries given as D-digit
    integers Q of shape (s, nq); the net is lifted to D digits.  Summed per
    query in float64."""
    Xd = to_depth(p, m, D, X)
    Q = np.asarray(Q, dtype=np.int64)
    c = np.asarray(c, dtype=np.float64)
    out = np.empty(Q.shape[1], dtype=np.float64)
    for t in range(Q.shape[1]):
        Kq = kernel_K(p, alpha, gamma, D, Q[:, t:t + 1], Xd)
        out[t] = float(np.sum(c * Kq))
    return out


def kernel_data(p, m, alpha, gamma, X):
    """(K(x_n, 0))_n, the kernel data whose DWT is K~ (Section 3.2)."""
    X = np.asarray(X, dtype=np.int64)
    return kernel_K(p, alpha, gamma, m, X, np.zeros_like(X))
