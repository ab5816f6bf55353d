"""Digital (t,m,s)-nets over Z_p (Section 1, Definition of a digital net,
Eq. (defy)) and their t-value (Section 1, the rank condition after the
definition).  Test infrastructure only; see the package docstring.

Conventions (the paper's):
  * point index n = n_0 + n_1 p + ... + n_{m-1} p^{m-1}, digit vector
    n_vec = (n_0, ..., n_{m-1}) (least significant digit first);
  * y_vec = C_j n_vec over Z_p, y_vec = (y_1, ..., y_m);
  * x_{j,n} = y_1 p^-1 + ... + y_m p^-m.
A generating matrix is stored as C[j][r][c] = entry in row r+1 (output digit
y_{r+1}) and column c (input digit n_c).  The integer form of a coordinate is
X_{j,n} = sum_r y_{r+1} p^{m-1-r}, so that x_{j,n} = X_{j,n} / p^m.
"""
import itertools

import numpy as np


def index_digits(p, m, n):
    """Base-p digits (n_0..n_{m-1}) of the indices ``n`` (array), LSB first.
    Returns an int64 array of shape (len(n), m)."""
    n = np.asarray(n, dtype=np.int64)
    out = np.empty(n.shape + (m,), dtype=np.int64)
    q = n.copy()
    for i in range(m):
        out[..., i] = q % p
        q //= p
    return out


def output_digits(p, m, C, n):
    """y_{j,n,r} for the indices ``n``: the matrix-vector products
    y_vec = C_j n_vec over Z_p of Eq. (defy).  Shape (s, len(n), m); the last
    axis is r = 1..m (most significant digit of x first)."""
    C = np.asarray(C, dtype=np.int64)
    nd = index_digits(p, m, n).astype(np.float64)          # (N, m)
    s = C.shape[0]
    y = np.empty((s, nd.shape[0], m), dtype=np.int64)
    for j in range(s):
        # float64 matmul of small integers is exact (|entries| < 2^53)
        prod = nd @ C[j].astype(np.float64).T                # (N, m): sum_c n_c C[r][c]
        y[j] = np.rint(prod).astype(np.int64) % p
    return y


def net_int(p, m, C, n=None, chunk=1 << 20):
    """Integer coordinates X_{j,n} = sum_r y_{j,n,r} p^{m-r}, shape (s, len(n)).
    With ``n`` None, all N = p^m points.  Evaluated in chunks so that large
    nets fit in memory."""
    N = p ** m
    if n is None:
        n = np.arange(N, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    C = np.asarray(C, dtype=np.int64)
    weights = np.array([p ** (m - 1 - r) for r in range(m)], dtype=np.int64)
    out = np.empty((C.shape[0], n.shape[0]), dtype=np.int64)
    for a in range(0, n.shape[0], chunk):
        y = output_digits(p, m, C, n[a:a + chunk])
        out[:, a:a + chunk] = y @ weights
    return out


def net_points(p, m, C, n=None):
    """x_{j,n} in float64, shape (s, len(n)) (Definition of a digital net)."""
    return net_int(p, m, C, n).astype(np.float64) / float(p ** m)


def rank_mod_p(A, p):
    """Rank over Z_p by Gaussian elimination."""
    A = np.array(A, dtype=np.int64) % p
    rows, cols = A.shape
    r = 0
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if A[i, c] != 0:
                piv = i
                break
        if piv is None:
            continue
        A[[r, piv]] = A[[piv, r]]
        inv = pow(int(A[r, c]), p - 2, p)
        A[r] = (A[r] * inv) % p
        for i in range(rows):
            if i != r and A[i, c] != 0:
                A[i] = (A[i] - A[i, c] * A[r]) % p
        r += 1
        if r == rows:
            break
    return r


def _compositions(total, parts):
    """All (d_1..d_parts) of non-negative integers with sum ``total``."""
    if parts == 1:
        yield (total,)
        return
    for first in range(total + 1):
        for rest in _compositions(total - first, parts - 1):
            yield (first,) + rest


def t_value(p, m, C):
    """Smallest t such that for every d_1+...+d_s = m-t the first d_j rows of
    the C_j are linearly independent over Z_p (Section 1, the t value)."""
    C = np.asarray(C, dtype=np.int64)
    s = C.shape[0]
    for t in range(0, m + 1):
        ok = True
        for d in _compositions(m - t, s):
            rows = [C[j, :d[j], :] for j in range(s) if d[j] > 0]
            if not rows:
                continue
            if rank_mod_p(np.concatenate(rows, axis=0), p) < m - t:
                ok = False
                break
        if ok:
            return t
    return m


def interval_counts(p, m, X, d):
    """Number of net points in each elementary interval
    prod_j [a_j p^-d_j, (a_j+1) p^-d_j): the point falls in the box given by
    the leading d_j base-p digits of each coordinate.  Returns a dict
    box -> count (boxes with no point are absent)."""
    X = np.asarray(X, dtype=np.int64)
    keys = [X[j] // (p ** (m - d[j])) for j in range(len(d))]
    counts = {}
    for key in zip(*keys):
        counts[key] = counts.get(key, 0) + 1
    return counts


def is_tms_net(p, m, X, t):
    """Geometric (t,m,s)-net property by exhaustive counting: every elementary
    interval of volume p^{t-m} holds exactly p^t points."""
    s = X.shape[0]
    for d in _compositions(m - t, s):
        cnt = interval_counts(p, m, X, d)
        nbox = p ** (m - t)
        if len(cnt) != nbox or any(v != p ** t for v in cnt.values()):
            return False
    return True


def t_value_geometric(p, m, X):
    """Smallest t for which the point set is a (t,m,s)-net, by counting."""
    for t in range(0, m + 1):
        if is_tms_net(p, m, X, t):
            return t
    return m


def all_generators(p, m):
    """Every m x m matrix over Z_p (only for tiny p, m in tests)."""
    for entries in itertools.product(range(p), repeat=m * m):
        yield np.array(entries, dtype=np.int64).reshape(m, m)
