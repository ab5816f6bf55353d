"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np


def announce(*parts):
    """Name the case before it touches the GPU (flushed, so a failing run
    still shows which case was running)."""
    print("[case]", *parts, file=sys.stderr, flush=True)


def nrel(a, b):
    """Normwise relative error ||a - b|| / ||b||."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def sample_indices(N, k, seed):
    """k random indices plus the corners; k is capped so that the oracle's
    O(N) per-coefficient sums stay within seconds at large N."""
    k = int(min(k, max(12, 4e8 // max(N, 1))))
    g = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([[0, N - 1, 1, N // 2], g.integers(0, N, k)]))
    return idx[idx < N]


def correctly_rounded_points(p, m, xo):
    """float32 x = RN(X p^-m) from the oracle's float64 quotient X / p^m.
    Casting the float64 quotient to float32 rounds twice, yet gives the
    correctly rounded value: X / p^m lies at least 2^-25 p^-m >= 2^-51
    (relative) away from every midpoint between two floats (for odd p,
    X 2^k - M p^m is a non-zero integer for odd M; for p = 2 the quotient is
    exact in float64), while the float64 quotient is within 2^-53 of it
    (pinned against exact rationals in tests/test_oracle_net.py)."""
    assert p ** m <= 2 ** 26
    return np.asarray(xo, dtype=np.float64).astype(np.float32)


def net_int_p2_doubling(m, C):
    """X_{j,n} of a p = 2 net at every n, from the Z_2-linearity of
    y = C_j n (Definition of a digital net): for n < 2^c,
    X_j(n + 2^c) = X_j(n) XOR X_j(2^c), where X_j(2^c) is column c of C_j read
    as an m-bit integer (row r -> bit m-1-r).  O(N) per coordinate, for inputs
    at sizes where oracle.net.net_int takes minutes; pinned against it in
    tests/test_oracle_net.py."""
    C = np.asarray(C, dtype=np.int64) % 2
    s = C.shape[0]
    w = np.int64(1) << (m - 1 - np.arange(m, dtype=np.int64))
    X = np.zeros((s, 1 << m), dtype=np.int64)
    for j in range(s):
        cols = C[j].T @ w
        for c in range(m):
            X[j, 1 << c:2 << c] = X[j, :1 << c] ^ cols[c]
    return X


def first_diff_digit_p2(D, a, b):
    """Index (1-based, most significant first) of the first binary digit in
    which the D-digit integers a and b differ, 0 when equal: D minus the bit
    length of a XOR b, plus one.  The same function as
    oracle.kernel.first_diff_digit for p = 2 (pinned in
    tests/test_oracle_net.py), vectorised through the bit length."""
    z = np.bitwise_xor(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))
    _, e = np.frexp(z.astype(np.float64))  # z = mant 2^e, mant in [0.5, 1): e = bit length (exact, z < 2^53)
    return np.where(z == 0, 0, D - e + 1).astype(np.int64)


def kernel_section_p2(alpha, gamma, D, X, Xv):
    """K(x_n, x_v) = prod_j [1 + gamma_j K'(x_{n,j} (-) x_{v,j}, 0)] (Section 4)
    for p = 2 points given as D-digit integers X (s, N) and Xv (s,), with the
    oracle's closed form of K'."""
    from oracle import kernel
    out = np.ones(X.shape[1])
    for j in range(X.shape[0]):
        out *= 1.0 + gamma[j] * kernel.kprime_closed(2, alpha, first_diff_digit_p2(D, X[j], Xv[j]))
    return out
