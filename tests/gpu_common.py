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
