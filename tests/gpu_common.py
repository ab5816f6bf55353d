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
