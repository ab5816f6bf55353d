"""Seeded synthetic inputs shared by the tests, the bench and the oracle
checks.  This module holds none of the method's arithmetic: it only draws
generating matrices, test-function parameters, raw data and query digits
with numpy's PCG64 generator.

Workload recipes (shapes and value distributions of the paper's experiments;
no published dataset is involved):
  * generating matrices: seeded random non-singular upper-triangular m x m
    matrices over Z_p, C[j][r][c] = 0 for c < r, diagonal in 1..p-1, entries
    above the diagonal uniform in 0..p-1 (the shape of Sobol' generators,
    which the paper uses but does not print);
  * test functions: the product family prod_j (1 + a_j (x_j - 1/2)), the
    exponential family exp(-sum_j w_j x_j^2) and the multiplicative function
    of the paper's Section 5.2;
  * queries: uniform D-digit base-p integers per coordinate (D = 32, 20, 13,
    11 for p = 2, 3, 5, 7).
"""
import math

import numpy as np

QUERY_DEPTH = {2: 32, 3: 20, 5: 13, 7: 11}


def rng(seed):
    return np.random.default_rng(seed)


def upper_triangular_generators(p, m, s, seed):
    """uint8 array (s, m, m): non-singular upper-triangular matrices over Z_p."""
    g = rng(seed)
    C = g.integers(0, p, size=(s, m, m), dtype=np.int64)
    C = np.triu(C, k=1)
    diag = g.integers(1, p, size=(s, m), dtype=np.int64)
    idx = np.arange(m)
    C[:, idx, idx] = diag
    return C.astype(np.uint8)


def identity_generators(p, m, s):
    """C_j = I for every coordinate (radical-inverse points)."""
    return np.broadcast_to(np.eye(m, dtype=np.uint8), (s, m, m)).copy()


def random_generators(p, m, s, seed):
    """Arbitrary (possibly singular) matrices over Z_p."""
    return rng(seed).integers(0, p, size=(s, m, m), dtype=np.int64).astype(np.uint8)


def uniform_int32(N, lo, hi, seed):
    """int32 values uniform in [lo, hi]."""
    return rng(seed).integers(lo, hi + 1, size=N, dtype=np.int64).astype(np.int32)


def uniform_float(N, seed, lo=-1.0, hi=1.0, dtype=np.float32):
    return rng(seed).uniform(lo, hi, size=N).astype(dtype)


def queries(p, s, nq, seed):
    """uint32 array (s, nq) of uniform D-digit base-p integers."""
    D = QUERY_DEPTH[p]
    top = p ** D
    return rng(seed).integers(0, top, size=(s, nq), dtype=np.int64).astype(np.uint32)


def kernel_weights(s, q=-2.0, beta=1.0):
    """gamma_j = beta j^q (the paper's Section 5.1 parameterisation)."""
    j = np.arange(1, s + 1, dtype=np.float64)
    return beta * j ** q


def family_params(kind, s, seed=None, **kw):
    """Per-coordinate parameters of a test-function family.
       product:  a_j = c j^-alpha_f  (c = kw 'scale', default 1; alpha_f from
                 kw 'alpha', or drawn uniform in [1, 3] with ``seed``)
       exp:      w_j = r^j          (r = kw 'ratio', default 0.1, or drawn
                 uniform in [0.05, 0.5] with ``seed``)
       wangfang: a_j = 1, j or j^2  (kw 'a' in {'1', 'k', 'k2'})."""
    j = np.arange(1, s + 1, dtype=np.float64)
    if kind == "product":
        if "const" in kw:
            return np.full(s, float(kw["const"]))
        if "alpha" in kw:
            alpha = kw["alpha"]
        elif seed is not None:
            alpha = rng(seed).uniform(1.0, 3.0)
        else:
            alpha = 2.0
        return kw.get("scale", 1.0) * j ** (-alpha)
    if kind == "exp":
        if "ratio" in kw:
            r = kw["ratio"]
        elif seed is not None:
            r = rng(seed).uniform(0.05, 0.5)
        else:
            r = 0.1
        return r ** j
    if kind == "wangfang":
        a = kw.get("a", "1")
        return {"1": np.ones(s), "k": j, "k2": j * j}[a]
    raise ValueError(kind)


def log_uniform_m(g, lo, hi, p, cap_points=1 << 26):
    """m = round(exp(U[ln lo, ln hi])), capped so that p^m <= cap_points."""
    m = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
    mmax = int(math.floor(math.log(cap_points) / math.log(p) + 1e-9))
    return max(1, min(m, mmax))


def batch_jobs(n, seed, m_lo=12, m_hi=22, s_lo=5, s_hi=50):
    """Ragged batch recipe: per job (m, s, alpha, generator seed) with m
    uniform in m_lo..m_hi, s uniform in s_lo..s_hi and the product family's
    alpha uniform in [1, 3]."""
    g = rng(seed)
    out = []
    for i in range(n):
        m = int(g.integers(m_lo, m_hi + 1))
        s = int(g.integers(s_lo, s_hi + 1))
        alpha = float(g.uniform(1.0, 3.0))
        out.append((m, s, alpha, 10_000 + 7 * seed + i))
    return out


def serving_workload(duration_s, rate, seed, n_nets=64, nq=4096, m_lo=10, m_hi=26, s_lo=2, s_hi=50,
                     cap_points=1 << 26):
    """Serving recipe: Poisson arrivals at `rate` per second for duration_s
    seconds; each request picks one of n_nets seeded nets (p uniform in
    {2, 3, 5}, m = round(exp(U[ln m_lo, ln m_hi])) capped so that p^m <=
    cap_points, s uniform in s_lo..s_hi), is an interpolation or an
    effective-dimension job with equal odds, and samples the product or the
    exponential family with equal odds (parameters drawn per request).
    Interpolation jobs carry nq uniform query points.  Returns (nets, reqs):
    nets[i] = (p, m, s, generator seed); reqs = list of dicts with keys t
    (arrival, s), net, kind, family, a, qseed."""
    g = rng(seed)
    nets = []
    for i in range(n_nets):
        p = int(g.choice([2, 3, 5]))
        m = log_uniform_m(g, m_lo, m_hi, p, cap_points)
        s = int(g.integers(s_lo, s_hi + 1))
        nets.append((p, m, s, 50_000 + 13 * seed + i))
    reqs = []
    t = 0.0
    k = 0
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= duration_s:
            break
        ni = int(g.integers(0, n_nets))
        kind = "interp" if g.random() < 0.5 else "eff_dim"
        family = "product" if g.random() < 0.5 else "exp"
        fseed = 70_000 + 17 * seed + k
        reqs.append({"t": t, "net": ni, "kind": kind, "family": family,
                     "a": family_params(family, nets[ni][2], seed=fseed), "qseed": fseed})
        k += 1
    return nets, reqs
