"""Fast CPU reference (o2.c): the paper's Algorithms 1 and 2, the kernel data,
the ANOVA variances through the kernel spectra, the spline coefficients and
the interpolant, as plain float64 / int64 loops in C with OpenMP.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: only ``tests/``, the
smoke check and the bench's CPU baseline load it; it shares no code with the
HIP library.  It is checked against the definitions in the Python oracle at
small sizes (tests/test_oracle_fast.py) and then stands in for them at full
size, where the O(N^2) definitions cannot run.

The shared library is built with gcc from ``o2.c`` next to this file (by
``build()``, or on first use when it is missing or older than its source).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "o2.c")
LIB = os.path.join(HERE, "libo2.so")
_L = None


def build(verbose=False):
    """Compile o2.c into libo2.so (gcc -O2 -fopenmp)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building the CPU reference failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        i32, i64, f64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        sig = {
            "o2_threads": ([], i32),
            "o2_set_threads": ([i32], None),
            "o2_net": ([i32, i32, i32, vp, i64, i64, vp], i32),
            "o2_sample": ([i32, i32, i32, i32, vp, vp, i64, vp], i32),
            "o2_fwt": ([i32, i32, i64, vp, vp, i32], i32),
            "o2_kernel_cols": ([i32, i32, i32, f64, vp, vp, i64, vp, vp, vp], i32),
            "o2_variances": ([i32, i32, i32, f64, vp, vp, vp, vp, vp, vp], i32),
            "o2_spline_coef": ([i32, i32, i32, f64, vp, vp, vp, vp, vp], i32),
            "o2_spline_eval": ([i32, i32, i32, f64, vp, vp, vp, i64, vp, i32, vp], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _L = L
    return _L


def _p(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s: error %d" % (what, rc))


def threads():
    return lib().o2_threads()


def set_threads(n):
    lib().o2_set_threads(int(n))


def net_int(p, m, C, n0=0, count=None):
    """X_{j,n} for n = n0 .. n0 + count - 1, int64 array (s, count)."""
    C = np.ascontiguousarray(np.asarray(C, dtype=np.int64) % p, dtype=np.int32)
    s = C.shape[0]
    if count is None:
        count = p ** m - n0
    X = np.empty((s, count), dtype=np.int64)
    _check(lib().o2_net(p, m, s, _p(C), n0, count, _p(X)), "o2_net")
    return X


def sample(kind, p, m, a, X):
    """f(x_n) in float64 for kind 'product' (prod_j (1 + a_j (x_j - 1/2))) or
    'exp' (exp(-sum_j a_j x_j^2)), x = X / p^m."""
    X = np.ascontiguousarray(X, dtype=np.int64)
    s, N = X.shape
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (s,):
        raise ValueError("one parameter per coordinate")
    f = np.empty(N)
    k = {"product": 0, "exp": 1}[kind]
    _check(lib().o2_sample(k, p, m, s, _p(a), _p(X), N, _p(f)), "o2_sample")
    return f


def fwt(p, m, x, inverse=False):
    """Algorithm 1 (forward, divided by p^m) or Algorithm 2 (inverse) of the
    last axis of ``x`` (length p^m; more leading axes are columns).  p = 2
    real data stay real; anything else is complex128."""
    x = np.asarray(x)
    N = p ** m
    if x.shape[-1] != N:
        raise ValueError("last axis must have p^m entries")
    cols = int(np.prod(x.shape[:-1], dtype=np.int64))
    if p == 2 and not np.iscomplexobj(x):
        re = np.ascontiguousarray(x, dtype=np.float64).copy()
        _check(lib().o2_fwt(p, m, cols, _p(re), None, int(inverse)), "o2_fwt")
        return re
    z = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(z.real).copy()
    im = np.ascontiguousarray(z.imag).copy()
    _check(lib().o2_fwt(p, m, cols, _p(re), _p(im), int(inverse)), "o2_fwt")
    return re + 1j * im


def _split(ft, p):
    if p == 2:
        if np.iscomplexobj(ft):
            raise ValueError("p = 2 spectra of real data are real")
        return np.ascontiguousarray(ft, dtype=np.float64), None
    ft = np.asarray(ft, dtype=np.complex128)
    return np.ascontiguousarray(ft.real), np.ascontiguousarray(ft.imag)


def kernel_cols(p, m, alpha, gamma, X):
    """(K, U, Q): K(x_n, 0) (N,), U_d = R_d - 1 (s, N), Q_j = e_j (s, N)."""
    X = np.ascontiguousarray(X, dtype=np.int64)
    s, N = X.shape
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    K = np.empty(N)
    U = np.empty((s, N))
    Q = np.empty((s, N))
    _check(lib().o2_kernel_cols(p, m, s, float(alpha), _p(g), _p(X), N, _p(K), _p(U), _p(Q)), "o2_kernel_cols")
    return K, U, Q


def variances(p, m, alpha, gamma, X, ft):
    """(var_trc[0..s], var_sup[0..s]) of the spline of f, from ft = the
    forward transform of f (Algorithm 1)."""
    X = np.ascontiguousarray(X, dtype=np.int64)
    s = X.shape[0]
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    re, im = _split(ft, p)
    vt = np.zeros(s + 1)
    vs = np.zeros(s + 1)
    _check(lib().o2_variances(p, m, s, float(alpha), _p(g), _p(X), _p(re), _p(im), _p(vt), _p(vs)), "o2_variances")
    return vt, vs


def spline_coef(p, m, alpha, gamma, X, ft):
    """Spline coefficients c (N,) from ft = the forward transform of f."""
    X = np.ascontiguousarray(X, dtype=np.int64)
    s = X.shape[0]
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    re, im = _split(ft, p)
    c = np.empty(p ** m)
    _check(lib().o2_spline_coef(p, m, s, float(alpha), _p(g), _p(X), _p(re), _p(im), _p(c)), "o2_spline_coef")
    return c


def spline_eval(p, m, alpha, gamma, X, c, Q, D):
    """Sf(q) at the D-digit queries Q (s, nq)."""
    X = np.ascontiguousarray(X, dtype=np.int64)
    s = X.shape[0]
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.int64)
    out = np.empty(Q.shape[1])
    _check(lib().o2_spline_eval(p, m, s, float(alpha), _p(g), _p(X), _p(c), Q.shape[1], _p(Q), int(D), _p(out)),
           "o2_spline_eval")
    return out
