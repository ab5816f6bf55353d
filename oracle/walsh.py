"""Walsh functions, the dual net and the discrete Walsh transform by its
definition (Section 1, Definitions of the Walsh functions and Eq.
(eq_dwalshcoeff); Section 2.1, the dual net, nu, digit-wise addition and the
representatives K(C); Section 3.3, the Lemma on the inverse).  Test
infrastructure only; see the package docstring.

The transforms here are the direct sums (O(N^2)).  Outputs are indexed by the
coset label h = h_0 + h_1 p + ... + h_{m-1} p^{m-1} of h_vec = C . k, which is
where Algorithm 1 leaves coefficient k (its final formula reads G^(m) at
(h_0, ..., h_{m-1})).
"""
import itertools

import numpy as np

from .net import index_digits, output_digits


def omega_table(p):
    """omega_p^e for e = 0..p-1 with omega_p = exp(2 pi i / p)."""
    e = np.arange(p)
    return np.exp(2j * np.pi * e / p)


def int_digits(p, k, count):
    """First ``count`` base-p digits of the integer k, LSB first."""
    out = []
    for _ in range(count):
        out.append(k % p)
        k //= p
    return out


def nu(p, k):
    """nu(0) = 0, nu(k) = 1 + index of the highest non-zero digit (Section 2.1)."""
    v = 0
    i = 0
    while k > 0:
        i += 1
        if k % p:
            v = i
        k //= p
    return v


def nu_vec(p, kvec):
    return sum(nu(p, k) for k in kvec)


def wal_exponent(p, k, xdig):
    """Exponent sum_i x_{i+1} k_i (mod p) of  pwal_k(x) = omega^(x_1 k_0 + ...)
    for x given by its digits xdig = (x_1, x_2, ...) (Definition of the Walsh
    function).  ``xdig`` may be an array (..., D); digits of k beyond D meet
    x-digits that are zero."""
    xdig = np.asarray(xdig, dtype=np.int64)
    D = xdig.shape[-1]
    kd = np.array(int_digits(p, k, D), dtype=np.int64)
    return (xdig @ kd) % p


def wal(p, k, xdig):
    """pwal_k(x) for x given by its base-p digits (x_1, x_2, ...)."""
    return omega_table(p)[wal_exponent(p, k, xdig)]


def wal_multi(p, kvec, ydig):
    """wal_k(x) = prod_j wal_{k_j}(x_j) (Definition for s >= 2).  ``ydig`` has
    shape (s, N, D): digits of every coordinate of every point."""
    e = np.zeros(ydig.shape[1], dtype=np.int64)
    for j, kj in enumerate(kvec):
        e = (e + wal_exponent(p, kj, ydig[j])) % p
    return omega_table(p)[e]


def coset_label(p, m, C, kvec):
    """h_vec = C . k = sum_j C_j^T k_vec_j^(m) over Z_p (Section 2.1), returned
    as the integer h = sum_i h_i p^i."""
    C = np.asarray(C, dtype=np.int64)
    h = np.zeros(m, dtype=np.int64)
    for j, kj in enumerate(kvec):
        kd = np.array(int_digits(p, kj, m), dtype=np.int64)
        h = (h + C[j].T @ kd) % p
    return int(sum(int(h[i]) * p ** i for i in range(m)))


def representatives(p, m, C):
    """K(C): in every coset D(h) the k of least nu(k), ties broken by the
    lexicographic order k_1 first (Section 2.1).  Brute force over
    [0, p^m)^s -- a representative never needs digits beyond the m-th, since
    dropping them keeps the coset and lowers nu.  Returns a list indexed by
    the label h.  Only for tiny p^(m s)."""
    C = np.asarray(C, dtype=np.int64)
    s = C.shape[0]
    N = p ** m
    best = [None] * N
    for kvec in itertools.product(range(N), repeat=s):
        h = coset_label(p, m, C, kvec)
        key = (nu_vec(p, kvec), kvec)
        if best[h] is None or key < best[h][0]:
            best[h] = (key, kvec)
    return [b[1] for b in best]


def dual_net_box(p, m, C, kmax):
    """Elements of the dual net D(C) = {k : C . k = 0} with all k_j < kmax."""
    C = np.asarray(C, dtype=np.int64)
    s = C.shape[0]
    return [k for k in itertools.product(range(kmax), repeat=s)
            if coset_label(p, m, C, k) == 0]


def inv_mod_p_matrix(A, p):
    """Inverse of a square matrix over Z_p (Gauss-Jordan); None if singular."""
    A = np.array(A, dtype=np.int64) % p
    n = A.shape[0]
    M = np.concatenate([A, np.eye(n, dtype=np.int64)], axis=1)
    for c in range(n):
        piv = next((i for i in range(c, n) if M[i, c] != 0), None)
        if piv is None:
            return None
        M[[c, piv]] = M[[piv, c]]
        M[c] = (M[c] * pow(int(M[c, c]), p - 2, p)) % p
        for i in range(n):
            if i != c and M[i, c] != 0:
                M[i] = (M[i] - M[i, c] * M[c]) % p
    return M[:, n:]


def coset_member(p, m, C, h):
    """Some wavenumber vector k with C . k = h: k_1 = (C_1^T)^-1 h_vec and
    k_j = 0 otherwise (needs C_1 non-singular).  Every member of a coset gives
    the same Walsh values on the net, so the DWT value does not depend on the
    member chosen (Section 2.2: the aliasing argument)."""
    C = np.asarray(C, dtype=np.int64)
    inv = inv_mod_p_matrix(C[0].T, p)
    if inv is None:
        raise ValueError("C_1 is singular")
    hv = np.array(int_digits(p, h, m), dtype=np.int64)
    kd = (inv @ hv) % p
    k1 = int(sum(int(kd[i]) * p ** i for i in range(m)))
    return (k1,) + (0,) * (C.shape[0] - 1)


def dwt_direct(p, m, C, f, hs=None, reps=None):
    """Discrete Walsh coefficients by their definition, Eq. (eq_dwalshcoeff):
        f~(k) = p^-m sum_{x in P(C)} f(x) conj(wal_k(x)),
    for k the representative of each coset label h in ``hs`` (all labels when
    None).  wal_k(x_n) is evaluated on the digits of the net points, not via
    the index identity of Section 2.2.  ``reps`` (from representatives())
    selects the K(C) members; otherwise coset_member() is used.  complex128.
    f may be real, complex or integer valued (integer data are summed exactly
    in int64 when p = 2)."""
    N = p ** m
    f = np.asarray(f)
    if hs is None:
        hs = range(N)
    hs = list(hs)
    ydig = output_digits(p, m, C, np.arange(N))
    integer = np.issubdtype(f.dtype, np.integer)
    out = np.zeros(len(hs), dtype=np.int64 if (integer and p == 2) else np.complex128)
    for t, h in enumerate(hs):
        kvec = reps[h] if reps is not None else coset_member(p, m, C, h)
        w = wal_multi(p, kvec, ydig)
        if integer and p == 2:
            out[t] = int(np.sum(f.astype(np.int64) * np.rint(w.real).astype(np.int64)))
        else:
            out[t] = np.sum(f * np.conj(w)) / N
    return out


_DIGIT_CACHE = {}


def _all_index_digits(p, m):
    """Digits n_i of every index n < p^m as an int8 array (m, N), computed
    once per (p, m) and reused across coefficients."""
    key = (p, m)
    if key not in _DIGIT_CACHE:
        _DIGIT_CACHE.clear()
        N = p ** m
        nd = np.empty((m, N), dtype=np.int8)
        q = np.arange(N, dtype=np.int64)
        for i in range(m):
            nd[i] = q % p
            q //= p
        _DIGIT_CACHE[key] = nd
    return _DIGIT_CACHE[key]


def phase_exponents(p, m, n, h):
    """n_vec . h_vec (mod p) for arrays of indices n and one label h."""
    hd = int_digits(p, h, m)
    if isinstance(n, np.ndarray) and n.shape == (p ** m,) and n[0] == 0 and n[-1] == p ** m - 1:
        nd = _all_index_digits(p, m)
        e = np.zeros(p ** m, dtype=np.int16)
        for i in range(m):
            if hd[i]:
                e += nd[i].astype(np.int16) * np.int16(hd[i])
                e %= p
        return e
    nd = index_digits(p, m, n)
    return (nd @ np.array(hd, dtype=np.int64)) % p


def dwt_phase(p, m, f, hs, normalise=True):
    """The same coefficients through the identity wal_k(x_n) = omega^(n.h)
    (Section 2.2):  f~ = p^-m sum_n f(x_n) omega^(-n.h).  For p = 2 the phase
    is (-1)^popcount(n & h) and integer data stay exact in int64 (no
    normalisation).  Used where the net is too large for dwt_direct; the two
    are checked against each other on small nets."""
    N = p ** m
    f = np.asarray(f)
    n = np.arange(N, dtype=np.int64)
    hs = list(hs)
    if p == 2:
        integer = np.issubdtype(f.dtype, np.integer)
        cplx = np.iscomplexobj(f)
        dt = np.int64 if integer else (np.complex128 if cplx else np.float64)
        out = np.zeros(len(hs), dtype=dt)
        fv = f.astype(dt)
        for t, h in enumerate(hs):
            sign = 1 - 2 * (np.bitwise_count(n & h) & 1).astype(np.int64)
            out[t] = np.sum(fv * sign)
        if not integer and normalise:
            out = out / N
        return out
    w = omega_table(p)
    out = np.zeros(len(hs), dtype=np.complex128)
    for t, h in enumerate(hs):
        e = phase_exponents(p, m, n, h)
        out[t] = np.sum(f * np.conj(w[e]))
    return out / N if normalise else out


def idwt_direct(p, m, C, ct, ns=None, reps=None):
    """Inverse by the Lemma of Section 3.3:  c_n = sum_{k in K(C)} c~(k) wal_k(x_n),
    with c~ indexed by the coset label h.  complex128."""
    N = p ** m
    ct = np.asarray(ct)
    if ns is None:
        ns = range(N)
    ns = np.array(list(ns), dtype=np.int64)
    ydig = output_digits(p, m, C, ns)
    out = np.zeros(len(ns), dtype=np.complex128)
    for h in range(N):
        kvec = reps[h] if reps is not None else coset_member(p, m, C, h)
        out += ct[h] * wal_multi(p, kvec, ydig)
    return out


def idwt_phase(p, m, ct, ns):
    """Inverse through the index identity: c_n = sum_h c~(h) omega^(+n.h);
    for p = 2 integer data stay exact in int64."""
    N = p ** m
    ct = np.asarray(ct)
    h = np.arange(N, dtype=np.int64)
    ns = list(ns)
    if p == 2:
        integer = np.issubdtype(ct.dtype, np.integer)
        cplx = np.iscomplexobj(ct)
        dt = np.int64 if integer else (np.complex128 if cplx else np.float64)
        out = np.zeros(len(ns), dtype=dt)
        cv = ct.astype(dt)
        for t, n in enumerate(ns):
            sign = 1 - 2 * (np.bitwise_count(h & n) & 1).astype(np.int64)
            out[t] = np.sum(cv * sign)
        return out
    w = omega_table(p)
    out = np.zeros(len(ns), dtype=np.complex128)
    for t, n in enumerate(ns):
        e = phase_exponents(p, m, h, n)
        out[t] = np.sum(ct * w[e])
    return out


def walsh_matrix(p, a):
    """W[k, X] = pwal_k(X / p^a) for k, X < p^a (one dimension, a digits)."""
    N = p ** a
    W = np.empty((N, N), dtype=np.complex128)
    for X in range(N):
        xd = int_digits(p, X, a)[::-1]       # x_1 .. x_a (most significant first)
        for k in range(N):
            W[k, X] = wal(p, k, np.array(xd))
    return W
