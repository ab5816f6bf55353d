"""Pins for oracle.walsh: Walsh functions, dual net, the DWT by its
definition (Eq. (eq_dwalshcoeff)) and its inverse (Lemma of Section 3.3)."""
import itertools

import numpy as np
import pytest
from scipy.linalg import hadamard

from oracle import net, walsh
from paper_0808_0487_amd import inputs


def bitrev(x, a):
    return int(format(x, "0%db" % a)[::-1], 2)


def digitrev(x, p, a):
    d = [(x // p ** i) % p for i in range(a)]
    return int(sum(d[i] * p ** (a - 1 - i) for i in range(a)))


@pytest.mark.parametrize("a", [1, 2, 3, 4])
def test_binary_walsh_matrix_is_sylvester_hadamard_with_bit_reversal(a):
    """p = 2: pwal_k(X / 2^a) = H[k, bitrev(X)] with H the Sylvester-Hadamard
    matrix (scipy), i.e. the Walsh-Paley ordering."""
    W = walsh.walsh_matrix(2, a)
    H = hadamard(2 ** a)
    perm = [bitrev(X, a) for X in range(2 ** a)]
    assert np.allclose(W.real, H[:, perm]) and np.allclose(W.imag, 0)


@pytest.mark.parametrize("p,a", [(3, 2), (5, 2), (3, 3)])
def test_walsh_matrix_is_kronecker_of_dft_with_digit_reversal(p, a):
    """wal_k(X/p^a) = prod_i omega^(k_i x_{i+1}): the Kronecker power of the
    p-point DFT matrix (numpy), columns in digit-reversed order; unitary up
    to p^a."""
    F = np.exp(2j * np.pi * np.outer(np.arange(p), np.arange(p)) / p)
    K = np.array([[1.0]])
    for _ in range(a):
        K = np.kron(F, K)        # k digit i <-> row digit i (LSB first)
    W = walsh.walsh_matrix(p, a)
    perm = [digitrev(X, p, a) for X in range(p ** a)]
    assert np.allclose(W, K[:, perm])
    assert np.allclose(W @ W.conj().T, p ** a * np.eye(p ** a))


def test_nu_values():
    assert walsh.nu(2, 0) == 0 and walsh.nu(2, 1) == 1 and walsh.nu(2, 2) == 2
    assert walsh.nu(2, 3) == 2 and walsh.nu(2, 8) == 4
    assert walsh.nu(3, 2) == 1 and walsh.nu(3, 3) == 2 and walsh.nu(3, 9) == 3


CASES = [(2, 3, 2, 1), (2, 4, 2, 2), (3, 2, 2, 3), (5, 1, 2, 4), (2, 2, 3, 5)]


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_representatives_cover_every_coset_and_start_at_zero(p, m, s, seed):
    C = inputs.upper_triangular_generators(p, m, s, seed)
    reps = walsh.representatives(p, m, C)
    assert len(reps) == p ** m
    assert reps[0] == (0,) * s
    for h, k in enumerate(reps):
        assert walsh.coset_label(p, m, C, k) == h


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_character_property_identifies_the_dual_net(p, m, s, seed):
    """Eq. (char): p^-m sum_x wal_k(x) = 1 if k in D(C) else 0, for every k in
    a box reaching past p^m."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    ydig = net.output_digits(p, m, C, np.arange(N))
    for k in itertools.product(range(min(p * N, 12)), repeat=s):
        avg = np.mean(walsh.wal_multi(p, k, ydig))
        expect = 1.0 if walsh.coset_label(p, m, C, k) == 0 else 0.0
        assert abs(avg - expect) < 1e-12


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_dwt_definition_equals_index_identity_form(p, m, s, seed):
    """The definition with the K(C) representatives, with another coset
    member, and the phase form omega^(-n.h) all agree (Section 2.2)."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    f = np.random.default_rng(seed).standard_normal(N)
    reps = walsh.representatives(p, m, C)
    a = walsh.dwt_direct(p, m, C, f, reps=reps)
    b = walsh.dwt_direct(p, m, C, f)
    c = walsh.dwt_phase(p, m, f, range(N))
    assert np.allclose(a, b, atol=1e-12) and np.allclose(a, c, atol=1e-12)


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_walsh_function_maps_to_delta_and_aliases(p, m, s, seed):
    """f = wal_k on the net gives f~ = delta at C.k; k (+) l with l in the
    dual net gives the same delta (Eqs. (char), (eq_aliasing))."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    ydig = net.output_digits(p, m, C, np.arange(N))
    dual = [l for l in walsh.dual_net_box(p, m, C, min(p * N, 9)) if any(l)]
    g = np.random.default_rng(seed)
    for _ in range(5):
        k = tuple(int(v) for v in g.integers(0, N, s))
        h = walsh.coset_label(p, m, C, k)
        for kk in [k] + [tuple(walsh_digit_add(p, a, b) for a, b in zip(k, l)) for l in dual[:3]]:
            f = walsh.wal_multi(p, kk, ydig)
            ft = walsh.dwt_phase(p, m, f, range(N))
            ref = np.zeros(N)
            ref[h] = 1.0
            assert np.allclose(ft, ref, atol=1e-12)


def walsh_digit_add(p, a, b):
    out, q = 0, 1
    while a or b:
        out += ((a % p + b % p) % p) * q
        a //= p
        b //= p
        q *= p
    return out


@pytest.mark.parametrize("p,m,s,seed", CASES + [(2, 7, 3, 6), (3, 4, 2, 7)])
def test_parseval_and_inverse_lemma(p, m, s, seed):
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    f = np.random.default_rng(seed).standard_normal(N)
    ft = walsh.dwt_direct(p, m, C, f)
    assert np.isclose(np.sum(np.abs(ft) ** 2), np.sum(f ** 2) / N)
    back = walsh.idwt_direct(p, m, C, ft)
    assert np.allclose(back, f, atol=1e-11)


@pytest.mark.parametrize("m", [3, 6, 8])
def test_one_dimensional_identity_net_is_the_hadamard_transform(m):
    """s = 1, C = I, p = 2: f~ = H f / N with H the Sylvester-Hadamard matrix."""
    p, N = 2, 2 ** m
    C = inputs.identity_generators(p, m, 1)
    f = np.random.default_rng(m).standard_normal(N)
    assert np.allclose(walsh.dwt_direct(p, m, C, f), hadamard(N) @ f / N, atol=1e-12)


@pytest.mark.parametrize("p,m", [(3, 3), (5, 2), (3, 5)])
def test_one_dimensional_identity_net_is_the_digit_tensor_fft(p, m):
    """s = 1, C = I, p odd: f~ is numpy's m-dimensional FFT over the digit
    tensor (n_0 fastest), divided by p^m."""
    N = p ** m
    C = inputs.identity_generators(p, m, 1)
    f = np.random.default_rng(m).standard_normal(N)
    ref = np.fft.fftn(f.reshape([p] * m, order="F")).reshape(N, order="F") / N
    assert np.allclose(walsh.dwt_direct(p, m, C, f), ref, atol=1e-12)


def test_integer_data_exact_for_p2():
    p, m, s = 2, 6, 3
    C = inputs.upper_triangular_generators(p, m, s, 9)
    f = inputs.uniform_int32(2 ** m, -1000, 1000, 9)
    a = walsh.dwt_direct(p, m, C, f)
    b = walsh.dwt_phase(p, m, f, range(2 ** m))
    assert a.dtype == np.int64 and np.array_equal(a, b)
    ref = hadamard(2 ** m).astype(np.int64) @ f.astype(np.int64)
    assert np.array_equal(b, ref)
    assert np.array_equal(walsh.idwt_phase(p, m, b, range(2 ** m)), (2 ** m) * f.astype(np.int64))
