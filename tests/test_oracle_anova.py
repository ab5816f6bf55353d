"""Pins for oracle.anova: effective dimensions and variances (Section 4)
against the analytic values printed in Tables 1 and 2 (Section 5.2), a
closed form for kernel sections, and the spectral route (Eq. (sig2sfu))."""
import json
import os

import numpy as np
import pytest

from oracle import anova, kernel, net
from paper_0808_0487_amd import inputs
from tests._libdwt import lib_dwt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_table2_exact.json")


def test_tables_1_and_2_exact_columns():
    rows = json.load(open(GOLDEN))["rows"]
    for row in rows:
        a = inputs.family_params("wangfang", row["s"], a=row["a"])
        v = anova.wangfang_component_variance(a)
        trc, sup, total = anova.product_anova(v)
        assert round(total, 4) == pytest.approx(row["var_f"], abs=1e-12), row
        assert anova.effective_dims(trc, sup, total) == (row["d_trc"], row["d_sup"]), row


def test_printed_sup_condition_with_trc_would_contradict_table_1():
    """Reading the d_sup condition literally (sigma^2_trc(d-1) < ...) cannot
    give Table 1's d_sup = 3 for a_k = 1, s = 10: trc(2) is far below the
    threshold, so the reading with sigma^2_sup is the consistent one."""
    v = anova.wangfang_component_variance(np.ones(10))
    trc, sup, total = anova.product_anova(v)
    assert trc[2] < 0.99 * total <= sup[3] and sup[2] < 0.99 * total


def test_small_configuration_analytic_values():
    """prod_j (1 + 0.5 (x_j - 1/2)), s = 4: component variance 1/48."""
    trc, sup, total = anova.product_anova(anova.product_family_component_variance(np.full(4, 0.5)))
    assert np.isclose(total, (1 + 1 / 48) ** 4 - 1)
    assert round(total, 6) == 0.085974
    assert anova.effective_dims(trc, sup, total) == (4, 2)


def test_esp_against_brute_force_subsets():
    import itertools
    v = np.random.default_rng(0).uniform(0, 1, 6)
    e = anova.esp(list(v))
    for j in range(7):
        brute = sum(np.prod([v[i] for i in u]) for u in itertools.combinations(range(6), j))
        assert np.isclose(e[j], brute)


CASES = [(2, 6, 3, 1), (2, 7, 4, 2), (3, 4, 3, 3), (5, 3, 3, 4)]


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_kernel_section_variances_closed_form(p, m, s, seed):
    """Sf = K(., y): sigma^2_trc(d) = prod_{j<=d}(1 + gamma_j^2 R'(0)) - 1 and
    sigma^2_sup(d) = sum_{j<=d} e_j(gamma_1^2 R'(0), ...), from the product
    form of K and int K' = 0."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    X = net.net_int(p, m, C)
    gam = inputs.kernel_weights(s, q=-1.0, beta=0.7)
    alpha = 1.7
    c = np.zeros(p ** m)
    c[3] = 1.0
    trc, sup = anova.variances_direct(p, m, alpha, gam, X, c)
    r0 = gam ** 2 * kernel.rprime_closed(p, alpha, 0)
    e = anova.esp(list(r0))
    for d in range(1, s + 1):
        assert np.isclose(trc[d], np.prod(1 + r0[:d]) - 1)
        assert np.isclose(sup[d], sum(e[1:d + 1]))


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_direct_double_sum_equals_spectral_route(p, m, s, seed):
    """Eq. (sig2sfu) summed over u in 1:d (Section 4):
    sigma^2_trc(d) = p^2m sum_h |c~(h)|^2 R~_d(h), with R_d - 1 in place of
    R_d (no constant term), and likewise with the symmetric-polynomial
    kernels for sigma^2_sup.  DWTs by numpy FFT."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    X = net.net_int(p, m, C)
    gam = inputs.kernel_weights(s)
    alpha = 2.0
    x = X / N
    f = np.exp(-np.sum(0.5 ** np.arange(1, s + 1)[:, None] * x ** 2, axis=0))
    c = kernel.spline_coef_dense(p, m, alpha, gam, X, f)
    trc, sup = anova.variances_direct(p, m, alpha, gam, X, c)
    ct2 = np.abs(lib_dwt(p, m, c)) ** 2
    i = [kernel.first_diff_digit(p, m, X[j], 0) for j in range(s)]
    r = [gam[j] ** 2 * kernel.rprime_closed(p, alpha, i[j]) for j in range(s)]
    prod = np.ones(N)
    e = anova.esp(r)
    acc = 0.0
    for d in range(1, s + 1):
        prod = prod * (1 + r[d - 1])
        Rt = lib_dwt(p, m, prod - 1.0)
        assert np.max(np.abs(Rt.imag)) < 1e-12
        assert np.isclose(trc[d], N * N * np.sum(ct2 * Rt.real), rtol=1e-9)
        acc += N * N * np.sum(ct2 * lib_dwt(p, m, e[d]).real)
        assert np.isclose(sup[d], acc, rtol=1e-9)


@pytest.mark.parametrize("p,m,s,seed", CASES)
def test_variance_chain_and_qmc_bound(p, m, s, seed):
    """0 <= trc(d) <= sup(d) <= total, both monotone (Section 4); and the bound
    of Section 5.2 in its exact form: the spline variance without the h = 0
    bin is at most sigma^2_QMC(f)."""
    C = inputs.upper_triangular_generators(p, m, s, seed)
    N = p ** m
    X = net.net_int(p, m, C)
    gam = inputs.kernel_weights(s)
    f = np.random.default_rng(seed).standard_normal(N)
    c = kernel.spline_coef_dense(p, m, 2.0, gam, X, f)
    trc, sup = anova.variances_direct(p, m, 2.0, gam, X, c)
    tol = 1e-12 * abs(trc[s])
    assert np.all(np.diff(trc) >= -tol) and np.all(np.diff(sup) >= -tol)
    assert np.all(trc <= sup + tol) and np.isclose(trc[s], sup[s])
    ft = lib_dwt(p, m, f)
    Kt = lib_dwt(p, m, kernel.kernel_data(p, m, 2.0, gam, X)).real
    i = [kernel.first_diff_digit(p, m, X[j], 0) for j in range(s)]
    R = np.prod([1 + gam[j] ** 2 * kernel.rprime_closed(p, 2.0, i[j]) for j in range(s)], axis=0)
    Rt = lib_dwt(p, m, R - 1.0).real
    rho = Rt / Kt ** 2
    assert np.all(rho >= -1e-12) and np.all(rho <= 1 + 1e-9)
    nz = np.sum(np.abs(ft[1:]) ** 2 * rho[1:])
    assert nz <= anova.var_qmc(f) * (1 + 1e-12)
    assert np.isclose(trc[s], nz + np.abs(ft[0]) ** 2 * rho[0], rtol=1e-9)
