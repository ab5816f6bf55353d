"""ANOVA variances of the spline and effective dimensions (Section 4), plus
the analytic ANOVA of product-form test functions used in Section 5.2.  Test
infrastructure only; see the package docstring.

Readings of the paper taken here (listed with reasons in the design notes):
  * the truncation kernel R_d sums over the non-empty u in 1:d only -- the
    constant u = {} carries no variance (Section 4, the vanishing constant
    term of the polynomial in beta^2);
  * the superposition dimension condition reads sigma^2_sup(d_sup - 1) <
    0.99 sigma^2 <= sigma^2_sup(d_sup); the printed sigma^2_trc in the first
    inequality is a typo (the analytic values of Table 1 need sigma^2_sup);
  * the coefficient Q~(k, j) carries the weights gamma~_u^2 inside the sum
    over |u| = j.
"""
import numpy as np

from .kernel import first_diff_digit, rprime_closed, weights_vec


def esp(values):
    """Elementary symmetric polynomials e_0..e_s of the list ``values``
    (arrays allowed) from the expansion prod_l (1 + t v_l) = sum_j t^j e_j."""
    s = len(values)
    e = [np.ones_like(np.asarray(values[0], dtype=np.float64))] + \
        [np.zeros_like(np.asarray(values[0], dtype=np.float64)) for _ in range(s)]
    for l, v in enumerate(values):
        for j in range(l + 1, 0, -1):
            e[j] = e[j] + v * e[j - 1]
    return e


def rprime_matrix(p, m, alpha, gamma, X):
    """gamma_j^2 R'(x_{n,j} (-) x_{v,j}, 0) for every coordinate and pair,
    shape (s, N, N)."""
    X = np.asarray(X, dtype=np.int64)
    s = X.shape[0]
    g = weights_vec(gamma, s)
    out = np.empty((s, X.shape[1], X.shape[1]))
    for j in range(s):
        i = first_diff_digit(p, m, X[j][:, None], X[j][None, :])
        out[j] = g[j] ** 2 * rprime_closed(p, alpha, i)
    return out


def variances_direct(p, m, alpha, gamma, X, c):
    """Truncation and superposition variances of the spline Sf = sum_n c_n
    K(., x_n) by the direct double sums of Section 4:
        sigma^2((Sf)_u) = gamma_u^2 sum_{n,v} c_n c_v R_u(x_n, x_v),
        sigma^2_trc(d)  = sum_{n,v} c_n c_v [prod_{j<=d}(1 + gamma_j^2 R'_j) - 1],
        sigma^2_sup(d)  = sum_{j<=d} sum_{n,v} c_n c_v e_j(gamma_1^2 R'_1, ...).
    Returns (var_trc[0..s], var_sup[0..s]); var_trc[s] = var_sup[s] = sigma^2(Sf)."""
    c = np.asarray(c, dtype=np.float64)
    r = rprime_matrix(p, m, alpha, gamma, X)
    s = r.shape[0]
    cc = np.outer(c, c)
    var_trc = np.zeros(s + 1)
    prod = np.ones_like(r[0])
    for d in range(1, s + 1):
        prod = prod * (1.0 + r[d - 1])
        var_trc[d] = float(np.sum(cc * (prod - 1.0)))
    e = esp([r[j] for j in range(s)])
    var_sup = np.zeros(s + 1)
    for d in range(1, s + 1):
        var_sup[d] = var_sup[d - 1] + float(np.sum(cc * e[d]))
    return var_trc, var_sup


def effective_dims(var_trc, var_sup, total=None, threshold=0.99):
    """d_trc = min{d : sigma^2_trc(d) >= 0.99 sigma^2},
    d_sup = min{d : sigma^2_sup(d) >= 0.99 sigma^2} (Section 4)."""
    var_trc = np.asarray(var_trc)
    var_sup = np.asarray(var_sup)
    s = len(var_trc) - 1
    if total is None:
        total = var_trc[s]
    target = threshold * total
    d_trc = next((d for d in range(s + 1) if var_trc[d] >= target), s)
    d_sup = next((d for d in range(s + 1) if var_sup[d] >= target), s)
    return d_trc, d_sup


def var_qmc(f):
    """sigma^2_QMC(f) = N^-1 sum f^2 - (N^-1 sum f)^2 (Section 5.2)."""
    f = np.asarray(f, dtype=np.float64)
    return float(np.mean(f * f) - np.mean(f) ** 2)


# ------------------------------------------------ analytic product functions
def product_anova(v):
    """ANOVA of f = prod_j g_j(x_j) with every g_j of mean one and variance
    v_j: sigma^2(f_u) = prod_{j in u} v_j.  Returns (var_trc[0..s],
    var_sup[0..s], total)."""
    v = np.asarray(v, dtype=np.float64)
    s = len(v)
    var_trc = np.zeros(s + 1)
    for d in range(1, s + 1):
        var_trc[d] = float(np.prod(1.0 + v[:d]) - 1.0)
    e = esp(list(v))
    var_sup = np.zeros(s + 1)
    for d in range(1, s + 1):
        var_sup[d] = var_sup[d - 1] + float(e[d])
    return var_trc, var_sup, var_trc[s]


def wangfang_component_variance(a):
    """Variance of g(x) = (|4x - 2| + a)/(1 + a) on [0,1] (Section 5.2 test
    function): |4x-2| is uniform on [0, 2], so its mean is 1 and its variance
    1/3, giving v = 1/(3 (1 + a)^2) with mean g = 1."""
    a = np.asarray(a, dtype=np.float64)
    return 1.0 / (3.0 * (1.0 + a) ** 2)


def product_family_component_variance(a):
    """Variance of g(x) = 1 + a (x - 1/2) on [0,1]: a^2/12, mean 1."""
    a = np.asarray(a, dtype=np.float64)
    return a * a / 12.0
