/* Fast CPU reference for the discrete Walsh transform on digital nets
 * (Liu, Dick and Hickernell, "A Multivariate Fast Discrete Walsh Transform
 * with an Application to Function Interpolation").
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the bench's CPU
 * baseline load this library.  It shares no code with the HIP library (no
 * headers, tables or helpers) and is built by gcc alone.
 *
 * Where the Python oracle writes out the plain definitions (O(N^2) sums,
 * dense solves, direct double sums), this file runs the paper's fast
 * algorithms as plain loops in float64 / int64, parallel over independent
 * sums with OpenMP, so that every output of a full-size configuration can be
 * compared and the CPU side can be timed at full size.  It is pinned to the
 * Python oracle at small sizes (tests/test_oracle_fast.py).
 *
 *   o2_net          the net's integer coordinates (Definition of a digital
 *                   net: y = C_j n mod p, X = sum_r y_r p^(m-r))
 *   o2_sample       the product and exponential test functions at the net
 *   o2_fwt          Algorithm 1 (forward, divided by p^m) and Algorithm 2
 *                   (inverse) over the m index digits, stage by stage
 *   o2_kernel_cols  K(x_n, 0), U_d = R_d(x_n, 0) - 1 and Q_j = e_j(gamma^2 R')
 *                   from the closed forms of K' and R' (Section 4)
 *   o2_variances    truncation and superposition variances of the spline
 *                   through the kernel spectra (Section 4, Eq. (sig2sfu)
 *                   summed over u, and Eq. (varSf))
 *   o2_spline_eval  Sf(q) = sum_n c_n K(q, x_n) (Section 3.2) at D-digit
 *                   queries
 *
 * Readings shared with the rest of the build: U_d sums over the non-empty
 * u only (the constant term of the polynomial in beta^2 vanishes); K~ is
 * clamped below at 1e-300 and rho = U~/K~^2 to [0, 1] (exact invariants,
 * enforced against rounding).
 *
 * Error returns: -1 for an invalid argument, -2 for a failed allocation.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O2_PMAX 64

static int64_t ipow64(int p, int m) {
  int64_t r = 1;
  for (int i = 0; i < m; ++i) r *= p;
  return r;
}

static int valid_pm(int p, int m) {
  if (p < 2 || p > O2_PMAX || m < 1) return 0;
  for (int d = 2; d * d <= p; ++d)
    if (p % d == 0) return 0;
  /* N = p^m must fit comfortably in int64 */
  double lg = m * log((double)p) / log(2.0);
  return lg <= 40.0;
}

int o2_threads(void) { return omp_get_max_threads(); }

void o2_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

/* ------------------------------------------------------------------ net */
/* X[j * count + i] = integer coordinate j of point n0 + i.  C holds s
 * matrices, C[(j m + r) m + c] = row r + 1 (output digit y_{r+1}), column c
 * (input digit n_c), entries in [0, p). */
int o2_net(int p, int m, int s, const int32_t* C, int64_t n0, int64_t count, int64_t* X) {
  if (!valid_pm(p, m) || s < 1 || count < 0 || n0 < 0 || n0 + count > ipow64(p, m)) return -1;
  if (p == 2) {
    /* Over Z_2, y = C n is the sum (XOR) of the columns c with n_c = 1. */
    int64_t* col = (int64_t*)malloc(sizeof(int64_t) * (size_t)s * m);
    if (!col) return -2;
    for (int j = 0; j < s; ++j)
      for (int c = 0; c < m; ++c) {
        int64_t v = 0;
        for (int r = 0; r < m; ++r) v = 2 * v + (C[((int64_t)j * m + r) * m + c] & 1);
        col[j * m + c] = v;
      }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
      const int64_t n = n0 + i;
      for (int j = 0; j < s; ++j) {
        int64_t x = 0;
        for (int c = 0; c < m; ++c)
          if ((n >> c) & 1) x ^= col[j * m + c];
        X[(int64_t)j * count + i] = x;
      }
    }
    free(col);
    return 0;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    int nd[64];
    int64_t q = n0 + i;
    for (int c = 0; c < m; ++c) {
      nd[c] = (int)(q % p);
      q /= p;
    }
    for (int j = 0; j < s; ++j) {
      int64_t x = 0;
      for (int r = 0; r < m; ++r) {
        const int32_t* row = C + ((int64_t)j * m + r) * m;
        int64_t acc = 0;
        for (int c = 0; c < m; ++c) acc += (int64_t)row[c] * nd[c];
        x = x * p + acc % p;
      }
      X[(int64_t)j * count + i] = x;
    }
  }
  return 0;
}

/* ------------------------------------------------------------- samples */
/* f(x_n), x_{n,j} = X_{j,n} / p^m, for two test-function families:
 * kind 0, product: prod_j (1 + a_j (x_j - 1/2));  kind 1, exp:
 * exp(-sum_j a_j x_j^2). */
int o2_sample(int kind, int p, int m, int s, const double* a, const int64_t* X, int64_t N, double* f) {
  if (!valid_pm(p, m) || s < 1 || N < 0 || (kind != 0 && kind != 1)) return -1;
  const double inv = 1.0 / (double)ipow64(p, m);
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double v = kind == 0 ? 1.0 : 0.0;
    for (int j = 0; j < s; ++j) {
      const double x = (double)X[(int64_t)j * N + n] * inv;
      if (kind == 0)
        v *= 1.0 + a[j] * (x - 0.5);
      else
        v += a[j] * x * x;
    }
    f[n] = kind == 0 ? v : exp(-v);
  }
  return 0;
}

/* ------------------------------------------------------------ transform */
/* One column of N = p^m values, in place.  Stage r (r = 1..m) replaces the
 * index digit in position r - 1 (weight p^(r-1)) by its frequency digit:
 * G_r(.., h_{r-1}, ..) = sum_{n_{r-1}} w^(-+ n_{r-1} h_{r-1}) G_{r-1}(.., n_{r-1}, ..),
 * w = exp(2 pi i / p), minus for Algorithm 1, plus for Algorithm 2.  The
 * result sits at the natural index h = sum h_i p^i.  im == NULL: real data,
 * p = 2 only. */
static void fwt_column(int p, int m, double* re, double* im, int inverse, const double* cw, const double* sw) {
  const int64_t N = ipow64(p, m);
  const double sgn = inverse ? 1.0 : -1.0;
  int64_t S = 1;
  for (int r = 1; r <= m; ++r) {
    const int64_t groups = N / p;
    if (p == 2) {
#pragma omp parallel for schedule(static)
      for (int64_t g = 0; g < groups; ++g) {
        const int64_t lo = g % S, hi = g / S;
        const int64_t a = hi * 2 * S + lo, b = a + S;
        const double ar = re[a], br = re[b];
        re[a] = ar + br;
        re[b] = ar - br;
        if (im) {
          const double ai = im[a], bi = im[b];
          im[a] = ai + bi;
          im[b] = ai - bi;
        }
      }
    } else {
#pragma omp parallel for schedule(static)
      for (int64_t g = 0; g < groups; ++g) {
        double vr[O2_PMAX], vi[O2_PMAX];
        const int64_t lo = g % S, hi = g / S;
        const int64_t base = hi * p * S + lo;
        for (int t = 0; t < p; ++t) {
          vr[t] = re[base + t * S];
          vi[t] = im[base + t * S];
        }
        for (int h = 0; h < p; ++h) {
          double accr = 0.0, acci = 0.0;
          for (int t = 0; t < p; ++t) {
            const int e = (t * h) % p;
            const double c = cw[e], sn = sgn * sw[e];
            accr += vr[t] * c - vi[t] * sn;
            acci += vr[t] * sn + vi[t] * c;
          }
          re[base + h * S] = accr;
          im[base + h * S] = acci;
        }
      }
    }
    S *= p;
  }
  if (!inverse) {
    const double inv = 1.0 / (double)N;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      re[i] *= inv;
      if (im) im[i] *= inv;
    }
  }
}

static void roots(int p, double* cw, double* sw) {
  const double pi = 3.14159265358979323846;
  for (int e = 0; e < p; ++e) {
    cw[e] = e == 0 ? 1.0 : cos(2.0 * pi * e / p);
    sw[e] = e == 0 ? 0.0 : sin(2.0 * pi * e / p);
  }
}

/* ncols columns of N values each (column c at re + c N, im + c N), in
 * place.  Forward (inverse == 0): Algorithm 1, divided by p^m.  Inverse:
 * Algorithm 2, not divided.  im may be NULL only for p = 2. */
int o2_fwt(int p, int m, int64_t ncols, double* re, double* im, int inverse) {
  if (!valid_pm(p, m) || ncols < 0 || !re || (!im && p != 2)) return -1;
  double cw[O2_PMAX], sw[O2_PMAX];
  roots(p, cw, sw);
  const int64_t N = ipow64(p, m);
  for (int64_t c = 0; c < ncols; ++c) fwt_column(p, m, re + c * N, im ? im + c * N : NULL, inverse, cw, sw);
  return 0;
}

/* 1 when every entry of a[0..n) lies in [0, lim). */
static int in_range(const int64_t* a, int64_t n, int64_t lim) {
  int ok = 1;
#pragma omp parallel for schedule(static) reduction(& : ok)
  for (int64_t i = 0; i < n; ++i) ok &= a[i] >= 0 && a[i] < lim;
  return ok;
}

/* --------------------------------------------------------- kernel data */
/* Position (1-based, most significant first) of the first non-zero base-p
 * digit of the D-digit integer z; 0 for z = 0.  For p = 2 the position of
 * the highest set bit. */
static int first_nonzero_digit(int p, int D, int64_t z) {
  if (z == 0) return 0;
  if (p == 2) return D - (63 - __builtin_clzll((unsigned long long)z));
  int i = D;
  while (z >= p) {
    z /= p;
    --i;
  }
  return i;
}

/* K'(z, 0) and R'(z, 0) for z whose first non-zero digit is z_i (Section 4,
 * the short forms after the Walsh series of K' and R'); i = 0 is z = 0,
 * where the series sum to K'(0, 0) = 1 and R'(0, 0) = (p^a - p)^2 /
 * ((p - 1)(p^2a - p)). */
static double kprime(int p, double alpha, int i) {
  if (i == 0) return 1.0;
  return 1.0 - pow((double)p, i * (1.0 - alpha)) * (pow((double)p, alpha) - 1.0) / (p - 1.0);
}

static double rprime(int p, double alpha, int i) {
  const double pa = pow((double)p, alpha), p2a = pow((double)p, 2.0 * alpha);
  const double A = (pa - p) * (pa - p) / ((p - 1.0) * (p2a - p));
  if (i == 0) return A;
  return A * (1.0 - pow((double)p, i * (1.0 - 2.0 * alpha)) * (p2a - 1.0) / (p - 1.0));
}

/* Per-coordinate tables over the first-digit index i = 0..m:
 * kt[j (m+1) + i] = 1 + gamma_j K'(i), rt[j (m+1) + i] = gamma_j^2 R'(i). */
static int tables(int p, int m, int s, double alpha, const double* gamma, double** kt, double** rt) {
  *kt = (double*)malloc(sizeof(double) * (size_t)s * (m + 1));
  *rt = (double*)malloc(sizeof(double) * (size_t)s * (m + 1));
  if (!*kt || !*rt) {
    free(*kt), free(*rt);
    return -2;
  }
  for (int j = 0; j < s; ++j)
    for (int i = 0; i <= m; ++i) {
      (*kt)[j * (m + 1) + i] = 1.0 + gamma[j] * kprime(p, alpha, i);
      (*rt)[j * (m + 1) + i] = gamma[j] * gamma[j] * rprime(p, alpha, i);
    }
  return 0;
}

/* For the N points with coordinates X (s x N, m-digit integers):
 *   K[n]        = prod_j [1 + gamma_j K'(x_{n,j}, 0)]                 (N)
 *   U[d-1][n]   = prod_{j<=d} [1 + gamma_j^2 R'(x_{n,j}, 0)] - 1, d = 1..s (s x N, may be NULL)
 *   Q[j-1][n]   = e_j(gamma_1^2 R'_1, ..., gamma_s^2 R'_s), j = 1..s   (s x N, may be NULL)
 * e_j by the expansion prod_l (1 + t v_l) = sum_j e_j t^j. */
int o2_kernel_cols(int p, int m, int s, double alpha, const double* gamma, const int64_t* X, int64_t N, double* K,
                   double* U, double* Q) {
  if (!valid_pm(p, m) || s < 1 || s > 256 || N < 0 || !(alpha > 1.0)) return -1;
  if (!in_range(X, (int64_t)s * N, ipow64(p, m))) return -1;
  double *kt, *rt;
  if (tables(p, m, s, alpha, gamma, &kt, &rt)) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double e[257];
    double k = 1.0, r = 1.0;
    e[0] = 1.0;
    for (int j = 1; j <= s; ++j) e[j] = 0.0;
    for (int j = 0; j < s; ++j) {
      const int i = first_nonzero_digit(p, m, X[(int64_t)j * N + n]);
      k *= kt[j * (m + 1) + i];
      const double v = rt[j * (m + 1) + i];
      r *= 1.0 + v;
      if (U) U[(int64_t)j * N + n] = r - 1.0;
      for (int t = j + 1; t >= 1; --t) e[t] += v * e[t - 1];
    }
    K[n] = k;
    if (Q)
      for (int j = 1; j <= s; ++j) Q[(int64_t)(j - 1) * N + n] = e[j];
  }
  free(kt), free(rt);
  return 0;
}

/* ------------------------------------------------------------ variances */
/* Truncation and superposition variances of the spline of f (Section 4):
 *   var_trc[d] = sum_h |f~(h)|^2 rho(U~_d)(h),   var_sup[d] = var_sup[d-1] + sum_h |f~(h)|^2 rho(Q~_d)(h),
 * rho(g~) = clamp(g~ / K~^2, 0, 1), all spectra by Algorithm 1 (divided by
 * p^m), d = 1..s; var_trc[0] = var_sup[0] = 0.  ft_re / ft_im: the forward
 * transform of f (ft_im NULL for p = 2).  Memory: s + 3 columns of N
 * doubles (2 s + 4 for p odd). */
int o2_variances(int p, int m, int s, double alpha, const double* gamma, const int64_t* X, const double* ft_re,
                 const double* ft_im, double* var_trc, double* var_sup) {
  if (!valid_pm(p, m) || s < 1 || s > 256 || !(alpha > 1.0) || (!ft_im && p != 2)) return -1;
  const int64_t N = ipow64(p, m);
  if (!in_range(X, (int64_t)s * N, N)) return -1;
  const int cplx = p != 2;
  double* K = (double*)calloc((size_t)N, sizeof(double));
  double* Q = (double*)calloc((size_t)N * s, sizeof(double));
  double* U = (double*)calloc((size_t)N, sizeof(double));
  double* P = (double*)malloc(sizeof(double) * (size_t)N);
  double* Ki = cplx ? (double*)calloc((size_t)N, sizeof(double)) : NULL;
  double* Ui = cplx ? (double*)calloc((size_t)N, sizeof(double)) : NULL;
  double* f2 = (double*)malloc(sizeof(double) * (size_t)N);
  double *kt = NULL, *rt = NULL;
  if (!K || !Q || !U || !P || !f2 || (cplx && (!Ki || !Ui)) || tables(p, m, s, alpha, gamma, &kt, &rt)) {
    free(K), free(Q), free(U), free(P), free(Ki), free(Ui), free(f2);
    return -2;
  }
  double cw[O2_PMAX], sw[O2_PMAX];
  roots(p, cw, sw);
  o2_kernel_cols(p, m, s, alpha, gamma, X, N, K, NULL, Q);
  fwt_column(p, m, K, Ki, 0, cw, sw);
#pragma omp parallel for schedule(static)
  for (int64_t h = 0; h < N; ++h) {
    const double a = ft_re[h], b = ft_im ? ft_im[h] : 0.0;
    f2[h] = a * a + b * b;
    P[h] = 1.0;
  }
  var_trc[0] = var_sup[0] = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int d = 1; d <= s; ++d) {
      if (pass == 0) {
        /* U_d = R_d - 1 from the running product over coordinates 1..d */
        const double* rj = rt + (d - 1) * (m + 1);
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
          P[n] *= 1.0 + rj[first_nonzero_digit(p, m, X[(int64_t)(d - 1) * N + n])];
          U[n] = P[n] - 1.0;
          if (cplx) Ui[n] = 0.0;
        }
      } else {
        memcpy(U, Q + (int64_t)(d - 1) * N, sizeof(double) * (size_t)N);
        if (cplx) memset(Ui, 0, sizeof(double) * (size_t)N);
      }
      fwt_column(p, m, U, Ui, 0, cw, sw);
      double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
      for (int64_t h = 0; h < N; ++h) {
        /* the spectra of real data that take equal values at x and its
         * digit-wise negative are real: only the real parts enter */
        const double k = fmax(K[h], 1e-300);
        double rho = U[h] / (k * k);
        rho = rho < 0.0 ? 0.0 : (rho > 1.0 ? 1.0 : rho);
        acc += f2[h] * rho;
      }
      if (pass == 0)
        var_trc[d] = acc;
      else
        var_sup[d] = var_sup[d - 1] + acc;
    }
  }
  free(K), free(Q), free(U), free(P), free(Ki), free(Ui), free(f2), free(kt), free(rt);
  return 0;
}

/* Spline coefficients (Section 3.2, Eq. (splinecoef)): c~ = f~ / (p^m K~)
 * with K~ the spectrum of K(x_n, 0) (clamped below at 1e-300), then
 * Algorithm 2.  ft_re / ft_im: forward transform of f (ft_im NULL for p = 2);
 * c: the real parts of the N coefficients. */
int o2_spline_coef(int p, int m, int s, double alpha, const double* gamma, const int64_t* X, const double* ft_re,
                   const double* ft_im, double* c) {
  if (!valid_pm(p, m) || s < 1 || s > 256 || !(alpha > 1.0) || (!ft_im && p != 2)) return -1;
  const int64_t N = ipow64(p, m);
  if (!in_range(X, (int64_t)s * N, N)) return -1;
  const int cplx = p != 2;
  double* K = (double*)calloc((size_t)N, sizeof(double));
  double* Ki = cplx ? (double*)calloc((size_t)N, sizeof(double)) : NULL;
  double* ci = cplx ? (double*)calloc((size_t)N, sizeof(double)) : NULL;
  if (!K || (cplx && (!Ki || !ci))) {
    free(K), free(Ki), free(ci);
    return -2;
  }
  double cw[O2_PMAX], sw[O2_PMAX];
  roots(p, cw, sw);
  o2_kernel_cols(p, m, s, alpha, gamma, X, N, K, NULL, NULL);
  fwt_column(p, m, K, Ki, 0, cw, sw);
#pragma omp parallel for schedule(static)
  for (int64_t h = 0; h < N; ++h) {
    const double den = (double)N * fmax(K[h], 1e-300);
    c[h] = ft_re[h] / den;
    if (cplx) ci[h] = ft_im[h] / den;
  }
  fwt_column(p, m, c, ci, 1, cw, sw);
  free(K), free(Ki), free(ci);
  return 0;
}

/* ------------------------------------------------------------ evaluation */
/* Sf(q) = sum_n c_n K(q, x_n) for nq queries given as D-digit integers
 * (Q: s x nq); the net's m-digit coordinates are lifted to D digits.  K(q, x)
 * = prod_j [1 + gamma_j K'(q_j (-) x_j, 0)], where the first non-zero digit
 * of q_j (-) x_j is the first digit in which q_j and x_j differ. */
int o2_spline_eval(int p, int m, int s, double alpha, const double* gamma, const int64_t* X, const double* c,
                   int64_t nq, const int64_t* Q, int D, double* out) {
  if (!valid_pm(p, m) || s < 1 || nq < 0 || D < m || !(alpha > 1.0)) return -1;
  if (D * log((double)p) / log(2.0) > 62.0) return -1;
  const int64_t N = ipow64(p, m), lift = ipow64(p, D - m);
  if (!in_range(X, (int64_t)s * N, N) || !in_range(Q, (int64_t)s * nq, ipow64(p, D))) return -1;
  double *kt, *rt;
  if (tables(p, D, s, alpha, gamma, &kt, &rt)) return -2;
  int64_t pw[64];
  pw[0] = 1;
  for (int k = 1; k <= D; ++k) pw[k] = pw[k - 1] * p;
  for (int64_t t = 0; t < nq; ++t) {
    double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
    for (int64_t n = 0; n < N; ++n) {
      double k = 1.0;
      for (int j = 0; j < s; ++j) {
        const int64_t a = Q[(int64_t)j * nq + t], b = X[(int64_t)j * N + n] * lift;
        /* first differing digit, most significant first: the first position
         * whose leading digits differ */
        int i = 0;
        if (a != b) {
          if (p == 2) {
            i = D - (63 - __builtin_clzll((unsigned long long)(a ^ b)));
          } else {
            for (int pos = 1; pos <= D; ++pos)
              if (a / pw[D - pos] != b / pw[D - pos]) {
                i = pos;
                break;
              }
          }
        }
        k *= kt[j * (D + 1) + i];
      }
      acc += c[n] * k;
    }
    out[t] = acc;
  }
  free(kt), free(rt);
  return 0;
}
