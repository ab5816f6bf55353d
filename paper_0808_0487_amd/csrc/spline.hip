// Walsh-kernel spline and ANOVA variances (Sections 3.2, 3.3 and 4).
//
//  * kernel data: K(x_n, 0) = prod_j [1 + gamma_j K'(x_{n,j}, 0)] and, for the
//    variances, U_d = R_d - 1 with R_d = prod_{j<=d} (1 + gamma_j^2 R'(x_{n,j}, 0))
//    and Q_j = e_j(gamma_1^2 R'_1, ..., gamma_s^2 R'_s) (elementary symmetric
//    polynomials), all in double-float.  K' and R' depend only on the index of
//    the first non-zero digit of x_{n,j}, so per-coordinate tables (computed
//    on the host in double) are indexed by a leading-zero count.
//  * their DWTs (the kernel spectra) are taken in double-float: their dynamic
//    range exceeds what float resolves (the small bins would lose all their
//    digits, and K~ must stay positive for the spectral solve).
//  * spectral solve, Eq. (splinecoef): c~ = f~ / (p^m K~), then Algorithm 2.
//  * variances, Eq. (sig2sfu) summed over u: with rho_g(h) = p^m g~(h)/K~u(h)^2
//    (K~u the unnormalised spectrum), sigma^2 = sum_h |f~(h)|^2 rho_g(h).
//    rho lies in [0, 1] exactly (0 <= g~ <= K~^2 because the Walsh
//    coefficients of R are the squares of those of K); the clamp only removes
//    rounding noise in bins where K~ is tiny.  These grouped sums are the
//    only float64 arithmetic on the device.
//  * evaluation, Sf(q) = sum_n c_n K(q, x_n), at query points given as D-digit
//    integers; the first differing digit of q and x_n is a leading-zero count
//    of their XOR (p = 2) or of their packed-digit XOR (p odd).
#include "dev_math.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace fdwt {

int fwt_run_tmp(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
                Kind out_kind, void* out, void* tmp, int batch, float scale, hipStream_t st);

constexpr int kTab = 33;  // entries per coordinate of the digit-indexed tables

__host__ __device__ static inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------- point indices
// Index t of the first non-zero digit (t = i - 1) of x_{n,j}, or m when
// x_{n,j} = 0, from the canonical integer (p = 2) or packed digits (p odd).
__device__ __forceinline__ int lead_p2(uint32_t X, int m) { return __clz(X) - (32 - m); }
__device__ __forceinline__ int lead_odd(uint64_t pk, int m) { return (__clzll(pk) - 64 + 4 * m) >> 2; }

// Same coordinate machinery as the net kernels (see net.hip).
template <int P>
__device__ __forceinline__ uint64_t addmod_packed_s(uint64_t a, uint64_t b) {
  constexpr uint64_t ones = 0x1111111111111111ull;
  uint64_t s = a + b;
  uint64_t ge = ((s + (8 - P) * ones) >> 3) & ones;
  return s - (uint64_t)P * ge;
}
template <int P>
__device__ __forceinline__ uint64_t packed_odd_s(const uint64_t* __restrict__ ptab, int j, int m, int64_t n) {
  uint64_t acc = 0;
  const uint64_t* t = ptab + (int64_t)j * m * P;
  for (int c = 0; c < m; ++c) {
    const int dgt = (int)(n % P);
    n /= P;
    acc = addmod_packed_s<P>(acc, t[c * P + dgt]);
  }
  return acc;
}

struct NetArgs {
  const uint32_t* xtab;  // p = 2
  const uint64_t* ptab;  // p odd
  int nbytes, s, m;
  int64_t N;
};

template <int P>
__device__ __forceinline__ int lead_index(const NetArgs& na, const uint32_t* lds_t0, int j, int64_t n,
                                          int64_t nw) {
  if constexpr (P == 2) {
    uint32_t u = 0;
    const uint32_t* base = na.xtab + (int64_t)j * na.nbytes * 256;
    for (int b = 1; b < na.nbytes; ++b) u ^= base[b * 256 + ((nw >> (8 * b)) & 255)];
    return lead_p2(lds_t0[j * 256 + (int)(n & 255)] ^ u, na.m);
  } else {
    (void)lds_t0;
    (void)nw;
    return lead_odd(packed_odd_s<P>(na.ptab, j, na.m, n), na.m);
  }
}

// ------------------------------------------------ kernel-data columns (DF)
// Column layout: 0 = K, 1..s = U_d (d = 1..s), s+1..2s = Q_j (j = 1..s).
// Writes columns [c0, c1) to out[(c - c0) * N + n].  ESP state lives in LDS
// (e_j of thread t at esp[j * blockDim + t]).
template <int P>
__global__ void __launch_bounds__(256) k_kernel_cols(NetArgs na, const df* __restrict__ tk,
                                                     const df* __restrict__ tr, int c0, int c1,
                                                     df* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* lds_t0 = reinterpret_cast<uint32_t*>(smem);
  const int s = na.s;
  const int tab_words = (P == 2) ? s * 256 : 0;
  df* esp = reinterpret_cast<df*>(smem + align_up((size_t)tab_words * 4));
  if constexpr (P == 2) {
    for (int i = threadIdx.x; i < s * 256; i += blockDim.x)
      lds_t0[i] = na.xtab[(int64_t)(i >> 8) * na.nbytes * 256 + (i & 255)];
    __syncthreads();
  }
  const bool need_r = c1 > 1;
  const bool need_q = c1 > s + 1;
  const int64_t N = na.N;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int T = blockDim.x;
  for (int64_t n0 = (int64_t)blockIdx.x * blockDim.x; n0 < N; n0 += stride) {
    const int64_t n = n0 + threadIdx.x;
    const int64_t nn = n < N ? n : N - 1;
    const int64_t nw = (int64_t)__builtin_amdgcn_readfirstlane((int)(nn >> 6)) << 6;
    df K = {1.0f, 0.0f}, u = {0.0f, 0.0f};
    if (need_q) {
      esp[threadIdx.x] = df{1.0f, 0.0f};
      for (int j = 1; j <= s; ++j) esp[j * T + threadIdx.x] = df{0.0f, 0.0f};
    }
    for (int j = 0; j < s; ++j) {
      const int t = lead_index<P>(na, lds_t0, j, nn, nw);
      K = mul(K, tk[j * kTab + t]);
      if (need_r) {
        const df r = tr[j * kTab + t];
        u = add(add(u, r), mul(u, r));  // (1 + u)(1 + r) - 1
        const int c = 1 + j;
        if (c >= c0 && c < c1 && n < N) out[(int64_t)(c - c0) * N + n] = u;
        if (need_q) {
          for (int i = j + 1; i >= 1; --i) {
            df e = esp[i * T + threadIdx.x];
            e = add(e, mul(r, esp[(i - 1) * T + threadIdx.x]));
            esp[i * T + threadIdx.x] = e;
          }
        }
      }
    }
    if (n < N) {
      if (c0 == 0) out[n] = K;
      if (need_q) {
        for (int j = 1; j <= s; ++j) {
          const int c = s + j;
          if (c >= c0 && c < c1) out[(int64_t)(c - c0) * N + n] = esp[j * T + threadIdx.x];
        }
      }
    }
  }
}

// ---------------------------------------------------- spectral division
template <int P>
__global__ void __launch_bounds__(256) k_spec_div(const void* __restrict__ ft, const void* __restrict__ gk,
                                                  int64_t N, void* __restrict__ ct) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < N; h += stride) {
    if constexpr (P == 2) {
      const df g = ((const df*)gk)[h];
      const float den = fmaxf(g.hi + g.lo, 1e-30f);
      ((float*)ct)[h] = ((const float*)ft)[h] / den;
    } else {
      const cdf g = ((const cdf*)gk)[h];
      const float den = fmaxf(g.re.hi + g.re.lo, 1e-30f);
      const float2 f = ((const float2*)ft)[h];
      ((float2*)ct)[h] = make_float2(f.x / den, f.y / den);
    }
  }
}

// ------------------------------------------------------- grouped sums
constexpr int kCB = 8;     // columns per reduction block
constexpr int kRedBlocks = 512;

template <int P>
__global__ void __launch_bounds__(256) k_effdim_reduce(const void* __restrict__ ft, const void* __restrict__ gk,
                                                       const void* __restrict__ G, int ncol, int64_t N,
                                                       double pm, double* __restrict__ partial,
                                                       double* __restrict__ qmc_partial) {
  __shared__ double red[256];
  const int cb = blockIdx.y * kCB;
  double acc[kCB];
#pragma unroll
  for (int k = 0; k < kCB; ++k) acc[k] = 0.0;
  double qmc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < N; h += stride) {
    double fsq, kk;
    if constexpr (P == 2) {
      const double f = (double)((const float*)ft)[h];
      fsq = f * f;
      kk = to_double(((const df*)gk)[h]);
    } else {
      const float2 f = ((const float2*)ft)[h];
      fsq = (double)f.x * f.x + (double)f.y * f.y;
      kk = to_double(((const cdf*)gk)[h].re);
    }
    const double w = kk > 0.0 ? pm / (kk * kk) : 0.0;
    if (h != 0) qmc += fsq;
#pragma unroll
    for (int k = 0; k < kCB; ++k) {
      const int c = cb + k;
      if (c < ncol) {
        double g;
        if constexpr (P == 2) g = to_double(((const df*)G)[(int64_t)c * N + h]);
        else g = to_double(((const cdf*)G)[(int64_t)c * N + h].re);
        const double rho = fmin(fmax(g * w, 0.0), 1.0);
        acc[k] += fsq * rho;
      }
    }
  }
  // Fixed-shape tree reduction (deterministic).
  for (int k = 0; k <= kCB; ++k) {
    const int c = cb + k;
    if (k < kCB && c >= ncol) continue;
    red[threadIdx.x] = (k < kCB) ? acc[k] : qmc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (k < kCB) partial[(int64_t)c * gridDim.x + blockIdx.x] = red[0];
      else if (blockIdx.y == 0) qmc_partial[blockIdx.x] = red[0];
    }
    __syncthreads();
  }
}

// Sum nblk partials per row in a fixed order: out[row] = sum_b in[row*nblk + b].
__global__ void __launch_bounds__(256) k_sum_rows(const double* __restrict__ in, int nblk, double* __restrict__ out) {
  __shared__ double red[256];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) a += in[(int64_t)blockIdx.x * nblk + b];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// --------------------------------------------------------- evaluation
constexpr int kNS = 64;  // points staged per step

template <int P>
__global__ void __launch_bounds__(256) k_query_prep(const uint32_t* __restrict__ q, int64_t nq, int s, int m,
                                                    int D, uint64_t* __restrict__ qh, uint32_t* __restrict__ qt) {
  const int64_t total = (int64_t)s * nq;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t Q = q[i];
    // digits d_1..d_D (most significant first)
    uint32_t dg[32];
    for (int l = D - 1; l >= 0; --l) {
      dg[l] = Q % P;
      Q /= P;
    }
    uint64_t head = 0;
    for (int l = 0; l < m; ++l) head |= (uint64_t)dg[l] << (4 * (m - 1 - l));
    uint32_t tail = (uint32_t)D;
    for (int l = D - 1; l >= m; --l)
      if (dg[l] != 0) tail = (uint32_t)l;
    qh[i] = head;
    qt[i] = tail;
  }
}

template <int P, int SMAX>
__global__ void __launch_bounds__(256) k_spline_eval(const void* __restrict__ Xp, const float* __restrict__ c,
                                                     int64_t N, int s, int m, const uint32_t* __restrict__ q,
                                                     const uint64_t* __restrict__ qh,
                                                     const uint32_t* __restrict__ qt, int64_t nq,
                                                     const float* __restrict__ te, int ntab, int64_t ppc,
                                                     df* __restrict__ partial) {
  using XT = typename std::conditional<P == 2, uint32_t, uint64_t>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  float* lte = reinterpret_cast<float*>(smem);
  XT* lx = reinterpret_cast<XT*>(smem + align_up((size_t)s * ntab * 4));
  float* lc = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(lx) + (size_t)s * kNS * sizeof(XT));
  for (int i = threadIdx.x; i < s * ntab; i += blockDim.x) lte[i] = te[i];

  const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t qq = qi < nq ? qi : nq - 1;
  XT qr[SMAX];
  uint32_t tl[SMAX];
#pragma unroll
  for (int j = 0; j < SMAX; ++j) {
    if (j < s) {
      if constexpr (P == 2) {
        qr[j] = q[(int64_t)j * nq + qq];
        tl[j] = 0;
      } else {
        qr[j] = qh[(int64_t)j * nq + qq];
        tl[j] = qt[(int64_t)j * nq + qq];
      }
    }
  }
  const int64_t nbeg = (int64_t)blockIdx.y * ppc;
  const int64_t nend = min(N, nbeg + ppc);
  df acc = {0.0f, 0.0f};
  for (int64_t n0 = nbeg; n0 < nend; n0 += kNS) {
    __syncthreads();
    for (int i = threadIdx.x; i < s * kNS; i += blockDim.x) {
      const int j = i / kNS, k = i % kNS;
      const int64_t n = n0 + k;
      lx[i] = n < nend ? ((const XT*)Xp)[(int64_t)j * N + n] : (XT)0;
    }
    for (int k = threadIdx.x; k < kNS; k += blockDim.x) lc[k] = (n0 + k < nend) ? c[n0 + k] : 0.0f;
    __syncthreads();
    float sub = 0.0f;
    for (int k = 0; k < kNS; ++k) {
      float prod = 1.0f;
#pragma unroll
      for (int j = 0; j < SMAX; ++j) {
        if (j < s) {
          const XT z = qr[j] ^ lx[j * kNS + k];
          int t;
          if constexpr (P == 2) t = __clz(z);
          else t = z ? ((__clzll(z) - 64 + 4 * m) >> 2) : (int)tl[j];
          prod *= lte[j * ntab + t];
        }
      }
      sub += lc[k] * prod;
    }
    acc = add(acc, df{sub, 0.0f});
  }
  if (qi < nq) partial[(int64_t)blockIdx.y * nq + qi] = acc;
}

__global__ void __launch_bounds__(256) k_eval_finish(const df* __restrict__ partial, int gy, int64_t nq,
                                                     float* __restrict__ sf) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += (int64_t)gridDim.x * blockDim.x) {
    df a = {0.0f, 0.0f};
    for (int y = 0; y < gy; ++y) a = add(a, partial[(int64_t)y * nq + i]);
    sf[i] = a.hi + a.lo;
  }
}

// =============================================================== host side
static df split_df(double v) {
  df r;
  r.hi = (float)v;
  r.lo = (float)(v - (double)r.hi);
  return r;
}

static NetArgs net_args(const Net& net) {
  return NetArgs{net.d_xtab, net.d_ptab, net.nbytes, net.s, net.m, net.N};
}

// Upload `bytes` from host `src` to device `dst` through the pinned staging
// buffer, ordered on `st`.
static int upload(Net& net, const void* src, size_t bytes, void* dst, hipStream_t st) {
  int rc = ensure_pin(net, bytes);
  if (rc) return rc;
  std::memcpy(net.pin, src, bytes);
  FDWT_HIP(hipMemcpyAsync(dst, net.pin, bytes, hipMemcpyHostToDevice, st));
  return pin_release(net, st);
}

// Kernel-data tables: tk[j][t] = 1 + gamma_j K'(t+1) for t < m, 1 + gamma_j for
// t >= m (x = 0); tr[j][t] = gamma_j^2 R'(t+1), gamma_j^2 R'(0).
static void kernel_tables(const Net& net, const fdwt_kernel* k, std::vector<df>& tk, std::vector<df>& tr) {
  tk.assign((size_t)net.s * kTab, df{0, 0});
  tr.assign((size_t)net.s * kTab, df{0, 0});
  for (int j = 0; j < net.s; ++j) {
    const double g = k->gamma[j];
    for (int t = 0; t < kTab; ++t) {
      const int i = t < net.m ? t + 1 : 0;
      tk[(size_t)j * kTab + t] = split_df(1.0 + g * kprime(net.p, k->alpha, i));
      tr[(size_t)j * kTab + t] = split_df(g * g * rprime(net.p, k->alpha, i));
    }
  }
}

static size_t kcols_lds(const Net& net, int threads, bool need_q) {
  size_t b = net.p == 2 ? align_up((size_t)net.s * 256 * 4) : 0;
  if (need_q) b += (size_t)(net.s + 1) * threads * sizeof(df);
  return b;
}

static int launch_kernel_cols(Net& net, const df* tk, const df* tr, int c0, int c1, df* out, hipStream_t st) {
  const bool need_q = c1 > net.s + 1;
  int threads = 256;
  while (threads > 64 && kcols_lds(net, threads, need_q) > 80 * 1024) threads /= 2;
  const size_t lds = kcols_lds(net, threads, need_q);
  const unsigned grid = (unsigned)std::min<int64_t>((net.N + threads - 1) / threads, 4096);
  NetArgs na = net_args(net);
  const void* fn;
  if (net.p == 2) fn = (const void*)k_kernel_cols<2>;
  else if (net.p == 3) fn = (const void*)k_kernel_cols<3>;
  else fn = (const void*)k_kernel_cols<5>;
  if (lds > 65536) FDWT_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (net.p == 2) hipLaunchKernelGGL(k_kernel_cols<2>, dim3(grid), dim3(threads), lds, st, na, tk, tr, c0, c1, out);
  else if (net.p == 3) hipLaunchKernelGGL(k_kernel_cols<3>, dim3(grid), dim3(threads), lds, st, na, tk, tr, c0, c1, out);
  else hipLaunchKernelGGL(k_kernel_cols<5>, dim3(grid), dim3(threads), lds, st, na, tk, tr, c0, c1, out);
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

// Unnormalised double-float spectra of `batch` real DF columns in `in`:
// p = 2 in place (out == in), p odd into complex DF `out`.
static int df_spectra(const Net& net, df* in, void* out, int batch, hipStream_t st) {
  if (net.p == 2) return fwt_run_tmp(2, net.m, false, K_DF, in, K_DF, K_DF, in, nullptr, batch, 1.0f, st);
  return fwt_run_tmp(net.p, net.m, false, K_DF, in, K_CDF, K_CDF, out, nullptr, batch, 1.0f, st);
}

static unsigned grid1(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 4096); }

int run_spline_coef(Net& net, const fdwt_kernel* kern, int ft_type, const void* ft, float* c, hipStream_t st) {
  (void)ft_type;
  const int64_t N = net.N;
  const size_t tab_b = align_up((size_t)net.s * kTab * sizeof(df));
  const size_t a_b = align_up((size_t)N * sizeof(df));
  const size_t g_b = net.p == 2 ? 0 : align_up((size_t)N * sizeof(cdf));
  const size_t ct_b = net.p == 2 ? 0 : align_up((size_t)N * sizeof(float2));
  int rc = ensure_ws(net, tab_b + a_b + g_b + ct_b, st);
  if (rc) return rc;
  char* w = (char*)net.ws;
  df* tk = (df*)w;
  df* A = (df*)(w + tab_b);
  void* GK = net.p == 2 ? (void*)A : (void*)(w + tab_b + a_b);
  void* ct = net.p == 2 ? (void*)c : (void*)(w + tab_b + a_b + g_b);
  std::vector<df> htk, htr;
  kernel_tables(net, kern, htk, htr);
  rc = upload(net, htk.data(), htk.size() * sizeof(df), tk, st);
  if (rc) return rc;
  rc = launch_kernel_cols(net, tk, tk, 0, 1, A, st);
  if (rc) return rc;
  rc = df_spectra(net, A, GK, 1, st);
  if (rc) return rc;
  if (net.p == 2) hipLaunchKernelGGL(k_spec_div<2>, dim3(grid1(N)), dim3(256), 0, st, ft, GK, N, ct);
  else if (net.p == 3) hipLaunchKernelGGL(k_spec_div<3>, dim3(grid1(N)), dim3(256), 0, st, ft, GK, N, ct);
  else hipLaunchKernelGGL(k_spec_div<5>, dim3(grid1(N)), dim3(256), 0, st, ft, GK, N, ct);
  FDWT_HIP(hipGetLastError());
  // Algorithm 2 (no normalisation); p odd returns the real part.
  if (net.p == 2) return fwt_run_tmp(2, net.m, true, K_F32, ct, K_F32, K_F32, c, nullptr, 1, 1.0f, st);
  return fwt_run_tmp(net.p, net.m, true, K_CF32, ct, K_CF32, K_F32, c, ct, 1, 1.0f, st);
}

template <int P>
static int launch_eval(Net& net, const void* Xp, const float* c, int64_t nq, const uint32_t* q,
                       const uint64_t* qh, const uint32_t* qt, const float* te, int ntab, df* partial,
                       int gy, int64_t ppc, size_t lds, hipStream_t st) {
  const dim3 grid((unsigned)((nq + 255) / 256), (unsigned)gy);
  const int s = net.s;
#define FDWT_EVAL(SM)                                                                              \
  {                                                                                                \
    auto fn = k_spline_eval<P, SM>;                                                                \
    if (lds > 65536) FDWT_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    hipLaunchKernelGGL(fn, grid, dim3(256), lds, st, Xp, c, net.N, s, net.m, q, qh, qt, nq, te,    \
                       ntab, ppc, partial);                                                        \
  }
  if (s <= 8) FDWT_EVAL(8)
  else if (s <= 16) FDWT_EVAL(16)
  else if (s <= 32) FDWT_EVAL(32)
  else FDWT_EVAL(64)
#undef FDWT_EVAL
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

int run_spline_eval(Net& net, const fdwt_kernel* kern, const float* c, int64_t nq, const uint32_t* q,
                    float* sf, hipStream_t st) {
  const int p = net.p, s = net.s, m = net.m;
  const int D = query_depth(p);
  const int ntab = D + 1;
  const int64_t N = net.N;
  const size_t xb = (p == 2) ? 4 : 8;
  // Grid: query blocks x point chunks, >= ~2048 workgroups in total.
  const int64_t qb = (nq + 255) / 256;
  int gy = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + qb - 1) / qb, (N + kNS - 1) / kNS));
  int64_t ppc = (N + gy - 1) / gy;
  ppc = (ppc + kNS - 1) / kNS * kNS;
  gy = (int)((N + ppc - 1) / ppc);
  const size_t te_b = align_up((size_t)s * ntab * 4);
  const size_t x_b = align_up((size_t)s * N * xb);
  const size_t qh_b = p == 2 ? 0 : align_up((size_t)s * nq * 8);
  const size_t qt_b = p == 2 ? 0 : align_up((size_t)s * nq * 4);
  const size_t pa_b = align_up((size_t)gy * nq * sizeof(df));
  int rc = ensure_ws(net, te_b + x_b + qh_b + qt_b + pa_b, st);
  if (rc) return rc;
  char* w = (char*)net.ws;
  float* te = (float*)w;
  void* Xp = w + te_b;
  uint64_t* qh = (uint64_t*)(w + te_b + x_b);
  uint32_t* qt = (uint32_t*)(w + te_b + x_b + qh_b);
  df* partial = (df*)(w + te_b + x_b + qh_b + qt_b);
  // te[j][t]: 1 + gamma_j K'(t+1) for t < D, 1 + gamma_j for t = D (equal digits).
  std::vector<float> hte((size_t)s * ntab);
  for (int j = 0; j < s; ++j)
    for (int t = 0; t < ntab; ++t)
      hte[(size_t)j * ntab + t] = (float)(1.0 + kern->gamma[j] * kprime(p, kern->alpha, t < D ? t + 1 : 0));
  rc = upload(net, hte.data(), hte.size() * 4, te, st);
  if (rc) return rc;
  rc = launch_net_packed(net, Xp, st);
  if (rc) return rc;
  if (p == 3) hipLaunchKernelGGL(k_query_prep<3>, dim3(grid1((int64_t)s * nq)), dim3(256), 0, st, q, nq, s, m, D, qh, qt);
  if (p == 5) hipLaunchKernelGGL(k_query_prep<5>, dim3(grid1((int64_t)s * nq)), dim3(256), 0, st, q, nq, s, m, D, qh, qt);
  FDWT_HIP(hipGetLastError());
  const size_t lds = te_b + (size_t)s * kNS * xb + kNS * 4;
  if (p == 2) rc = launch_eval<2>(net, Xp, c, nq, q, nullptr, nullptr, te, ntab, partial, gy, ppc, lds, st);
  else if (p == 3) rc = launch_eval<3>(net, Xp, c, nq, q, qh, qt, te, ntab, partial, gy, ppc, lds, st);
  else rc = launch_eval<5>(net, Xp, c, nq, q, qh, qt, te, ntab, partial, gy, ppc, lds, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_eval_finish, dim3(grid1(nq)), dim3(256), 0, st, partial, gy, nq, sf);
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

int run_eff_dim(Net& net, const fdwt_kernel* kern, int ft_type, const void* ft, fdwt_effdim* out, hipStream_t st) {
  (void)ft_type;
  const int p = net.p, s = net.s;
  const int64_t N = net.N;
  const size_t eb = sizeof(df), cb = (p == 2) ? sizeof(df) : sizeof(cdf);
  const int ncols = 2 * s;  // U_1..U_s, Q_1..Q_s  (column c+1 of the generator layout)
  // Columns per chunk within a workspace budget.
  const size_t budget = (size_t)8 << 30;
  const size_t per_col = (size_t)N * (eb + (p == 2 ? 0 : cb));
  int ch = (int)std::max<size_t>(1, std::min<size_t>((size_t)ncols, budget / per_col));
  const size_t tab_b = align_up((size_t)2 * s * kTab * sizeof(df));
  const size_t gk_b = align_up((size_t)N * cb) + (p == 2 ? 0 : align_up((size_t)N * eb));
  const size_t a_b = align_up((size_t)ch * N * eb);
  const size_t b_b = p == 2 ? 0 : align_up((size_t)ch * N * cb);
  const size_t part_b = align_up((size_t)(ncols + 1) * kRedBlocks * sizeof(double));
  const size_t res_b = align_up((size_t)(ncols + 1) * sizeof(double));
  const size_t h0_b = align_up(64);
  int rc = ensure_ws(net, tab_b + gk_b + a_b + b_b + part_b + res_b + h0_b, st);
  if (rc) return rc;
  char* w = (char*)net.ws;
  df* tk = (df*)w;
  df* tr = tk + (size_t)s * kTab;
  char* gkbase = w + tab_b;
  void* GK = gkbase;                                   // DF (p = 2) or CDF spectrum of K
  df* gk_in = p == 2 ? (df*)gkbase : (df*)(gkbase + align_up((size_t)N * cb));
  df* A = (df*)(w + tab_b + gk_b);
  void* B = p == 2 ? (void*)A : (void*)(w + tab_b + gk_b + a_b);
  double* partial = (double*)(w + tab_b + gk_b + a_b + b_b);
  double* qmc_partial = partial + (size_t)ncols * kRedBlocks;
  double* res = (double*)(w + tab_b + gk_b + a_b + b_b + part_b);
  char* h0 = w + tab_b + gk_b + a_b + b_b + part_b + res_b;

  std::vector<df> htab, htr;
  kernel_tables(net, kern, htab, htr);
  htab.insert(htab.end(), htr.begin(), htr.end());
  rc = upload(net, htab.data(), htab.size() * sizeof(df), tk, st);
  if (rc) return rc;
  // K~ (unnormalised).
  rc = launch_kernel_cols(net, tk, tr, 0, 1, gk_in, st);
  if (!rc) rc = df_spectra(net, gk_in, GK, 1, st);
  if (rc) return rc;
  const double pm = (double)N;
  for (int c0 = 0; c0 < ncols; c0 += ch) {
    const int c1 = std::min(ncols, c0 + ch);
    rc = launch_kernel_cols(net, tk, tr, c0 + 1, c1 + 1, A, st);
    if (!rc) rc = df_spectra(net, A, B, c1 - c0, st);
    if (rc) return rc;
    const dim3 grid(kRedBlocks, (unsigned)((c1 - c0 + kCB - 1) / kCB));
    double* part_c = partial + (size_t)c0 * kRedBlocks;
    if (p == 2) hipLaunchKernelGGL(k_effdim_reduce<2>, grid, dim3(256), 0, st, ft, GK, B, c1 - c0, N, pm, part_c, qmc_partial);
    else if (p == 3) hipLaunchKernelGGL(k_effdim_reduce<3>, grid, dim3(256), 0, st, ft, GK, B, c1 - c0, N, pm, part_c, qmc_partial);
    else hipLaunchKernelGGL(k_effdim_reduce<5>, grid, dim3(256), 0, st, ft, GK, B, c1 - c0, N, pm, part_c, qmc_partial);
    FDWT_HIP(hipGetLastError());
    // The h = 0 bin of U_s (for the h = 0 share of the total).
    if (s - 1 >= c0 && s - 1 < c1)
      FDWT_HIP(hipMemcpyAsync(h0 + 32, (char*)B + (size_t)(s - 1 - c0) * N * cb, cb, hipMemcpyDeviceToDevice, st));
  }
  hipLaunchKernelGGL(k_sum_rows, dim3(ncols + 1), dim3(256), 0, st, partial, kRedBlocks, res);
  FDWT_HIP(hipGetLastError());
  FDWT_HIP(hipMemcpyAsync(h0, ft, p == 2 ? 4 : 8, hipMemcpyDeviceToDevice, st));
  FDWT_HIP(hipMemcpyAsync(h0 + 8, GK, cb, hipMemcpyDeviceToDevice, st));
  // Results to the host.
  const size_t nres = (size_t)(ncols + 1) * sizeof(double);
  rc = ensure_pin(net, nres + 64);
  if (rc) return rc;
  FDWT_HIP(hipMemcpyAsync(net.pin, res, nres, hipMemcpyDeviceToHost, st));
  FDWT_HIP(hipMemcpyAsync((char*)net.pin + nres, h0, 64, hipMemcpyDeviceToHost, st));
  FDWT_HIP(hipStreamSynchronize(st));
  const double* r = (const double*)net.pin;
  const char* hz = (const char*)net.pin + nres;
  out->var_trc[0] = 0.0;
  out->var_sup[0] = 0.0;
  for (int d = 1; d <= s; ++d) {
    out->var_trc[d] = r[d - 1];
    out->var_sup[d] = out->var_sup[d - 1] + r[s + d - 1];
  }
  out->var_total = out->var_trc[s];
  out->var_qmc = r[ncols];
  {
    double fsq, kk, g;
    if (p == 2) {
      float f;
      df k0, g0;
      std::memcpy(&f, hz, 4);
      std::memcpy(&k0, hz + 8, sizeof(df));
      std::memcpy(&g0, hz + 32, sizeof(df));
      fsq = (double)f * f;
      kk = (double)k0.hi + k0.lo;
      g = (double)g0.hi + g0.lo;
    } else {
      float f[2];
      cdf k0, g0;
      std::memcpy(f, hz, 8);
      std::memcpy(&k0, hz + 8, sizeof(cdf));
      std::memcpy(&g0, hz + 32, sizeof(cdf));
      fsq = (double)f[0] * f[0] + (double)f[1] * f[1];
      kk = (double)k0.re.hi + k0.re.lo;
      g = (double)g0.re.hi + g0.re.lo;
    }
    const double rho = kk > 0 ? std::min(1.0, std::max(0.0, pm * g / (kk * kk))) : 0.0;
    out->var_total_h0 = fsq * rho;
  }
  const double target = 0.99 * out->var_total;
  out->d_trc = s;
  out->d_sup = s;
  for (int d = 0; d <= s; ++d)
    if (out->var_trc[d] >= target) {
      out->d_trc = d;
      break;
    }
  for (int d = 0; d <= s; ++d)
    if (out->var_sup[d] >= target) {
      out->d_sup = d;
      break;
    }
  return FDWT_OK;
}

}  // namespace fdwt
