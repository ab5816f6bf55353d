// Walsh-kernel spline and ANOVA variances (Sections 3.2, 3.3 and 4).
//
//  * kernel data: K(x_n, 0) = prod_j [1 + gamma_j K'(x_{n,j}, 0)] and, for the
//    variances, U_d = R_d - 1 with R_d = prod_{j<=d} (1 + gamma_j^2 R'(x_{n,j}, 0))
//    and Q_j = e_j(gamma_1^2 R'_1, ..., gamma_s^2 R'_s) (elementary symmetric
//    polynomials), all in float64.  K' and R' depend only on the index of the
//    first non-zero digit of x_{n,j}, so per-coordinate tables (computed on
//    the host) are indexed by a leading-zero count.
//  * their DWTs (the kernel spectra) are taken in float64: their dynamic
//    range exceeds what float resolves (the small bins would lose all their
//    digits, and K~ must stay positive for the spectral solve).  On MI355X
//    float64 vector arithmetic runs at half the float32 rate, far cheaper than
//    emulating the extra precision with float pairs.
//  * spectral solve, Eq. (splinecoef): c~ = f~ / (p^m K~), then Algorithm 2.
//  * variances, Eq. (sig2sfu) summed over u: with rho_g(h) = p^m g~(h)/K~u(h)^2
//    (K~u the unnormalised spectrum), sigma^2 = sum_h |f~(h)|^2 rho_g(h).
//    rho lies in [0, 1] exactly (0 <= g~ <= K~^2 because the Walsh
//    coefficients of R are the squares of those of K); the clamp only removes
//    rounding noise in bins where K~ is tiny.  The sums run in float64 inside
//    the last pass of the spectra's transform (nothing is stored).
//  * evaluation, Sf(q) = sum_n c_n K(q, x_n), at query points given as D-digit
//    integers; the first differing digit of q and x_n is a leading-zero count
//    of their XOR (p = 2) or of their packed-digit XOR (p odd).
#include "coords.h"
#include "dev_math.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>

namespace fdwt {

constexpr int kTab = 33;  // entries per coordinate of the digit-indexed tables

__host__ __device__ static inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct NetArgs {
  const uint32_t* xtab;  // p = 2
  const uint64_t* ptab;  // p odd
  int nbytes, s, m;
  int64_t N;
};

// ------------------------------------------------ kernel-data columns (f64)
// Column layout: 0 = K, 1..s = U_d (d = 1..s), s+1..2s = Q_j (j = 1..s).
// Writes columns [c0, c1) to out[(c - c0) * N + n].  The elementary symmetric
// polynomials e_0..e_SMAX live in registers (updates unrolled, truncated per
// chunk of coordinates where the higher ones are still zero).
template <int P, int SMAX>
__global__ void __launch_bounds__(kChunk) k_kernel_cols(NetArgs na, const double* __restrict__ tk,
                                                        const double* __restrict__ tr, int c0, int c1,
                                                        double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int s = na.s;
  double* ltk = reinterpret_cast<double*>(smem);       // [s][kTab]
  double* ltr = ltk + s * kTab;                         // [s][kTab]
  uint32_t* lt0 = reinterpret_cast<uint32_t*>(ltr + s * kTab);
  for (int i = threadIdx.x; i < s * kTab; i += blockDim.x) {
    ltk[i] = tk[i];
    ltr[i] = tr[i];
  }
  P2Coords pc{na.xtab, na.nbytes, s, lt0, lt0 + s * 256};
  uint64_t* lodd = reinterpret_cast<uint64_t*>(ltr + s * kTab);
  OddCoords<P == 2 ? 3 : P> oc{na.ptab, s, na.m, lodd, lodd + s * OddCoords<P == 2 ? 3 : P>::PK};
  if constexpr (P == 2) pc.stage_tables();
  else oc.stage_tables();
  const bool need_r = c1 > 1;
  const bool need_q = c1 > s + 1;
  const int64_t N = na.N;
  const int m = na.m;
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < N; base += (int64_t)gridDim.x * kChunk) {
    __syncthreads();
    if constexpr (P == 2) pc.stage_group(base);
    else oc.stage_group(base);
    __syncthreads();
    const int64_t n = base + threadIdx.x;
    const int64_t nn = n < N ? n : N - 1;
    int orr = 0, ok = 0;
    if constexpr (P != 2) oc.split(nn, orr, ok);
    double K = 1.0, u = 0.0;
    double e[SMAX + 1];
#pragma unroll
    for (int i = 0; i <= SMAX; ++i) e[i] = i == 0 ? 1.0 : 0.0;
    // Coordinates in chunks of 4 (SMAX is a multiple of 4): after chunk q
    // only e[1..4(q + 1)] can be non-zero, so the update of the symmetric
    // polynomials stops there (a compile-time bound per chunk).  The last
    // chunk runs to s: s > SMAX only when no symmetric polynomial is wanted
    // (K and the U_d alone).
#pragma unroll
    for (int q = 0; q < SMAX / 4; ++q) {
      const int je = (q == SMAX / 4 - 1 || 4 * q + 4 > s) ? s : 4 * q + 4;
      for (int j = 4 * q; j < je; ++j) {
        int t;
        if constexpr (P == 2) t = lead_p2(pc.X(j, nn), m);
        else t = lead_odd(oc.X(j, orr, ok), m);
        K *= ltk[j * kTab + t];
        if (need_r) {
          const double r = ltr[j * kTab + t];
          u = u + r + u * r;  // (1 + u)(1 + r) - 1
          const int c = 1 + j;
          if (c >= c0 && c < c1 && n < N) out[(int64_t)(c - c0) * N + n] = u;
          if (need_q) {
#pragma unroll
            for (int i = 4 * q + 4; i >= 1; --i) e[i] += r * e[i - 1];
          }
        }
      }
    }
    if (n < N) {
      if (c0 == 0) out[n] = K;
      if (need_q) {
#pragma unroll
        for (int j = 1; j <= SMAX; ++j) {
          const int c = s + j;
          if (j <= s && c >= c0 && c < c1) out[(int64_t)(c - c0) * N + n] = e[j];
        }
      }
    }
  }
}

// p = 2, N a multiple of 512: the same columns as k_kernel_cols with two
// adjacent points per thread, stored 16 bytes per lane (a store-bound
// kernel: about 4% faster than one point per thread at 2^24 points, s = 20).
// A 512-point group is two 256-point halves, each with its own XOR of the
// upper-byte tables.
template <int SMAX>
__global__ void __launch_bounds__(kChunk) k_kernel_cols2(NetArgs na, const double* __restrict__ tk,
                                                         const double* __restrict__ tr, int c0, int c1,
                                                         double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int s = na.s;
  double* ltk = reinterpret_cast<double*>(smem);
  double* ltr = ltk + s * kTab;
  uint32_t* lt0 = reinterpret_cast<uint32_t*>(ltr + s * kTab);  // [s][256]
  uint32_t* lu = lt0 + s * 256;                                  // [2][s]
  for (int i = threadIdx.x; i < s * kTab; i += blockDim.x) {
    ltk[i] = tk[i];
    ltr[i] = tr[i];
  }
  P2Coords pc{na.xtab, na.nbytes, s, lt0, lu};
  pc.stage_tables();
  const bool need_r = c1 > 1;
  const bool need_q = c1 > s + 1;
  const int64_t N = na.N;
  const int m = na.m;
  const int half = threadIdx.x >> 7;
  const int lo = (2 * threadIdx.x) & 255;
  for (int64_t base = (int64_t)blockIdx.x * 512; base < N; base += (int64_t)gridDim.x * 512) {
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * s; i += blockDim.x) {
      const int h = i / s, j = i - h * s;
      const int64_t b = base + 256 * h;
      const uint32_t* tj = na.xtab + (int64_t)j * na.nbytes * 256;
      uint32_t v = 0;
      for (int bb = 1; bb < na.nbytes; ++bb) v ^= tj[bb * 256 + (int)((b >> (8 * bb)) & 255)];
      lu[h * s + j] = v;
    }
    __syncthreads();
    const int64_t n = base + 2 * threadIdx.x;
    double K0 = 1.0, K1 = 1.0, u0 = 0.0, u1 = 0.0;
    double e0[SMAX + 1], e1[SMAX + 1];
#pragma unroll
    for (int i = 0; i <= SMAX; ++i) e0[i] = e1[i] = i == 0 ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < SMAX / 4; ++q) {
      const int je = (q == SMAX / 4 - 1 || 4 * q + 4 > s) ? s : 4 * q + 4;
      for (int j = 4 * q; j < je; ++j) {
        const uint32_t uj = lu[half * s + j];
        const int t0 = lead_p2(lt0[j * 256 + lo] ^ uj, m);
        const int t1 = lead_p2(lt0[j * 256 + lo + 1] ^ uj, m);
        K0 *= ltk[j * kTab + t0];
        K1 *= ltk[j * kTab + t1];
        if (need_r) {
          const double r0 = ltr[j * kTab + t0], r1 = ltr[j * kTab + t1];
          u0 = u0 + r0 + u0 * r0;
          u1 = u1 + r1 + u1 * r1;
          const int c = 1 + j;
          if (c >= c0 && c < c1) {
            double2 w;
            w.x = u0;
            w.y = u1;
            *reinterpret_cast<double2*>(out + (int64_t)(c - c0) * N + n) = w;
          }
          if (need_q) {
#pragma unroll
            for (int i = 4 * q + 4; i >= 1; --i) {
              e0[i] += r0 * e0[i - 1];
              e1[i] += r1 * e1[i - 1];
            }
          }
        }
      }
    }
    if (c0 == 0) {
      double2 w;
      w.x = K0;
      w.y = K1;
      *reinterpret_cast<double2*>(out + n) = w;
    }
    if (need_q) {
#pragma unroll
      for (int j = 1; j <= SMAX; ++j) {
        const int c = s + j;
        if (j <= s && c >= c0 && c < c1) {
          double2 w;
          w.x = e0[j];
          w.y = e1[j];
          *reinterpret_cast<double2*>(out + (int64_t)(c - c0) * N + n) = w;
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
      const double g = fmax(((const double*)gk)[h], 1e-300);
      ((float*)ct)[h] = (float)((double)((const float*)ft)[h] / g);
    } else {
      const double g = fmax(((const double2*)gk)[h].x, 1e-300);
      const float2 f = ((const float2*)ft)[h];
      ((float2*)ct)[h] = make_float2((float)((double)f.x / g), (float)((double)f.y / g));
    }
  }
}

// ------------------------------------------------------- grouped sums
// Weights of the grouped sums: wts[h] = (|f~(h)|^2, p^m / K~u(h)^2), with
// K~u the unnormalised kernel spectrum (so that rho = g~u * wts.y is the
// normalised ratio of Eq. (sig2sfu)), and the sample variance
// sum_{h != 0} |f~(h)|^2 as block partials.
constexpr int kRedBlocks = 1024;

template <int P>
__global__ void __launch_bounds__(256) k_effdim_weights(const void* __restrict__ ft, const void* __restrict__ gk,
                                                        int64_t N, double pm, float2* __restrict__ wts,
                                                        double* __restrict__ qmc_partial, int blkF, int m) {
  __shared__ double red[256];
  double qmc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < N; b += stride) {
    // wts[b] is the weight of coefficient h: b = h, or (blkF > 0) the blocked
    // position of h for a first pass of 2^blkF elements (PassDesc::oblk).
    int64_t h = b;
    if (blkF > 0) {
      const int64_t w = b & 15, hi = (b >> 4) & ((int64_t(1) << (m - blkF)) - 1), mid = b >> (4 + m - blkF);
      h = (hi << blkF) + mid * 16 + w;
    }
    double fsq, kk;
    if constexpr (P == 2) {
      const double f = (double)((const float*)ft)[h];
      fsq = f * f;
      kk = ((const double*)gk)[h];
    } else {
      const float2 f = ((const float2*)ft)[h];
      fsq = (double)f.x * f.x + (double)f.y * f.y;
      kk = ((const double2*)gk)[h].x;
    }
    const double kinv = kk > 0.0 ? fmin(pm / (kk * kk), 3.0e38) : 0.0;
    wts[b] = make_float2((float)fsq, (float)kinv);
    if (h != 0) qmc += fsq;
  }
  red[threadIdx.x] = qmc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) qmc_partial[blockIdx.x] = red[0];
}

// Sum nblk partials per row in a fixed order: out[row] = sum_b in[row*nblk + b].
constexpr int kSumThreads = 1024;
__global__ void __launch_bounds__(kSumThreads) k_sum_rows(const double* __restrict__ in, int nblk,
                                                          double* __restrict__ out) {
  __shared__ double red[kSumThreads];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kSumThreads) a += in[(int64_t)blockIdx.x * nblk + b];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = kSumThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// --------------------------------------------------------- evaluation
// Points staged in LDS per step of the evaluation: 256 for up to 16
// coordinates (fewer barriers and staging rounds per evaluation), 64 above
// (the staged strings of many coordinates would otherwise limit how many
// workgroups share a CU).  Point chunks are rounded to kNSMax.
constexpr int kNSMax = 256;
template <int SMAX>
constexpr int eval_ns() { return SMAX <= 16 ? 256 : 64; }

// Query digit strings, p odd: the D digits of q[j][i] (most significant
// first) in the layout of eval_string_odd.
template <int P>
__global__ void __launch_bounds__(256) k_query_prep(const uint32_t* __restrict__ q, int64_t nq, int s, int D,
                                                    uint64_t* __restrict__ qs) {
  const int64_t total = (int64_t)s * nq;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t Q = q[i];
    uint64_t v = 0;
    for (int f = D - 1; f >= 0; --f) {
      v |= (uint64_t)(Q % P) << (63 - kStrBits<P> * (f + 1));
      Q /= P;
    }
    qs[i] = v;
  }
}

// Leading-zero count with all ones for a zero argument (v_ffbh_u32).
__device__ __forceinline__ int ffbh_raw(uint32_t z) {
  int c;
  asm("v_ffbh_u32 %0, %1" : "=v"(c) : "v"(z));
  return c;
}

// Sf at queries as partial sums over point chunks (blockIdx.y): each thread
// takes one query; the points of a chunk are staged in LDS kNS at a time and
// read as 16-byte broadcasts, 8 points a group (two reads per coordinate:
// with 4 points a group the table reads' latency was not hidden, 8 reach the
// VALU issue limit).  The factor 1 + gamma_j K'(.) of
// coordinate j is entry (c + 1) of a per-coordinate table in LDS (kTabE
// floats a row, copied from ftab), where c is the leading-zero count of the
// XOR of the query's and the point's digit strings (one v_add_lshl_u32 makes
// the byte offset; distinct entries of a row lie in distinct banks):
//   p = 2: the first differing bit c (all equal: v_ffbh_u32 gives -1, entry 0);
//   p odd: c = Bt + 1..Bt + B for first differing digit t (B = 2 for p = 3,
//          3 otherwise: coords.h), 64 when all D digits agree.  c comes from
//          the high 32 bits of the strings; a lane whose high words agree for
//          some (point, coordinate) of a group of 8 points (the first 15 or 10
//          digits equal, rare) redoes that group exactly, taking c from the
//          low words there.  Entry 0 (c = -1: high words equal) is a NaN,
//          which the group's products keep, so one test per point after the
//          coordinate loop detects it without work in the loop.
constexpr int kTabE = 68;  // table entries per coordinate (p odd uses 0..65)

template <int P, int SMAX>
__global__ void __launch_bounds__(256) k_spline_eval(const void* __restrict__ Xp, const float* __restrict__ c,
                                                     int64_t N, int s, const void* __restrict__ qv, int64_t nq,
                                                     const float* __restrict__ ftab, int64_t ppc,
                                                     df* __restrict__ partial) {
  constexpr bool ODD = P != 2;
  constexpr int V = 8;  // points per group (two 16-byte LDS reads per coordinate)
  constexpr int kNS = eval_ns<SMAX>();
  constexpr int kSub = 64;  // points per float partial sum (then double-float)
  extern __shared__ __align__(16) unsigned char smem[];
  float* lt = reinterpret_cast<float*>(smem);                              // [s][kTabE]
  uint32_t* lxh = reinterpret_cast<uint32_t*>(lt + (size_t)s * kTabE);     // [s][kNS] (p odd: high words)
  uint32_t* lxl = lxh + (size_t)s * kNS;                                  // [s][kNS] p odd: low words
  float* lc = reinterpret_cast<float*>(lxh + (size_t)(ODD ? 2 : 1) * s * kNS);  // [kNS]
  for (int i = threadIdx.x; i < s * kTabE; i += blockDim.x) lt[i] = ftab[i];
  const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t qq = qi < nq ? qi : nq - 1;
  // Query high words stay in registers; the low words (needed only on the
  // rare path) are read from memory there.
  uint32_t qh[SMAX];
#pragma unroll
  for (int j = 0; j < SMAX; ++j) {
    if (j < s) {
      if constexpr (ODD) {
        qh[j] = (uint32_t)(((const uint64_t*)qv)[(int64_t)j * nq + qq] >> 32);
      } else {
        qh[j] = ((const uint32_t*)qv)[(int64_t)j * nq + qq];
      }
    }
  }
  auto factor = [&](int j, int cl) {  // cl in [-1, 64]
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(lt + j * kTabE) +
                                           ((uint32_t)(cl + 1) << 2));
  };
  const int64_t nbeg = (int64_t)blockIdx.y * ppc;
  const int64_t nend = min(N, nbeg + ppc);
  df acc = {0.0f, 0.0f};
  for (int64_t n0 = nbeg; n0 < nend; n0 += kNS) {
    __syncthreads();
    for (int i = threadIdx.x; i < s * kNS; i += blockDim.x) {
      const int j = i / kNS, k = i % kNS;
      const int64_t n = n0 + k;
      if constexpr (ODD) {
        const uint64_t v = n < nend ? ((const uint64_t*)Xp)[(int64_t)j * N + n] : 0ull;
        lxh[i] = (uint32_t)(v >> 32);
        lxl[i] = (uint32_t)v;
      } else {
        lxh[i] = n < nend ? ((const uint32_t*)Xp)[(int64_t)j * N + n] : 0u;
      }
    }
    for (int k = threadIdx.x; k < kNS; k += blockDim.x) lc[k] = (n0 + k < nend) ? c[n0 + k] : 0.0f;
    __syncthreads();
    for (int kb = 0; kb < kNS; kb += kSub) {  // float partial sums over kSub points
      float sub = 0.0f;
      for (int k = kb; k < kb + kSub; k += V) {
        float pr[V];
#pragma unroll
        for (int u = 0; u < V; ++u) pr[u] = 1.0f;
#pragma unroll
        for (int j = 0; j < SMAX; ++j) {
          if (j < s) {
            const uint4 xv = *reinterpret_cast<const uint4*>(lxh + j * kNS + k);
            const uint4 xw = *reinterpret_cast<const uint4*>(lxh + j * kNS + k + 4);
            const uint32_t xs[V] = {xv.x, xv.y, xv.z, xv.w, xw.x, xw.y, xw.z, xw.w};
#pragma unroll
            for (int u = 0; u < V; ++u) pr[u] *= factor(j, ffbh_raw(qh[j] ^ xs[u]));
          }
        }
        if constexpr (ODD) {
          // Equal high words (leading-zero count -1) pick a NaN table entry,
          // which the product keeps: one test per point instead of one per
          // coordinate finds the groups that need the low words.
          bool rare = false;
#pragma unroll
          for (int u = 0; u < V; ++u) rare |= __builtin_isnan(pr[u]);
          if (rare) {
            // Rare: some high words agree; redo the group from the full strings.
            // The empty asm keeps the query loads on this path.
            int64_t qo = qq;
            asm volatile("" : "+v"(qo));
#pragma unroll
            for (int u = 0; u < V; ++u) pr[u] = 1.0f;
            for (int j = 0; j < s; ++j) {
              const uint64_t qs = ((const uint64_t*)qv + (int64_t)j * nq)[qo];
              const uint32_t qhi = (uint32_t)(qs >> 32), qlo = (uint32_t)qs;
              for (int u = 0; u < V; ++u) {
                const uint32_t zh = qhi ^ lxh[j * kNS + k + u];
                int cl;
                if (zh) {
                  cl = ffbh_raw(zh);
                } else {
                  const uint32_t zl = qlo ^ lxl[j * kNS + k + u];
                  cl = zl ? 32 + ffbh_raw(zl) : 64;
                }
                pr[u] *= factor(j, cl);
              }
            }
          }
        }
#pragma unroll
        for (int u = 0; u < V; ++u) sub += lc[k + u] * pr[u];
      }
      acc = add(acc, df{sub, 0.0f});
    }
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

// ------------------------------------------------ kernel-parameter cost
// Section 5.1, p = 2.  g(u) = K(x_u (+) x_N, 0) over the first half (an
// m-digit net, tables of `na`): coordinate j of x_u (+) x_N as an
// (m+1)-digit integer is (X_j(u) << 1) ^ delta_j; the factor comes from its
// first non-zero digit, tk2[j][t] = 1 + gamma_j K'(t+1) (t < m+1) and
// tk2[j][m+1] = 1 + gamma_j (all digits zero).
__global__ void __launch_bounds__(kChunk) k_kernel_shift_p2(NetArgs na, const uint32_t* __restrict__ delta,
                                                            const double* __restrict__ tk2, int m2,
                                                            double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int s = na.s;
  double* ltk = reinterpret_cast<double*>(smem);                       // [s][kTab]
  uint32_t* ld = reinterpret_cast<uint32_t*>(ltk + s * kTab);           // [s]
  uint32_t* lt0 = ld + ((s + 1) & ~1);
  for (int i = threadIdx.x; i < s * kTab; i += blockDim.x) ltk[i] = tk2[i];
  for (int i = threadIdx.x; i < s; i += blockDim.x) ld[i] = delta[i];
  P2Coords pc{na.xtab, na.nbytes, s, lt0, lt0 + s * 256};
  pc.stage_tables();
  const int64_t N = na.N;
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < N; base += (int64_t)gridDim.x * kChunk) {
    __syncthreads();
    pc.stage_group(base);
    __syncthreads();
    const int64_t n = base + threadIdx.x;
    if (n < N) {
      double K = 1.0;
      for (int j = 0; j < s; ++j) {
        const uint32_t z = (pc.X(j, n) << 1) ^ ld[j];
        const int t = z ? (int)__clz(z) - (32 - m2) : m2;
        K *= ltk[j * kTab + t];
      }
      out[n] = K;
    }
  }
}

// P(h) = f~(h) G(h) / K_u(h) in place of G (K_u > 0; clamped against rounding).
__global__ void __launch_bounds__(256) k_split_combine(const float* __restrict__ ft, const double* __restrict__ ku,
                                                       double* __restrict__ g, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < N; h += stride)
    g[h] = (double)ft[h] * g[h] / fmax(ku[h], 1e-300);
}

// Block partials of sum_n (fval[n] - sf[n])^2 in float64; sf_out (nullable)
// receives sf as float.
__global__ void __launch_bounds__(256) k_sq_diff(const float* __restrict__ fval, const double* __restrict__ sf,
                                                 int64_t N, double* __restrict__ partial, float* __restrict__ sf_out) {
  __shared__ double red[256];
  double a = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
    const double d = (double)fval[n] - sf[n];
    a += d * d;
    if (sf_out) sf_out[n] = (float)sf[n];
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// =============================================================== host side
static NetArgs net_args(const Net& net) {
  return NetArgs{net.d_xtab, net.d_ptab, net.nbytes, net.s, net.m, net.N};
}

// Kernel-data tables: tk[j][t] = 1 + gamma_j K'(t+1) for t < m, 1 + gamma_j for
// t >= m (x = 0); tr[j][t] = gamma_j^2 R'(t+1), gamma_j^2 R'(0).  Laid out as
// tk then tr, each [s][kTab].
static std::vector<double> kernel_tables(const Net& net, const fdwt_kernel* k) {
  std::vector<double> t((size_t)2 * net.s * kTab, 0.0);
  for (int j = 0; j < net.s; ++j) {
    const double g = k->gamma[j];
    for (int i = 0; i < kTab; ++i) {
      const int dig = i < net.m ? i + 1 : 0;
      t[(size_t)j * kTab + i] = 1.0 + g * kprime(net.p, k->alpha, dig);
      t[(size_t)(net.s + j) * kTab + i] = g * g * rprime(net.p, k->alpha, dig);
    }
  }
  return t;
}

size_t kernel_tables_bytes(const Net& net) { return (size_t)2 * net.s * kTab * sizeof(double); }

// Consecutive slices of a workspace; with base == nullptr it only measures.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    void* r = base ? base + off : nullptr;
    off += align_up(bytes);
    return r;
  }
};

template <int P, int SMAX>
static int kcols_launch(const Net& net, const double* tk, const double* tr, int c0, int c1, double* out,
                        hipStream_t st) {
  const size_t lds = (size_t)2 * net.s * kTab * 8 +
                     (P == 2 ? (size_t)net.s * 257 * 4 : OddCoords<P == 2 ? 3 : P>::lds_bytes(net.s));
  if (int rc = allow_lds((const void*)k_kernel_cols<P, SMAX>, lds)) return rc;
  NetArgs na = net_args(net);
  void* args[] = {(void*)&na, (void*)&tk, (void*)&tr, (void*)&c0, (void*)&c1, (void*)&out};
  if constexpr (P == 2) {
    if (net.N % 512 == 0) {
      const size_t lds2 = (size_t)2 * net.s * kTab * 8 + (size_t)net.s * 258 * 4;
      if (int rc = allow_lds((const void*)k_kernel_cols2<SMAX>, lds2)) return rc;
      const unsigned grid2 = (unsigned)std::min<int64_t>(net.N / 512, 4096);
      return launch_timed((const void*)k_kernel_cols2<SMAX>, dim3(grid2), dim3(kChunk), args, lds2, st,
                          FDWT_TC_KCOLS, 8.0 * (double)net.N * (c1 - c0));
    }
  }
  const unsigned grid = (unsigned)std::min<int64_t>((net.N + kChunk - 1) / kChunk, 2048);
  return launch_timed((const void*)k_kernel_cols<P, SMAX>, dim3(grid), dim3(kChunk), args, lds, st, FDWT_TC_KCOLS,
                      8.0 * (double)net.N * (c1 - c0));
}

// SMAX: register length of the symmetric-polynomial state (>= s; 8 when only
// K and the U_d columns are wanted).
template <int P>
static int kcols_p(const Net& net, const double* tk, const double* tr, int c0, int c1, double* out,
                   hipStream_t st) {
  const int s = net.s;
  if (c1 <= s + 1 || s <= 8) return kcols_launch<P, 8>(net, tk, tr, c0, c1, out, st);
  if (s <= 16) return kcols_launch<P, 16>(net, tk, tr, c0, c1, out, st);
  if (s <= 24) return kcols_launch<P, 24>(net, tk, tr, c0, c1, out, st);
  if (s <= 32) return kcols_launch<P, 32>(net, tk, tr, c0, c1, out, st);
  if (s <= 48) return kcols_launch<P, 48>(net, tk, tr, c0, c1, out, st);
  return kcols_launch<P, 64>(net, tk, tr, c0, c1, out, st);
}

static int launch_kernel_cols(const Net& net, const double* tk, const double* tr, int c0, int c1, double* out,
                              hipStream_t st) {
  if (net.p == 2) return kcols_p<2>(net, tk, tr, c0, c1, out, st);
  if (net.p == 3) return kcols_p<3>(net, tk, tr, c0, c1, out, st);
  if (net.p == 5) return kcols_p<5>(net, tk, tr, c0, c1, out, st);
  return kcols_p<7>(net, tk, tr, c0, c1, out, st);
}

static unsigned grid1(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 4096); }

int fwt_reduce_f64(int p, int m, const double* in, void* tmp, int batch, const float2* wts, double* partial,
                   double* h0_out, int h0_col, int64_t* parts, hipStream_t st);
int64_t fwt_reduce_parts(int p, int m, size_t elem_bytes);
bool fwt_p2_split_ok(int m);
bool fwt_p2_blocked_ok(int m);
int fwt_p2_first_loge(int m);
int fwt_p2_f64_first(int m, const double* in, double* out, int batch, bool blocked, hipStream_t st);
int fwt_p2_f64_reduce_rest(int m, double* data, int batch, const float2* wts, double* partial, double* h0_out,
                           int h0_col, bool blocked, hipStream_t st);
int fwt_p2_gen_first(int m, int s, const uint32_t* xtab, int nbytes, const double* tab, int ktab, bool kcol,
                     int d0, int d1, double* out, bool blocked, hipStream_t st);
int fwt_p2_f64_rest(int m, double* data, int batch, hipStream_t st);

// ------------------------------------------------------ kernel spectrum
// Unnormalised float64 spectrum of the kernel data K(x_n, 0): p = 2, N
// doubles; p odd, N complex doubles.
size_t spectrum_bytes(const Net& net) { return (size_t)net.N * (net.p == 2 ? 8 : 16); }

struct SpecWs {
  double* tab;  // kernel tables
  double* A;    // kernel data (p odd; p = 2 transforms in place in the spectrum)
};
static void spec_layout(const Net& net, Carve& cv, SpecWs& w) {
  w.tab = (double*)cv.take((size_t)2 * net.s * kTab * sizeof(double));
  w.A = net.p == 2 ? nullptr : (double*)cv.take((size_t)net.N * 8);
}
size_t spectrum_ws_bytes(const Net& net) {
  Carve cv(nullptr);
  SpecWs w;
  spec_layout(net, cv, w);
  return cv.off;
}

// Computes the spectrum into gk (spectrum_bytes); the tables and, for p odd,
// the data go through the first spectrum_ws_bytes of ws.  tab_dev: tables
// already on the device (then they are not staged again), or nullptr.
static int spectrum_into(Net& net, Scratch& sc, const fdwt_kernel* kern, void* ws, void* gk, hipStream_t st,
                         const double* tab_dev = nullptr) {
  Carve cv(ws);
  SpecWs w;
  spec_layout(net, cv, w);
  int rc = FDWT_OK;
  const double* tab = tab_dev;
  if (!tab) {
    const std::vector<double> htab = kernel_tables(net, kern);
    rc = upload(sc, htab.data(), htab.size() * sizeof(double), w.tab, st);
    if (rc) return rc;
    tab = w.tab;
  }
  if (net.p == 2 && fwt_p2_split_ok(net.m)) {
    // K generated inside the first pass of its transform (no column in memory).
    if ((rc = fwt_p2_gen_first(net.m, net.s, net.d_xtab, net.nbytes, tab, kTab, true, 0, 0, (double*)gk, false,
                               st)))
      return rc;
    return fwt_p2_f64_rest(net.m, (double*)gk, 1, st);
  }
  double* A = net.p == 2 ? (double*)gk : w.A;
  rc = launch_kernel_cols(net, tab, tab + (size_t)net.s * kTab, 0, 1, A, st);
  if (rc) return rc;
  if (net.p == 2) return fwt_run_tmp(2, net.m, false, K_F64, A, K_F64, K_F64, A, nullptr, 1, 1.0, st);
  return fwt_run_tmp(net.p, net.m, false, K_F64, A, K_CF64, K_CF64, gk, nullptr, 1, 1.0, st);
}

int run_spectrum(Net& net, Scratch& sc, const fdwt_kernel* kern, void* gk, hipStream_t st) {
  int rc = ensure_ws(sc, spectrum_ws_bytes(net), st);
  if (rc) return rc;
  return spectrum_into(net, sc, kern, sc.ws, gk, st);
}

int cached_spectrum(Net& net, const fdwt_kernel* kern, const void** gk, hipStream_t st) {
  std::vector<double> key(1 + net.s);
  key[0] = kern->alpha;
  for (int j = 0; j < net.s; ++j) key[1 + j] = kern->gamma[j];
  const bool hit = net.spec && key.size() == net.spec_key.size() &&
                   std::memcmp(key.data(), net.spec_key.data(), key.size() * sizeof(double)) == 0;
  if (!hit) {
    const size_t need = spectrum_bytes(net);
    if (net.spec && net.spec_bytes < need) {
      FDWT_HIP(hipStreamSynchronize(st));
      FDWT_HIP(hipFree(net.spec));
      net.spec = nullptr;
    }
    if (!net.spec) {
      if (hipMalloc(&net.spec, need) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FDWT_ENOMEM, "kernel spectrum allocation failed");
      }
      net.spec_bytes = need;
    }
    if (!net.spec_ready) FDWT_HIP(hipEventCreateWithFlags(&net.spec_ready, hipEventDisableTiming));
    net.spec_key.clear();  // invalid until computed
    if (int rc = run_spectrum(net, net.sc, kern, net.spec, st)) return rc;
    FDWT_HIP(hipEventRecord(net.spec_ready, st));
    net.spec_key = key;
  } else {
    FDWT_HIP(hipStreamWaitEvent(st, net.spec_ready, 0));
  }
  *gk = net.spec;
  return FDWT_OK;
}

void drop_spectrum(Net& net) { net.spec_key.clear(); }

void release_spectrum(Net& net) {
  if (net.spec) {
    (void)hipDeviceSynchronize();
    (void)hipFree(net.spec);
  }
  if (net.spec_ready) (void)hipEventDestroy(net.spec_ready);
  net.spec = nullptr;
  net.spec_bytes = 0;
  net.spec_ready = nullptr;
  net.spec_key.clear();
}

// ------------------------------------------------- spline coefficients
struct CoefWs {
  void* gk;  // spectrum (when not given)
  void* sw;  // its workspace
  float2* ct;  // p odd: c~ (complex)
};
static void coef_layout(const Net& net, bool have_gk, Carve& cv, CoefWs& w) {
  w.gk = have_gk ? nullptr : cv.take(spectrum_bytes(net));
  w.sw = have_gk ? nullptr : cv.take(spectrum_ws_bytes(net));
  w.ct = net.p == 2 ? nullptr : (float2*)cv.take((size_t)net.N * sizeof(float2));
}
size_t spline_coef_ws_bytes(const Net& net, bool have_spectrum) {
  Carve cv(nullptr);
  CoefWs w;
  coef_layout(net, have_spectrum, cv, w);
  return cv.off;
}

int run_spline_coef(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* gk_given, const void* ft, float* c,
                    hipStream_t st) {
  const int64_t N = net.N;
  int rc = ensure_ws(sc, spline_coef_ws_bytes(net, gk_given != nullptr), st);
  if (rc) return rc;
  Carve cv(sc.ws);
  CoefWs w;
  coef_layout(net, gk_given != nullptr, cv, w);
  const void* GK = gk_given;
  if (!GK) {
    rc = spectrum_into(net, sc, kern, w.sw, w.gk, st);
    if (rc) return rc;
    GK = w.gk;
  }
  void* ct = net.p == 2 ? (void*)c : (void*)w.ct;
  if (net.p == 2) hipLaunchKernelGGL(k_spec_div<2>, dim3(grid1(N)), dim3(256), 0, st, ft, GK, N, ct);
  else hipLaunchKernelGGL(k_spec_div<3>, dim3(grid1(N)), dim3(256), 0, st, ft, GK, N, ct);  // any odd p
  FDWT_HIP(hipGetLastError());
  // Algorithm 2 (no normalisation); p odd returns the real part.
  if (net.p == 2) return fwt_run_tmp(2, net.m, true, K_F32, ct, K_F32, K_F32, c, nullptr, 1, 1.0, st);
  return fwt_run_tmp(net.p, net.m, true, K_CF32, ct, K_CF32, K_F32, c, ct, 1, 1.0, st);
}

// ----------------------------------------------------------- evaluation
template <int P>
static int launch_eval(Net& net, const void* Xp, const float* c, int64_t nq, const void* qv, const float* tl,
                       df* partial, int gy, int64_t ppc, hipStream_t st) {
  const dim3 grid((unsigned)((nq + 255) / 256), (unsigned)gy);
  const int s = net.s;
  const size_t xb = P == 2 ? 4 : 8;  // staged bytes per point and coordinate
  // Tables, then the staged points (p odd: high and low words of the strings).
#define FDWT_EVAL(SM)                                                                              \
  {                                                                                                \
    auto fn = k_spline_eval<P, SM>;                                                                \
    constexpr size_t ns_ = eval_ns<SM>();                                                          \
    const size_t lds = (size_t)s * kTabE * 4 + (size_t)s * ns_ * xb + ns_ * 4;                     \
    if (int rc_ = allow_lds((const void*)fn, lds)) return rc_;                                     \
    hipLaunchKernelGGL(fn, grid, dim3(256), lds, st, Xp, c, net.N, s, qv, nq, tl, ppc, partial);   \
  }
  if (s <= 8) FDWT_EVAL(8)
  else if (s <= 16) FDWT_EVAL(16)
  else if (s <= 32) FDWT_EVAL(32)
  else FDWT_EVAL(64)
#undef FDWT_EVAL
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

size_t eval_tables_bytes(const Net& net) { return (size_t)net.s * kTabE * 4; }

size_t packed_bytes(const Net& net) { return (size_t)net.s * net.N * (net.p == 2 ? 4 : 8); }

// Grid of the evaluation: query blocks x point chunks, >= ~2048 workgroups in
// total; it depends on (N, nq) only, so a result never depends on where or
// alongside what it runs.
static void eval_grid(int64_t N, int64_t nq, int* gy_out, int64_t* ppc_out) {
  const int64_t qb = (nq + 255) / 256;
  int gy = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + qb - 1) / qb, (N + kNSMax - 1) / kNSMax));
  int64_t ppc = (N + gy - 1) / gy;
  ppc = (ppc + kNSMax - 1) / kNSMax * kNSMax;
  gy = (int)((N + ppc - 1) / ppc);
  *gy_out = gy;
  *ppc_out = ppc;
}

struct EvalWs {
  float* tl;     // factor tables [s][kTabE]
  void* Xp;      // packed coordinates (when not given)
  uint64_t* qs;  // p odd: query digit strings [s][nq]
  df* partial;
};
static void eval_layout(const Net& net, int64_t nq, bool have_packed, Carve& cv, EvalWs& w) {
  const int p = net.p, s = net.s;
  int gy;
  int64_t ppc;
  eval_grid(net.N, nq, &gy, &ppc);
  w.tl = (float*)cv.take(eval_tables_bytes(net));
  w.Xp = have_packed ? nullptr : cv.take(packed_bytes(net));
  w.qs = p == 2 ? nullptr : (uint64_t*)cv.take((size_t)s * nq * 8);
  w.partial = (df*)cv.take((size_t)gy * nq * sizeof(df));
}
size_t spline_eval_ws_bytes(const Net& net, int64_t nq, bool have_packed) {
  Carve cv(nullptr);
  EvalWs w;
  eval_layout(net, nq, have_packed, cv, w);
  return cv.off;
}

int run_spline_eval(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* packed, const float* c, int64_t nq,
                    const uint32_t* q, float* sf, hipStream_t st) {
  const int p = net.p, s = net.s, m = net.m;
  const int D = query_depth(p);
  const int64_t N = net.N;
  int gy;
  int64_t ppc;
  eval_grid(N, nq, &gy, &ppc);
  int rc = ensure_ws(sc, spline_eval_ws_bytes(net, nq, packed != nullptr), st);
  if (rc) return rc;
  Carve cv(sc.ws);
  EvalWs w;
  eval_layout(net, nq, packed != nullptr, cv, w);
  // Factor 1 + gamma_j K'(t+1) of first differing digit t < D, and 1 + gamma_j
  // when all D digits agree, at entry c + 1 of the leading-zero count c that
  // k_spline_eval computes (p = 2: c = t, or -1 when equal; p odd: c = Bt+1..Bt+B,
  // or 64 when equal).  For p odd, entry 0 (high words equal, c = -1) is a
  // NaN: it marks the points whose low words must be read.
  const int B = p == 3 ? kStrBits<3> : kStrBits<5>;  // digit-string field width (coords.h)
  std::vector<float> htl((size_t)s * kTabE, 1.0f);
  for (int j = 0; j < s; ++j) {
    float* row = htl.data() + (size_t)j * kTabE;
    const float eq = (float)(1.0 + kern->gamma[j] * kprime(p, kern->alpha, 0));
    for (int t = 0; t < D; ++t) {
      const float v = (float)(1.0 + kern->gamma[j] * kprime(p, kern->alpha, t + 1));
      if (p == 2) row[t + 1] = v;
      else for (int l = B * t + 1; l <= B * t + B; ++l) row[l + 1] = v;
    }
    row[p == 2 ? 0 : 65] = eq;
    if (p != 2) row[0] = std::numeric_limits<float>::quiet_NaN();
  }
  rc = upload(sc, htl.data(), htl.size() * 4, w.tl, st);
  if (rc) return rc;
  const void* Xp = packed;
  if (!Xp) {
    rc = launch_net_packed(net, w.Xp, st);
    if (rc) return rc;
    Xp = w.Xp;
  }
  const void* qv = q;
  if (p != 2) {
    if (p == 3) hipLaunchKernelGGL(k_query_prep<3>, dim3(grid1((int64_t)s * nq)), dim3(256), 0, st, q, nq, s, D, w.qs);
    else if (p == 5) hipLaunchKernelGGL(k_query_prep<5>, dim3(grid1((int64_t)s * nq)), dim3(256), 0, st, q, nq, s, D, w.qs);
    else hipLaunchKernelGGL(k_query_prep<7>, dim3(grid1((int64_t)s * nq)), dim3(256), 0, st, q, nq, s, D, w.qs);
    FDWT_HIP(hipGetLastError());
    qv = w.qs;
  }
  hipEvent_t tb = timed_begin(st);
  if (p == 2) rc = launch_eval<2>(net, Xp, c, nq, qv, w.tl, w.partial, gy, ppc, st);
  else rc = launch_eval<3>(net, Xp, c, nq, qv, w.tl, w.partial, gy, ppc, st);  // any odd p: digit strings
  if (rc) return rc;
  timed_end(tb, st, FDWT_TC_EVAL, (double)nq * (double)N * s);
  hipLaunchKernelGGL(k_eval_finish, dim3(grid1(nq)), dim3(256), 0, st, w.partial, gy, nq, sf);
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

// -------------------------------------------------- effective dimension
// Columns of kernel data per chunk so that data (8 B) + intermediate (8 or
// 16 B) per column stay within `budget` bytes.  The variances do not depend
// on the chunking: every column is transformed and reduced on its own.
int eff_dim_chunk(const Net& net, size_t budget) {
  const size_t wb = (net.p == 2) ? 8 : 16;
  const size_t per_col = (size_t)net.N * (8 + wb);
  return (int)std::max<size_t>(1, std::min<size_t>((size_t)2 * net.s, budget / per_col));
}

size_t eff_dim_res_bytes(const Net& net) { return (size_t)(2 * net.s + 2) * sizeof(double); }

// Blocked intermediate layout of the p = 2 variance transforms
// (FDWT_EFFDIM_BLOCKED = 0 turns it off: each grouped-sum tile holds the same
// elements either way, so the variances are bit-identical).
static bool effdim_blocked() {  // read at each call
  const char* e = getenv("FDWT_EFFDIM_BLOCKED");
  return e ? atoi(e) != 0 : true;
}

struct EffWs {
  void* gk;
  void* sw;
  double* tab;
  float2* wts;
  double* A;
  void* B;
  double* partial;
  double* qmc_partial;
  double* res;
};
// Columns transformed for the variances: U_1..U_s and Q_1..Q_{s-1}.  Q_s is
// not needed: sigma^2_sup(s) = sigma^2_trc(s) = sigma^2(Sf) (Section 4), so
// its increment is the total minus sigma^2_sup(s - 1).
static int effdim_cols(int s) { return 2 * s - 1; }

static void eff_layout(const Net& net, bool have_gk, int ch, Carve& cv, EffWs& w) {
  const int ncols = effdim_cols(net.s);
  const size_t wb = (net.p == 2) ? sizeof(double) : sizeof(double2);
  const int64_t parts = fwt_reduce_parts(net.p, net.m, wb);
  w.gk = have_gk ? nullptr : cv.take(spectrum_bytes(net));
  w.sw = have_gk ? nullptr : cv.take(spectrum_ws_bytes(net));
  w.tab = (double*)cv.take((size_t)2 * net.s * kTab * sizeof(double));
  w.wts = (float2*)cv.take((size_t)net.N * sizeof(float2));
  w.A = (double*)cv.take((size_t)ch * net.N * 8);
  w.B = cv.take((size_t)ch * net.N * wb);
  w.partial = (double*)cv.take((size_t)ncols * parts * sizeof(double) + kRedBlocks * sizeof(double));
  w.qmc_partial = w.partial ? w.partial + (size_t)ncols * parts : nullptr;
  w.res = (double*)cv.take(eff_dim_res_bytes(net));
}
size_t eff_dim_ws_bytes(const Net& net, bool have_spectrum, int chunk) {
  Carve cv(nullptr);
  EffWs w;
  eff_layout(net, have_spectrum, chunk, cv, w);
  return cv.off;
}

// Enqueues the whole variance computation on st; the 2s + 2 result doubles
// (sigma^2_trc(d) for d = 1..s, the superposition increments for j = 1..s-1,
// an unused slot, sigma^2_QMC and the h = 0 share) land in res_host (pinned)
// when st reaches this point (when res_host is given; *res_dev receives their
// device copy).
// gk_given: a cached spectrum, or nullptr to compute it here.
int eff_dim_enqueue(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* gk_given, const void* ft, int ch,
                    double* res_host, const double** res_dev, hipStream_t st) {
  const int p = net.p, s = net.s;
  const int64_t N = net.N;
  const size_t wb = (p == 2) ? sizeof(double) : sizeof(double2);
  const int ncols = effdim_cols(s);  // U_1..U_s, Q_1..Q_{s-1} (generator columns 1..2s-1)
  const int64_t parts = fwt_reduce_parts(p, net.m, wb);  // partial sums per column
  int rc = ensure_ws(sc, eff_dim_ws_bytes(net, gk_given != nullptr, ch), st);
  if (rc) return rc;
  Carve cv(sc.ws);
  EffWs w;
  eff_layout(net, gk_given != nullptr, ch, cv, w);
  const std::vector<double> htab = kernel_tables(net, kern);
  rc = upload(sc, htab.data(), htab.size() * sizeof(double), w.tab, st);
  if (rc) return rc;
  const void* GK = gk_given;
  if (!GK) {
    rc = spectrum_into(net, sc, kern, w.sw, w.gk, st, w.tab);
    if (rc) return rc;
    GK = w.gk;
  }
  double* h0 = w.res + 2 * s + 1;  // h = 0 share of the total
  const double pm = (double)N;
  // p = 2 two-pass plans keep the intermediate columns in the blocked layout
  // (the grouped-sum pass then reads contiguous tiles and weights).
  const bool blk = p == 2 && fwt_p2_blocked_ok(net.m) && effdim_blocked();
  const int blkF = blk ? fwt_p2_first_loge(net.m) : 0;
  if (p == 2) hipLaunchKernelGGL(k_effdim_weights<2>, dim3(kRedBlocks), dim3(256), 0, st, ft, GK, N, pm, w.wts, w.qmc_partial, blkF, net.m);
  else hipLaunchKernelGGL(k_effdim_weights<3>, dim3(kRedBlocks), dim3(256), 0, st, ft, GK, N, pm, w.wts, w.qmc_partial, 0, net.m);  // any odd p
  FDWT_HIP(hipGetLastError());
  const int h0c = s - 1;  // U_s: its h = 0 term is the h = 0 share of the total
  const double* tr = w.tab + (size_t)s * kTab;
  for (int c0 = 0; c0 < ncols; c0 += ch) {
    const int c1 = std::min(ncols, c0 + ch);
    const int h0_col = (h0c >= c0 && h0c < c1) ? h0c - c0 : -1;
    if (p == 2 && fwt_p2_split_ok(net.m)) {
      // Chunk columns [c0, c1): the U_d among them are generated inside the
      // first pass of their transforms (B columns 0..nu-1); only the Q_j go
      // through memory (kernel data in A, first pass into B after the U_d).
      double* B = (double*)w.B;
      const int u1 = std::min(c1, s), nu = std::max(0, u1 - c0);
      if (nu > 0 && (rc = fwt_p2_gen_first(net.m, s, net.d_xtab, net.nbytes, tr, kTab, false, c0, u1, B, blk, st)))
        return rc;
      const int q0 = std::max(c0, s);
      if (q0 < c1) {
        if ((rc = launch_kernel_cols(net, w.tab, tr, q0 + 1, c1 + 1, w.A, st))) return rc;
        if ((rc = fwt_p2_f64_first(net.m, w.A, B + (size_t)nu * N, c1 - q0, blk, st))) return rc;
      }
      rc = fwt_p2_f64_reduce_rest(net.m, B, c1 - c0, w.wts, w.partial + (size_t)c0 * parts, h0, h0_col, blk, st);
    } else {
      rc = launch_kernel_cols(net, w.tab, tr, c0 + 1, c1 + 1, w.A, st);
      if (rc) return rc;
      int64_t t = 0;
      rc = fwt_reduce_f64(p, net.m, w.A, w.B, c1 - c0, w.wts, w.partial + (size_t)c0 * parts, h0, h0_col, &t, st);
    }
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_sum_rows, dim3(ncols), dim3(kSumThreads), 0, st, w.partial, (int)parts, w.res);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kSumThreads), 0, st, w.qmc_partial, kRedBlocks, w.res + 2 * s);
  FDWT_HIP(hipGetLastError());
  if (res_dev) *res_dev = w.res;
  if (res_host) FDWT_HIP(hipMemcpyAsync(res_host, w.res, eff_dim_res_bytes(net), hipMemcpyDeviceToHost, st));
  return FDWT_OK;
}

// Variances and dimensions from the 2s + 2 result doubles (Section 5's
// definitions: the smallest d whose variance reaches 0.99 sigma^2).
void eff_dim_finish(int s, const double* r, fdwt_effdim* out) {
  out->var_trc[0] = 0.0;
  out->var_sup[0] = 0.0;
  for (int d = 1; d <= s; ++d) {
    out->var_trc[d] = r[d - 1];
    out->var_sup[d] = d < s ? out->var_sup[d - 1] + r[s + d - 1] : r[s - 1];  // sup(s) = trc(s)
  }
  out->var_total = out->var_trc[s];
  out->var_qmc = r[2 * s];
  out->var_total_h0 = r[2 * s + 1];
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
}

// Column budget of the one-call eff_dim (FDWT_EFFDIM_CHUNK_MB overrides the
// 12 GiB default; results do not depend on it).
static size_t effdim_budget() {
  static const size_t b = [] {
    const char* e = getenv("FDWT_EFFDIM_CHUNK_MB");
    const long v = e ? atol(e) : 12 * 1024;
    return (size_t)std::max(1L, v) << 20;
  }();
  return b;
}

int run_eff_dim(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* ft, fdwt_effdim* out, hipStream_t st) {
  const int ch = eff_dim_chunk(net, effdim_budget());
  const double* res_dev = nullptr;
  const void* gk = nullptr;
  int rc = cached_spectrum(net, kern, &gk, st);
  if (rc) return rc;
  rc = eff_dim_enqueue(net, sc, kern, gk, ft, ch, nullptr, &res_dev, st);
  if (rc) return rc;
  std::vector<double> res(2 * net.s + 2);
  FDWT_HIP(hipStreamSynchronize(st));
  FDWT_HIP(hipMemcpy(res.data(), res_dev, eff_dim_res_bytes(net), hipMemcpyDeviceToHost));
  eff_dim_finish(net.s, res.data(), out);
  return FDWT_OK;
}

// ------------------------------------------------------ query depth
// Queries of q_depth digits, Q p^-q_depth, as queries of the full depth D:
// Q p^(D - q_depth) (the same point; its digits past q_depth are zero).
__global__ void __launch_bounds__(256) k_lift_queries(const uint32_t* __restrict__ q, int64_t n, uint32_t mul,
                                                      uint32_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = q[i] * mul;
}

int lift_queries(const Net& net, const uint32_t* q, int64_t nq, int q_depth, uint32_t* out, hipStream_t st) {
  const int D = query_depth(net.p);
  if (q_depth < 1 || q_depth > D) return fail(FDWT_EINVAL, "q_depth must be in 1.." + std::to_string(D));
  uint32_t mul = 1;
  for (int i = q_depth; i < D; ++i) mul *= (uint32_t)net.p;
  const int64_t n = nq * net.s;
  if (n > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_lift_queries, dim3(grid), dim3(256), 0, st, q, n, mul, out);
    FDWT_HIP(hipGetLastError());
  }
  return FDWT_OK;
}

// ------------------------------------------------------- split cost
int run_split_cost(Net& tr, Scratch& sc, const uint32_t* delta, const float* ft, const float* fval,
                   const fdwt_kernel* kern, float* sf_out, double* cost, hipStream_t st) {
  const int s = tr.s, m2 = tr.m + 1;
  const int64_t N = tr.N;
  Carve need(nullptr);
  need.take(spectrum_bytes(tr));
  need.take(spectrum_ws_bytes(tr));
  need.take((size_t)s * kTab * sizeof(double));
  need.take((size_t)s * 4);
  need.take((size_t)N * 8);
  need.take(kRedBlocks * sizeof(double));
  need.take(sizeof(double));
  if (int rc = ensure_ws(sc, need.off, st)) return rc;
  Carve cv(sc.ws);
  double* gk = (double*)cv.take(spectrum_bytes(tr));
  void* sw = cv.take(spectrum_ws_bytes(tr));
  double* tk2 = (double*)cv.take((size_t)s * kTab * sizeof(double));
  uint32_t* dd = (uint32_t*)cv.take((size_t)s * 4);
  double* g = (double*)cv.take((size_t)N * 8);
  double* partial = (double*)cv.take(kRedBlocks * sizeof(double));
  double* res = (double*)cv.take(sizeof(double));
  int rc = spectrum_into(tr, sc, kern, sw, gk, st);  // K_u, unnormalised
  if (rc) return rc;
  std::vector<double> h2((size_t)s * kTab, 1.0);
  for (int j = 0; j < s; ++j)
    for (int t = 0; t <= m2; ++t)
      h2[(size_t)j * kTab + t] = 1.0 + kern->gamma[j] * kprime(2, kern->alpha, t < m2 ? t + 1 : 0);
  if ((rc = upload(sc, h2.data(), h2.size() * sizeof(double), tk2, st))) return rc;
  if ((rc = upload(sc, delta, (size_t)s * 4, dd, st))) return rc;
  const size_t lds = (size_t)s * kTab * 8 + (size_t)((s + 1) & ~1) * 4 + (size_t)s * 257 * 4;
  if ((rc = allow_lds((const void*)k_kernel_shift_p2, lds))) return rc;
  const unsigned grid = (unsigned)std::min<int64_t>((N + kChunk - 1) / kChunk, 2048);
  hipLaunchKernelGGL(k_kernel_shift_p2, dim3(grid), dim3(kChunk), lds, st, net_args(tr), dd, tk2, m2, g);
  FDWT_HIP(hipGetLastError());
  if ((rc = fwt_run_tmp(2, tr.m, false, K_F64, g, K_F64, K_F64, g, nullptr, 1, 1.0, st))) return rc;
  hipLaunchKernelGGL(k_split_combine, dim3(grid1(N)), dim3(256), 0, st, ft, gk, g, N);
  FDWT_HIP(hipGetLastError());
  if ((rc = fwt_run_tmp(2, tr.m, true, K_F64, g, K_F64, K_F64, g, nullptr, 1, 1.0, st))) return rc;
  hipLaunchKernelGGL(k_sq_diff, dim3(kRedBlocks), dim3(256), 0, st, fval, g, N, partial, sf_out);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kSumThreads), 0, st, partial, kRedBlocks, res);
  FDWT_HIP(hipGetLastError());
  FDWT_HIP(hipStreamSynchronize(st));
  FDWT_HIP(hipMemcpy(cost, res, sizeof(double), hipMemcpyDeviceToHost));
  return FDWT_OK;
}

}  // namespace fdwt
