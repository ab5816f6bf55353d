// Digital net generation and test-function sampling on the device
// (Definition of a digital net, Eq. (defy): y_vec = C_j n_vec over Z_p,
// x_{j,n} = sum_r y_{j,n,r} p^-r).
//
// Coordinates come from the table machinery of coords.h (byte tables and
// per-group XORs for p = 2, packed digits for p odd).
//
// Points in float are x = X p^-m rounded once to nearest.  p = 2: (float)X
// rounds (only for m > 24) and the power of two scales exactly.  p odd:
// x_d = (double)X * (double)p^-m is within 2^-52 (relative) of X / p^m, and
// X / p^m is at least 2^-25 p^-m >= 2^-51 (relative) away from every
// midpoint between two floats (a midpoint is M 2^-k with M odd, and
// X 2^k - M p^m is a non-zero integer since M p^m is odd), so rounding x_d
// to float gives the correctly rounded point.
#include "coords.h"
#include "dev_math.h"
#include "family.h"

#include <cmath>

namespace fdwt {

// ------------------------------------------------------------- kernels
// Output modes of the coordinate kernel.
enum CoordMode { CM_DIGITS = 0, CM_POINTS = 1, CM_SHIFTED = 2 };

template <int MODE>
__global__ void __launch_bounds__(kChunk) k_coords_p2(const uint32_t* xtab, int nbytes, int s, int m,
                                                      int64_t N, void* out) {
  extern __shared__ uint32_t lds_t0[];
  P2Coords pc{xtab, nbytes, s, lds_t0, lds_t0 + s * 256};
  pc.stage_tables();
  const float inv = 1.0f / (float)(1u << m);  // exact power of two
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < N; base += (int64_t)gridDim.x * kChunk) {
    __syncthreads();
    pc.stage_group(base);
    __syncthreads();
    const int64_t n = base + threadIdx.x;
    if (n < N) {
      for (int j = 0; j < s; ++j) {
        const uint32_t X = pc.X(j, n);
        if (MODE == CM_DIGITS) ((uint32_t*)out)[(int64_t)j * N + n] = X;
        if (MODE == CM_POINTS) ((float*)out)[(int64_t)j * N + n] = (float)X * inv;
        if (MODE == CM_SHIFTED) ((uint32_t*)out)[(int64_t)j * N + n] = X << (32 - m);
      }
    }
  }
}

template <int P, int MODE>
__global__ void __launch_bounds__(kChunk) k_coords_odd(const uint64_t* ptab, int s, int m, int64_t N,
                                                       double inv_pm, void* out) {
  extern __shared__ __align__(16) uint64_t lds_odd[];
  OddCoords<P> oc{ptab, s, m, lds_odd, lds_odd + s * OddCoords<P>::PK};
  oc.stage_tables();
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < N; base += (int64_t)gridDim.x * kChunk) {
    __syncthreads();
    oc.stage_group(base);
    __syncthreads();
    const int64_t n = base + threadIdx.x;
    if (n < N) {
      int r, k;
      oc.split(n, r, k);
      for (int j = 0; j < s; ++j) {
        const uint64_t pk = oc.X(j, r, k);
        if (MODE == CM_DIGITS) ((uint32_t*)out)[(int64_t)j * N + n] = canon_odd<P>(pk, m);
        if (MODE == CM_POINTS) ((float*)out)[(int64_t)j * N + n] = (float)((double)canon_odd<P>(pk, m) * inv_pm);
        if (MODE == CM_SHIFTED) ((uint64_t*)out)[(int64_t)j * N + n] = eval_string_odd<P>(pk, m);
      }
    }
  }
}

// p = 2: a workgroup takes blocks of kSampleBlock = 4096 consecutive points;
// thread t owns base + t + 256 k (k < 16).  X_j is linear over Z_2 in the bits
// of n and base, t and 256 k occupy disjoint bits, so X_j(n) is the XOR of
// X_j(base) (uniform), X_j(t) (one table read per coordinate) and X_j(256 k)
// (four 16-byte broadcasts per coordinate): about one XOR per point and
// coordinate besides the family's arithmetic.
constexpr int kSampleBlock = 4096;
template <int FAM>
__global__ void __launch_bounds__(256) k_sample_p2(const uint32_t* xtab, int nbytes, FamilyArgs fa, int m,
                                                   int64_t N, float* f) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int s = fa.s;
  uint32_t* t0 = lds;               // [s][256]: X_j(t)
  uint32_t* t1 = t0 + s * 256;      // [s][16]:  X_j(256 k)
  uint32_t* ub = t1 + s * 16;       // [s]: X_j(base)
  float* la = reinterpret_cast<float*>(ub + kMaxS);
  float* li = la + kMaxS;
  const int tid = threadIdx.x;
  for (int i = tid; i < s * 256; i += 256) t0[i] = xtab[(size_t)(i >> 8) * nbytes * 256 + (i & 255)];
  for (int i = tid; i < s * 16; i += 256) t1[i] = nbytes > 1 ? xtab[((size_t)(i >> 4) * nbytes + 1) * 256 + (i & 15)] : 0u;
  for (int j = tid; j < s; j += 256) {
    la[j] = fa.a[j];
    li[j] = fa.inv1a[j];
  }
  const float inv = 1.0f / (float)(1u << m);
  for (int64_t base = (int64_t)blockIdx.x * kSampleBlock; base < N; base += (int64_t)gridDim.x * kSampleBlock) {
    __syncthreads();
    for (int j = tid; j < s; j += 256) {
      uint32_t v = 0;
      const uint32_t* tj = xtab + (size_t)j * nbytes * 256;
      for (int b = 1; b < nbytes; ++b) v ^= tj[b * 256 + (int)((base >> (8 * b)) & 255)];
      ub[j] = v;
    }
    __syncthreads();
    typename FamState<FAM>::T acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = fam_init<FAM>(fa);
    for (int j = 0; j < s; ++j) {
      const uint32_t xl = t0[j * 256 + tid] ^ ub[j];
      const uint4* r = reinterpret_cast<const uint4*>(t1 + j * 16);
      const uint4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
      const uint32_t kx[16] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                               r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w};
      const float a = la[j], ia = li[j];
#pragma unroll
      for (int k = 0; k < 16; ++k) fam_step<FAM, false>(acc[k], fa, a, ia, xl ^ kx[k], inv, (double)inv);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t n = base + tid + 256 * k;
      if (n < N) f[n] = fam_final<FAM>(acc[k], fa);
    }
  }
}

template <int P, int FAM>
__global__ void __launch_bounds__(kChunk) k_sample_odd(const uint64_t* ptab, FamilyArgs fa, int m, int64_t N,
                                                       double inv_pm_d, float* f) {
  extern __shared__ __align__(16) uint64_t lds_odd[];
  const int s = fa.s;
  OddCoords<P> oc{ptab, s, m, lds_odd, lds_odd + s * OddCoords<P>::PK};
  float* la = reinterpret_cast<float*>(lds_odd + OddCoords<P>::lds_bytes(s) / 8);
  float* li = la + kMaxS;
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    la[j] = fa.a[j];
    li[j] = fa.inv1a[j];
  }
  oc.stage_tables();
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < N; base += (int64_t)gridDim.x * kChunk) {
    __syncthreads();
    oc.stage_group(base);
    __syncthreads();
    const int64_t n = base + threadIdx.x;
    if (n < N) {
      int r, k;
      oc.split(n, r, k);
      auto acc = fam_init<FAM>(fa);
      for (int j = 0; j < s; ++j)
        fam_step<FAM, true>(acc, fa, la[j], li[j], canon_odd<P>(oc.X(j, r, k), m), 0.0f, inv_pm_d);
      f[n] = fam_final<FAM>(acc, fa);
    }
  }
}

// ----------------------------------------------------------- launchers
// Enough workgroups to fill the chip several times over, few enough that the
// per-workgroup table staging is amortised over many point groups.
static unsigned grid_for(int64_t N, int threads) {
  int64_t b = (N + threads - 1) / threads;
  return (unsigned)std::min<int64_t>(b, 2048);
}

static double inv_pm(const Net& net) { return 1.0 / (double)net.N; }

template <int MODE>
static int coords(const Net& net, void* out, hipStream_t st) {
  const unsigned g = grid_for(net.N, 256);
  if (net.p == 2) {
    if (int rc = allow_lds((const void*)k_coords_p2<MODE>, (size_t)net.s * 257 * 4)) return rc;
    hipLaunchKernelGGL(k_coords_p2<MODE>, dim3(g), dim3(kChunk), (size_t)net.s * 257 * 4, st, net.d_xtab,
                       net.nbytes, net.s, net.m, net.N, out);
  } else if (net.p == 3) {
    const size_t lds = OddCoords<3>::lds_bytes(net.s);
    if (int rc = allow_lds((const void*)k_coords_odd<3, MODE>, lds)) return rc;
    hipLaunchKernelGGL((k_coords_odd<3, MODE>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, net.s, net.m,
                       net.N, inv_pm(net), out);
  } else if (net.p == 5) {
    const size_t lds = OddCoords<5>::lds_bytes(net.s);
    if (int rc = allow_lds((const void*)k_coords_odd<5, MODE>, lds)) return rc;
    hipLaunchKernelGGL((k_coords_odd<5, MODE>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, net.s, net.m,
                       net.N, inv_pm(net), out);
  } else {
    const size_t lds = OddCoords<7>::lds_bytes(net.s);
    if (int rc = allow_lds((const void*)k_coords_odd<7, MODE>, lds)) return rc;
    hipLaunchKernelGGL((k_coords_odd<7, MODE>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, net.s, net.m,
                       net.N, inv_pm(net), out);
  }
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

int launch_net_digits(const Net& net, uint32_t* X, hipStream_t st) { return coords<CM_DIGITS>(net, X, st); }
int launch_net_points(const Net& net, float* x, hipStream_t st) { return coords<CM_POINTS>(net, x, st); }
int launch_net_packed(const Net& net, void* out, hipStream_t st) { return coords<CM_SHIFTED>(net, out, st); }

template <int FAM>
static int sample_fam(const Net& net, const FamilyArgs& fa, float* f, unsigned g, hipStream_t st) {
  if (net.p == 2) {
    const size_t lds = (size_t)net.s * (256 + 16) * 4 + kMaxS * 4 + 2 * kMaxS * 4;
    const unsigned g2 = (unsigned)std::min<int64_t>((net.N + kSampleBlock - 1) / kSampleBlock, 4096);
    if (int rc = allow_lds((const void*)k_sample_p2<FAM>, lds)) return rc;
    hipLaunchKernelGGL(k_sample_p2<FAM>, dim3(g2), dim3(256), lds, st, net.d_xtab, net.nbytes, fa, net.m,
                       net.N, f);
  } else if (net.p == 3) {
    const size_t lds = OddCoords<3>::lds_bytes(net.s) + 2 * kMaxS * 4;
    if (int rc = allow_lds((const void*)k_sample_odd<3, FAM>, lds)) return rc;
    hipLaunchKernelGGL((k_sample_odd<3, FAM>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, fa, net.m, net.N,
                       inv_pm(net), f);
  } else if (net.p == 5) {
    const size_t lds = OddCoords<5>::lds_bytes(net.s) + 2 * kMaxS * 4;
    if (int rc = allow_lds((const void*)k_sample_odd<5, FAM>, lds)) return rc;
    hipLaunchKernelGGL((k_sample_odd<5, FAM>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, fa, net.m, net.N,
                       inv_pm(net), f);
  } else {
    const size_t lds = OddCoords<7>::lds_bytes(net.s) + 2 * kMaxS * 4;
    if (int rc = allow_lds((const void*)k_sample_odd<7, FAM>, lds)) return rc;
    hipLaunchKernelGGL((k_sample_odd<7, FAM>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, fa, net.m, net.N,
                       inv_pm(net), f);
  }
  return FDWT_OK;
}

FamilyArgs make_family_args(const Net& net, int family, const double* a) {
  FamilyArgs fa;
  fa.s = net.s;
  if (family == FDWT_FAMILY_ASIAN) {
    // a = (S0, K, sigma, r, T)
    const double dt = a[4] / net.s;
    fa.g[0] = std::log(a[0]);
    fa.g[1] = a[1];
    fa.g[2] = (a[3] - 0.5 * a[2] * a[2]) * dt;
    fa.g[3] = a[2] * std::sqrt(dt);
    fa.g[4] = std::exp(-a[3] * a[4]);
    fa.g[5] = 1.0 / (net.s + 1);
  } else {
    for (int j = 0; j < net.s; ++j) {
      fa.a[j] = (float)a[j];
      fa.inv1a[j] = (float)(1.0 / (1.0 + a[j]));
    }
  }
  return fa;
}

int launch_sample(const Net& net, int family, const double* a, float* f, hipStream_t st) {
  const FamilyArgs fa = make_family_args(net, family, a);
  const unsigned g = grid_for(net.N, 256);
  hipEvent_t tb = timed_begin(st);
  int rc;
  if (family == FDWT_FAMILY_PRODUCT) rc = sample_fam<FDWT_FAMILY_PRODUCT>(net, fa, f, g, st);
  else if (family == FDWT_FAMILY_EXP) rc = sample_fam<FDWT_FAMILY_EXP>(net, fa, f, g, st);
  else if (family == FDWT_FAMILY_ASIAN) rc = sample_fam<FDWT_FAMILY_ASIAN>(net, fa, f, g, st);
  else rc = sample_fam<FDWT_FAMILY_WANGFANG>(net, fa, f, g, st);
  if (rc) return rc;
  FDWT_HIP(hipGetLastError());
  timed_end(tb, st, FDWT_TC_SAMPLE, 4.0 * (double)net.N);
  return FDWT_OK;
}

}  // namespace fdwt
