// Digital net generation and test-function sampling on the device
// (Definition of a digital net, Eq. (defy): y_vec = C_j n_vec over Z_p,
// x_{j,n} = sum_r y_{j,n,r} p^-r).
//
// Coordinates come from the table machinery of coords.h (byte tables and
// per-group XORs for p = 2, packed digits for p odd).
#include "coords.h"
#include "dev_math.h"

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
                                                       float inv_pm, void* out) {
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
        if (MODE == CM_POINTS) ((float*)out)[(int64_t)j * N + n] = (float)canon_odd<P>(pk, m) * inv_pm;
        if (MODE == CM_SHIFTED) ((uint64_t*)out)[(int64_t)j * N + n] = eval_string_odd(pk, m);
      }
    }
  }
}

// Test-function families (float arithmetic).
struct FamilyArgs {
  int s;
  float a[kMaxS];
  float inv1a[kMaxS];  // 1 / (1 + a_j), Section 5.2 function
};

template <int FAM>
__device__ __forceinline__ float fam_init() {
  return FAM == FDWT_FAMILY_EXP ? 0.0f : 1.0f;
}
template <int FAM>
__device__ __forceinline__ float fam_step(float acc, float a, float inv1a, float x) {
  if constexpr (FAM == FDWT_FAMILY_PRODUCT) return acc * (1.0f + a * (x - 0.5f));
  else if constexpr (FAM == FDWT_FAMILY_EXP) return acc + a * x * x;
  else return acc * ((fabsf(4.0f * x - 2.0f) + a) * inv1a);
}
template <int FAM>
__device__ __forceinline__ float fam_final(float acc) {
  if constexpr (FAM == FDWT_FAMILY_EXP) return expf(-acc);
  else return acc;
}

template <int FAM>
__global__ void __launch_bounds__(kChunk) k_sample_p2(const uint32_t* xtab, int nbytes, FamilyArgs fa, int m,
                                                      int64_t N, float* f) {
  extern __shared__ uint32_t lds[];
  const int s = fa.s;
  P2Coords pc{xtab, nbytes, s, lds, lds + s * 256};
  float* la = reinterpret_cast<float*>(lds + s * 256 + kMaxS);
  float* li = la + kMaxS;
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    la[j] = fa.a[j];
    li[j] = fa.inv1a[j];
  }
  pc.stage_tables();
  const float inv = 1.0f / (float)(1u << m);
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < N; base += (int64_t)gridDim.x * kChunk) {
    __syncthreads();
    pc.stage_group(base);
    __syncthreads();
    const int64_t n = base + threadIdx.x;
    float acc = fam_init<FAM>();
    for (int j = 0; j < s; ++j) acc = fam_step<FAM>(acc, la[j], li[j], (float)pc.X(j, n) * inv);
    if (n < N) f[n] = fam_final<FAM>(acc);
  }
}

template <int P, int FAM>
__global__ void __launch_bounds__(kChunk) k_sample_odd(const uint64_t* ptab, FamilyArgs fa, int m, int64_t N,
                                                       float inv_pm, float* f) {
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
      float acc = fam_init<FAM>();
      for (int j = 0; j < s; ++j) {
        const uint32_t X = canon_odd<P>(oc.X(j, r, k), m);
        acc = fam_step<FAM>(acc, la[j], li[j], (float)X * inv_pm);
      }
      f[n] = fam_final<FAM>(acc);
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

static float inv_pm(const Net& net) { return (float)(1.0 / (double)net.N); }

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
  } else {
    const size_t lds = OddCoords<5>::lds_bytes(net.s);
    if (int rc = allow_lds((const void*)k_coords_odd<5, MODE>, lds)) return rc;
    hipLaunchKernelGGL((k_coords_odd<5, MODE>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, net.s, net.m,
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
    const size_t lds = (size_t)net.s * 257 * 4 + 2 * kMaxS * 4 + 4 * kMaxS;
    if (int rc = allow_lds((const void*)k_sample_p2<FAM>, lds)) return rc;
    hipLaunchKernelGGL(k_sample_p2<FAM>, dim3(g), dim3(kChunk), lds, st, net.d_xtab, net.nbytes, fa, net.m,
                       net.N, f);
  } else if (net.p == 3) {
    const size_t lds = OddCoords<3>::lds_bytes(net.s) + 2 * kMaxS * 4;
    if (int rc = allow_lds((const void*)k_sample_odd<3, FAM>, lds)) return rc;
    hipLaunchKernelGGL((k_sample_odd<3, FAM>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, fa, net.m, net.N,
                       inv_pm(net), f);
  } else {
    const size_t lds = OddCoords<5>::lds_bytes(net.s) + 2 * kMaxS * 4;
    if (int rc = allow_lds((const void*)k_sample_odd<5, FAM>, lds)) return rc;
    hipLaunchKernelGGL((k_sample_odd<5, FAM>), dim3(g), dim3(kChunk), lds, st, net.d_ptab, fa, net.m, net.N,
                       inv_pm(net), f);
  }
  return FDWT_OK;
}

int launch_sample(const Net& net, int family, const double* a, float* f, hipStream_t st) {
  FamilyArgs fa;
  fa.s = net.s;
  for (int j = 0; j < net.s; ++j) {
    fa.a[j] = (float)a[j];
    fa.inv1a[j] = (float)(1.0 / (1.0 + a[j]));
  }
  const unsigned g = grid_for(net.N, 256);
  hipEvent_t tb = timed_begin(st);
  int rc;
  if (family == FDWT_FAMILY_PRODUCT) rc = sample_fam<FDWT_FAMILY_PRODUCT>(net, fa, f, g, st);
  else if (family == FDWT_FAMILY_EXP) rc = sample_fam<FDWT_FAMILY_EXP>(net, fa, f, g, st);
  else rc = sample_fam<FDWT_FAMILY_WANGFANG>(net, fa, f, g, st);
  if (rc) return rc;
  FDWT_HIP(hipGetLastError());
  timed_end(tb, st, FDWT_TC_SAMPLE, 4.0 * (double)net.N);
  return FDWT_OK;
}

}  // namespace fdwt
