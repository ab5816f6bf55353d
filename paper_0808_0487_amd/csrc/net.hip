// Digital net generation and test-function sampling on the device
// (Definition of a digital net, Eq. (defy): y_vec = C_j n_vec over Z_p,
// x_{j,n} = sum_r y_{j,n,r} p^-r).
//
// p = 2: the map n -> X_j(n) is linear over Z_2, so X_j(n) is the XOR of the
//   generator columns selected by the set bits of n.  The library keeps, per
//   coordinate and per byte of n, a 256-entry table of those XORs.  Inside a
//   wavefront (64 consecutive n, aligned) the bytes above the lowest one are
//   uniform, so their contribution is fetched once per wave with scalar
//   loads; only the low-byte table is read per lane, from LDS.
// p odd: digits are kept packed in 4-bit fields (digit y_{r+1} at bits
//   4(m-1-r)); column contributions v * C_j[:, c] mod p come from a table and
//   are added field-wise modulo p without carries between fields.
#include "dev_math.h"

namespace fdwt {

// Field-wise (a + b) mod P for packed 4-bit digits < P (P <= 7): the sum of
// two fields is <= 2P - 2 < 16, and adding 8 - P sets bit 3 of a field
// exactly when the field is >= P.
template <int P>
__device__ __forceinline__ uint64_t addmod_packed(uint64_t a, uint64_t b) {
  constexpr uint64_t ones = 0x1111111111111111ull;
  uint64_t s = a + b;
  uint64_t ge = ((s + (8 - P) * ones) >> 3) & ones;
  return s - (uint64_t)P * ge;
}

// Packed digits of X_j(n), p odd.
template <int P>
__device__ __forceinline__ uint64_t packed_odd(const uint64_t* __restrict__ ptab, int j, int m, int64_t n) {
  uint64_t acc = 0;
  const uint64_t* t = ptab + (int64_t)j * m * P;
  for (int c = 0; c < m; ++c) {
    const int dgt = (int)(n % P);
    n /= P;
    acc = addmod_packed<P>(acc, t[c * P + dgt]);
  }
  return acc;
}

// Canonical integer sum_r y_{r+1} p^{m-1-r} from packed fields.
template <int P>
__device__ __forceinline__ uint32_t canon_odd(uint64_t packed, int m) {
  uint32_t X = 0;
  for (int r = 0; r < m; ++r) X = X * P + (uint32_t)((packed >> (4 * (m - 1 - r))) & 15u);
  return X;
}

// p = 2 helpers: per-wave uniform part and per-lane low-byte part.
struct P2Tabs {
  const uint32_t* xtab;  // [s][nbytes][256]
  int nbytes;
};

__device__ __forceinline__ uint32_t p2_uniform(const P2Tabs& t, int j, int64_t nwave) {
  // nwave: wave-uniform index whose bytes >= 1 equal those of every lane.
  uint32_t u = 0;
  const uint32_t* base = t.xtab + (int64_t)j * t.nbytes * 256;
  for (int b = 1; b < t.nbytes; ++b) u ^= base[b * 256 + ((nwave >> (8 * b)) & 255)];
  return u;
}

// Stage the low-byte tables of all coordinates in LDS: lds[j*256 + v].
__device__ __forceinline__ void p2_stage(const P2Tabs& t, int s, uint32_t* lds) {
  for (int i = threadIdx.x; i < s * 256; i += blockDim.x)
    lds[i] = t.xtab[(int64_t)(i >> 8) * t.nbytes * 256 + (i & 255)];
  __syncthreads();
}

// ------------------------------------------------------------- kernels
// Output modes of the coordinate kernel.
enum CoordMode { CM_DIGITS = 0, CM_POINTS = 1, CM_SHIFTED = 2 };

template <int MODE>
__global__ void __launch_bounds__(256) k_coords_p2(P2Tabs t, int s, int m, int64_t N, void* out) {
  extern __shared__ uint32_t lds_t0[];
  p2_stage(t, s, lds_t0);
  const float inv = 1.0f / (float)(1u << m);  // exact power of two
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n0 = (int64_t)blockIdx.x * blockDim.x; n0 < N; n0 += stride) {
    const int64_t n = n0 + threadIdx.x;
    const int64_t nw = (int64_t)__builtin_amdgcn_readfirstlane((int)(n >> 6)) << 6;
    for (int j = 0; j < s; ++j) {
      const uint32_t u = p2_uniform(t, j, nw);
      if (n < N) {
        const uint32_t X = lds_t0[j * 256 + (int)(n & 255)] ^ u;
        if (MODE == CM_DIGITS) ((uint32_t*)out)[(int64_t)j * N + n] = X;
        if (MODE == CM_POINTS) ((float*)out)[(int64_t)j * N + n] = (float)X * inv;
        if (MODE == CM_SHIFTED) ((uint32_t*)out)[(int64_t)j * N + n] = X << (32 - m);
      }
    }
  }
}

template <int P, int MODE>
__global__ void __launch_bounds__(256) k_coords_odd(const uint64_t* ptab, int s, int m, int64_t N,
                                                    float inv_pm, void* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
    for (int j = 0; j < s; ++j) {
      const uint64_t pk = packed_odd<P>(ptab, j, m, n);
      if (MODE == CM_DIGITS) ((uint32_t*)out)[(int64_t)j * N + n] = canon_odd<P>(pk, m);
      if (MODE == CM_POINTS) ((float*)out)[(int64_t)j * N + n] = (float)canon_odd<P>(pk, m) * inv_pm;
      if (MODE == CM_SHIFTED) ((uint64_t*)out)[(int64_t)j * N + n] = pk;
    }
  }
}

// Test-function families (float arithmetic).
struct FamilyArgs {
  int kind;
  int s;
  float a[kMaxS];
  float inv1a[kMaxS];  // 1 / (1 + a_j), Section 5.2 function
};

__device__ __forceinline__ void fam_init(const FamilyArgs& fa, float& acc) {
  acc = (fa.kind == FDWT_FAMILY_EXP) ? 0.0f : 1.0f;
}
__device__ __forceinline__ void fam_step(const FamilyArgs& fa, int j, float x, float& acc) {
  if (fa.kind == FDWT_FAMILY_PRODUCT) acc *= 1.0f + fa.a[j] * (x - 0.5f);
  else if (fa.kind == FDWT_FAMILY_EXP) acc += fa.a[j] * x * x;
  else acc *= (fabsf(4.0f * x - 2.0f) + fa.a[j]) * fa.inv1a[j];
}
__device__ __forceinline__ float fam_final(const FamilyArgs& fa, float acc) {
  return (fa.kind == FDWT_FAMILY_EXP) ? expf(-acc) : acc;
}

__global__ void __launch_bounds__(256) k_sample_p2(P2Tabs t, FamilyArgs fa, int m, int64_t N, float* f) {
  extern __shared__ uint32_t lds_t0[];
  p2_stage(t, fa.s, lds_t0);
  const float inv = 1.0f / (float)(1u << m);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n0 = (int64_t)blockIdx.x * blockDim.x; n0 < N; n0 += stride) {
    const int64_t n = n0 + threadIdx.x;
    const int64_t nw = (int64_t)__builtin_amdgcn_readfirstlane((int)(n >> 6)) << 6;
    float acc;
    fam_init(fa, acc);
    for (int j = 0; j < fa.s; ++j) {
      const uint32_t u = p2_uniform(t, j, nw);
      const uint32_t X = lds_t0[j * 256 + (int)(n & 255)] ^ u;
      fam_step(fa, j, (float)X * inv, acc);
    }
    if (n < N) f[n] = fam_final(fa, acc);
  }
}

template <int P>
__global__ void __launch_bounds__(256) k_sample_odd(const uint64_t* ptab, FamilyArgs fa, int m, int64_t N,
                                                    float inv_pm, float* f) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
    float acc;
    fam_init(fa, acc);
    for (int j = 0; j < fa.s; ++j) {
      const uint32_t X = canon_odd<P>(packed_odd<P>(ptab, j, m, n), m);
      fam_step(fa, j, (float)X * inv_pm, acc);
    }
    f[n] = fam_final(fa, acc);
  }
}

// ----------------------------------------------------------- launchers
static unsigned grid_for(int64_t N, int threads) {
  int64_t b = (N + threads - 1) / threads;
  return (unsigned)std::min<int64_t>(b, 8192);
}

static float inv_pm(const Net& net) { return (float)(1.0 / (double)net.N); }

template <int MODE>
static int coords(const Net& net, void* out, hipStream_t st) {
  const unsigned g = grid_for(net.N, 256);
  if (net.p == 2) {
    P2Tabs t{net.d_xtab, net.nbytes};
    hipLaunchKernelGGL(k_coords_p2<MODE>, dim3(g), dim3(256), (size_t)net.s * 256 * 4, st, t, net.s,
                       net.m, net.N, out);
  } else if (net.p == 3) {
    hipLaunchKernelGGL((k_coords_odd<3, MODE>), dim3(g), dim3(256), 0, st, net.d_ptab, net.s, net.m,
                       net.N, inv_pm(net), out);
  } else {
    hipLaunchKernelGGL((k_coords_odd<5, MODE>), dim3(g), dim3(256), 0, st, net.d_ptab, net.s, net.m,
                       net.N, inv_pm(net), out);
  }
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

int launch_net_digits(const Net& net, uint32_t* X, hipStream_t st) { return coords<CM_DIGITS>(net, X, st); }
int launch_net_points(const Net& net, float* x, hipStream_t st) { return coords<CM_POINTS>(net, x, st); }
int launch_net_packed(const Net& net, void* out, hipStream_t st) { return coords<CM_SHIFTED>(net, out, st); }

int launch_sample(const Net& net, int family, const double* a, float* f, hipStream_t st) {
  FamilyArgs fa;
  fa.kind = family;
  fa.s = net.s;
  for (int j = 0; j < net.s; ++j) {
    fa.a[j] = (float)a[j];
    fa.inv1a[j] = (float)(1.0 / (1.0 + a[j]));
  }
  const unsigned g = grid_for(net.N, 256);
  if (net.p == 2) {
    P2Tabs t{net.d_xtab, net.nbytes};
    hipLaunchKernelGGL(k_sample_p2, dim3(g), dim3(256), (size_t)net.s * 256 * 4, st, t, fa, net.m, net.N, f);
  } else if (net.p == 3) {
    hipLaunchKernelGGL(k_sample_odd<3>, dim3(g), dim3(256), 0, st, net.d_ptab, fa, net.m, net.N,
                       inv_pm(net), f);
  } else {
    hipLaunchKernelGGL(k_sample_odd<5>, dim3(g), dim3(256), 0, st, net.d_ptab, fa, net.m, net.N,
                       inv_pm(net), f);
  }
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

}  // namespace fdwt
