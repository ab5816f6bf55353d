// Device-side evaluation of net coordinates X_{j,n} (Definition of a digital
// net, Eq. (defy)) shared by the sampling, coordinate and kernel-data kernels.
//
// p = 2: X_j(n) is the XOR of the generator columns selected by the set bits
//   of n.  Tables hold, per coordinate and per byte b of n, the XOR for each
//   byte value.  A workgroup of 256 threads handles 256 consecutive points
//   (aligned) at a time: the bytes above the lowest are then common to the
//   whole group, so their XOR (one value per coordinate) is computed once per
//   group into LDS, and each thread adds only its low-byte table entry (also
//   in LDS).
// p odd: digits are packed in 4-bit fields, digit y_{r+1} at bits 4(m-1-r);
//   the contribution v * (column c of C_j) mod p of each index digit v comes
//   from a table and is added field-wise modulo p.
#pragma once

#include "fdwt_internal.h"

namespace fdwt {

constexpr int kChunk = 256;  // points per group (= threads per workgroup)

struct P2Coords {
  const uint32_t* xtab;  // [s][nbytes][256]
  int nbytes, s;
  uint32_t* t0;          // LDS [s][256]
  uint32_t* u;           // LDS [s]

  // Low-byte tables into LDS (call once per workgroup; ends with a barrier).
  __device__ __forceinline__ void stage_tables() const {
    for (int i = threadIdx.x; i < s * 256; i += blockDim.x)
      t0[i] = xtab[(int64_t)(i >> 8) * nbytes * 256 + (i & 255)];
    __syncthreads();
  }
  // XOR of the upper-byte tables for the group starting at `base` (a multiple
  // of 256).  Callers put a barrier before (LDS reuse) and after.
  __device__ __forceinline__ void stage_group(int64_t base) const {
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
      uint32_t v = 0;
      const uint32_t* tj = xtab + (int64_t)j * nbytes * 256;
      for (int b = 1; b < nbytes; ++b) v ^= tj[b * 256 + (int)((base >> (8 * b)) & 255)];
      u[j] = v;
    }
  }
  __device__ __forceinline__ uint32_t X(int j, int64_t n) const { return t0[j * 256 + (int)(n & 255)] ^ u[j]; }
};

// Field-wise (a + b) mod P of packed 4-bit digits < P (P <= 7): a field sum
// is <= 2P - 2 < 16, and adding 8 - P sets bit 3 of a field exactly when the
// field is >= P.
template <int P>
__device__ __forceinline__ uint64_t addmod_packed(uint64_t a, uint64_t b) {
  constexpr uint64_t ones = 0x1111111111111111ull;
  const uint64_t s = a + b;
  const uint64_t ge = ((s + (8 - P) * ones) >> 3) & ones;
  return s - (uint64_t)P * ge;
}

// Packed digits of X_j(n), p odd.  ptab: [s][m][P].
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

// Index t of the first non-zero digit (t = i - 1) of x_{n,j}, or m when
// x_{n,j} = 0.
__device__ __forceinline__ int lead_p2(uint32_t X, int m) { return __clz(X) - (32 - m); }
__device__ __forceinline__ int lead_odd(uint64_t pk, int m) { return (__clzll(pk) - 64 + 4 * m) >> 2; }

}  // namespace fdwt
