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
//   from a table and is added field-wise modulo p.  OddCoords splits the
//   index as n = h p^K + r: a workgroup table (LDS) holds the packed sum over
//   the K low digits for every r < p^K, and per group of 256 consecutive
//   points the few high parts h that occur are summed once into LDS, so a
//   coordinate costs one field-wise addition.
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

// Packed digits of X_j(n) through workgroup tables (see the file comment).
// Layout in LDS: t0 [s][PK] then u [s][NH] (uint64).
template <int P>
struct OddCoords {
  static constexpr int K = P == 3 ? 4 : 2;               // low digits per table entry
  static constexpr int PK = P == 3 ? 81 : P * P;         // P^K
  static constexpr int NH = kChunk / PK + 2;             // high parts per group (at most)
  static constexpr size_t lds_bytes(int s) { return (size_t)s * (PK + NH) * 8; }
  const uint64_t* ptab;  // [s][m][P] (global)
  int s, m;
  uint64_t* t0;          // LDS [s][PK]
  uint64_t* u;           // LDS [s][NH]
  uint32_t hi0 = 0;

  // Low-digit tables (once per workgroup; ends with a barrier).
  __device__ __forceinline__ void stage_tables() const {
    for (int i = threadIdx.x; i < s * PK; i += blockDim.x) {
      const int j = i / PK;
      int r = i - j * PK;
      const uint64_t* t = ptab + (int64_t)j * m * P;
      uint64_t acc = 0;
      for (int c = 0; c < K && c < m; ++c) {
        acc = addmod_packed<P>(acc, t[c * P + r % P]);
        r /= P;
      }
      t0[i] = acc;
    }
    __syncthreads();
  }
  // High parts of the group starting at `base` (a multiple of kChunk).
  // Callers put a barrier before (LDS reuse) and after.
  __device__ __forceinline__ void stage_group(int64_t base) {
    hi0 = (uint32_t)(base / PK);
    const int nh = (int)((base + kChunk - 1) / PK - hi0 + 1);
    for (int i = threadIdx.x; i < s * nh; i += blockDim.x) {
      const int j = i / nh, k = i - (i / nh) * nh;
      uint32_t h = hi0 + k;
      const uint64_t* t = ptab + (int64_t)j * m * P;
      uint64_t acc = 0;
      for (int c = K; c < m; ++c) {
        acc = addmod_packed<P>(acc, t[c * P + h % P]);
        h /= P;
      }
      u[j * NH + k] = acc;
    }
  }
  // Index split of point n (n < 2^26) for X(): r = n mod PK, h - hi0.
  __device__ __forceinline__ void split(int64_t n, int& r, int& k) const {
    const uint32_t nn = (uint32_t)n;
    const uint32_t h = nn / PK;
    r = (int)(nn - h * PK);
    k = (int)(h - hi0);
  }
  __device__ __forceinline__ uint64_t X(int j, int r, int k) const {
    return addmod_packed<P>(t0[j * PK + r], u[j * NH + k]);
  }
};

// Canonical integer sum_r y_{r+1} p^{m-1-r} from packed fields.
template <int P>
__device__ __forceinline__ uint32_t canon_odd(uint64_t packed, int m) {
  uint32_t X = 0;
  for (int r = 0; r < m; ++r) X = X * P + (uint32_t)((packed >> (4 * (m - 1 - r))) & 15u);
  return X;
}

// Digit strings for the interpolant evaluation: fields of B bits under one
// zero bit, B = 2 for p = 3 and 3 for p = 5, 7 (the fewest that hold a
// digit), digit y_{f+1} in bits [62 - B f, 63 - B (f + 1)].  The leading-zero
// count of the XOR of two strings is then B f + 1..B f + B when digit f + 1
// is the first that differs, and 64 when none does; the first 32 bits hold
// 15 digits (p = 3) or 10 (p = 5, 7).
template <int P>
constexpr int kStrBits = P == 3 ? 2 : 3;
template <int P>
__device__ __forceinline__ uint64_t eval_string_odd(uint64_t pk, int m) {
  constexpr int B = kStrBits<P>;
  uint64_t v = 0;
  for (int f = 0; f < m; ++f) v |= ((pk >> (4 * (m - 1 - f))) & 7ull) << (63 - B * (f + 1));
  return v;
}

// Index t of the first non-zero digit (t = i - 1) of x_{n,j}, or m when
// x_{n,j} = 0.
__device__ __forceinline__ int lead_p2(uint32_t X, int m) { return __clz(X) - (32 - m); }
__device__ __forceinline__ int lead_odd(uint64_t pk, int m) { return (__clzll(pk) - 64 + 4 * m) >> 2; }

}  // namespace fdwt
