// Building blocks of the static-shape p = 2 passes (fwt.hip: fwt_p2,
// fwt_p2_gen, fwt_p2_fam; batch.hip: the one-launch batch tiles).
#pragma once

#include "pass_core.h"

namespace fdwt {

// -------------------------------------------- p = 2 passes, static shape
// For p = 2 the tile shape (2^LOGE elements, rows of 2^WDIG contiguous
// elements) is a template parameter, so every LDS and global offset inside a
// tile is a compile-time constant added to a per-thread base: the per-element
// work is the butterfly itself.  Padded LDS index pad(e) = e + e/32; for the
// element sets used here pad(e0 + j*stride) = pad(e0) + pad(j*stride) holds
// exactly (checked exhaustively for every shape), so the offsets fold.
__host__ __device__ constexpr int cpad(int e) { return e + (e >> 5); }
__host__ __device__ constexpr int cilog2(int v) { return v <= 1 ? 0 : 1 + cilog2(v >> 1); }
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

template <int LOGE, int WDIG>
struct P2Shape {
  static constexpr int E = 1 << LOGE;
  static constexpr int W = 1 << WDIG;
  static constexpr int RD = LOGE - WDIG;                 // digits transformed
  static constexpr int THREADS = E / 16 < 64 ? 64 : (E / 16 > 1024 ? 1024 : E / 16);
  static constexpr int EPT = E / THREADS;                // elements per thread
  static constexpr int KGMAX = cmin(4, cilog2(EPT));     // digits per register group
  static_assert(EPT >= 2 && THREADS % W == 0, "unsupported shape");
};

// Register groups over row digits [Q, Q+KG), then the next group.  KGM caps
// the group size (fewer live registers when other values must stay live).
template <int LOGE, int WDIG, int Q, class T, int KGM = 4, int RDL = P2Shape<LOGE, WDIG>::RD,
          bool DONE = (Q >= RDL)>
struct P2Groups {
  static __device__ __forceinline__ void run(T* lds, int tid) {
    using S = P2Shape<LOGE, WDIG>;
    constexpr int KG = cmin(cmin(S::KGMAX, KGM), RDL - Q);
    constexpr int R = 1 << KG;
    constexpr int STQ = S::W << Q;                      // element stride of digit Q
    constexpr int GPT = (S::E >> KG) / S::THREADS;      // groups per thread
#pragma unroll
    for (int t = 0; t < GPT; ++t) {
      const int g = tid + t * S::THREADS;
      const int c = g & (S::W - 1);
      const int rem = g >> WDIG;
      const int il = rem & ((1 << Q) - 1);
      const int ih = rem >> Q;
      const int e0 = c + S::W * (il + (ih << (Q + KG)));
      T* base = lds + cpad(e0);
      T x[R];
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = base[cpad(j * STQ)];
#pragma unroll
      for (int b = 0; b < KG; ++b) {
#pragma unroll
        for (int j0 = 0; j0 < R; ++j0) {
          if (((j0 >> b) & 1) == 0) {
            const T u = x[j0], v = x[j0 + (1 << b)];
            x[j0] = add(u, v);
            x[j0 + (1 << b)] = sub(u, v);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j) base[cpad(j * STQ)] = x[j];
    }
    lds_barrier();
    P2Groups<LOGE, WDIG, Q + KG, T, KGM, RDL>::run(lds, tid);
  }
};
template <int LOGE, int WDIG, int Q, class T, int KGM, int RDL>
struct P2Groups<LOGE, WDIG, Q, T, KGM, RDL, true> {
  static __device__ __forceinline__ void run(T*, int) {}
};

// Radix-2 stages over register-index bits [0, NB) of v.
template <int NB, class T, int N>
__device__ __forceinline__ void reg_bfly(T (&v)[N]) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int j0 = 0; j0 < N; ++j0) {
      if (((j0 >> b) & 1) == 0) {
        const T u = v[j0], w = v[j0 + (1 << b)];
        v[j0] = add(u, w);
        v[j0 + (1 << b)] = sub(u, w);
      }
    }
  }
}

// Radix-2 stages over register-index bits [LO, HI) of v.
template <int LO, int HI, class T, int N>
__device__ __forceinline__ void reg_bfly_bits(T (&v)[N]) {
#pragma unroll
  for (int b = LO; b < HI; ++b) {
#pragma unroll
    for (int j0 = 0; j0 < N; ++j0) {
      if (((j0 >> b) & 1) == 0) {
        const T u = v[j0], w = v[j0 + (1 << b)];
        v[j0] = add(u, w);
        v[j0 + (1 << b)] = sub(u, w);
      }
    }
  }
}

}  // namespace fdwt
