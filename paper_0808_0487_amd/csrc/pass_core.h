// Device building blocks shared by the transform passes (fwt.hip) and the
// batched persistent kernel (batch.hip): pass descriptor, element-type
// conversions, the padded LDS index and the runtime-geometry register groups.
#pragma once

#include "dev_math.h"

namespace fdwt {

struct PassDesc {
  int64_t col_in;   // elements between batch columns of the input
  int64_t col_out;  // elements between batch columns of the output
  int64_t sd0;      // p^d0: index stride of the pass's first digit
  int64_t shi;      // p^(d0+r): index stride of the digits above the pass
  int32_t r;        // digits transformed by this pass
  int32_t wdig;     // w = p^wdig contiguous elements per tile row
  int32_t w;
  int32_t nlo;      // p^d0 / w tiles side by side along the low digits
  int32_t E;        // tile size p^r * w
  int32_t kreg;     // digits per register group
  int32_t xcd;      // 1: consecutive tiles are kept on one XCD
  int32_t ntiles;   // tiles per column
  int32_t batch;    // columns
  float scale;      // multiplies float-based outputs (last pass only)
  double scale64;   // the same factor for double-based outputs
  // Grouped-sum epilogue (EPI_REDUCE): instead of storing, accumulate
  // sum_h wts[h].x * clamp(value(h) * wts[h].y, 0, 1) per column into
  // partial sums: partial[col * ntiles + tile] (generic pass) or one per wave,
  // partial[(col * ntiles + tile) * waves + wave] (static p = 2 pass); the
  // value at h = 0 of column h0_col goes to *h0_out as well.
  const float2* wts;
  double* partial;
  double* h0_out;
  int32_t h0_col;
  // Grouped-sum order of the static p = 2 pass (requires ntiles % grid == 0):
  // when nonzero, block l (grid size G) is column (l / G) % batch of tile
  // ((l / G) / batch) * G + l % G, so a workgroup takes every column of one
  // tile in successive rounds and keeps that tile's weights in registers.
  int32_t wkeep;
  // Blocked output of a contiguous first pass (LOGE >= 10, WDIG 0): when
  // nonzero, element e of tile t is stored at (e >> 4) * oblk + 16 t + (e & 15),
  // oblk = 16 * ntiles, so that each tile of a following strided pass (rows of
  // 16) is one contiguous block.
  int64_t oblk;
  // Column pointer tables (store passes of static p = 2 shapes): when set,
  // column c reads in_tab[c] and writes out_tab[c] instead of in/out plus
  // c times the column stride (a group of equal-size jobs anywhere in memory).
  const void* const* in_tab;
  void* const* out_tab;
};

enum Epilogue { EPI_STORE = 0, EPI_REDUCE = 1 };

// Pointers in the global address space.  A pointer read from memory (a
// column table) is generic to the compiler, and accesses through it become
// flat instructions, which the LDS wait counter also tracks: every wait for
// LDS would then wait for the tile prefetch and the stores in flight as well.
// Accesses through a gptr are global instructions.
template <class T>
using gptr = T __attribute__((address_space(1)))*;
template <class T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}
// Entry i of a column pointer table.  The tables are written before a launch
// and never by a kernel, so they are read through the constant address
// space: with a uniform index that is a scalar load, which the vector
// memory counter does not track (a vector load of the pointer would make
// the wait for it drain every load and store issued before it).
template <class T>
__device__ __forceinline__ T* col_ptr(const void* const* tab, int i) {
  using cptr = const void* const __attribute__((address_space(4)))*;
  return (T*)((cptr)tab)[i];
}

// ------------------------------------------------------------ conversions
template <class Tin, class T>
__device__ __forceinline__ T cvt_in(Tin v);
template <> __device__ __forceinline__ float cvt_in<float, float>(float v) { return v; }
template <> __device__ __forceinline__ uint32_t cvt_in<uint32_t, uint32_t>(uint32_t v) { return v; }
template <> __device__ __forceinline__ float2 cvt_in<float, float2>(float v) { return make_float2(v, 0.0f); }
template <> __device__ __forceinline__ float2 cvt_in<float2, float2>(float2 v) { return v; }
template <> __device__ __forceinline__ double cvt_in<double, double>(double v) { return v; }
template <> __device__ __forceinline__ double2 cvt_in<double, double2>(double v) { return make_double2(v, 0.0); }
template <> __device__ __forceinline__ double2 cvt_in<double2, double2>(double2 v) { return v; }

// sc scales float-based outputs, sc64 double-based ones.
template <class T, class Tout>
__device__ __forceinline__ Tout cvt_out(T v, float sc, double sc64);
template <> __device__ __forceinline__ float cvt_out<float, float>(float v, float sc, double) { return v * sc; }
template <> __device__ __forceinline__ uint32_t cvt_out<uint32_t, uint32_t>(uint32_t v, float, double) { return v; }
template <> __device__ __forceinline__ float2 cvt_out<float2, float2>(float2 v, float sc, double) { return make_float2(v.x * sc, v.y * sc); }
template <> __device__ __forceinline__ float cvt_out<float2, float>(float2 v, float sc, double) { return v.x * sc; }
template <> __device__ __forceinline__ double cvt_out<double, double>(double v, float, double sc) { return v * sc; }
template <> __device__ __forceinline__ double2 cvt_out<double2, double2>(double2 v, float, double sc) { return make_double2(v.x * sc, v.y * sc); }
template <> __device__ __forceinline__ double cvt_out<double2, double>(double2 v, float, double sc) { return v.x * sc; }

// Real part as double (the grouped-sum epilogue).
__device__ __forceinline__ double real_of(double v) { return v; }
__device__ __forceinline__ double real_of(double2 v) { return v.x; }
__device__ __forceinline__ double real_of(float v) { return v; }
__device__ __forceinline__ double real_of(float2 v) { return v.x; }
__device__ __forceinline__ double real_of(uint32_t v) { return (double)v; }

// LDS index with one padding element per 32 (spreads the stride-p^k
// register-group accesses over the banks).
__device__ __forceinline__ int pad(int e) { return e + (e >> 5); }

template <int P>
struct Ix {
  // a / p^k and a % p^k for powers of p given by their exponent and value.
  static __device__ __forceinline__ int div(int a, int k, int pk) {
    if constexpr (P == 2) return a >> k; else return a / pk;
  }
  static __device__ __forceinline__ int mod(int a, int k, int pk) {
    if constexpr (P == 2) return a & (pk - 1); else return a % pk;
  }
};

// Quotient and remainder of 0 <= a < 2^22 by 1 <= dv < 2^22 given
// inv = 1.0f / dv (correctly rounded): a * inv is within 0.5 of a / dv (a
// relative error below 2^-23 on a value below 2^22), so its truncation is
// the quotient or one off, and one correction step makes it exact.  The
// emulation of these float operations on the host checks every (a, dv) the
// pass geometries use.  Replaces the integer division (a long instruction
// sequence) on the passes' per-group index arithmetic.
__host__ __device__ __forceinline__ void divmod_small(int a, int dv, float inv, int& q, int& r) {
  q = (int)((float)a * inv);
  r = a - q * dv;
  if (r < 0) {
    --q;
    r += dv;
  } else if (r >= dv) {
    ++q;
    r -= dv;
  }
}

template <int P, int K>
struct PowC {
  static constexpr int v = P * PowC<P, K - 1>::v;
};
template <int P>
struct PowC<P, 0> {
  static constexpr int v = 1;
};

__device__ __forceinline__ int ipow_d(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// One register group: the KK digits [q, q+KK) of the tile row index.  Each
// thread takes p^KK elements that differ only in those digits, applies the
// KK radix-p stages in registers and writes them back.  inv_w = 1.0f / w
// (odd p: see divmod_small).
template <int P, bool INV, class T, int KK>
__device__ __forceinline__ void run_group(T* lds, const PassDesc& d, int q, float inv_w = 0.0f) {
  constexpr int R = PowC<P, KK>::v;
  const int pq = ipow_d(P, q);
  const int ng = d.E / R;
  const int stq = d.w * pq;  // LDS stride of digit q
  const float inv_pq = P == 2 ? 0.0f : 1.0f / (float)pq;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    int c, rem, il, ih;
    if constexpr (P == 2) {
      c = Ix<P>::mod(g, d.wdig, d.w);
      rem = Ix<P>::div(g, d.wdig, d.w);
      il = Ix<P>::mod(rem, q, pq);
      ih = Ix<P>::div(rem, q, pq);
    } else {
      divmod_small(g, d.w, inv_w, rem, c);
      divmod_small(rem, pq, inv_pq, ih, il);
    }
    const int e0 = c + d.w * (il + pq * R * ih);
    T x[R];
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = lds[pad(e0 + j * stq)];
#pragma unroll
    for (int t = 0, st = 1; t < KK; ++t, st *= P) {
#pragma unroll
      for (int j0 = 0; j0 < R; ++j0) {
        if ((j0 / st) % P == 0) Dft<P, INV>::run(x + j0, st);
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) lds[pad(e0 + j * stq)] = x[j];
  }
}


}  // namespace fdwt
