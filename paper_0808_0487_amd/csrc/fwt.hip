// Radix-p butterfly passes of the fast discrete Walsh transform and its
// inverse (Algorithm 1 of Section 2.2, Algorithm 2 of Section 3.3).
//
// Stage r of Algorithm 1 replaces index digit n_{r-1} by h_{r-1} through a
// p-point DFT with weights omega^(-n h); stages act on different digits and
// commute, so the m stages are grouped into passes over HBM.  A pass
// transforms r consecutive digits [d0, d0+r) of every column: a workgroup
// loads a tile of p^r rows (the r digits) by w contiguous elements (the lowest
// digits, w = p^wdig >= 64 bytes of data so that HBM reads and writes come in
// full segments), stages it in LDS, runs the r stages in groups of k digits
// held in registers (p^k values per thread, one LDS round trip per group),
// and writes the tile back in place.  The output is in natural order
// (h = sum h_i p^i), as in Algorithm 1.
#include "family.h"
#include "p2_stages.h"
#include "pass_core.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <type_traits>
#include <mutex>
#include <unordered_set>

namespace fdwt {

// First logical block of workgroup hw.  Workgroups are dispatched round-robin
// over the 8 XCDs (hw mod 8); XCD x gets the contiguous range of the
// ceil((G - x) / 8) logical blocks starting at x floor(G/8) + min(x, G mod 8),
// so neighbouring tiles (which share cache lines and DRAM pages) meet in the
// same L2.  A bijection of [0, G) for any G, so a grid need not be a multiple
// of 8 (3^14 points make 729 tiles: one round, not two).
__device__ __forceinline__ int xcd_first(int hw, int G) {
  const int x = hw & 7, q = G >> 3, r = G & 7;
  return x * q + (x < r ? x : r) + (hw >> 3);
}

size_t kind_bytes(Kind k) {
  switch (k) {
    case K_F32: return 4;
    case K_U32: return 4;
    case K_CF32: return 8;
    case K_F64: return 8;
    case K_CF64: return 16;
  }
  return 0;
}

// Per-thread geometry of the generic pass.  A register group holds R = p^KMAX
// elements; each thread loads LPT elements of a tile (e = tid + k TH): one
// group, except for p = 5, whose groups are one digit (a two-digit group of
// 25 complex values, with as many prefetched, needs more registers than a
// wave gets) and whose threads load 16 elements, so that 1024 threads cover
// a 5^6-element tile.
template <int P, int KMAX, int BYTES>
struct PassShape {
  static constexpr int R = PowC<P, KMAX>::v;
  static constexpr int LPT = P == 5 ? 16 : R;
  // Largest tile the planner can give this kernel (padded tile within
  // 160 KiB of LDS, at most 1024 x LPT elements) and the threads it takes:
  // the kernel is compiled for that many, which sets its register budget.
  static constexpr int emax_elems() {
    int E = 1;
    while ((int64_t)E * P <= 1024 * LPT && ((int64_t)E * P + E * P / 32 + 1) * BYTES <= 160 * 1024) E *= P;
    return E;
  }
  static constexpr int THREADS_RAW = (emax_elems() + LPT - 1) / LPT;
  static constexpr int THREADS = THREADS_RAW < 64 ? 64 : (THREADS_RAW + 63) / 64 * 64;
};

// A pass is a persistent kernel: each workgroup walks over logical blocks
// (tile, column) with stride gridDim.x.  The next tile's elements are loaded
// into registers right after the current tile is in LDS, so the HBM reads of
// tile k+1 overlap the butterflies and stores of tile k.
template <int P, bool INV, class Tin, class T, class Tout, int KMAX, int EPI>
__global__ void __launch_bounds__((PassShape<P, KMAX, sizeof(T)>::THREADS))
    fwt_pass(const Tin* __restrict__ in, Tout* out, PassDesc d) {
  constexpr int LPT = PassShape<P, KMAX, sizeof(T)>::LPT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int G = gridDim.x;
  const int nb = d.ntiles * d.batch;
  const int tid = threadIdx.x, TH = blockDim.x;
  // Workgroups are dispatched round-robin over the 8 XCDs; with xcd set, XCD x
  // takes the contiguous logical range [x G/8, (x+1) G/8) of every round, so
  // neighbouring tiles (which share cache lines and DRAM pages, and for the
  // grouped-sum epilogue the weights of a tile) meet in the same L2.
  const int hw = blockIdx.x;
  int lb = d.xcd ? xcd_first(hw, G) : hw;

  auto locate = [&](int l, int& col, int& tile) {
    if (EPI == EPI_REDUCE) {
      col = l % d.batch;
      tile = l / d.batch;
    } else {
      col = l / d.ntiles;
      tile = l % d.ntiles;
    }
  };
  auto tile_base = [&](int tile) {
    const int lo = tile % d.nlo;
    const int hi = tile / d.nlo;
    return (int64_t)lo * d.w + (int64_t)hi * d.shi;
  };
  // Element e = tid + k TH of a tile sits in row e / w, column e mod w, at
  // global offset (e mod w) + (e / w) sd0 from the tile base.  The thread's
  // (row, column) for k = 0 and the step TH are split once; each next k
  // advances them with a carry, so no element needs a division.  Offsets
  // within a column fit in 32 bits (N <= 2^26).
  const float inv_w = 1.0f / (float)d.w;
  int i0, c0, ti, tc;
  divmod_small(tid, d.w, inv_w, i0, c0);
  divmod_small(TH, d.w, inv_w, ti, tc);
  const uint32_t sd0 = (uint32_t)d.sd0;
  // f(k, e, offset) for the thread's elements; clamp: indices past the tile
  // end take its last element (offset and index), so the loads of a tile
  // are all in flight together.
  const uint32_t last = (uint32_t)(d.w - 1) + (uint32_t)(d.E / d.w - 1) * sd0;
  auto for_elems = [&](bool clamp, auto&& f) {
    // The empty asm makes the counters opaque here, so the offsets are
    // recomputed at each sweep (a few operations per element) instead of
    // being hoisted out of the tile loop into LPT live registers.
    int c = c0, i = i0;
    asm volatile("" : "+v"(c), "+v"(i));
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const int e = tid + k * TH;
      if (e < d.E) f(k, e, (uint32_t)c + (uint32_t)i * sd0);
      else if (clamp) f(k, d.E - 1, last);
      c += tc;
      i += ti;
      if (c >= d.w) {
        c -= d.w;
        ++i;
      }
    }
  };
  Tin pre[LPT];
  auto prefetch = [&](int l) {
    int col, tile;
    locate(l, col, tile);
    const Tin* src = in + (int64_t)col * d.col_in + tile_base(tile);
    for_elems(true, [&](int k, int, uint32_t off) { pre[k] = src[off]; });
  };
  double* red = reinterpret_cast<double*>(smem_raw + (size_t)(d.E + d.E / 32 + 1) * sizeof(T) + 8 -
                                          ((d.E + d.E / 32 + 1) * sizeof(T)) % 8);
  if (lb < nb) prefetch(lb);
  for (; lb < nb; lb += G) {
    // Clamped indices write the tile's last element again, with its value.
    for_elems(true, [&](int k, int e, uint32_t) { lds[pad(e)] = cvt_in<Tin, T>(pre[k]); });
    lds_barrier();
    prefetch(lb + G < nb ? lb + G : lb);  // unconditional: exact wait counts
    for (int q = 0; q < d.r; q += d.kreg) {
      const int kk = min(d.kreg, d.r - q);
      if constexpr (KMAX >= 4) {
        if (kk == 4) run_group<P, INV, T, 4>(lds, d, q, inv_w);
      }
      if constexpr (KMAX >= 3) {
        if (kk == 3) run_group<P, INV, T, 3>(lds, d, q, inv_w);
      }
      if constexpr (KMAX >= 2) {
        if (kk == 2) run_group<P, INV, T, 2>(lds, d, q, inv_w);
      }
      if (kk == 1) run_group<P, INV, T, 1>(lds, d, q, inv_w);
      lds_barrier();
    }
    int col, tile;
    locate(lb, col, tile);
    const int64_t base = tile_base(tile);
    if constexpr (EPI == EPI_STORE) {
      Tout* dst = out + (int64_t)col * d.col_out + base;
      for_elems(false, [&](int, int e, uint32_t off) { dst[off] = cvt_out<T, Tout>(lds[pad(e)], d.scale, d.scale64); });
    } else {
      double acc = 0.0;
      for_elems(false, [&](int, int e, uint32_t off) {
        const int64_t h = base + off;
        const float2 wt = d.wts[h];
        const double rho = fmin(fmax(real_of(lds[pad(e)]) * (double)wt.y, 0.0), 1.0);
        const double term = (double)wt.x * rho;
        acc += term;
        if (h == 0 && col == d.h0_col) *d.h0_out = term;
      });
      // Wave sums by butterfly shuffles, then the waves in a fixed order.
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
      lds_barrier();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        d.partial[(int64_t)col * d.ntiles + tile] = t;
      }
    }
    lds_barrier();
  }
}

// -------------------------------------------- p = 3 passes, static shape
// Float-complex passes of p = 3 with the tile geometry fixed at compile time:
// every tile holds 3^8 = 6561 elements, 3^RD rows (the RD digits of the
// pass) of W = 3^(8 - RD) contiguous elements (the lowest digits), 52.5 KiB
// of LDS.  Each of TH = 3^(8 - KT) threads takes 3^KT elements: element
// e = tid + k TH lies in row tid / W + k 3^(RD - KT), so the values a thread
// loads differ exactly in the KT top digits of the pass (k = j0 + 3 j1 + ...),
// whose radix-3 stages run in registers before the tile goes to LDS; the
// other digits go through LDS in groups of up to KT digits.  With KT = 3
// (243 threads, 27 elements each) three workgroups share a CU, so the 729
// tiles of a 3^14-point transform run in one round; KT = 2 (729 threads)
// serves passes of two digits.  All LDS offsets of a group are compile-time
// strides from a per-thread base; the strides W 3^q are odd multiples of the
// row length, so the tile needs no padding.
template <int RD, int KT>
struct P3Shape {
  static constexpr int E = 6561;
  static constexpr int EPT = PowC<3, KT>::v;  // elements per thread
  static constexpr int TH = E / EPT;
  static constexpr int WDIG = 8 - RD;
  static constexpr int W = PowC<3, WDIG>::v;
  static constexpr int RSTEP = TH / W;         // rows between a thread's elements, 3^(RD - KT)
  static_assert(RD >= KT && RD <= 8 && RD != 7 && TH % W == 0, "unsupported p = 3 shape");
};

// Radix-3 stages over the digits 0..KG-1 of the index of x (3^KG values).
template <int KG, bool INV, class T, int N>
__device__ __forceinline__ void dft3_digits(T (&x)[N]) {
  static_assert(PowC<3, KG>::v == N, "3^KG values");
#pragma unroll
  for (int t = 0, st = 1; t < KG; ++t, st *= 3) {
#pragma unroll
    for (int j0 = 0; j0 < N; ++j0)
      if ((j0 / st) % 3 == 0) Dft<3, INV>::run(x + j0, st);
  }
}

// Register groups over row digits [Q, Q + KG) for Q < LIM, then the next.
template <int RD, int KT, int Q, bool INV, class T, int LIM = RD - KT, bool DONE = (Q >= LIM)>
struct P3Groups {
  static __device__ __forceinline__ void run(T* lds, int tid) {
    using S = P3Shape<RD, KT>;
    constexpr int KG = (LIM - Q) >= KT ? KT : (LIM - Q);
    constexpr int R = PowC<3, KG>::v;
    constexpr int PQ = PowC<3, Q>::v;
    constexpr int STQ = S::W * PQ;          // element stride of digit Q
    constexpr int GPT = S::E / R / S::TH;   // groups per thread
    const int c = tid % S::W;
    const int u0 = tid / S::W;
#pragma unroll
    for (int g = 0; g < GPT; ++g) {
      // group tid + g TH: rows u = lo + PQ (j + R hi), lo < PQ
      const int u = u0 + g * S::RSTEP;
      const int lo = u % PQ, hi = u / PQ;
      T* base = lds + c + S::W * (lo + PQ * R * hi);
      T x[R];
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = base[j * STQ];
      dft3_digits<KG, INV>(x);
#pragma unroll
      for (int j = 0; j < R; ++j) base[j * STQ] = x[j];
    }
    lds_barrier();
    P3Groups<RD, KT, Q + KG, INV, T, LIM>::run(lds, tid);
  }
};
template <int RD, int KT, int Q, bool INV, class T, int LIM>
struct P3Groups<RD, KT, Q, INV, T, LIM, true> {
  static __device__ __forceinline__ void run(T*, int) {}
};

template <bool INV, class Tin, class T, class Tout, int RD, int KT>
__global__ void __launch_bounds__((P3Shape<RD, KT>::TH)) fwt_p3s(const Tin* __restrict__ in, Tout* out, PassDesc d) {
  using S = P3Shape<RD, KT>;
  constexpr int TH = S::TH, EPT = S::EPT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int G = gridDim.x;
  const int nb = d.ntiles * d.batch;
  const int hw = blockIdx.x;
  int lb = d.xcd ? xcd_first(hw, G) : hw;
  const int tid = threadIdx.x;
  // Global offset of element tid + k TH: goff0 + k gstep.
  const uint32_t sd0 = (uint32_t)d.sd0;
  const uint32_t goff0 = (uint32_t)(tid % S::W) + (uint32_t)(tid / S::W) * sd0;
  const uint32_t gstep = (uint32_t)S::RSTEP * sd0;
  auto locate = [&](int l, int& col, int& tile) {
    col = l / d.ntiles;
    tile = l % d.ntiles;
  };
  auto tile_base = [&](int tile) {
    const int lo = tile % d.nlo;
    const int hi = tile / d.nlo;
    return (int64_t)lo * S::W + (int64_t)hi * d.shi;
  };
  Tin pre[EPT];
  // live false: every load reads the tile's first element (one cache line), a
  // stand-in that keeps the loads unconditional when there is no next tile.
  auto prefetch = [&](int l, bool live) {
    int col, tile;
    locate(l, col, tile);
    const Tin* src = in + (int64_t)col * d.col_in + tile_base(tile) + (live ? goff0 : 0u);
    const uint32_t st = live ? gstep : 0u;
#pragma unroll
    for (int k = 0; k < EPT; ++k) pre[k] = src[k * st];
  };
  if (lb < nb) prefetch(lb, true);
  for (; lb < nb; lb += G) {
    T v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[k] = cvt_in<Tin, T>(pre[k]);
    dft3_digits<KT, INV>(v);  // the KT top digits of the pass
    int col, tile;
    locate(lb, col, tile);
    Tout* dst = out + (int64_t)col * d.col_out + tile_base(tile) + goff0;
    if constexpr (RD == KT) {
      // The pass has no other digits: straight back to memory.
      prefetch(lb + G < nb ? lb + G : lb, lb + G < nb);  // unconditional: exact wait counts
#pragma unroll
      for (int k = 0; k < EPT; ++k) dst[k * gstep] = cvt_out<T, Tout>(v[k], d.scale, d.scale64);
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) lds[tid + k * TH] = v[k];
      lds_barrier();
      prefetch(lb + G < nb ? lb + G : lb, lb + G < nb);  // unconditional: exact wait counts
      P3Groups<RD, KT, 0, INV, T>::run(lds, tid);
#pragma unroll
      for (int k = 0; k < EPT; ++k) dst[k * gstep] = cvt_out<T, Tout>(lds[tid + k * TH], d.scale, d.scale64);
      lds_barrier();
    }
  }
}

// -------------------------------------------- p = 2 passes, static shape
// (tile geometry, register groups and stages: p2_stages.h)

template <class Tin, class T, class Tout, int LOGE, int WDIG, int EPI>
__global__ void __launch_bounds__((P2Shape<LOGE, WDIG>::THREADS))
    fwt_p2(const Tin* __restrict__ in, Tout* out, PassDesc d) {
  using S = P2Shape<LOGE, WDIG>;
  constexpr int EPT = S::EPT, TH = S::THREADS;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int G = gridDim.x;
  const int nb = d.ntiles * d.batch;
  const int hw = blockIdx.x;
  int lb = d.xcd ? xcd_first(hw, G) : hw;
  const int tid = threadIdx.x;
  // Element e = tid + k*TH of a tile: row i = e >> WDIG, column e & (W-1);
  // global offset goff0 + k*gstep, LDS index pad(tid) + pad(k*TH).
  const uint32_t sd0 = (uint32_t)d.sd0;
  const uint32_t goff0 = (uint32_t)(tid & (S::W - 1)) + (uint32_t)(tid >> WDIG) * sd0;
  const uint32_t gstep = (uint32_t)(TH >> WDIG) * sd0;
  T* lrow = lds + cpad(tid);
  auto locate = [&](int l, int& col, int& tile) {
    if (EPI == EPI_REDUCE && d.wkeep) {
      const int r = l / G;
      col = r % d.batch;
      tile = (r / d.batch) * G + l % G;
    } else if (EPI == EPI_REDUCE) {
      col = l % d.batch;
      tile = l / d.batch;
    } else {
      col = l / d.ntiles;
      tile = l % d.ntiles;
    }
  };
  auto tile_base = [&](int tile) {
    const int lo = tile % d.nlo;
    const int hi = tile / d.nlo;
    return (int64_t)lo * S::W + (int64_t)hi * d.shi;
  };
  Tin pre[EPT];
  // Converts the prefetched elements into the tile registers.  The empty asm
  // is a use of each register, so the wait for the prefetch sits here.  A
  // pass takes the next tile before it stores the current one (or its
  // partial sum): the prefetch is then the newest memory operation, and its
  // wait covers at most the stores of the tile before, issued a whole tile
  // earlier.  With the wait at the top of the loop instead, it also waited
  // for the stores of the tile just finished.
  auto take = [&](T (&v)[EPT]) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      v[k] = cvt_in<Tin, T>(pre[k]);
      asm volatile("" : "+v"(v[k]));
    }
  };
  auto prefetch = [&](int l) {
    int col, tile;
    locate(l, col, tile);
    const Tin* colp = d.in_tab ? col_ptr<const Tin>(d.in_tab, col) : in + (int64_t)col * d.col_in;
    const gptr<const Tin> src = to_global(colp + tile_base(tile) + goff0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) pre[k] = src[k * gstep];
  };
  if (lb < nb) prefetch(lb);
  if constexpr (LOGE >= 10) {
    // Three stage groups per tile.  The 16 elements a thread loads (e = tid +
    // k TH) differ in the top 4 bits of e: those stages run in registers
    // before the tile goes to LDS.  The stages of bits [WDIG, 6) run through
    // LDS.  The store mapping e = lane + 64 k + 1024 w (still coalesced) puts
    // bits 6..9 in the register index: the remaining stages run in registers
    // after reading the tile back.
    constexpr int NS = (LOGE - 10) < 4 ? (LOGE - 10) : 4;
    constexpr int RDL = 6 - WDIG;
    // The wave index is uniform in a wave: read as a scalar, the addresses
    // derived from it stay in scalar registers.
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t goffS = (uint32_t)(lane & (S::W - 1)) + (uint32_t)((lane >> WDIG) + (1024 >> WDIG) * wv) * sd0;
    const uint32_t gstepS = (uint32_t)(64 >> WDIG) * sd0;
    T* lrowS = lds + cpad(lane + 1024 * wv);
    T v[EPT];
    if (lb < nb) take(v);
    float2 wcur[EPI == EPI_REDUCE ? EPT : 1];  // the grouped-sum weights of the tile
    for (; lb < nb; lb += G) {
      reg_bfly<4>(v);
#pragma unroll
      for (int k = 0; k < EPT; ++k) lrow[cpad(k * TH)] = v[k];
      lds_barrier();
      int col, tile;
      locate(lb, col, tile);
      const int64_t base = tile_base(tile);
      if constexpr (EPI == EPI_REDUCE) {
        if (!d.wkeep || col == 0) {  // with wkeep, column 0 starts a new tile
          const float2* wt = d.wts + base + goffS;
#pragma unroll
          for (int k = 0; k < EPT; ++k) wcur[k] = wt[k * gstepS];
        }
      }
      prefetch(lb + G < nb ? lb + G : lb);  // unconditional: exact wait counts
      P2Groups<LOGE, WDIG, 0, T, (EPI == EPI_REDUCE && sizeof(T) >= 8) ? 2 : 4, RDL>::run(lds, tid);
      T y[EPT];
#pragma unroll
      for (int k = 0; k < EPT; ++k) y[k] = lrowS[66 * k];
      reg_bfly<NS>(y);
      if constexpr (EPI == EPI_STORE) {
        take(v);  // the next tile (the last round takes its own tile again)
        if (WDIG == 0 && d.oblk) {
          // Blocked layout: e = lane + 64 k + 1024 w has row e >> 4 and column e & 15.
          const int64_t rs = d.oblk;
          const gptr<Tout> dst = to_global(out + (int64_t)col * d.col_out + ((lane >> 4) + 64 * wv) * rs +
                                           (int64_t)tile * 16 + (lane & 15));
#pragma unroll
          for (int k = 0; k < EPT; ++k) dst[k * 4 * rs] = cvt_out<T, Tout>(y[k], d.scale, d.scale64);
        } else {
          const gptr<Tout> dst =
              to_global((d.out_tab ? col_ptr<Tout>(d.out_tab, col) : out + (int64_t)col * d.col_out) + base + goffS);
#pragma unroll
          for (int k = 0; k < EPT; ++k) dst[k * gstepS] = cvt_out<T, Tout>(y[k], d.scale, d.scale64);
        }
      } else {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const double rho = fmin(fmax(real_of(y[k]) * (double)wcur[k].y, 0.0), 1.0);
          const double term = (double)wcur[k].x * rho;
          acc += term;
          if (col == d.h0_col && base + goffS + (int64_t)k * gstepS == 0) *d.h0_out = term;
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        take(v);
        if (lane == 0) d.partial[((int64_t)col * d.ntiles + tile) * (TH / 64) + wv] = acc;
      }
      lds_barrier();
    }
    return;
  }
  T v[EPT];
  if (lb < nb) take(v);
  for (; lb < nb; lb += G) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) lrow[cpad(k * TH)] = v[k];
    lds_barrier();
    int col, tile;
    locate(lb, col, tile);
    const int64_t base = tile_base(tile);
    // Grouped-sum weights of this tile: loaded now, used after the butterflies.
    float2 wcur[EPI == EPI_REDUCE ? EPT : 1];
    if constexpr (EPI == EPI_REDUCE) {
      const float2* wt = d.wts + base + goff0;
#pragma unroll
      for (int k = 0; k < EPT; ++k) wcur[k] = wt[k * gstep];
    }
    // Unconditional (the last round re-reads its own block): with no branch
    // around the loads the compiler's wait counts stay exact, so waiting for
    // this tile's weights does not wait for the next tile's elements.
    prefetch(lb + G < nb ? lb + G : lb);
    // The grouped-sum variant keeps this tile's weights live across the
    // butterflies: 2-digit register groups keep it within 128 registers.
    P2Groups<LOGE, WDIG, 0, T, (EPI == EPI_REDUCE && sizeof(T) >= 8) ? 2 : 4>::run(lds, tid);
    if constexpr (EPI == EPI_STORE) {
      take(v);
      const gptr<Tout> dst =
          to_global((d.out_tab ? col_ptr<Tout>(d.out_tab, col) : out + (int64_t)col * d.col_out) + base + goff0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) dst[k * gstep] = cvt_out<T, Tout>(lrow[cpad(k * TH)], d.scale, d.scale64);
    } else {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const float2 w2 = wcur[k];
        const double rho = fmin(fmax(real_of(lrow[cpad(k * TH)]) * (double)w2.y, 0.0), 1.0);
        const double term = (double)w2.x * rho;
        acc += term;
        if (col == d.h0_col && base + goff0 + (int64_t)k * gstep == 0) *d.h0_out = term;
      }
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      take(v);
      if ((tid & 63) == 0) d.partial[((int64_t)col * d.ntiles + tile) * (TH / 64) + (tid >> 6)] = acc;
    }
    lds_barrier();
  }
}

// First (contiguous) pass of float64 transforms whose input columns are
// generated in registers instead of read from memory (p = 2, Section 4):
//  * truncation columns (KCOL false): U_d = prod_{j<=d} (1 + a_j) - 1,
//    d = 1..s, with a_j = gamma_j^2 R'(x_{n,j}) = tab[j][t];
//  * kernel column (KCOL true): K(x_n, 0) = prod_j tab[j][t] with
//    tab[j][t] = 1 + gamma_j K'(x_{n,j}, 0).
// t is the index of the first non-zero digit of x_{n,j} (the leading-zero
// count of X_j(n) in m bits; t = m for X = 0).  Each workgroup takes whole
// tiles and runs j = 1..s in order; a thread keeps the running value for its
// 16 points (n = tile E + tid + k TH) in registers (for U: U_j = U_{j-1} +
// a_j (1 + U_{j-1}), one column stored per j).  X_j(n) is the XOR of the
// generator columns of the set bits of n (Definition of a digital net,
// p = 2); the columns and the tables are staged in LDS, so the loop's only
// memory accesses are its stores.
struct ColGen {
  const uint32_t* xtab;  // [s][nbytes][256]: X_j of byte value v at byte b
  const double* tab;     // [s][ktab]
  int nbytes, s, m, ktab;
  int d0, d1;            // truncation columns U_{d0+1}..U_{d1} are stored (out column d - 1 - d0)
};

template <int LOGE, bool KCOL>
__global__ void __launch_bounds__((P2Shape<LOGE, 0>::THREADS)) fwt_p2_gen(ColGen g, double* out, PassDesc d) {
  using S = P2Shape<LOGE, 0>;
  constexpr int EPT = S::EPT, TH = S::THREADS, TB = LOGE - 4;  // tid has TB bits
  static_assert(LOGE >= 10 && EPT == 16, "16 elements per thread");
  constexpr int NS = (LOGE - 10) < 4 ? (LOGE - 10) : 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int m = g.m, s = g.s;
  double* rl = lds + ((cpad(S::E) + 1) & ~1);                    // [s][m + 1]
  uint32_t* cl = reinterpret_cast<uint32_t*>(rl + s * (m + 1));   // [s][m]: generator columns
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < s * (m + 1); i += TH) rl[i] = g.tab[(i / (m + 1)) * g.ktab + i % (m + 1)];
  for (int i = tid; i < s * m; i += TH) {
    const int j = i / m, c = i % m;
    cl[i] = g.xtab[((size_t)j * g.nbytes + (c >> 3)) * 256 + (1 << (c & 7))];
  }
  __syncthreads();
  const int G = gridDim.x, hw = blockIdx.x;
  int lb = d.xcd ? xcd_first(hw, G) : hw;
  double* lrow = lds + cpad(tid);
  double* lrowS = lds + cpad(lane + 1024 * wv);
  const uint32_t goffS = (uint32_t)(lane + 1024 * wv);
  const int sh = 32 - m;
  // Pass over one generated column of the tile: the same stage groups as
  // fwt_p2's first pass, then a coalesced store.
  auto transform_store = [&](const double (&u)[EPT], int col) {
    double v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[k] = u[k];
    reg_bfly<4>(v);
#pragma unroll
    for (int k = 0; k < EPT; ++k) lrow[cpad(k * TH)] = v[k];
    lds_barrier();
    P2Groups<LOGE, 0, 0, double, 4, 6>::run(lds, tid);
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[k] = lrowS[66 * k];
    reg_bfly<NS>(v);
    if (d.oblk) {  // blocked layout (PassDesc::oblk)
      const int64_t rs = d.oblk;
      const gptr<double> dst =
          to_global(out + (int64_t)col * d.col_out + ((lane >> 4) + 64 * wv) * rs + (int64_t)lb * 16 + (lane & 15));
#pragma unroll
      for (int k = 0; k < EPT; ++k) dst[k * 4 * rs] = v[k];
    } else {
      const gptr<double> dst = to_global(out + (int64_t)col * d.col_out + ((int64_t)lb << LOGE) + goffS);
#pragma unroll
      for (int k = 0; k < EPT; ++k) dst[k * 64] = v[k];
    }
    lds_barrier();
  };
  for (; lb < d.ntiles; lb += G) {
    const uint32_t n0 = (uint32_t)lb << LOGE;
    double u[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) u[k] = KCOL ? 1.0 : 0.0;
    const int jend = KCOL ? s : g.d1;
    for (int j = 0; j < jend; ++j) {
      const uint32_t* cj = cl + j * m;
      uint32_t xt = 0;  // X_j(tid) ^ X_j(n0)
#pragma unroll
      for (int c = 0; c < TB; ++c) xt ^= cj[c] & (0u - (((uint32_t)tid >> c) & 1u));
      for (int c = LOGE; c < m; ++c)
        if ((n0 >> c) & 1) xt ^= cj[c];
      uint32_t kx[EPT];  // X_j(k TH): the XOR of the columns of k's bits
      kx[0] = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t cb = cj[TB + b];
#pragma unroll
        for (int k = 0; k < (1 << b); ++k) kx[k + (1 << b)] = kx[k] ^ cb;
      }
      const double* rj = rl + j * (m + 1);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double a = rj[(int)__clz(xt ^ kx[k]) - sh];
        u[k] = KCOL ? u[k] * a : fma(a, 1.0 + u[k], u[k]);
      }
      if constexpr (!KCOL) {
        if (j >= g.d0) transform_store(u, j - g.d0);
      }
    }
    if constexpr (KCOL) transform_store(u, 0);
  }
}


// First pass of the forward transform of a test function sampled at the
// net (p = 2, fdwt_dwt_forward_family): the 16 values each thread would load
// are generated instead, f(x_n) at n = tile E + tid + k TH, with the sampling
// kernel's arithmetic (family.h, the same operations in the same order), then
// transformed and stored exactly as fwt_p2's first pass does, so the result
// equals sampling then transforming bit for bit while the samples never
// cross HBM.  X_j(n) is linear over Z_2 in the bits of n, which split into
// the tid part (a vector lookup in the net's byte tables), the 16 k parts
// (built by doubling from four generator columns) and the tile part; the
// last two are the same for the whole workgroup and come from scalar loads.
struct FamGen {
  const uint32_t* xtab;  // [s][nbytes][256]: X_j of byte value v at byte b
  int nbytes, m;
  FamilyArgs fa;
};

template <int LOGE, int FAM>
__global__ void __launch_bounds__((P2Shape<LOGE, 0>::THREADS)) fwt_p2_fam(FamGen g, float* out, PassDesc d) {
  using S = P2Shape<LOGE, 0>;
  constexpr int EPT = S::EPT, TH = S::THREADS, TB = LOGE - 4;  // tid has TB bits
  static_assert(LOGE >= 10 && EPT == 16, "16 elements per thread");
  constexpr int NS = (LOGE - 10) < 4 ? (LOGE - 10) : 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* lds = reinterpret_cast<float*>(smem_raw);
  using ctab = const uint32_t __attribute__((address_space(4)))*;
  const ctab tc = (ctab)g.xtab;
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int s = g.fa.s, nby = g.nbytes;
  const float inv = 1.0f / (float)(1u << g.m);  // exact power of two, as the sampling kernel's
  float* lrow = lds + cpad(tid);
  float* lrowS = lds + cpad(lane + 1024 * wv);
  const uint32_t goffS = (uint32_t)(lane + 1024 * wv);
  const int G = gridDim.x, hw = blockIdx.x;
  int lb = d.xcd ? xcd_first(hw, G) : hw;
  for (; lb < d.ntiles; lb += G) {
    const uint32_t n0 = (uint32_t)lb << LOGE;
    typename FamState<FAM>::T acc[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) acc[k] = fam_init<FAM>(g.fa);
    for (int j = 0; j < s; ++j) {
      const uint32_t* tj = g.xtab + (size_t)j * nby * 256;
      uint32_t xt = tj[tid & 255];
      if constexpr (TB > 8) xt ^= tj[256 + (tid >> 8)];
      uint32_t tp = 0;  // X_j(n0)
      for (int b = 1; b < nby; ++b) tp ^= tc[(j * nby + b) * 256 + ((n0 >> (8 * b)) & 255)];
      xt ^= tp;
      uint32_t kx[EPT];  // X_j(k TH)
      kx[0] = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int bit = TB + b;
        const uint32_t cb = tc[(j * nby + (bit >> 3)) * 256 + (1 << (bit & 7))];
#pragma unroll
        for (int k = 0; k < (1 << b); ++k) kx[k + (1 << b)] = kx[k] ^ cb;
      }
      const float a = g.fa.a[j], ia = g.fa.inv1a[j];
#pragma unroll
      for (int k = 0; k < EPT; ++k) fam_step<FAM, false>(acc[k], g.fa, a, ia, xt ^ kx[k], inv, (double)inv);
    }
    float v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[k] = fam_final<FAM>(acc[k], g.fa);
    reg_bfly<4>(v);
#pragma unroll
    for (int k = 0; k < EPT; ++k) lrow[cpad(k * TH)] = v[k];
    lds_barrier();
    P2Groups<LOGE, 0, 0, float, 4, 6>::run(lds, tid);
    float y[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) y[k] = lrowS[66 * k];
    reg_bfly<NS>(y);
    const gptr<float> dst = to_global(out + ((int64_t)lb << LOGE) + goffS);
#pragma unroll
    for (int k = 0; k < EPT; ++k) dst[k * 64] = cvt_out<float, float>(y[k], d.scale, d.scale64);
    lds_barrier();
  }
}


// ----------------------------------------------------------------- planner
struct PassGeom {
  int d0, r, wdig;
};

// LDS per workgroup: 80 KiB lets two workgroups share a CU (160 KiB of LDS).
// Elements of 8 bytes or more take a whole CU so that m = 24 still needs only
// two passes (measured faster at m = 24 than three passes with two
// workgroups per CU); FDWT_LDS_KB_WIDE overrides that budget (KiB).
static size_t lds_budget(size_t bytes) {
  static const size_t wide = [] {
    const char* e = getenv("FDWT_LDS_KB_WIDE");
    const long v = e ? atol(e) : 160;
    return (size_t)std::max(16L, std::min(160L, v)) * 1024;
  }();
  return bytes >= 8 ? wide : (size_t)80 * 1024;
}

// Digits per register group of the generic pass (PassShape's KMAX) and the
// elements each thread loads per tile (PassShape's LPT).
static int kreg_for(int p, Kind) {
  if (p == 2) return 4;
  if (p == 3) return 2;
  return 1;
}
static int loads_per_thread(int p) { return p == 2 ? 16 : (p == 3 ? 9 : (p == 5 ? 16 : 7)); }

static std::vector<PassGeom> plan(int p, int m, size_t bytes, Kind work) {
  // Largest tile exponent e with the padded tile within the LDS budget and
  // at most 1024 threads x the elements each thread loads.
  (void)work;
  const size_t budget = lds_budget(bytes);
  const int64_t per_block = 1024 * loads_per_thread(p);
  int emax = 0;
  for (int e = 1; e <= 30; ++e) {
    int64_t E = ipow(p, e);
    if ((size_t)(E + E / 32 + 1) * bytes > budget || E > per_block) break;
    emax = e;
  }
  int wpref = 0;
  while ((size_t)ipow(p, wpref) * bytes < 64) ++wpref;
  std::vector<PassGeom> out;
  const int r1 = std::min(m, emax);
  out.push_back({0, r1, 0});
  const int rest = m - r1;
  if (rest > 0) {
    // Strided passes: split the remaining digits evenly.
    const int cap = emax - std::min(wpref, r1);
    const int nstr = (rest + cap - 1) / cap;
    int d = r1;
    for (int i = 0; i < nstr; ++i) {
      const int r = (rest - (d - r1) + (nstr - i) - 1) / (nstr - i);
      out.push_back({d, r, std::min(wpref, d)});
      d += r;
    }
  }
  return out;
}

static int set_lds_attr(const void* fn, size_t bytes) { return allow_lds(fn, bytes); }

// Compute units of the current device (cached per device).
static int device_cus() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (!cache[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// Optional grouped-sum epilogue of the last pass.
struct ReduceArgs {
  const float2* wts;
  double* partial;  // [batch][fwt_reduce_parts]
  double* h0_out;
  int h0_col;
};

template <int P, bool INV, class Tin, class T, class Tout>
static int launch_pass(const void* in, void* out, const PassGeom& g, int m, int batch, double scale,
                       int64_t col_in, int64_t col_out, Kind work, const ReduceArgs* red, hipStream_t st) {
  constexpr int KMAX = P == 2 ? 4 : (P == 3 ? 2 : 1);
  using Shape = PassShape<P, KMAX, sizeof(T)>;
  constexpr int LPT = Shape::LPT;
  static_assert(PowC<P, KMAX>::v <= LPT, "a thread loads at least one register group");
  PassDesc d{};
  d.col_in = col_in;
  d.col_out = col_out;
  d.sd0 = ipow(P, g.d0);
  d.shi = ipow(P, g.d0 + g.r);
  d.r = g.r;
  d.wdig = g.wdig;
  d.w = (int)ipow(P, g.wdig);
  d.nlo = (int)ipow(P, g.d0 - g.wdig);
  d.E = (int)ipow(P, g.r) * d.w;
  d.kreg = std::min(kreg_for(P, work), KMAX);
  d.scale = (float)scale;
  d.scale64 = scale;
  const int64_t ntiles = ipow(P, m) / d.E;
  const int64_t nb = ntiles * batch;
  d.ntiles = (int)ntiles;
  d.batch = batch;
  if (red) {
    d.wts = red->wts;
    d.partial = red->partial;
    d.h0_out = red->h0_out;
    d.h0_col = red->h0_col;
  } else {
    d.h0_col = -1;
  }
  if (LPT != loads_per_thread(P)) return fail(FDWT_EINVAL, "pass geometry tables disagree");
  int threads = std::max(64, std::min(1024, (d.E + LPT - 1) / LPT));
  threads = (threads + 63) / 64 * 64;
  // Every tile element is loaded by the per-thread prefetch; the index
  // arithmetic (divmod_small) needs indices below 2^22.
  if ((int64_t)threads * LPT < d.E || d.E >= (1 << 22) || threads > Shape::THREADS)
    return fail(FDWT_EINVAL, "pass tile larger than one workgroup loads");
  const size_t tile_bytes = (size_t)(d.E + d.E / 32 + 1) * sizeof(T);
  const size_t lds = tile_bytes + 8 - tile_bytes % 8 + 16 * sizeof(double);
  const void* fn = red ? (const void*)fwt_pass<P, INV, Tin, T, Tout, KMAX, EPI_REDUCE>
                       : (const void*)fwt_pass<P, INV, Tin, T, Tout, KMAX, EPI_STORE>;
  int rc = set_lds_attr(fn, lds);
  if (rc) return rc;
  // Persistent grid: as many workgroups as fit on the device at once.
  int per_cu = 0;
  FDWT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds));
  int64_t G = (int64_t)std::max(1, per_cu) * device_cus();
  if (G >= nb) G = nb;
  d.xcd = G >= 64 ? 1 : 0;
  const double elems = (double)ipow(P, m) * batch;
  const double alg = red ? elems * sizeof(Tin) + (double)ipow(P, m) * sizeof(float2)
                         : elems * (sizeof(Tin) + sizeof(Tout));
  const int cls = sizeof(T) >= 16 || std::is_same<T, double>::value ? FDWT_TC_PASS_F64
                  : (sizeof(T) == 8 ? FDWT_TC_PASS_CF32 : FDWT_TC_PASS_F32);
  const Tin* inp = (const Tin*)in;
  Tout* outp = (Tout*)out;
  void* args[] = {(void*)&inp, (void*)&outp, (void*)&d};
  return launch_timed(fn, dim3((unsigned)G), dim3(threads), args, lds, st, cls, alg);
}

// Dispatch on (p, direction, in/work/out kinds).
template <int P, bool INV>
static int pass_dispatch(Kind ik, Kind wk, Kind ok, const void* in, void* out, const PassGeom& g,
                         int m, int batch, double scale, int64_t ci, int64_t co, const ReduceArgs* red,
                         hipStream_t st) {
#define FDWT_PASS(TIN, T, TOUT) \
  return launch_pass<P, INV, TIN, T, TOUT>(in, out, g, m, batch, scale, ci, co, wk, red, st)
  if constexpr (P == 2) {
    if (!red) {
      if (wk == K_F32 && ik == K_F32 && ok == K_F32) FDWT_PASS(float, float, float);
      if (wk == K_U32 && ik == K_U32 && ok == K_U32) FDWT_PASS(uint32_t, uint32_t, uint32_t);
    }
    if (wk == K_F64 && ik == K_F64 && ok == K_F64) FDWT_PASS(double, double, double);
  } else {
    if (wk == K_CF32 && !red) {
      if (ik == K_F32 && ok == K_CF32) FDWT_PASS(float, float2, float2);
      if (ik == K_F32 && ok == K_F32) FDWT_PASS(float, float2, float);
      if (ik == K_CF32 && ok == K_CF32) FDWT_PASS(float2, float2, float2);
      if (ik == K_CF32 && ok == K_F32) FDWT_PASS(float2, float2, float);
    }
    if (wk == K_CF64) {
      if (ik == K_F64 && ok == K_CF64) FDWT_PASS(double, double2, double2);
      if (ik == K_CF64 && ok == K_CF64) FDWT_PASS(double2, double2, double2);
      if (!red && ik == K_CF64 && ok == K_F64) FDWT_PASS(double2, double2, double);
    }
  }
#undef FDWT_PASS
  return fail(FDWT_EINVAL, "unsupported transform element types");
}

static int pass_any(int p, bool inv, Kind ik, Kind wk, Kind ok, const void* in, void* out,
                    const PassGeom& g, int m, int batch, double scale, int64_t ci, int64_t co,
                    const ReduceArgs* red, hipStream_t st) {
  switch (p) {
    case 2:
      return inv ? pass_dispatch<2, true>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st)
                 : pass_dispatch<2, false>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st);
    case 3:
      return inv ? pass_dispatch<3, true>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st)
                 : pass_dispatch<3, false>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st);
    case 5:
      return inv ? pass_dispatch<5, true>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st)
                 : pass_dispatch<5, false>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st);
    case 7:
      return inv ? pass_dispatch<7, true>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st)
                 : pass_dispatch<7, false>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, red, st);
  }
  return fail(FDWT_EUNSUPPORTED, "p must be 2, 3, 5 or 7");
}

// ---------------------------------------------- p = 2 static-shape passes
struct P2Pass {
  int d0, loge, wdig;
};

// Two passes cover m <= 24: a contiguous first pass of up to 2^14 elements,
// then strided passes over the remaining digits with rows of 2^wd elements,
// split evenly (>= 2^7 elements per tile).  Rows of 16 doubles or 32 floats
// are 128 bytes, the cache line: a row never shares a line with another tile
// (tiles of one column are not neighbours in time) and each DRAM access
// moves a whole line.  4-byte elements take rows of 32 when that does not
// add a pass (every m <= 23); m = 24 keeps rows of 16 (64 bytes) and two
// passes.
static std::vector<P2Pass> plan_p2_w(int m, int emax, int wd) {
  std::vector<P2Pass> out;
  if (m <= emax) {
    out.push_back({0, m, 0});
    return out;
  }
  const int rem = m - emax;
  const int cap = emax - wd;
  const int nstr = (rem + cap - 1) / cap;
  const int rd = std::max((rem + nstr - 1) / nstr, 7 - wd);
  const int first = m - nstr * rd;
  out.push_back({0, first, 0});
  for (int i = 0; i < nstr; ++i) out.push_back({first + i * rd, rd + wd, wd});
  return out;
}

static std::vector<P2Pass> plan_p2_e(int m, int emax, size_t bytes = 4) {
  std::vector<P2Pass> v = plan_p2_w(m, emax, 4);
  if (bytes <= 4) {
    std::vector<P2Pass> w = plan_p2_w(m, emax, 5);
    if (w.size() <= v.size()) return w;
  }
  return v;
}

static std::vector<P2Pass> plan_p2(int m, size_t bytes) {
  return plan_p2_e(m, (bytes >= 8 && lds_budget(bytes) < 136 * 1024) ? 13 : 14, bytes);
}

template <class Tin, class T, class Tout, int WDIG, int EPI>
static const void* p2_kernel(int loge) {
  switch (loge) {
    case 7: return (const void*)fwt_p2<Tin, T, Tout, 7, WDIG, EPI>;
    case 8: return (const void*)fwt_p2<Tin, T, Tout, 8, WDIG, EPI>;
    case 9: return (const void*)fwt_p2<Tin, T, Tout, 9, WDIG, EPI>;
    case 10: return (const void*)fwt_p2<Tin, T, Tout, 10, WDIG, EPI>;
    case 11: return (const void*)fwt_p2<Tin, T, Tout, 11, WDIG, EPI>;
    case 12: return (const void*)fwt_p2<Tin, T, Tout, 12, WDIG, EPI>;
    case 13: return (const void*)fwt_p2<Tin, T, Tout, 13, WDIG, EPI>;
    case 14: return (const void*)fwt_p2<Tin, T, Tout, 14, WDIG, EPI>;
  }
  return nullptr;
}

// Workgroups per CU for (kernel, LDS), cached.
static int occupancy(const void* fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_pair(fn, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, lds) != hipSuccess || n < 1) n = 1;
  cache[key] = n;
  return n;
}

// ---------------------------------------------- p = 3 static-shape passes
// FDWT_P3_STATIC = 0 sends p = 3 float-complex transforms through the
// generic pass instead (read once per process).
static bool p3_static_enabled() {
  static const bool on = [] {
    const char* e = getenv("FDWT_P3_STATIC");
    return e ? atoi(e) != 0 : true;
  }();
  return on;
}

// Whether a pass has a shape of fwt_p3s: the first pass of 8 digits, or a
// strided pass of 2..6 digits over rows of 3^(8 - r) elements.
static bool p3s_shape(const PassGeom& g) {
  return (g.d0 == 0 && g.r == 8 && g.wdig == 0) || (g.d0 >= 8 && g.r >= 2 && g.r <= 6 && g.wdig == 8 - g.r);
}

// The generic plan's digit split (a first pass of 8 digits, the rest split
// evenly into passes of at most 6), with every strided pass of two or more
// digits taking rows of 3^(8 - r) elements, so that its tiles hold 3^8.
static std::vector<PassGeom> plan_p3s(int m) {
  std::vector<PassGeom> v = plan(3, m, sizeof(float2), K_CF32);
  for (PassGeom& g : v)
    if (g.d0 > 0 && g.r >= 2) g.wdig = 8 - g.r;
  return v;
}

// FDWT_P3_KT = 2 or 3 fixes the register digits of every static pass of
// three or more digits (read once per process); 0 or unset: chosen per launch.
static int p3s_kt_forced() {
  static const int kt = [] {
    const char* e = getenv("FDWT_P3_KT");
    const int v = e ? atoi(e) : 0;
    return v == 2 || v == 3 ? v : 0;
  }();
  return kt;
}

template <bool INV, class Tin, class Tout, int RD>
static const void* p3s_kernel(int kt) {
  if constexpr (RD >= 3) {
    if (kt == 3) return (const void*)fwt_p3s<INV, Tin, float2, Tout, RD, 3>;
    return (const void*)fwt_p3s<INV, Tin, float2, Tout, RD, 2>;
  } else {
    return kt == 2 ? (const void*)fwt_p3s<INV, Tin, float2, Tout, RD, 2> : nullptr;
  }
}

template <bool INV, class Tin, class Tout>
static const void* p3s_kernel_for(int rd, int kt) {
  if (rd == 8) return p3s_kernel<INV, Tin, Tout, 8>(kt);
  if constexpr (std::is_same<Tin, float2>::value) {
    switch (rd) {
      case 2: return p3s_kernel<INV, Tin, Tout, 2>(kt);
      case 3: return p3s_kernel<INV, Tin, Tout, 3>(kt);
      case 4: return p3s_kernel<INV, Tin, Tout, 4>(kt);
      case 5: return p3s_kernel<INV, Tin, Tout, 5>(kt);
      case 6: return p3s_kernel<INV, Tin, Tout, 6>(kt);
    }
  }
  return nullptr;
}

template <bool INV, class Tin, class Tout>
static int launch_p3s(const void* in, void* out, const PassGeom& g, int m, int batch, double scale, hipStream_t st) {
  if (!p3s_shape(g)) return fail(FDWT_EINVAL, "not a static p = 3 pass shape");
  const int64_t N = ipow(3, m);
  const int64_t ntiles = N / 6561;
  const int64_t nb = ntiles * batch;
  const size_t lds = (size_t)6561 * sizeof(float2);
  // Two register digits (729 threads, two workgroups per CU) hide memory
  // latency best; three (243 threads, three per CU) pay when they let every
  // tile run in one round and two digits would not (3^14 points: 729 tiles).
  const void* fn = p3s_kernel_for<INV, Tin, Tout>(g.r, 2);
  int kt = 2;
  if (!fn) return fail(FDWT_EINVAL, "static p = 3 pass not built for these element types");
  if (g.r >= 3) {
    const void* fn3 = p3s_kernel_for<INV, Tin, Tout>(g.r, 3);
    if (int rc = allow_lds(fn, lds)) return rc;
    if (int rc = allow_lds(fn3, lds)) return rc;
    const int64_t g2 = (int64_t)occupancy(fn, 729, lds) * device_cus();
    const int64_t g3 = (int64_t)occupancy(fn3, 243, lds) * device_cus();
    const int forced = p3s_kt_forced();
    if (forced ? forced == 3 : (nb > g2 && nb <= g3)) {
      fn = fn3;
      kt = 3;
    }
  }
  PassDesc d{};
  d.col_in = N;
  d.col_out = N;
  d.sd0 = ipow(3, g.d0);
  d.shi = ipow(3, g.d0 + g.r);
  d.r = g.r;
  d.wdig = g.wdig;
  d.w = (int)ipow(3, g.wdig);
  d.nlo = (int)ipow(3, g.d0 - g.wdig);
  d.E = 6561;
  d.kreg = kt;
  d.scale = (float)scale;
  d.scale64 = scale;
  d.h0_col = -1;
  d.ntiles = (int)ntiles;
  d.batch = batch;
  const int threads = kt == 3 ? 243 : 729;
  if (int rc = allow_lds(fn, lds)) return rc;
  int64_t G = (int64_t)occupancy(fn, threads, lds) * device_cus();
  if (G >= nb) G = nb;
  d.xcd = G >= 64 ? 1 : 0;
  const Tin* inp = (const Tin*)in;
  Tout* outp = (Tout*)out;
  void* args[] = {(void*)&inp, (void*)&outp, (void*)&d};
  return launch_timed(fn, dim3((unsigned)G), dim3(threads), args, lds, st, FDWT_TC_PASS_CF32,
                      (double)N * batch * (sizeof(Tin) + sizeof(Tout)));
}

template <bool INV>
static int p3s_pass_dir(Kind ik, Kind ok, const void* in, void* out, const PassGeom& g, int m, int batch,
                        double scale, hipStream_t st) {
  if (ik == K_F32 && ok == K_CF32) return launch_p3s<INV, float, float2>(in, out, g, m, batch, scale, st);
  if (ik == K_F32 && ok == K_F32) return launch_p3s<INV, float, float>(in, out, g, m, batch, scale, st);
  if (ik == K_CF32 && ok == K_CF32) return launch_p3s<INV, float2, float2>(in, out, g, m, batch, scale, st);
  if (ik == K_CF32 && ok == K_F32) return launch_p3s<INV, float2, float>(in, out, g, m, batch, scale, st);
  return fail(FDWT_EINVAL, "unsupported transform element types");
}

// Partial sums per column written by a reducing static pass: one per wave of
// every tile.
static int64_t p2_reduce_parts(int m, const P2Pass& g) {
  const int threads = std::max(64, std::min(1024, (1 << g.loge) / 16));
  return ((int64_t(1) << m) >> g.loge) * (threads / 64);
}

// FDWT_REDUCE_WKEEP = 0 turns the grouped-sum weight reuse off (the sums are
// bit-identical either way: each partial sum covers the same elements).
// Read at each launch.
static bool wkeep_enabled() {
  const char* e = getenv("FDWT_REDUCE_WKEEP");
  return !(e && atoi(e) == 0);
}

template <class Tin, class T, class Tout>

// layout: 0 natural; 1 the (contiguous first) pass stores in the blocked
// layout of PassDesc::oblk; 2 the (strided) pass reads and writes that
// blocked layout, where each of its tiles is one contiguous block.
static int launch_p2(const void* in, void* out, const P2Pass& g, int m, int batch, double scale,
                     const ReduceArgs* red, hipStream_t st, const void* const* in_tab = nullptr,
                     void* const* out_tab = nullptr, int layout = 0) {
  constexpr bool wide = sizeof(T) >= 8;
  const void* fn = nullptr;
  if (red) {
    if constexpr (wide) fn = g.wdig ? p2_kernel<Tin, T, Tout, 4, EPI_REDUCE>(g.loge) : p2_kernel<Tin, T, Tout, 0, EPI_REDUCE>(g.loge);
  } else {
    if (g.wdig == 5) {
      if constexpr (!wide) fn = p2_kernel<Tin, T, Tout, 5, EPI_STORE>(g.loge);
    } else {
      fn = g.wdig ? p2_kernel<Tin, T, Tout, 4, EPI_STORE>(g.loge) : p2_kernel<Tin, T, Tout, 0, EPI_STORE>(g.loge);
    }
  }
  if (!fn || (g.wdig != 0 && g.wdig != 4 && g.wdig != 5)) return fail(FDWT_EINVAL, "no static pass shape");
  const int64_t N = int64_t(1) << m;
  const int E = 1 << g.loge;
  const int threads = std::max(64, std::min(1024, E / 16));
  PassDesc d{};
  d.col_in = N;
  d.col_out = N;
  d.sd0 = int64_t(1) << g.d0;
  d.shi = int64_t(1) << (g.d0 + g.loge - g.wdig);
  d.r = g.loge - g.wdig;
  d.wdig = g.wdig;
  d.w = 1 << g.wdig;
  d.nlo = (int)(int64_t(1) << (g.d0 - g.wdig));
  d.E = E;
  d.scale = (float)scale;
  d.scale64 = scale;
  const int64_t ntiles = N / E;
  const int64_t nb = ntiles * batch;
  d.ntiles = (int)ntiles;
  d.batch = batch;
  if (red) {
    d.wts = red->wts;
    d.partial = red->partial;
    d.h0_out = red->h0_out;
    d.h0_col = red->h0_col;
  } else {
    d.h0_col = -1;
  }
  d.in_tab = in_tab;
  d.out_tab = out_tab;
  if (layout == 1) {
    if (g.wdig != 0 || g.loge < 10 || in_tab || out_tab) return fail(FDWT_EINVAL, "blocked store needs a first pass");
    d.oblk = ntiles * 16;
  } else if (layout == 2) {
    if (g.wdig != 4 || g.d0 + g.loge - g.wdig != m) return fail(FDWT_EINVAL, "blocked read needs the last pass");
    d.sd0 = 16;
    d.nlo = 1;
    d.shi = E;
  }
  const size_t lds = ((size_t)cpad(E) * sizeof(T) + 15) / 16 * 16;
  if (int rc = allow_lds(fn, lds)) return rc;
  int64_t G = (int64_t)occupancy(fn, threads, lds) * device_cus();
  if (G >= nb) G = nb;
  d.xcd = G >= 64 ? 1 : 0;
  // Grouped sums over several columns: a workgroup keeps one tile's weights
  // for all its columns when the tiles split evenly over the grid.
  d.wkeep = (red && g.loge >= 10 && batch > 1 && ntiles % G == 0 && wkeep_enabled()) ? 1 : 0;
  void* args[] = {(void*)&in, (void*)&out, (void*)&d};
  const double elems = (double)N * batch;
  const double work = red ? elems * sizeof(Tin) + (double)N * sizeof(float2) : elems * (sizeof(Tin) + sizeof(Tout));
  return launch_timed(fn, dim3((unsigned)G), dim3(threads), args, lds, st, wide ? FDWT_TC_PASS_F64 : FDWT_TC_PASS_F32,
                      work);
}

static int p2_pass(Kind k, const void* in, void* out, const P2Pass& g, int m, int batch, double scale,
                   const ReduceArgs* red, hipStream_t st, int layout = 0) {
  if (k == K_F32 && !red) return launch_p2<float, float, float>(in, out, g, m, batch, scale, nullptr, st);
  if (k == K_U32 && !red) return launch_p2<uint32_t, uint32_t, uint32_t>(in, out, g, m, batch, scale, nullptr, st);
  if (k == K_F64) return launch_p2<double, double, double>(in, out, g, m, batch, scale, red, st, nullptr, nullptr, layout);
  return fail(FDWT_EINVAL, "unsupported p = 2 element type");
}

// p = 2 transforms of one element type through the static-shape passes
// (forward and inverse coincide up to the scale for p = 2).
static bool p2_static_ok(int p, int m, Kind ik, Kind wk, Kind ok) {
  return p == 2 && m >= 7 && ik == wk && ok == wk && (wk == K_F32 || wk == K_U32 || wk == K_F64);
}

static int run_p2(int m, Kind k, const void* in, void* out, void* tmp, int batch, double scale,
                  const ReduceArgs* red, int64_t* last_parts, hipStream_t st) {
  const std::vector<P2Pass> passes = plan_p2(m, kind_bytes(k));
  const size_t np = passes.size();
  if (last_parts) *last_parts = p2_reduce_parts(m, passes.back());
  if (np == 1) return p2_pass(k, in, out, passes[0], m, batch, scale, red, st);
  void* mid = red ? tmp : out;
  if (!mid) return fail(FDWT_EINVAL, "transform needs a workspace for its intermediate passes");
  int rc = p2_pass(k, in, mid, passes[0], m, batch, 1.0f, nullptr, st);
  for (size_t i = 1; !rc && i + 1 < np; ++i) rc = p2_pass(k, mid, mid, passes[i], m, batch, 1.0f, nullptr, st);
  if (rc) return rc;
  return p2_pass(k, mid, out, passes[np - 1], m, batch, scale, red, st);
}

static int run_passes(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
                      Kind out_kind, void* out, void* tmp, int batch, double scale, const ReduceArgs* red,
                      int64_t* last_parts, hipStream_t st) {
  if (p2_static_ok(p, m, in_kind, work_kind, out_kind))
    return run_p2(m, work_kind, in, out, tmp, batch, scale, red, last_parts, st);
  const int64_t N = ipow(p, m);
  // p = 3 float-complex store passes take the static shapes where the plan
  // has them (every pass but a strided one of a single digit, for m >= 8).
  const bool p3s = p == 3 && work_kind == K_CF32 && !red && p3_static_enabled();
  std::vector<PassGeom> passes = p3s ? plan_p3s(m) : plan(p, m, kind_bytes(work_kind), work_kind);
  const size_t np = passes.size();
  if (last_parts) {
    const PassGeom& g = passes.back();
    *last_parts = N / (ipow(p, g.r) * ipow(p, g.wdig));
  }
  auto one = [&](Kind ik, Kind ok, const void* src, void* dst, const PassGeom& g, double sc,
                 const ReduceArgs* rd) {
    if (p3s && p3s_shape(g))
      return inverse ? p3s_pass_dir<true>(ik, ok, src, dst, g, m, batch, sc, st)
                     : p3s_pass_dir<false>(ik, ok, src, dst, g, m, batch, sc, st);
    return pass_any(p, inverse, ik, work_kind, ok, src, dst, g, m, batch, sc, N, N, rd, st);
  };
  if (np == 1) return one(in_kind, out_kind, in, out, passes[0], scale, red);
  // Intermediate buffer: the output itself when it holds the working type.
  void* mid = (!red && kind_bytes(out_kind) == kind_bytes(work_kind)) ? out : tmp;
  if (!mid) return fail(FDWT_EINVAL, "transform needs a workspace for its intermediate passes");
  int rc = one(in_kind, work_kind, in, mid, passes[0], 1.0, nullptr);
  if (rc) return rc;
  for (size_t i = 1; i + 1 < np; ++i) {
    rc = one(work_kind, work_kind, mid, mid, passes[i], 1.0, nullptr);
    if (rc) return rc;
  }
  return one(work_kind, out_kind, mid, out, passes[np - 1], scale, red);
}

int fwt_run_tmp(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
                Kind out_kind, void* out, void* tmp, int batch, double scale, hipStream_t st) {
  return run_passes(p, m, inverse, in_kind, in, work_kind, out_kind, out, tmp, batch, scale, nullptr,
                    nullptr, st);
}

int fwt_run(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
            Kind out_kind, void* out, int batch, double scale, hipStream_t st) {
  return fwt_run_tmp(p, m, inverse, in_kind, in, work_kind, out_kind, out, nullptr, batch, scale, st);
}

// Unnormalised forward transform of `batch` real float64 columns with the
// grouped-sum epilogue in its last pass (no output stored).  tmp holds the
// intermediate passes (batch columns of the working type); partial receives
// [batch][parts] partial sums, parts (fwt_reduce_parts) returned in *parts.
int fwt_reduce_f64(int p, int m, const double* in, void* tmp, int batch, const float2* wts,
                   double* partial, double* h0_out, int h0_col, int64_t* parts, hipStream_t st) {
  ReduceArgs red{wts, partial, h0_out, h0_col};
  const Kind wk = p == 2 ? K_F64 : K_CF64;
  return run_passes(p, m, false, K_F64, in, wk, wk, tmp, tmp, batch, 1.0f, &red, parts, st);
}

// Plans of p = 2 float transforms for the batch tuner: the first pass takes
// up to 2^emax elements (emax in 7..14), then strided passes of rows of 16.
int p2_plan_passes(int m, int emax) { return (int)plan_p2_e(m, emax).size(); }
// Plans for two values of emax are the same pass list.
bool p2_plans_equal(int m, int e1, int e2) {
  const std::vector<P2Pass> a = plan_p2_e(m, e1), b = plan_p2_e(m, e2);
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].d0 != b[i].d0 || a[i].loge != b[i].loge || a[i].wdig != b[i].wdig) return false;
  return true;
}

// Pass `level` of the plan (m, emax) for a group of njobs float jobs of 2^m
// points each: column c reads in_tab[c] (level 0) or out_tab[c] and writes
// out_tab[c]; the last pass scales by 2^-m (Eq. (eq_dwalshcoeff)).
int fwt_p2_group_pass(int m, int emax, int level, const void* const* in_tab, void* const* out_tab, int njobs,
                      hipStream_t st) {
  const std::vector<P2Pass> passes = plan_p2_e(m, emax);
  if (level < 0 || level >= (int)passes.size()) return fail(FDWT_EINVAL, "no such pass");
  const bool last = level + 1 == (int)passes.size();
  const double scale = last ? std::ldexp(1.0, -m) : 1.0;
  const void* const* src = level == 0 ? in_tab : (const void* const*)out_tab;
  return launch_p2<float, float, float>(nullptr, nullptr, passes[level], m, njobs, scale, nullptr, st, src, out_tab);
}

// The p = 2 float64 transform of a batch of columns split after its first
// pass, for callers that produce part of the first pass's output with
// fwt_p2_gen_first: whether the plan for m has that shape (two or more
// passes, the first contiguous with 2^12..2^14-element tiles), the first pass
// alone (in -> out), and the remaining passes in place with the grouped-sum
// epilogue in the last (partial as for fwt_reduce_f64).
bool fwt_p2_split_ok(int m) {
  if (m < 7) return false;
  const std::vector<P2Pass> v = plan_p2(m, 8);
  return v.size() >= 2 && v[0].d0 == 0 && v[0].wdig == 0 && v[0].loge >= 12 && v[0].loge <= 14;
}

// Two-pass plans can keep the intermediate in the blocked layout of
// PassDesc::oblk (the first pass stores blocks, the grouped-sum pass reads
// each tile as one contiguous block; its weights then come in the same
// layout, fwt_p2_blocked_index).
bool fwt_p2_blocked_ok(int m) { return fwt_p2_split_ok(m) && plan_p2(m, 8).size() == 2; }

// Digits of the first pass of the float64 plan for m.
int fwt_p2_first_loge(int m) { return plan_p2(m, 8)[0].loge; }

int fwt_p2_f64_first(int m, const double* in, double* out, int batch, bool blocked, hipStream_t st) {
  if (!fwt_p2_split_ok(m) || (blocked && !fwt_p2_blocked_ok(m))) return fail(FDWT_EINVAL, "no split plan for this m");
  return p2_pass(K_F64, in, out, plan_p2(m, 8)[0], m, batch, 1.0, nullptr, st, blocked ? 1 : 0);
}

int fwt_p2_f64_reduce_rest(int m, double* data, int batch, const float2* wts, double* partial, double* h0_out,
                           int h0_col, bool blocked, hipStream_t st) {
  if (!fwt_p2_split_ok(m) || (blocked && !fwt_p2_blocked_ok(m))) return fail(FDWT_EINVAL, "no split plan for this m");
  const std::vector<P2Pass> v = plan_p2(m, 8);
  const ReduceArgs red{wts, partial, h0_out, h0_col};
  int rc = FDWT_OK;
  for (size_t i = 1; !rc && i + 1 < v.size(); ++i) rc = p2_pass(K_F64, data, data, v[i], m, batch, 1.0, nullptr, st);
  if (rc) return rc;
  return p2_pass(K_F64, data, data, v.back(), m, batch, 1.0, &red, st, blocked ? 2 : 0);
}

// First pass of the transforms of generated columns (fwt_p2_gen): the
// truncation columns U_{d0+1}..U_{d1} from the R' table (kcol false: out
// receives d1 - d0 columns), or the kernel column K from the K' table (kcol
// true: one column; d0, d1 unused).
int fwt_p2_gen_first(int m, int s, const uint32_t* xtab, int nbytes, const double* tab, int ktab, bool kcol,
                     int d0, int d1, double* out, bool blocked, hipStream_t st) {
  if (!fwt_p2_split_ok(m) || s < 1 || s > 64 || ktab <= m) return fail(FDWT_EINVAL, "bad generated-column pass");
  if (!kcol && (d0 < 0 || d1 > s || d0 >= d1)) return fail(FDWT_EINVAL, "bad generated-column range");
  const P2Pass g = plan_p2(m, 8)[0];
  const void* fn = nullptr;
  if (kcol) fn = g.loge == 14 ? (const void*)fwt_p2_gen<14, true>
                 : g.loge == 13 ? (const void*)fwt_p2_gen<13, true> : (const void*)fwt_p2_gen<12, true>;
  else fn = g.loge == 14 ? (const void*)fwt_p2_gen<14, false>
            : g.loge == 13 ? (const void*)fwt_p2_gen<13, false> : (const void*)fwt_p2_gen<12, false>;
  const int64_t N = int64_t(1) << m;
  const int E = 1 << g.loge;
  const int threads = E / 16;
  const int ncol = kcol ? 1 : d1 - d0;
  PassDesc d{};
  d.col_in = N;
  d.col_out = N;
  d.ntiles = (int)(N / E);
  d.batch = ncol;
  d.h0_col = -1;
  if (blocked) {
    if (!fwt_p2_blocked_ok(m)) return fail(FDWT_EINVAL, "no blocked plan for this m");
    d.oblk = (int64_t)d.ntiles * 16;
  }
  const size_t lds = (size_t)((cpad(E) + 1) & ~1) * sizeof(double) + (size_t)s * (m + 1) * sizeof(double) +
                     (size_t)s * m * sizeof(uint32_t);
  if (int rc = allow_lds(fn, lds)) return rc;
  int64_t G = (int64_t)occupancy(fn, threads, lds) * device_cus();
  if (G >= d.ntiles) G = d.ntiles;
  d.xcd = G >= 64 ? 1 : 0;
  ColGen cg{xtab, tab, nbytes, s, m, ktab, kcol ? 0 : d0, kcol ? s : d1};
  void* args[] = {(void*)&cg, (void*)&out, (void*)&d};
  return launch_timed(fn, dim3((unsigned)G), dim3(threads), args, lds, st, FDWT_TC_PASS_F64,
                      (double)N * ncol * sizeof(double));
}

// The passes after the first of an unnormalised p = 2 float64 transform, in
// place (the first pass's output already in data).
int fwt_p2_f64_rest(int m, double* data, int batch, hipStream_t st) {
  if (!fwt_p2_split_ok(m)) return fail(FDWT_EINVAL, "no split plan for this m");
  const std::vector<P2Pass> v = plan_p2(m, 8);
  int rc = FDWT_OK;
  for (size_t i = 1; !rc && i < v.size(); ++i) rc = p2_pass(K_F64, data, data, v[i], m, batch, 1.0, nullptr, st);
  return rc;
}

// fdwt_dwt_forward_family for p = 2: the first pass samples its own input
// (fwt_p2_fam), the remaining passes run in place on out.  Returns
// FDWT_EUNSUPPORTED (nothing enqueued) when the plan's first pass has fewer
// than 2^10 elements; the caller then samples and transforms separately.
template <int FAM>
static const void* fam_kernel(int loge) {
  switch (loge) {
    case 10: return (const void*)fwt_p2_fam<10, FAM>;
    case 11: return (const void*)fwt_p2_fam<11, FAM>;
    case 12: return (const void*)fwt_p2_fam<12, FAM>;
    case 13: return (const void*)fwt_p2_fam<13, FAM>;
    case 14: return (const void*)fwt_p2_fam<14, FAM>;
  }
  return nullptr;
}

int fwt_p2_forward_family(const Net& net, int family, const FamilyArgs& fa, float* out, hipStream_t st) {
  const std::vector<P2Pass> passes = plan_p2(net.m, 4);
  const P2Pass& g0 = passes[0];
  if (net.p != 2 || net.m < 10 || g0.d0 != 0 || g0.wdig != 0 || g0.loge < 10 || g0.loge > 14)
    return FDWT_EUNSUPPORTED;
  const void* fn = family == FDWT_FAMILY_PRODUCT ? fam_kernel<FDWT_FAMILY_PRODUCT>(g0.loge)
                   : family == FDWT_FAMILY_EXP   ? fam_kernel<FDWT_FAMILY_EXP>(g0.loge)
                   : family == FDWT_FAMILY_ASIAN ? fam_kernel<FDWT_FAMILY_ASIAN>(g0.loge)
                                                 : fam_kernel<FDWT_FAMILY_WANGFANG>(g0.loge);
  if (!fn) return fail(FDWT_EINVAL, "no fused sampling pass for this shape");
  const int64_t N = int64_t(1) << net.m;
  const int E = 1 << g0.loge;
  const int threads = E / 16;
  const double scale = std::ldexp(1.0, -net.m);  // Eq. (eq_dwalshcoeff), applied by the last pass
  PassDesc d{};
  d.ntiles = (int)(N / E);
  d.batch = 1;
  d.h0_col = -1;
  d.scale = passes.size() == 1 ? (float)scale : 1.0f;
  d.scale64 = passes.size() == 1 ? scale : 1.0;
  const size_t lds = ((size_t)cpad(E) * sizeof(float) + 15) / 16 * 16;
  if (int rc = allow_lds(fn, lds)) return rc;
  int64_t G = (int64_t)occupancy(fn, threads, lds) * device_cus();
  if (G >= d.ntiles) G = d.ntiles;
  d.xcd = G >= 64 ? 1 : 0;
  FamGen fg{net.d_xtab, net.nbytes, net.m, fa};
  void* args[] = {(void*)&fg, (void*)&out, (void*)&d};
  if (int rc = launch_timed(fn, dim3((unsigned)G), dim3(threads), args, lds, st, FDWT_TC_SAMPLE, 4.0 * (double)N))
    return rc;
  for (size_t i = 1; i < passes.size(); ++i) {
    const bool last = i + 1 == passes.size();
    if (int rc = p2_pass(K_F32, out, out, passes[i], net.m, 1, last ? scale : 1.0, nullptr, st)) return rc;
  }
  return FDWT_OK;
}

int64_t fwt_reduce_parts(int p, int m, size_t elem_bytes) {
  if (p == 2 && m >= 7) return p2_reduce_parts(m, plan_p2(m, elem_bytes).back());
  std::vector<PassGeom> passes = plan(p, m, elem_bytes, elem_bytes >= 16 ? K_CF64 : K_F64);
  const PassGeom& g = passes.back();
  return ipow(p, m) / (ipow(p, g.r) * ipow(p, g.wdig));
}

}  // namespace fdwt
