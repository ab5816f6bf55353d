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
#include "dev_math.h"

#include <algorithm>
#include <mutex>
#include <unordered_set>

namespace fdwt {

size_t kind_bytes(Kind k) {
  switch (k) {
    case K_F32: return 4;
    case K_U32: return 4;
    case K_CF32: return 8;
    case K_DF: return 8;
    case K_CDF: return 16;
  }
  return 0;
}

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
  float scale;      // multiplies float-based outputs (last pass only)
};

// ------------------------------------------------------------ conversions
template <class Tin, class T>
__device__ __forceinline__ T cvt_in(Tin v);
template <> __device__ __forceinline__ float cvt_in<float, float>(float v) { return v; }
template <> __device__ __forceinline__ uint32_t cvt_in<uint32_t, uint32_t>(uint32_t v) { return v; }
template <> __device__ __forceinline__ float2 cvt_in<float, float2>(float v) { return make_float2(v, 0.0f); }
template <> __device__ __forceinline__ float2 cvt_in<float2, float2>(float2 v) { return v; }
template <> __device__ __forceinline__ df cvt_in<df, df>(df v) { return v; }
template <> __device__ __forceinline__ cdf cvt_in<df, cdf>(df v) { return cdf{v, df{0.0f, 0.0f}}; }
template <> __device__ __forceinline__ cdf cvt_in<cdf, cdf>(cdf v) { return v; }

template <class T, class Tout>
__device__ __forceinline__ Tout cvt_out(T v, float sc);
template <> __device__ __forceinline__ float cvt_out<float, float>(float v, float sc) { return v * sc; }
template <> __device__ __forceinline__ uint32_t cvt_out<uint32_t, uint32_t>(uint32_t v, float) { return v; }
template <> __device__ __forceinline__ float2 cvt_out<float2, float2>(float2 v, float sc) { return make_float2(v.x * sc, v.y * sc); }
template <> __device__ __forceinline__ float cvt_out<float2, float>(float2 v, float sc) { return v.x * sc; }
template <> __device__ __forceinline__ df cvt_out<df, df>(df v, float) { return v; }
template <> __device__ __forceinline__ cdf cvt_out<cdf, cdf>(cdf v, float) { return v; }
template <> __device__ __forceinline__ df cvt_out<cdf, df>(cdf v, float) { return v.re; }

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
// KK radix-p stages in registers and writes them back.
template <int P, bool INV, class T, int KK>
__device__ __forceinline__ void run_group(T* lds, const PassDesc& d, int q) {
  constexpr int R = PowC<P, KK>::v;
  const int pq = ipow_d(P, q);
  const int ng = d.E / R;
  const int stq = d.w * pq;  // LDS stride of digit q
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    const int c = Ix<P>::mod(g, d.wdig, d.w);
    const int rem = Ix<P>::div(g, d.wdig, d.w);
    const int il = Ix<P>::mod(rem, q, pq);
    const int ih = Ix<P>::div(rem, q, pq);
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

template <int P, bool INV, class Tin, class T, class Tout, int KMAX>
__global__ void __launch_bounds__(1024) fwt_pass(const Tin* __restrict__ in, Tout* out, PassDesc d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  int b = blockIdx.x;
  if (d.xcd) {
    // Workgroups are dispatched round-robin over the 8 XCDs; remap so that
    // consecutive tiles (which share cache lines at tile edges and DRAM pages)
    // run on the same XCD and share its L2.
    const int nb = gridDim.x;
    b = (b & 7) * (nb >> 3) + (b >> 3);
  }
  const int lo = b % d.nlo;
  const int hi = b / d.nlo;
  const int64_t base = (int64_t)lo * d.w + (int64_t)hi * d.shi;
  const Tin* src = in + (int64_t)blockIdx.y * d.col_in + base;
  Tout* dst = out + (int64_t)blockIdx.y * d.col_out + base;

  for (int e = threadIdx.x; e < d.E; e += blockDim.x) {
    const int c = Ix<P>::mod(e, d.wdig, d.w);
    const int i = Ix<P>::div(e, d.wdig, d.w);
    lds[pad(e)] = cvt_in<Tin, T>(src[c + (int64_t)i * d.sd0]);
  }
  __syncthreads();
  for (int q = 0; q < d.r; q += d.kreg) {
    const int kk = min(d.kreg, d.r - q);
    if constexpr (KMAX >= 4) {
      if (kk == 4) run_group<P, INV, T, 4>(lds, d, q);
    }
    if constexpr (KMAX >= 3) {
      if (kk == 3) run_group<P, INV, T, 3>(lds, d, q);
    }
    if constexpr (KMAX >= 2) {
      if (kk == 2) run_group<P, INV, T, 2>(lds, d, q);
    }
    if (kk == 1) run_group<P, INV, T, 1>(lds, d, q);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < d.E; e += blockDim.x) {
    const int c = Ix<P>::mod(e, d.wdig, d.w);
    const int i = Ix<P>::div(e, d.wdig, d.w);
    dst[c + (int64_t)i * d.sd0] = cvt_out<T, Tout>(lds[pad(e)], d.scale);
  }
}

// ----------------------------------------------------------------- planner
struct PassGeom {
  int d0, r, wdig;
};

static constexpr size_t kLdsBudget = 80 * 1024;  // two workgroups per CU

static int kreg_for(int p, Kind work) {
  if (p == 2) return 4;
  if (p == 3) return 2;
  return work == K_CF32 ? 2 : 1;
}

static std::vector<PassGeom> plan(int p, int m, size_t bytes) {
  // Largest tile exponent e with the padded tile within the LDS budget.
  int emax = 0;
  for (int e = 1; e <= 30; ++e) {
    int64_t E = ipow(p, e);
    if ((size_t)(E + E / 32 + 1) * bytes > kLdsBudget) break;
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

template <class F>
static int set_lds_attr(F* fn, size_t bytes) {
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  std::lock_guard<std::mutex> g(mu);
  if (bytes <= 65536 || done.count((const void*)fn)) return FDWT_OK;
  FDWT_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done.insert((const void*)fn);
  return FDWT_OK;
}

template <int P, bool INV, class Tin, class T, class Tout>
static int launch_pass(const void* in, void* out, const PassGeom& g, int m, int batch, float scale,
                       int64_t col_in, int64_t col_out, Kind work, hipStream_t st) {
  constexpr int KMAX = (P == 2) ? 4 : ((P == 3 || sizeof(T) <= 8) ? 2 : 1);
  PassDesc d;
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
  d.scale = scale;
  const int64_t ntiles = ipow(P, m) / d.E;
  d.xcd = (ntiles % 8 == 0 && ntiles >= 64) ? 1 : 0;
  const int R = (int)ipow(P, d.kreg);
  int threads = std::max(64, std::min(1024, (d.E + R - 1) / R));
  threads = (threads + 63) / 64 * 64;
  const size_t lds = (size_t)(d.E + d.E / 32 + 1) * sizeof(T);
  auto fn = fwt_pass<P, INV, Tin, T, Tout, KMAX>;
  int rc = set_lds_attr(fn, lds);
  if (rc) return rc;
  hipLaunchKernelGGL(fn, dim3((unsigned)ntiles, (unsigned)batch), dim3(threads), lds, st,
                     (const Tin*)in, (Tout*)out, d);
  FDWT_HIP(hipGetLastError());
  return FDWT_OK;
}

// Dispatch on (p, direction, in/work/out kinds).
template <int P, bool INV>
static int pass_dispatch(Kind ik, Kind wk, Kind ok, const void* in, void* out, const PassGeom& g,
                         int m, int batch, float scale, int64_t ci, int64_t co, hipStream_t st) {
#define FDWT_PASS(TIN, T, TOUT) \
  return launch_pass<P, INV, TIN, T, TOUT>(in, out, g, m, batch, scale, ci, co, wk, st)
  if constexpr (P == 2) {
    if (wk == K_F32 && ik == K_F32 && ok == K_F32) FDWT_PASS(float, float, float);
    if (wk == K_U32 && ik == K_U32 && ok == K_U32) FDWT_PASS(uint32_t, uint32_t, uint32_t);
    if (wk == K_DF && ik == K_DF && ok == K_DF) FDWT_PASS(df, df, df);
  } else {
    if (wk == K_CF32) {
      if (ik == K_F32 && ok == K_CF32) FDWT_PASS(float, float2, float2);
      if (ik == K_F32 && ok == K_F32) FDWT_PASS(float, float2, float);
      if (ik == K_CF32 && ok == K_CF32) FDWT_PASS(float2, float2, float2);
      if (ik == K_CF32 && ok == K_F32) FDWT_PASS(float2, float2, float);
    }
    if (wk == K_CDF) {
      if (ik == K_DF && ok == K_CDF) FDWT_PASS(df, cdf, cdf);
      if (ik == K_DF && ok == K_DF) FDWT_PASS(df, cdf, df);
      if (ik == K_CDF && ok == K_CDF) FDWT_PASS(cdf, cdf, cdf);
      if (ik == K_CDF && ok == K_DF) FDWT_PASS(cdf, cdf, df);
    }
  }
#undef FDWT_PASS
  return fail(FDWT_EINVAL, "unsupported transform element types");
}

static int pass_any(int p, bool inv, Kind ik, Kind wk, Kind ok, const void* in, void* out,
                    const PassGeom& g, int m, int batch, float scale, int64_t ci, int64_t co,
                    hipStream_t st) {
  switch (p) {
    case 2:
      return inv ? pass_dispatch<2, true>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, st)
                 : pass_dispatch<2, false>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, st);
    case 3:
      return inv ? pass_dispatch<3, true>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, st)
                 : pass_dispatch<3, false>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, st);
    case 5:
      return inv ? pass_dispatch<5, true>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, st)
                 : pass_dispatch<5, false>(ik, wk, ok, in, out, g, m, batch, scale, ci, co, st);
  }
  return fail(FDWT_EUNSUPPORTED, "p must be 2, 3 or 5");
}

int fwt_run_tmp(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
                Kind out_kind, void* out, void* tmp, int batch, float scale, hipStream_t st) {
  const int64_t N = ipow(p, m);
  std::vector<PassGeom> passes = plan(p, m, kind_bytes(work_kind));
  const size_t np = passes.size();
  if (np == 1)
    return pass_any(p, inverse, in_kind, work_kind, out_kind, in, out, passes[0], m, batch, scale,
                    N, N, st);
  // Intermediate buffer: the output itself when it holds the working type.
  void* mid = (kind_bytes(out_kind) == kind_bytes(work_kind)) ? out : tmp;
  if (!mid) return fail(FDWT_EINVAL, "transform needs a workspace for a narrowing output");
  int rc = pass_any(p, inverse, in_kind, work_kind, work_kind, in, mid, passes[0], m, batch, 1.0f,
                    N, N, st);
  if (rc) return rc;
  for (size_t i = 1; i + 1 < np; ++i) {
    rc = pass_any(p, inverse, work_kind, work_kind, work_kind, mid, mid, passes[i], m, batch, 1.0f,
                  N, N, st);
    if (rc) return rc;
  }
  return pass_any(p, inverse, work_kind, work_kind, out_kind, mid, out, passes[np - 1], m, batch,
                  scale, N, N, st);
}

int fwt_run(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
            Kind out_kind, void* out, int batch, float scale, hipStream_t st) {
  return fwt_run_tmp(p, m, inverse, in_kind, in, work_kind, out_kind, out, nullptr, batch, scale,
                     st);
}

}  // namespace fdwt
