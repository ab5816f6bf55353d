// Device arithmetic for the transform element types -- float, uint32 (mod
// 2^32), complex float (float2), double and complex double (double2) -- the
// radix-p DFT codelets the butterfly stages apply, and a double-float pair
// (df) used for compensated partial sums.
#pragma once

#include "fdwt_internal.h"

namespace fdwt {

// Workgroup barrier that orders LDS only.  __syncthreads() fences every
// address space, which makes each wave wait for all of its outstanding global
// loads and stores at the barrier; the transform passes only exchange data
// through LDS, so their barriers wait for LDS traffic alone and global
// prefetches stay in flight across them.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------- double-float
// Error-free transformations (Knuth's TwoSum, Dekker's FastTwoSum).
// Contraction is switched off so the compiler keeps every rounding step.
__device__ __forceinline__ df two_sum(float a, float b) {
#pragma clang fp contract(off)
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ df fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}
__device__ __forceinline__ df add(df a, df b) {
#pragma clang fp contract(off)
  df s = two_sum(a.hi, b.hi);
  df t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ double to_double(df a) { return (double)a.hi + (double)a.lo; }

// ----------------------------------------------------------- plain types
__host__ __device__ __forceinline__ float add(float a, float b) { return a + b; }
__host__ __device__ __forceinline__ float sub(float a, float b) { return a - b; }
__host__ __device__ __forceinline__ uint32_t add(uint32_t a, uint32_t b) { return a + b; }
__host__ __device__ __forceinline__ uint32_t sub(uint32_t a, uint32_t b) { return a - b; }

__host__ __device__ __forceinline__ float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 scale(float2 a, float c) { return make_float2(a.x * c, a.y * c); }
__host__ __device__ __forceinline__ float2 half(float2 a) { return make_float2(0.5f * a.x, 0.5f * a.y); }
// a + i*sg*b for sg = +1 or -1 (multiplication by +-i folded in).
__host__ __device__ __forceinline__ float2 add_i(float2 a, float2 b, int sg) {
  return sg > 0 ? make_float2(a.x - b.y, a.y + b.x) : make_float2(a.x + b.y, a.y - b.x);
}

__host__ __device__ __forceinline__ double add(double a, double b) { return a + b; }
__host__ __device__ __forceinline__ double sub(double a, double b) { return a - b; }
__host__ __device__ __forceinline__ double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 scale(double2 a, double c) { return make_double2(a.x * c, a.y * c); }
__host__ __device__ __forceinline__ double2 half(double2 a) { return make_double2(0.5 * a.x, 0.5 * a.y); }
__host__ __device__ __forceinline__ double2 add_i(double2 a, double2 b, int sg) {
  return sg > 0 ? make_double2(a.x - b.y, a.y + b.x) : make_double2(a.x + b.y, a.y - b.x);
}

// ---------------------------------------------------- codelet constants
// Real constants of the p-point DFT (values of sin and cos at multiples of
// 2 pi / p), converted to the element's real type.
constexpr double kSin60 = 0.86602540378443864676;   // sin(2 pi / 3)
constexpr double kCos72 = 0.30901699437494742410;   // cos(2 pi / 5)
constexpr double kSin72 = 0.95105651629515357212;   // sin(2 pi / 5)
constexpr double kCos144 = -0.80901699437494742410; // cos(4 pi / 5)
constexpr double kSin144 = 0.58778525229247312917;  // sin(4 pi / 5)

template <class C>
struct RealOf;
template <>
struct RealOf<float2> {
  using T = float;
};
template <>
struct RealOf<double2> {
  using T = double;
};
#define FDWT_K(C, v) ((typename RealOf<C>::T)(v))

// p-point DFT of x[0], x[st], ..., x[(p-1) st] in place:
//   y_h = sum_n x_n w^(n h),  w = exp(-2 pi i / p) (forward) or exp(+2 pi i / p)
// (inverse).  For p = 2 any ring element type works.
template <int P, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  template <class T>
  static __host__ __device__ __forceinline__ void run(T* x, int st) {
    T a = x[0], b = x[st];
    x[0] = add(a, b);
    x[st] = sub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  // y0 = x0 + t, y1,2 = (x0 - t/2) -+ i sin60 (x1 - x2) (forward signs).
  template <class C>
  static __host__ __device__ __forceinline__ void run(C* x, int st) {
    C x0 = x[0], x1 = x[st], x2 = x[2 * st];
    C t = add(x1, x2);
    C d = sub(x1, x2);
    C a = sub(x0, half(t));
    C b = scale(d, FDWT_K(C, kSin60));
    const int sg = INV ? 1 : -1;
    x[0] = add(x0, t);
    x[st] = add_i(a, b, sg);
    x[2 * st] = add_i(a, b, -sg);
  }
};

template <bool INV>
struct Dft<5, INV> {
  // With t1 = x1 + x4, t2 = x2 + x3, d1 = x1 - x4, d2 = x2 - x3:
  //   a1 = x0 + c72 t1 + c144 t2, a2 = x0 + c144 t1 + c72 t2,
  //   b1 = s72 d1 + s144 d2,       b2 = s144 d1 - s72 d2,
  //   y1 = a1 -+ i b1, y4 = a1 +- i b1, y2 = a2 -+ i b2, y3 = a2 +- i b2.
  template <class C>
  static __host__ __device__ __forceinline__ void run(C* x, int st) {
    C x0 = x[0], x1 = x[st], x2 = x[2 * st], x3 = x[3 * st], x4 = x[4 * st];
    C t1 = add(x1, x4), t2 = add(x2, x3);
    C d1 = sub(x1, x4), d2 = sub(x2, x3);
    const auto c1 = FDWT_K(C, kCos72), c2 = FDWT_K(C, kCos144);
    const auto s1 = FDWT_K(C, kSin72), s2 = FDWT_K(C, kSin144);
    C a1 = add(x0, add(scale(t1, c1), scale(t2, c2)));
    C a2 = add(x0, add(scale(t1, c2), scale(t2, c1)));
    C b1 = add(scale(d1, s1), scale(d2, s2));
    C b2 = sub(scale(d1, s2), scale(d2, s1));
    const int sg = INV ? 1 : -1;
    x[0] = add(x0, add(t1, t2));
    x[st] = add_i(a1, b1, sg);
    x[4 * st] = add_i(a1, b1, -sg);
    x[2 * st] = add_i(a2, b2, sg);
    x[3 * st] = add_i(a2, b2, -sg);
  }
};

// Complex product.
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// 6-point DFT (exp(-2 pi i a k / 6), or exp(+...) when INV6) by the
// Good-Thomas map a = 3 a1 + 2 a2, k = 3 k1 + 4 k2 (mod 6): 3-point DFTs over
// a2, then 2-point DFTs over a1, no twiddle factors.
template <bool INV6, class C>
__host__ __device__ __forceinline__ void dft6(const C (&in)[6], C (&out)[6]) {
  C c0[3] = {in[0], in[2], in[4]};  // a1 = 0
  C c1[3] = {in[3], in[5], in[1]};  // a1 = 1
  Dft<3, INV6>::run(c0, 1);
  Dft<3, INV6>::run(c1, 1);
  out[0] = add(c0[0], c1[0]);
  out[3] = sub(c0[0], c1[0]);
  out[4] = add(c0[1], c1[1]);
  out[1] = sub(c0[1], c1[1]);
  out[2] = add(c0[2], c1[2]);
  out[5] = sub(c0[2], c1[2]);
}

// DFT6 of v_c = w^(3^-c mod 7), c = 0..5, divided by 6 (w = exp(-2 pi i / 7)
// forward, exp(+2 pi i / 7) inverse): the kernel of the Rader convolution.
// V_0 = -1/6 (the six non-trivial 7th roots sum to -1); V_3 is imaginary.
constexpr double kRader7Fwd[6][2] = {{-1.0 / 6.0, 0.0},
                                     {0.4066888930575896, -0.17043646531196566},
                                     {0.3950782342627002, -0.1958510486474644},
                                     {0.0, -0.4409585518440986},
                                     {0.39507823426270006, 0.1958510486474646},
                                     {-0.4066888930575896, -0.17043646531196588}};
constexpr double kRader7Inv[6][2] = {{-1.0 / 6.0, 0.0},
                                     {-0.4066888930575896, 0.1704364653119659},
                                     {0.39507823426270006, -0.1958510486474646},
                                     {0.0, 0.4409585518440985},
                                     {0.3950782342627002, 0.1958510486474644},
                                     {0.40668889305758965, 0.17043646531196566}};

template <bool INV>
struct Dft<7, INV> {
  // Rader's algorithm (the remark after Algorithm 1): with the primitive
  // root 3, n = 3^a and h = 3^-b (mod 7) turn y_h - x_0 (h != 0) into the
  // length-6 cyclic convolution z_b = sum_a u_a v_(b-a) of u_a = x_(3^a) with
  // v_c = w^(3^-c); it runs as DFT6, a product with DFT6(v)/6, and an inverse
  // DFT6.  3^a mod 7 = 1, 3, 2, 6, 4, 5; 3^-b mod 7 = 1, 5, 4, 6, 2, 3.
  template <class C>
  static __host__ __device__ __forceinline__ void run(C* x, int st) {
    using R = typename RealOf<C>::T;
    const C x0 = x[0];
    const C u[6] = {x[st], x[3 * st], x[2 * st], x[6 * st], x[4 * st], x[5 * st]};
    C U[6];
    dft6<false>(u, U);
    const C y0 = add(x0, U[0]);  // U_0 = sum of u
    C Z[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      C v;
      v.x = (R)(INV ? kRader7Inv[k][0] : kRader7Fwd[k][0]);
      v.y = (R)(INV ? kRader7Inv[k][1] : kRader7Fwd[k][1]);
      Z[k] = cmul(U[k], v);
    }
    C z[6];
    dft6<true>(Z, z);
    x[0] = y0;
    x[st] = add(x0, z[0]);
    x[5 * st] = add(x0, z[1]);
    x[4 * st] = add(x0, z[2]);
    x[6 * st] = add(x0, z[3]);
    x[2 * st] = add(x0, z[4]);
    x[3 * st] = add(x0, z[5]);
  }
};

}  // namespace fdwt
