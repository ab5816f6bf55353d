// Internal declarations of libfdwt (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fdwt.h"

namespace fdwt {

// ------------------------------------------------------------------ errors
struct Error {
  int code;
  std::string msg;
};
void set_error(int code, const std::string& msg);
int fail(int code, const std::string& msg);  // sets and returns code
#define FDWT_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::fdwt::fail(FDWT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxS = 64;
constexpr int kMaxLog2N = 26;

// ------------------------------------------------------------ value types
// Double-float: value = hi + lo with |lo| <= ulp(hi)/2 (about 48 bits).
struct df {
  float hi, lo;
};

// ------------------------------------------------------------------- net
struct Net {
  int p = 0, m = 0, s = 0;
  int64_t N = 0;
  int device = 0;
  int nbytes = 0;           // p = 2: bytes of n used by the XOR tables
  // p = 2: uint32 [s][nbytes][256], XOR of generator columns per byte of n.
  uint32_t* d_xtab = nullptr;
  // p odd: uint64 [s][m][p]: packed digits (4-bit fields, digit y_{r+1} at
  // bits 4(m-1-r)) of v * column c of C_j mod p.
  uint64_t* d_ptab = nullptr;
  // Grow-only workspace owned by the handle.
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // Pinned host staging for small per-call tables and results.
  void* pin = nullptr;
  size_t pin_bytes = 0;
  hipEvent_t pin_done = nullptr;  // last copy out of/into `pin` finished
};

}  // namespace fdwt

struct fdwt_net {
  fdwt::Net n;
};

namespace fdwt {

int64_t ipow(int64_t b, int e);

// Launch timing (see fdwt_timing_enable).  timed_begin returns an event (or
// nullptr when timing is off) recorded on st; timed_end records the closing
// event and files the launch under class cls with its algorithmic work.
hipEvent_t timed_begin(hipStream_t st);
void timed_end(hipEvent_t begin, hipStream_t st, int cls, double work);
// Allows a kernel more than the default 64 KiB of dynamic LDS (once per kernel).
int allow_lds(const void* fn, size_t bytes);
int ensure_ws(Net& net, size_t bytes, hipStream_t st);
int ensure_pin(Net& net, size_t bytes);
int pin_acquire(Net& net);          // waits until `pin` is free again
int pin_release(Net& net, hipStream_t st);

// --------------------------------------------------------- kernel launchers
// net.hip
int launch_net_digits(const Net& net, uint32_t* X, hipStream_t st);
int launch_net_points(const Net& net, float* x, hipStream_t st);
int launch_net_packed(const Net& net, void* out, hipStream_t st);  // p=2: uint32 X<<(32-m); p odd: uint64 packed
int launch_sample(const Net& net, int family, const double* a, float* f, hipStream_t st);

// fwt.hip: element kinds
enum Kind { K_F32 = 0, K_U32 = 1, K_CF32 = 2, K_F64 = 3, K_CF64 = 4 };
size_t kind_bytes(Kind k);
// Transform `batch` columns of N elements (column stride = N elements of the
// respective type).  in_kind may differ from the working kind only as
// F32 -> CF32 and F64 -> CF64 (p odd, real input).  out_kind may differ only
// as CF32 -> F32 and CF64 -> F64 (real part).
// scale multiplies float-based outputs of the last pass (1 = none).
int fwt_run(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
            Kind out_kind, void* out, int batch, double scale, hipStream_t st);

// spline.hip / effdim.hip
int run_spline_coef(Net& net, const fdwt_kernel* kern, int ft_type, const void* ft, float* c,
                    hipStream_t st);
int run_spline_eval(Net& net, const fdwt_kernel* kern, const float* c, int64_t nq,
                    const uint32_t* q, float* sf, hipStream_t st);
int run_eff_dim(Net& net, const fdwt_kernel* kern, int ft_type, const void* ft, fdwt_effdim* out,
                hipStream_t st);

// Host tables of the kernel closed forms in double, for coordinates j and
// first-differing-digit index i (0 = no differing digit).
double kprime(int p, double alpha, int i);
double rprime(int p, double alpha, int i);
int query_depth(int p);

}  // namespace fdwt
