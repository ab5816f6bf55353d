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

// --------------------------------------------------------------- scratch
// Device workspace and pinned host staging used by one chain of calls.
// Owned mode (fixed = false): grow-only, reused call after call; a staging
// upload waits until the previous one has left `pin`.  Lent mode (fixed =
// true, the server's jobs): both areas are carved out by the caller at their
// final size; a request beyond them fails with FDWT_EBUDGET, and staging is
// handed out in consecutive slices (pin_used) that are never reused while the
// chain runs, so nothing waits on the host.
struct Scratch {
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool fixed = false;
  void* pin = nullptr;
  size_t pin_bytes = 0;
  size_t pin_used = 0;
  hipEvent_t pin_done = nullptr;  // owned mode: last copy through `pin` finished
};

// ------------------------------------------------------------------- net
struct Net {
  int p = 0, m = 0, s = 0;
  int64_t N = 0;
  int device = 0;
  int nbytes = 0;           // p = 2: bytes of n used by the XOR tables
  std::vector<uint8_t> C;   // the generators, [s][m][m] as given
  // p = 2: uint32 [s][nbytes][256], XOR of generator columns per byte of n.
  uint32_t* d_xtab = nullptr;
  // p odd: uint64 [s][m][p]: packed digits (4-bit fields, digit y_{r+1} at
  // bits 4(m-1-r)) of v * column c of C_j mod p.
  uint64_t* d_ptab = nullptr;
  // Workspace and staging of the handle's own calls (grow-only).
  Scratch sc;
  // Cached kernel spectrum (Section 3.2's K~, unnormalised float64) of the
  // kernel whose (alpha, gamma) bytes are spec_key; spec_ready is recorded on
  // the stream that computed it.
  void* spec = nullptr;
  size_t spec_bytes = 0;
  std::vector<double> spec_key;
  hipEvent_t spec_ready = nullptr;
};

}  // namespace fdwt

struct fdwt_net {
  fdwt::Net n;
};

namespace fdwt {

int64_t ipow(int64_t b, int e);

// Makes a device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Launch timing (see fdwt_timing_enable).  timed_begin returns an event (or
// nullptr when timing is off) recorded on st; timed_end records the closing
// event and files the launch under class cls with its algorithmic work.
hipEvent_t timed_begin(hipStream_t st);
void timed_end(hipEvent_t begin, hipStream_t st, int cls, double work);
// Launches one kernel (hipLaunchKernel arguments); while timing is on, with
// start and stop events attached to the dispatch itself (hipExtLaunchKernel),
// so the recorded duration is the kernel's alone, filed under cls.
int launch_timed(const void* fn, dim3 grid, dim3 block, void** args, size_t lds, hipStream_t st, int cls,
                 double work);
// Allows a kernel more than the default 64 KiB of dynamic LDS (once per kernel).
int allow_lds(const void* fn, size_t bytes);
int ensure_ws(Scratch& sc, size_t bytes, hipStream_t st);
// Host staging of `bytes` for one copy on st: *host receives the slice; call
// pin_release after enqueuing the copy.
int pin_take(Scratch& sc, size_t bytes, void** host);
int pin_release(Scratch& sc, hipStream_t st);
// Enqueues a host-to-device copy of `bytes` from src through the staging.
int upload(Scratch& sc, const void* src, size_t bytes, void* dst, hipStream_t st);
void scratch_release(Scratch& sc);  // owned mode: frees both areas
inline size_t align_ws(size_t b) { return (b + 255) & ~(size_t)255; }  // workspace slice alignment

// --------------------------------------------------------- kernel launchers
// net.hip
int launch_net_digits(const Net& net, uint32_t* X, hipStream_t st);
int launch_net_points(const Net& net, float* x, hipStream_t st);
int launch_net_packed(const Net& net, void* out, hipStream_t st);  // p=2: uint32 X<<(32-m); p odd: uint64 packed
int launch_sample(const Net& net, int family, const double* a, float* f, hipStream_t st);

// fwt.hip: element kinds
enum Kind { K_F32 = 0, K_U32 = 1, K_CF32 = 2, K_F64 = 3, K_CF64 = 4 };
size_t kind_bytes(Kind k);
// Transform with an explicit intermediate buffer `tmp` (needed when the
// output is narrower than the working type: N elements of work_kind).
int fwt_run_tmp(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
                Kind out_kind, void* out, void* tmp, int batch, double scale, hipStream_t st);
// api.cpp: the element kinds of fdwt_dwt_forward / fdwt_dwt_inverse for the
// ABI types (validated: FDWT_EINVAL otherwise), and the bytes of the
// intermediate buffer that transform needs (0 when the output holds it).
int transform_kinds(const Net& net, bool inverse, int in_type, const void* in, int out_type, const void* out,
                    Kind* ik, Kind* wk, Kind* ok);
size_t transform_tmp_bytes(const Net& net, Kind wk, Kind ok);
// Transform `batch` columns of N elements (column stride = N elements of the
// respective type).  in_kind may differ from the working kind only as
// F32 -> CF32 and F64 -> CF64 (p odd, real input).  out_kind may differ only
// as CF32 -> F32 and CF64 -> F64 (real part).
// scale multiplies float-based outputs of the last pass (1 = none).
int fwt_run(int p, int m, bool inverse, Kind in_kind, const void* in, Kind work_kind,
            Kind out_kind, void* out, int batch, double scale, hipStream_t st);

// spline.hip.  Every step takes an explicit Scratch; *_ws_bytes return the
// workspace a step needs (the step lays it out the same way), so a caller
// can lend exactly that much.
size_t kernel_tables_bytes(const Net& net);  // staged kernel tables (K' and R' per coordinate)
size_t spectrum_bytes(const Net& net);     // kernel spectrum: N doubles (p = 2), N complex doubles
size_t spectrum_ws_bytes(const Net& net);
int run_spectrum(Net& net, Scratch& sc, const fdwt_kernel* kern, void* gk, hipStream_t st);
// The net's cached spectrum for kern, computed on st if absent or for another
// kernel; st waits for it.  *gk receives the device pointer.
int cached_spectrum(Net& net, const fdwt_kernel* kern, const void** gk, hipStream_t st);
void drop_spectrum(Net& net);     // forget the cached spectrum (memory kept)
void release_spectrum(Net& net);  // free it
size_t spline_coef_ws_bytes(const Net& net, bool have_spectrum);
int run_spline_coef(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* gk, const void* ft, float* c,
                    hipStream_t st);
size_t packed_bytes(const Net& net);       // packed coordinates of all points (launch_net_packed)
size_t eval_tables_bytes(const Net& net);  // staged per-lane factor tables of the evaluation
size_t spline_eval_ws_bytes(const Net& net, int64_t nq, bool have_packed);
int run_spline_eval(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* packed, const float* c,
                    int64_t nq, const uint32_t* q, float* sf, hipStream_t st);
int eff_dim_chunk(const Net& net, size_t budget);
size_t eff_dim_res_bytes(const Net& net);
size_t eff_dim_ws_bytes(const Net& net, bool have_spectrum, int chunk);
int eff_dim_enqueue(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* gk, const void* ft, int chunk,
                    double* res_host, const double** res_dev, hipStream_t st);
void eff_dim_finish(int s, const double* res, fdwt_effdim* out);
int run_eff_dim(Net& net, Scratch& sc, const fdwt_kernel* kern, const void* ft, fdwt_effdim* out, hipStream_t st);

// Section 5.1 (p = 2): Sf on the second half of a 2^(m+1)-point net from the
// spline fitted on the first half (the m-digit net `tr`), as the inverse
// transform of f~ G / K_u, and the cost sum (f - Sf)^2.  delta: the second
// half's shift x_N, per coordinate as an (m+1)-digit integer (host array).
// ft: forward transform of the first half's values; fval: second half's
// values; sf_out (nullable) receives Sf there.  Synchronises st.
int run_split_cost(Net& tr, Scratch& sc, const uint32_t* delta, const float* ft, const float* fval,
                   const fdwt_kernel* kern, float* sf_out, double* cost, hipStream_t st);

// tune.cpp (Section 5.1): cost of (alpha, beta, q) = prm, and the
// Nelder-Mead selection from `start`, for a p = 2 net of m + 1 digits.
int split_cost_call(const Net& n2, const float* f2, const double prm[3], float* sf, double* cost, hipStream_t st);
int kernel_tune_call(const Net& n2, const float* f2, const double start[3], int max_evals, fdwt_kernel_fit* out,
                     hipStream_t st);

// Host tables of the kernel closed forms in double, for coordinates j and
// first-differing-digit index i (0 = no differing digit).
double kprime(int p, double alpha, int i);
double rprime(int p, double alpha, int i);
int query_depth(int p);
// Queries of q_depth digits lifted to the full depth (spline.hip).
int lift_queries(const Net& net, const uint32_t* q, int64_t nq, int q_depth, uint32_t* out, hipStream_t st);

}  // namespace fdwt
