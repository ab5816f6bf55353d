// C ABI of libfdwt: argument validation, net handles, workspace ownership and
// dispatch to the HIP kernels.  Every entry point returns a status code and
// never lets an exception escape.
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <unordered_set>

#include <hip/hip_ext.h>

#include "family.h"
#include "fdwt_internal.h"

namespace fdwt {

static thread_local std::string g_err;

void set_error(int code, const std::string& msg) {
  (void)code;
  g_err = msg;
}
int fail(int code, const std::string& msg) {
  set_error(code, msg);
  return code;
}

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

int allow_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  if (bytes <= 65536) return FDWT_OK;
  std::lock_guard<std::mutex> g(mu);
  if (done.count(fn)) return FDWT_OK;
  FDWT_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done.insert(fn);
  return FDWT_OK;
}

// ------------------------------------------------------------ timing
namespace {
struct TimedRec {
  hipEvent_t a, b;
  int cls;
  double work;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedRec> g_recs;

void drop_records() {
  for (auto& r : g_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
}
}  // namespace

hipEvent_t timed_begin(hipStream_t st) {
  {
    std::lock_guard<std::mutex> g(g_tmu);
    if (!g_timing) return nullptr;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  if (hipEventRecord(e, st) != hipSuccess) {
    (void)hipEventDestroy(e);
    return nullptr;
  }
  return e;
}

void timed_end(hipEvent_t begin, hipStream_t st, int cls, double work) {
  if (!begin) return;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, st) != hipSuccess) {
    (void)hipEventDestroy(begin);
    if (e) (void)hipEventDestroy(e);
    return;
  }
  std::lock_guard<std::mutex> g(g_tmu);
  g_recs.push_back({begin, e, cls, work});
}

int launch_timed(const void* fn, dim3 grid, dim3 block, void** args, size_t lds, hipStream_t st, int cls,
                 double work) {
  bool on;
  {
    std::lock_guard<std::mutex> g(g_tmu);
    on = g_timing;
  }
  hipEvent_t a = nullptr, b = nullptr;
  if (on && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)) {
    (void)hipGetLastError();
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    a = b = nullptr;
    on = false;
  }
  if (!on) {
    FDWT_HIP(hipLaunchKernel(fn, grid, block, args, lds, st));
    return FDWT_OK;
  }
  const hipError_t e = hipExtLaunchKernel(fn, grid, block, args, lds, st, a, b, 0);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return fail(FDWT_EDEVICE, std::string("hipExtLaunchKernel: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> g(g_tmu);
  g_recs.push_back({a, b, cls, work});
  return FDWT_OK;
}

int query_depth(int p) { return p == 2 ? 32 : (p == 3 ? 20 : (p == 5 ? 13 : (p == 7 ? 11 : 0))); }

// K'(z,0) and R'(z,0) of Section 4 for z whose first non-zero base-p digit is
// digit i (i = 0: z = 0).
double kprime(int p, double alpha, int i) {
  if (i == 0) return 1.0;
  return 1.0 - std::pow((double)p, i * (1.0 - alpha)) * (std::pow((double)p, alpha) - 1.0) / (p - 1.0);
}
double rprime(int p, double alpha, int i) {
  const double pa = std::pow((double)p, alpha), p2a = std::pow((double)p, 2.0 * alpha);
  const double A = (pa - p) * (pa - p) / ((p - 1.0) * (p2a - p));
  if (i == 0) return A;
  return A * (1.0 - std::pow((double)p, i * (1.0 - 2.0 * alpha)) * (p2a - 1.0) / (p - 1.0));
}

int ensure_ws(Scratch& sc, size_t bytes, hipStream_t st) {
  if (sc.ws_bytes >= bytes) return FDWT_OK;
  if (sc.fixed)
    return fail(FDWT_EBUDGET, "workspace of " + std::to_string(bytes) + " bytes exceeds the lent " +
                                  std::to_string(sc.ws_bytes));
  if (sc.ws) {
    FDWT_HIP(hipStreamSynchronize(st));
    FDWT_HIP(hipFree(sc.ws));
    sc.ws = nullptr;
    sc.ws_bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FDWT_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  sc.ws = p;
  sc.ws_bytes = bytes;
  return FDWT_OK;
}

int pin_take(Scratch& sc, size_t bytes, void** host) {
  if (sc.fixed) {
    const size_t b = align_ws(bytes);
    if (sc.pin_used + b > sc.pin_bytes) return fail(FDWT_EBUDGET, "lent staging area exhausted");
    *host = (char*)sc.pin + sc.pin_used;
    sc.pin_used += b;
    return FDWT_OK;
  }
  if (sc.pin_done) FDWT_HIP(hipEventSynchronize(sc.pin_done));
  if (sc.pin_bytes < bytes) {
    if (sc.pin) FDWT_HIP(hipHostFree(sc.pin));
    sc.pin = nullptr;
    sc.pin_bytes = 0;
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FDWT_ENOMEM, "pinned staging allocation failed");
    }
    sc.pin = p;
    sc.pin_bytes = bytes;
  }
  *host = sc.pin;
  return FDWT_OK;
}

int pin_release(Scratch& sc, hipStream_t st) {
  if (sc.fixed) return FDWT_OK;
  if (!sc.pin_done) FDWT_HIP(hipEventCreateWithFlags(&sc.pin_done, hipEventDisableTiming));
  FDWT_HIP(hipEventRecord(sc.pin_done, st));
  return FDWT_OK;
}

int upload(Scratch& sc, const void* src, size_t bytes, void* dst, hipStream_t st) {
  void* h = nullptr;
  if (int rc = pin_take(sc, bytes, &h)) return rc;
  std::memcpy(h, src, bytes);
  FDWT_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, st));
  return pin_release(sc, st);
}

void scratch_release(Scratch& sc) {
  if (sc.fixed) return;
  if (sc.ws || sc.pin_done) (void)hipDeviceSynchronize();
  if (sc.ws) (void)hipFree(sc.ws);
  if (sc.pin) (void)hipHostFree(sc.pin);
  if (sc.pin_done) (void)hipEventDestroy(sc.pin_done);
  sc = Scratch{};
}

static bool is_prime(int p) {
  if (p < 2) return false;
  for (int d = 2; d * d <= p; ++d)
    if (p % d == 0) return false;
  return true;
}

static int check_net(const fdwt_net* h) {
  if (!h) return fail(FDWT_EINVAL, "net handle is NULL");
  return FDWT_OK;
}

static int check_kernel(const Net& net, const fdwt_kernel* k) {
  if (!k || !k->gamma) return fail(FDWT_EINVAL, "kernel or its gamma is NULL");
  if (k->s != net.s) return fail(FDWT_EINVAL, "kernel s differs from the net's s");
  if (!(k->alpha > 1.0) || !std::isfinite(k->alpha)) return fail(FDWT_EINVAL, "alpha must be > 1");
  for (int j = 0; j < k->s; ++j)
    if (!(k->gamma[j] > 0.0) || !std::isfinite(k->gamma[j]))
      return fail(FDWT_EINVAL, "gamma_j must be positive and finite");
  return FDWT_OK;
}

static int check_family(const Net& net, int family, const double* a) {
  if (family == FDWT_FAMILY_ASIAN) {
    for (int i = 0; i < 5; ++i)
      if (!std::isfinite(a[i])) return fail(FDWT_EINVAL, "family parameter out of range");
    if (!(a[0] > 0.0) || a[1] < 0.0 || !(a[2] > 0.0) || !(a[4] > 0.0))
      return fail(FDWT_EINVAL, "Asian parameters need S0 > 0, K >= 0, sigma > 0, T > 0");
    return FDWT_OK;
  }
  if (family != FDWT_FAMILY_PRODUCT && family != FDWT_FAMILY_EXP && family != FDWT_FAMILY_WANGFANG)
    return fail(FDWT_EINVAL, "unknown family");
  for (int j = 0; j < net.s; ++j)
    if (!std::isfinite(a[j]) || (family == FDWT_FAMILY_WANGFANG && a[j] <= -1.0))
      return fail(FDWT_EINVAL, "family parameter out of range");
  return FDWT_OK;
}

static Kind to_kind(int t) {
  switch (t) {
    case FDWT_F32: return K_F32;
    case FDWT_I32: return K_U32;
    case FDWT_CF32: return K_CF32;
    case FDWT_F64: return K_F64;
    case FDWT_CF64: return K_CF64;
  }
  return (Kind)-1;
}

int transform_kinds(const Net& net, bool inverse, int in_type, const void* in, int out_type, const void* out,
                    Kind* ik_out, Kind* wk_out, Kind* ok_out) {
  if (!in || !out) return fail(FDWT_EINVAL, "NULL data pointer");
  Kind ik = to_kind(in_type), ok = to_kind(out_type), wk;
  if ((int)ik < 0 || (int)ok < 0) return fail(FDWT_EINVAL, "unknown element type");
  if (net.p == 2) {
    if (!((ik == K_F32 && ok == K_F32) || (ik == K_U32 && ok == K_U32) || (ik == K_F64 && ok == K_F64)))
      return fail(FDWT_EINVAL, "p = 2 transforms are F32 -> F32, I32 -> I32 or F64 -> F64");
    wk = ik;
  } else {
    const bool dbl = (ik == K_F64 || ik == K_CF64);
    const Kind re = dbl ? K_F64 : K_F32, cx = dbl ? K_CF64 : K_CF32;
    const bool okf = inverse ? (ik == cx && (ok == cx || ok == re))
                             : ((ik == re || ik == cx) && ok == cx);
    if (!okf || ik == K_U32)
      return fail(FDWT_EINVAL, inverse ? "odd-p inverse takes CF32 to CF32 or F32 (CF64 to CF64 or F64)"
                                       : "odd-p forward takes F32 or CF32 to CF32 (F64 or CF64 to CF64)");
    wk = cx;
  }
  if (in == out && kind_bytes(ik) != kind_bytes(ok))
    return fail(FDWT_EINVAL, "in-place transform needs equal input and output element sizes");
  *ik_out = ik;
  *wk_out = wk;
  *ok_out = ok;
  return FDWT_OK;
}

size_t transform_tmp_bytes(const Net& net, Kind wk, Kind ok) {
  return kind_bytes(ok) < kind_bytes(wk) ? (size_t)net.N * kind_bytes(wk) : 0;
}

static int transform(Net& net, bool inverse, int in_type, const void* in, int out_type, void* out,
                     hipStream_t st) {
  Kind ik, wk, ok;
  if (int rc = transform_kinds(net, inverse, in_type, in, out_type, out, &ik, &wk, &ok)) return rc;
  void* tmp = nullptr;
  if (transform_tmp_bytes(net, wk, ok)) {
    int rc = ensure_ws(net.sc, (size_t)net.N * kind_bytes(wk), st);
    if (rc) return rc;
    tmp = net.sc.ws;
  }
  const double scale = (!inverse && wk != K_U32) ? 1.0 / (double)net.N : 1.0;  // Eq. (eq_dwalshcoeff)
  return fwt_run_tmp(net.p, net.m, inverse, ik, in, wk, ok, out, tmp, 1, scale, st);
}

}  // namespace fdwt

using namespace fdwt;

#define FDWT_GUARD_BEGIN try {
#define FDWT_GUARD_END                                                        \
  }                                                                           \
  catch (const std::bad_alloc&) {                                             \
    return fail(FDWT_ENOMEM, "host allocation failed");                       \
  }                                                                           \
  catch (const std::exception& e) {                                           \
    return fail(FDWT_EDEVICE, std::string("internal error: ") + e.what());    \
  }                                                                           \
  catch (...) {                                                               \
    return fail(FDWT_EDEVICE, "internal error");                              \
  }

extern "C" {

const char* fdwt_last_error(void) { return g_err.c_str(); }

int fdwt_timing_enable(int on) {
  std::lock_guard<std::mutex> g(g_tmu);
  drop_records();
  g_timing = on != 0;
  return FDWT_OK;
}

int fdwt_timing_query(int cls, double* total_ms, int64_t* launches, double* work) {
  if (cls < 0 || cls >= FDWT_TC_COUNT) return fail(FDWT_EINVAL, "unknown timing class");
  std::lock_guard<std::mutex> g(g_tmu);
  double ms = 0.0, w = 0.0;
  int64_t n = 0;
  for (auto& r : g_recs) {
    if (r.cls != cls) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(FDWT_EDEVICE, "event synchronisation failed");
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(FDWT_EDEVICE, "event timing failed");
    ms += t;
    w += r.work;
    ++n;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (work) *work = w;
  return FDWT_OK;
}

int fdwt_query_depth(int p) { return query_depth(p); }

int fdwt_net_generate(int p, int m, int s, const uint8_t* C_host, fdwt_net** out) {
  FDWT_GUARD_BEGIN
  g_err.clear();
  if (!out || !C_host) return fail(FDWT_EINVAL, "NULL argument");
  *out = nullptr;
  if (!is_prime(p)) return fail(FDWT_EINVAL, "p must be prime");
  if (p != 2 && p != 3 && p != 5 && p != 7) return fail(FDWT_EUNSUPPORTED, "only p = 2, 3, 5, 7 are supported");
  if (m < 1) return fail(FDWT_EINVAL, "m must be >= 1");
  if (s < 1 || s > kMaxS) return fail(FDWT_EINVAL, "s must be in 1..64");
  if (ipow(p, m) > (int64_t(1) << kMaxLog2N)) return fail(FDWT_EINVAL, "p^m must be <= 2^26");
  for (int64_t i = 0; i < (int64_t)s * m * m; ++i)
    if (C_host[i] >= p) return fail(FDWT_EINVAL, "generator entry >= p");
  auto* h = new fdwt_net();
  Net& net = h->n;
  net.p = p;
  net.m = m;
  net.s = s;
  net.N = ipow(p, m);
  if (hipGetDevice(&net.device) != hipSuccess) {
    delete h;
    return fail(FDWT_EDEVICE, "no HIP device");
  }
  net.C.assign(C_host, C_host + (size_t)s * m * m);
  auto C = [&](int j, int r, int c) { return (int)C_host[((int64_t)j * m + r) * m + c]; };
  if (p == 2) {
    // Column c of C_j as an m-bit integer (row r -> bit m-1-r); per byte b of n,
    // the XOR of the columns selected by each byte value.
    net.nbytes = (m + 7) / 8;
    std::vector<uint32_t> tab((size_t)s * net.nbytes * 256, 0);
    for (int j = 0; j < s; ++j) {
      uint32_t col[32] = {0};
      for (int c = 0; c < m; ++c)
        for (int r = 0; r < m; ++r)
          if (C(j, r, c) & 1) col[c] |= 1u << (m - 1 - r);
      for (int b = 0; b < net.nbytes; ++b)
        for (int v = 0; v < 256; ++v) {
          uint32_t x = 0;
          for (int t = 0; t < 8; ++t)
            if ((v >> t) & 1 && 8 * b + t < m) x ^= col[8 * b + t];
          tab[((size_t)j * net.nbytes + b) * 256 + v] = x;
        }
    }
    if (hipMalloc(&net.d_xtab, tab.size() * 4) != hipSuccess) {
      delete h;
      return fail(FDWT_ENOMEM, "table allocation failed");
    }
    if (hipMemcpy(net.d_xtab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(net.d_xtab);
      delete h;
      return fail(FDWT_EDEVICE, "table upload failed");
    }
  } else {
    // Packed digits of v * (column c of C_j) mod p, digit y_{r+1} at bits 4(m-1-r).
    std::vector<uint64_t> tab((size_t)s * m * p, 0);
    for (int j = 0; j < s; ++j)
      for (int c = 0; c < m; ++c)
        for (int v = 0; v < p; ++v) {
          uint64_t x = 0;
          for (int r = 0; r < m; ++r) x |= (uint64_t)((v * C(j, r, c)) % p) << (4 * (m - 1 - r));
          tab[((size_t)j * m + c) * p + v] = x;
        }
    if (hipMalloc(&net.d_ptab, tab.size() * 8) != hipSuccess) {
      delete h;
      return fail(FDWT_ENOMEM, "table allocation failed");
    }
    if (hipMemcpy(net.d_ptab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(net.d_ptab);
      delete h;
      return fail(FDWT_EDEVICE, "table upload failed");
    }
  }
  *out = h;
  return FDWT_OK;
  FDWT_GUARD_END
}

int fdwt_net_info(const fdwt_net* h, int* p, int* m, int* s, int64_t* n_points) {
  if (int rc = check_net(h)) return rc;
  if (p) *p = h->n.p;
  if (m) *m = h->n.m;
  if (s) *s = h->n.s;
  if (n_points) *n_points = h->n.N;
  return FDWT_OK;
}

void fdwt_net_free(fdwt_net* h) {
  if (!h) return;
  Net& n = h->n;
  DeviceGuard g(n.device);
  scratch_release(n.sc);
  release_spectrum(n);
  if (n.d_xtab || n.d_ptab) (void)hipDeviceSynchronize();
  if (n.d_xtab) (void)hipFree(n.d_xtab);
  if (n.d_ptab) (void)hipFree(n.d_ptab);
  delete h;
}

int fdwt_net_drop_spectrum(fdwt_net* h) {
  if (int rc = check_net(h)) return rc;
  drop_spectrum(h->n);
  return FDWT_OK;
}

int fdwt_net_digits(const fdwt_net* h, uint32_t* X_dev, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (!X_dev) return fail(FDWT_EINVAL, "NULL output");
  DeviceGuard g(h->n.device);
  return launch_net_digits(h->n, X_dev, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_net_points(const fdwt_net* h, float* x_dev, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (!x_dev) return fail(FDWT_EINVAL, "NULL output");
  DeviceGuard g(h->n.device);
  return launch_net_points(h->n, x_dev, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_sample(const fdwt_net* h, int family, const double* a_host, float* f_dev, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (!a_host || !f_dev) return fail(FDWT_EINVAL, "NULL argument");
  if (int rc = check_family(h->n, family, a_host)) return rc;
  DeviceGuard g(h->n.device);
  return launch_sample(h->n, family, a_host, f_dev, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_dwt_forward(const fdwt_net* h, int in_type, const void* in_dev, int out_type, void* out_dev,
                     void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  DeviceGuard g(h->n.device);
  return transform(const_cast<Net&>(h->n), false, in_type, in_dev, out_type, out_dev,
                   (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_dwt_forward_family(const fdwt_net* h, int family, const double* a_host, int out_type, void* out_dev,
                            void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (!a_host || !out_dev) return fail(FDWT_EINVAL, "NULL argument");
  if (int rc = check_family(h->n, family, a_host)) return rc;
  Net& net = const_cast<Net&>(h->n);
  if (out_type != (net.p == 2 ? FDWT_F32 : FDWT_CF32))
    return fail(FDWT_EINVAL, "coefficients are F32 (p = 2) or CF32 (p odd)");
  DeviceGuard g(net.device);
  hipStream_t st = (hipStream_t)stream;
  // p = 2 samples inside the first pass (m >= 10), or into the output and
  // transforms in place; p odd samples into the workspace (the complex
  // output is twice as wide).
  if (net.p == 2) {
    const int rc = fwt_p2_forward_family(net, family, make_family_args(net, family, a_host), (float*)out_dev, st);
    if (rc != FDWT_EUNSUPPORTED) return rc;
  }
  float* f = (float*)out_dev;
  if (net.p != 2) {
    if (int rc = ensure_ws(net.sc, (size_t)net.N * sizeof(float), st)) return rc;
    f = (float*)net.sc.ws;
  }
  if (int rc = launch_sample(net, family, a_host, f, st)) return rc;
  return transform(net, false, FDWT_F32, f, out_type, out_dev, st);
  FDWT_GUARD_END
}

int fdwt_dwt_inverse(const fdwt_net* h, int in_type, const void* in_dev, int out_type, void* out_dev,
                     void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  DeviceGuard g(h->n.device);
  return transform(const_cast<Net&>(h->n), true, in_type, in_dev, out_type, out_dev,
                   (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_spline_coef(const fdwt_net* h, const fdwt_kernel* kern, int ft_type, const void* ft_dev,
                     float* c_dev, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (int rc = check_kernel(h->n, kern)) return rc;
  if (!ft_dev || !c_dev) return fail(FDWT_EINVAL, "NULL data pointer");
  if (ft_type != (h->n.p == 2 ? FDWT_F32 : FDWT_CF32))
    return fail(FDWT_EINVAL, "coefficients must be F32 (p = 2) or CF32 (p odd)");
  DeviceGuard g(h->n.device);
  Net& net = const_cast<Net&>(h->n);
  const void* gk = nullptr;
  if (int rc = cached_spectrum(net, kern, &gk, (hipStream_t)stream)) return rc;
  return run_spline_coef(net, net.sc, kern, gk, ft_dev, c_dev, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_spline_eval(const fdwt_net* h, const fdwt_kernel* kern, const float* c_dev, int64_t nq,
                     const uint32_t* q_dev, float* sf_dev, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (int rc = check_kernel(h->n, kern)) return rc;
  if (nq < 0 || nq > (int64_t(1) << 28)) return fail(FDWT_EINVAL, "nq must be in 0..2^28");
  if (nq == 0) return FDWT_OK;
  if (!c_dev || !q_dev || !sf_dev) return fail(FDWT_EINVAL, "NULL data pointer");
  DeviceGuard g(h->n.device);
  Net& net = const_cast<Net&>(h->n);
  return run_spline_eval(net, net.sc, kern, nullptr, c_dev, nq, q_dev, sf_dev, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_walsh_interp_depth(const fdwt_net* h, const fdwt_kernel* kern, const float* f_dev, float* c_dev,
                            int64_t nq, const uint32_t* q_dev, int q_depth, float* sf_dev, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  const Net& net = h->n;
  const int D = query_depth(net.p);
  if (q_depth < 1 || q_depth > D) return fail(FDWT_EINVAL, "q_depth must be in 1.." + std::to_string(D));
  if (nq < 0 || nq > (int64_t(1) << 28)) return fail(FDWT_EINVAL, "nq must be in 0..2^28");
  if (q_depth == D || nq == 0) return fdwt_walsh_interp(h, kern, f_dev, c_dev, nq, q_dev, sf_dev, stream);
  if (!q_dev) return fail(FDWT_EINVAL, "NULL query pointer");
  DeviceGuard g(net.device);
  hipStream_t st = (hipStream_t)stream;
  uint32_t* ql = nullptr;
  if (hipMallocAsync((void**)&ql, (size_t)nq * net.s * sizeof(uint32_t), st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FDWT_ENOMEM, "query allocation failed");
  }
  int rc = lift_queries(net, q_dev, nq, q_depth, ql, st);
  if (!rc) rc = fdwt_walsh_interp(h, kern, f_dev, c_dev, nq, ql, sf_dev, stream);
  (void)hipFreeAsync(ql, st);
  return rc;
  FDWT_GUARD_END
}

int fdwt_walsh_interp(const fdwt_net* h, const fdwt_kernel* kern, const float* f_dev, float* c_dev,
                      int64_t nq, const uint32_t* q_dev, float* sf_dev, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (int rc = check_kernel(h->n, kern)) return rc;
  if (!f_dev) return fail(FDWT_EINVAL, "NULL data pointer");
  if (nq < 0 || nq > (int64_t(1) << 28)) return fail(FDWT_EINVAL, "nq must be in 0..2^28");
  if (nq > 0 && (!q_dev || !sf_dev)) return fail(FDWT_EINVAL, "NULL query or output pointer");
  Net& net = const_cast<Net&>(h->n);
  DeviceGuard g(net.device);
  hipStream_t st = (hipStream_t)stream;
  // ft and c live in the caller's c buffer when given, else in a scratch
  // allocation owned by this call.
  const size_t ftb = (size_t)net.N * (net.p == 2 ? 4 : 8);
  void* ft = nullptr;
  float* c = c_dev;
  if (hipMallocAsync(&ft, ftb + (c_dev ? 0 : (size_t)net.N * 4), st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FDWT_ENOMEM, "interpolation scratch allocation failed");
  }
  if (!c) c = (float*)((char*)ft + ftb);
  int rc = transform(net, false, FDWT_F32, f_dev, net.p == 2 ? FDWT_F32 : FDWT_CF32, ft, st);
  const void* gk = nullptr;
  if (!rc) rc = cached_spectrum(net, kern, &gk, st);
  if (!rc) rc = run_spline_coef(net, net.sc, kern, gk, ft, c, st);
  if (!rc && nq > 0) rc = run_spline_eval(net, net.sc, kern, nullptr, c, nq, q_dev, sf_dev, st);
  (void)hipFreeAsync(ft, st);
  return rc;
  FDWT_GUARD_END
}

int fdwt_split_cost(const fdwt_net* h, const float* f2_dev, double alpha, double beta, double q, float* sf_dev,
                    double* cost, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (!f2_dev || !cost) return fail(FDWT_EINVAL, "NULL argument");
  if (!(alpha > 1.0) || !std::isfinite(alpha) || !(beta > 0.0) || !std::isfinite(beta) || !std::isfinite(q))
    return fail(FDWT_EINVAL, "need alpha > 1, beta > 0 and finite q");
  DeviceGuard g(h->n.device);
  const double prm[3] = {alpha, beta, q};
  return split_cost_call(h->n, f2_dev, prm, sf_dev, cost, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_kernel_tune(const fdwt_net* h, const float* f2_dev, const double* start, int max_evals,
                     fdwt_kernel_fit* out, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (!f2_dev || !start || !out) return fail(FDWT_EINVAL, "NULL argument");
  if (!(start[0] > 1.0) || !std::isfinite(start[0]) || !(start[1] > 0.0) || !std::isfinite(start[1]) ||
      !std::isfinite(start[2]))
    return fail(FDWT_EINVAL, "need alpha > 1, beta > 0 and finite q at the start");
  if (max_evals < 4 || max_evals > 100000) return fail(FDWT_EINVAL, "max_evals must be in 4..100000");
  DeviceGuard g(h->n.device);
  return kernel_tune_call(h->n, f2_dev, start, max_evals, out, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_eff_dim(const fdwt_net* h, const fdwt_kernel* kern, int ft_type, const void* ft_dev,
                 fdwt_effdim* out, void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (int rc = check_kernel(h->n, kern)) return rc;
  if (!ft_dev || !out || !out->var_trc || !out->var_sup) return fail(FDWT_EINVAL, "NULL argument");
  if (ft_type != (h->n.p == 2 ? FDWT_F32 : FDWT_CF32))
    return fail(FDWT_EINVAL, "coefficients must be F32 (p = 2) or CF32 (p odd)");
  DeviceGuard g(h->n.device);
  Net& net = const_cast<Net&>(h->n);
  return run_eff_dim(net, net.sc, kern, ft_dev, out, (hipStream_t)stream);
  FDWT_GUARD_END
}

int fdwt_eff_dim_data(const fdwt_net* h, const fdwt_kernel* kern, const float* f_dev, fdwt_effdim* out,
                      void* stream) {
  FDWT_GUARD_BEGIN
  if (int rc = check_net(h)) return rc;
  if (int rc = check_kernel(h->n, kern)) return rc;
  if (!f_dev || !out || !out->var_trc || !out->var_sup) return fail(FDWT_EINVAL, "NULL argument");
  Net& net = const_cast<Net&>(h->n);
  DeviceGuard g(net.device);
  hipStream_t st = (hipStream_t)stream;
  // The transform of the data lives in a stream-ordered allocation of this
  // call (the net's workspace holds eff_dim's own columns).
  void* ft = nullptr;
  if (hipMallocAsync(&ft, (size_t)net.N * (net.p == 2 ? 4 : 8), st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FDWT_ENOMEM, "eff_dim transform allocation failed");
  }
  const int ft_type = net.p == 2 ? FDWT_F32 : FDWT_CF32;
  int rc = transform(net, false, FDWT_F32, f_dev, ft_type, ft, st);
  if (!rc) rc = run_eff_dim(net, net.sc, kern, ft, out, st);
  (void)hipFreeAsync(ft, st);
  return rc;
  FDWT_GUARD_END
}

}  // extern "C"
