// No-allocation variant of fdwt_dwt_inverse (for callers that cannot
// allocate device memory: code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The inverse transform with a real output from complex coefficients (p odd,
// CF32 -> F32 or CF64 -> F64) keeps its intermediate passes in a buffer of N
// elements of the complex working type; fdwt_dwt_inverse takes it from the
// net's workspace, which grows (hipMalloc) on first need.  This variant takes
// it from `scratch`, a fixed device array of kNoAllocScratchBytes in this
// library's code object.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address is resolved once per device with
// hipGetSymbolAddress and only that address is handed to kernels.
#include <mutex>
#include <vector>

#include "fdwt_internal.h"

namespace fdwt {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on the current device (resolved on the first
// call for that device, then cached; the array itself lives as long as the
// process).
static int scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;
  std::lock_guard<std::mutex> g(mu);
  if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(FDWT_EDEVICE, std::string("scratch address lookup failed: ") + hipGetErrorString(e));
    }
    addr[device] = p;
  }
  *out = addr[device];
  return FDWT_OK;
}

}  // namespace fdwt

using namespace fdwt;

extern "C" int fdwt_dwt_inverse_noalloc(const fdwt_net* h, int in_type, const void* in_dev, int out_type,
                                        void* out_dev, void* stream) {
  try {
    if (!h) return fail(FDWT_EINVAL, "net handle is NULL");
    const Net& net = h->n;
    Kind ik, wk, ok;
    if (int rc = transform_kinds(net, true, in_type, in_dev, out_type, out_dev, &ik, &wk, &ok)) return rc;
    const size_t need = transform_tmp_bytes(net, wk, ok);
    if (need > kNoAllocScratchBytes)
      return fail(FDWT_EBUDGET, "the inverse needs " + std::to_string(need) +
                                    " bytes of scratch; the no-allocation entry point holds " +
                                    std::to_string(kNoAllocScratchBytes));
    DeviceGuard g(net.device);
    if (!g.ok) return fail(FDWT_EDEVICE, "cannot select the net's device");
    void* tmp = nullptr;
    if (need) {
      if (int rc = scratch_address(net.device, &tmp)) return rc;
    }
    return fwt_run_tmp(net.p, net.m, true, ik, in_dev, wk, ok, out_dev, tmp, 1, 1.0, (hipStream_t)stream);
  } catch (...) {
    return fail(FDWT_EDEVICE, "internal error");
  }
}
