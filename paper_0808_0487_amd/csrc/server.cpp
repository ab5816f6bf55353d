// Serving loop: interpolation and effective-dimension requests of any
// (p, m, s) admitted against a device-memory budget and run concurrently.
//
// One scheduler thread owns every HIP call of the server.  Device memory is
// one arena (a single allocation of the budget) carved by a best-fit
// allocator with coalescing; nets (their generator tables), kernel spectra
// (per net and kernel) and packed point coordinates (per net) stay resident
// in it between requests and are evicted least-recently-used when a new
// request needs room and no running job holds them.  Each admitted job gets
// one lane (a non-blocking HIP stream of default priority), a slice of the
// arena for its buffers and workspace, and a slice of the lane's pinned
// staging; its steps are enqueued at once and the lane's completion event is
// polled, so requests that arrive while others run are admitted as soon as a
// lane and memory are free and their kernels overlap on the device.  A job
// whose cache entry is being computed by another running job waits for that
// entry's ready event on the device, not on the host.
//
// Admission is first-come first-served with bounded overtaking: a waiting
// job that does not fit may be passed by later jobs at most max_bypass
// times; after that nothing is admitted before it.  Every launch of a job
// depends only on the job's own (p, m, s, data, kernel, queries), so a
// result is bit-identical whether the job runs alone or in a mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "arena.h"
#include "fdwt_internal.h"

namespace fdwt {

namespace {

// ------------------------------------------------------------------ jobs
struct Request {
  int kind, p, m, s, family;
  uint64_t net_key;
  std::vector<uint8_t> C;
  std::vector<double> a, gamma;
  double alpha;
  int64_t nq;
  std::vector<uint32_t> q;
};

// Device bytes a request needs: its own buffers and workspace (job) and the
// cache entries it may have to create (spectrum, packed coordinates).
struct Sizes {
  size_t job = 0, spectrum = 0, packed = 0, f = 0, ft = 0, c = 0, qd = 0, sf = 0, ws = 0, pin = 0;
  int chunk = 1;
};

Net shape_net(int p, int m, int s) {
  Net n;
  n.p = p;
  n.m = m;
  n.s = s;
  n.N = ipow(p, m);
  return n;
}

Sizes request_sizes(const Request& r, size_t chunk_bytes) {
  const Net n = shape_net(r.p, r.m, r.s);
  Sizes z;
  z.spectrum = spectrum_bytes(n);
  z.f = (size_t)n.N * 4;
  z.ft = (size_t)n.N * (r.p == 2 ? 4 : 8);
  size_t ws = spectrum_ws_bytes(n);
  const size_t tab_pin = align_ws(kernel_tables_bytes(n));
  if (r.kind == FDWT_JOB_INTERP) {
    z.packed = packed_bytes(n);
    z.c = (size_t)n.N * 4;
    z.qd = (size_t)r.s * r.nq * 4;
    z.sf = (size_t)r.nq * 4;
    ws = std::max(ws, spline_coef_ws_bytes(n, true));
    ws = std::max(ws, spline_eval_ws_bytes(n, r.nq, true));
    z.pin = tab_pin + align_ws(eval_tables_bytes(n)) + align_ws(z.qd) + align_ws(z.sf);
  } else {
    z.chunk = eff_dim_chunk(n, chunk_bytes);
    ws = std::max(ws, eff_dim_ws_bytes(n, true, z.chunk));
    z.pin = 2 * tab_pin + align_ws(eff_dim_res_bytes(n));
  }
  z.ws = ws;
  z.job = align_ws(z.f) + align_ws(z.ft) + align_ws(z.c) + align_ws(z.qd) + align_ws(z.sf) + align_ws(z.ws);
  return z;
}

int check_request(const fdwt_request* q) {
  if (!q) return fail(FDWT_EINVAL, "NULL request");
  if (q->kind != FDWT_JOB_INTERP && q->kind != FDWT_JOB_EFFDIM) return fail(FDWT_EINVAL, "unknown job kind");
  if (q->p != 2 && q->p != 3 && q->p != 5 && q->p != 7)
    return fail(FDWT_EUNSUPPORTED, "only p = 2, 3, 5, 7 are supported");
  if (q->m < 1 || ipow(q->p, q->m) > (int64_t(1) << kMaxLog2N)) return fail(FDWT_EINVAL, "need 1 <= m, p^m <= 2^26");
  if (q->s < 1 || q->s > kMaxS) return fail(FDWT_EINVAL, "s must be in 1..64");
  if (!q->C_host || !q->a_host || !q->gamma_host) return fail(FDWT_EINVAL, "NULL request array");
  for (int64_t i = 0; i < (int64_t)q->s * q->m * q->m; ++i)
    if (q->C_host[i] >= q->p) return fail(FDWT_EINVAL, "generator entry >= p");
  if (q->family != FDWT_FAMILY_PRODUCT && q->family != FDWT_FAMILY_EXP && q->family != FDWT_FAMILY_WANGFANG &&
      q->family != FDWT_FAMILY_ASIAN)
    return fail(FDWT_EINVAL, "unknown family");
  if (!(q->alpha > 1.0) || !std::isfinite(q->alpha)) return fail(FDWT_EINVAL, "alpha must be > 1");
  for (int j = 0; j < q->s; ++j)
    if (!(q->gamma_host[j] > 0.0) || !std::isfinite(q->gamma_host[j]))
      return fail(FDWT_EINVAL, "gamma_j must be positive and finite");
  if (q->kind == FDWT_JOB_INTERP) {
    if (q->nq < 1 || q->nq > (int64_t(1) << 24)) return fail(FDWT_EINVAL, "nq must be in 1..2^24");
    if (!q->q_host) return fail(FDWT_EINVAL, "NULL queries");
  }
  return FDWT_OK;
}

Request copy_request(const fdwt_request* q) {
  Request r;
  r.kind = q->kind;
  r.p = q->p;
  r.m = q->m;
  r.s = q->s;
  r.family = q->family;
  r.net_key = q->net_key;
  r.C.assign(q->C_host, q->C_host + (size_t)q->s * q->m * q->m);
  r.a.assign(q->a_host, q->a_host + (q->family == FDWT_FAMILY_ASIAN ? 5 : q->s));
  r.gamma.assign(q->gamma_host, q->gamma_host + q->s);
  r.alpha = q->alpha;
  r.nq = q->kind == FDWT_JOB_INTERP ? q->nq : 0;
  if (r.nq) r.q.assign(q->q_host, q->q_host + (size_t)q->s * r.nq);
  return r;
}

}  // namespace

// Resident objects.  refs counts running jobs that read or write the entry.
struct CacheEntry {
  size_t off = kNone, bytes = 0;
  int refs = 0;
  bool valid = false;  // its computation was enqueued without error
  uint64_t last_use = 0;
  hipEvent_t ready = nullptr;  // recorded after the entry was computed
};

struct NetEntry {
  fdwt_net* h = nullptr;
  int p = 0, m = 0, s = 0;
  std::vector<uint8_t> C;
  CacheEntry packed;
};

struct Job {
  int64_t id = 0;
  Request r;
  Sizes z;
  int status = FDWT_OK;
  std::string err;
  bool done = false;
  int bypassed = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int spectrum_hit = 0, packed_hit = 0;
  size_t job_off = kNone;
  int lane = -1;
  NetEntry* net = nullptr;
  CacheEntry* spec = nullptr;
  bool holds_packed = false;
  void* pin_out = nullptr;  // lane staging slice of the result
  std::vector<float> sf;
  std::vector<double> res;
};

struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  void* pin = nullptr;
  size_t pin_bytes = 0;
  std::shared_ptr<Job> job;
};

}  // namespace fdwt

using namespace fdwt;

struct fdwt_server {
  fdwt_server_config cfg{};
  int device = 0;
  char* base = nullptr;
  Arena arena;
  std::vector<Lane> lanes;
  std::unordered_map<uint64_t, std::unique_ptr<NetEntry>> nets;  // scheduler thread only
  std::map<std::string, std::unique_ptr<CacheEntry>> spectra;    // key: net key + kernel bytes
  uint64_t tick = 0;

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<std::shared_ptr<Job>> pending;  // arrival order
  std::unordered_map<int64_t, std::shared_ptr<Job>> jobs;
  std::unordered_map<uint64_t, std::vector<uint8_t>> net_keys;  // key -> (p, m, s, C) signature
  int64_t next_id = 1;
  bool stop = false;
  int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_rejected = 0;  // guarded by mu
  // Written by the scheduler thread only.
  std::atomic<int64_t> spec_hits{0}, spec_misses{0}, packed_hits{0}, packed_misses{0}, evictions{0}, nets_built{0};
  std::atomic<int> in_flight{0};
  // Job ids whose device work fails with FDWT_ENOMEM after the kernel
  // spectrum step (FDWT_SERVER_INJECT_ENOMEM; failure-isolation tests).
  std::unordered_set<int64_t> inject_enomem;
  std::thread th;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void loop();
  bool try_admit(const std::shared_ptr<Job>& j, int lane);
  void finish(int lane);
  bool evict_one();
  size_t alloc_evicting(size_t bytes);
  int enqueue(Job& j, Lane& L);
};

static std::string sig_of(int p, int m, int s, const std::vector<uint8_t>& C) {
  std::string k((const char*)&p, sizeof p);
  k.append((const char*)&m, sizeof m);
  k.append((const char*)&s, sizeof s);
  k.append((const char*)C.data(), C.size());
  return k;
}

static std::string spectrum_key(const Request& r) {
  std::string k((const char*)&r.net_key, sizeof r.net_key);
  k.append((const char*)&r.alpha, sizeof r.alpha);
  k.append((const char*)r.gamma.data(), r.gamma.size() * sizeof(double));
  return k;
}

// Drops the least recently used entry that no running job holds.
bool fdwt_server::evict_one() {
  CacheEntry* best = nullptr;
  std::string best_key;
  for (auto& kv : spectra)
    if (kv.second->refs == 0 && kv.second->off != kNone && (!best || kv.second->last_use < best->last_use)) {
      best = kv.second.get();
      best_key = kv.first;
    }
  NetEntry* bnet = nullptr;
  for (auto& kv : nets) {
    CacheEntry& c = kv.second->packed;
    if (c.refs == 0 && c.off != kNone && (!best || c.last_use < best->last_use)) {
      best = &c;
      bnet = kv.second.get();
    }
  }
  if (!best) return false;
  arena.release(best->off, best->bytes);
  best->off = kNone;
  ++evictions;
  if (!bnet) {
    if (best->ready) (void)hipEventDestroy(best->ready);
    spectra.erase(best_key);
  }
  return true;
}

size_t fdwt_server::alloc_evicting(size_t bytes) {
  for (;;) {
    const size_t off = arena.alloc(bytes);
    if (off != kNone) return off;
    if (!evict_one()) return kNone;
  }
}

// Reserves everything job j needs and enqueues it on lane `lane`; false when
// the memory is not there (nothing is kept then).
bool fdwt_server::try_admit(const std::shared_ptr<Job>& jp, int lane) {
  Job& j = *jp;
  const Request& r = j.r;
  // Net handle (generator tables; small, kept for the server's lifetime).
  NetEntry* ne = nullptr;
  auto it = nets.find(r.net_key);
  if (it == nets.end()) {
    fdwt_net* h = nullptr;
    if (fdwt_net_generate(r.p, r.m, r.s, r.C.data(), &h) != FDWT_OK) {
      j.status = FDWT_EDEVICE;
      j.err = std::string("net generation failed: ") + fdwt_last_error();
      return true;  // completes as failed
    }
    auto e = std::make_unique<NetEntry>();
    e->h = h;
    e->p = r.p;
    e->m = r.m;
    e->s = r.s;
    e->C = r.C;
    ne = e.get();
    nets[r.net_key] = std::move(e);
    ++nets_built;
  } else {
    ne = it->second.get();
  }
  // Pin what this job reuses so that the allocations below cannot evict it.
  const std::string sk = spectrum_key(r);
  auto si = spectra.find(sk);
  CacheEntry* spec = (si != spectra.end() && si->second->off != kNone && si->second->valid) ? si->second.get() : nullptr;
  if (!spec && si != spectra.end()) {
    // An invalid entry still held by a running job cannot be replaced yet.
    if (si->second->refs > 0) return false;
    if (si->second->off != kNone) arena.release(si->second->off, si->second->bytes);
    if (si->second->ready) (void)hipEventDestroy(si->second->ready);
    spectra.erase(si);
  }
  const bool want_packed = r.kind == FDWT_JOB_INTERP;
  if (want_packed && ne->packed.off != kNone && !ne->packed.valid) {
    if (ne->packed.refs > 0) return false;
    arena.release(ne->packed.off, ne->packed.bytes);
    ne->packed.off = kNone;
  }
  const bool packed_hit = want_packed && ne->packed.off != kNone;
  if (spec) ++spec->refs;
  if (packed_hit) ++ne->packed.refs;
  size_t spec_off = kNone, packed_off = kNone, job_off = kNone;
  bool ok = true;
  if (!spec) ok = (spec_off = alloc_evicting(j.z.spectrum)) != kNone;
  if (ok && want_packed && !packed_hit) ok = (packed_off = alloc_evicting(j.z.packed)) != kNone;
  if (ok) ok = (job_off = alloc_evicting(j.z.job)) != kNone;
  if (!ok) {
    if (spec) --spec->refs;
    if (packed_hit) --ne->packed.refs;
    if (spec_off != kNone) arena.release(spec_off, j.z.spectrum);
    if (packed_off != kNone) arena.release(packed_off, j.z.packed);
    return false;
  }
  const bool spec_hit = spec != nullptr;
  if (!spec) {
    auto e = std::make_unique<CacheEntry>();
    e->off = spec_off;
    e->bytes = j.z.spectrum;
    e->refs = 1;
    e->valid = true;
    spec = e.get();
    spectra[sk] = std::move(e);
  }
  if (want_packed && !packed_hit) {
    ne->packed.off = packed_off;
    ne->packed.bytes = j.z.packed;
    ne->packed.refs = 1;
    ne->packed.valid = true;
  }
  spec->last_use = ++tick;
  if (want_packed) ne->packed.last_use = tick;
  j.net = ne;
  j.spec = spec;
  j.holds_packed = want_packed;
  j.job_off = job_off;
  j.spectrum_hit = spec_hit;
  j.packed_hit = packed_hit;
  j.lane = lane;
  j.t_admit = now();
  if (spec_hit) ++spec_hits; else ++spec_misses;
  if (want_packed) {
    if (packed_hit) ++packed_hits; else ++packed_misses;
  }
  Lane& L = lanes[lane];
  L.job = jp;
  const int rc = enqueue(j, L);
  if (rc != FDWT_OK) {
    j.status = rc;
    j.err = fdwt_last_error();
    // Entries this job was to compute may be incomplete: nobody may use them.
    if (!spec_hit) spec->valid = false;
    if (want_packed && !packed_hit) ne->packed.valid = false;
  }
  // The completion event closes whatever was enqueued, failed or not.
  if (hipEventRecord(L.done, L.st) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(L.st);
  }
  ++in_flight;
  return true;
}

int fdwt_server::enqueue(Job& j, Lane& L) {
  const Request& r = j.r;
  Net& net = j.net->h->n;
  const hipStream_t st = L.st;
  if (L.pin_bytes < j.z.pin) {
    if (L.pin) FDWT_HIP(hipHostFree(L.pin));
    L.pin = nullptr;
    L.pin_bytes = 0;
    FDWT_HIP(hipHostMalloc(&L.pin, j.z.pin, hipHostMallocDefault));
    L.pin_bytes = j.z.pin;
  }
  char* jb = base + j.job_off;
  size_t o = 0;
  auto take = [&](size_t b) {
    char* p = jb + o;
    o += align_ws(b);
    return (void*)p;
  };
  float* f = (float*)take(j.z.f);
  void* ft = take(j.z.ft);
  float* c = (float*)take(j.z.c);
  uint32_t* qd = (uint32_t*)take(j.z.qd);
  float* sf = (float*)take(j.z.sf);
  Scratch sc;
  sc.fixed = true;
  sc.ws = take(j.z.ws);
  sc.ws_bytes = j.z.ws;
  sc.pin = L.pin;
  sc.pin_bytes = L.pin_bytes;
  fdwt_kernel kern{r.alpha, r.gamma.data(), r.s};
  void* gk = base + j.spec->off;
  // Kernel spectrum: computed by this job, or awaited on the device.
  if (!j.spectrum_hit) {
    if (!j.spec->ready) FDWT_HIP(hipEventCreateWithFlags(&j.spec->ready, hipEventDisableTiming));
    if (int rc = run_spectrum(net, sc, &kern, gk, st)) return rc;
    FDWT_HIP(hipEventRecord(j.spec->ready, st));
  } else {
    FDWT_HIP(hipStreamWaitEvent(st, j.spec->ready, 0));
  }
  if (inject_enomem.count(j.id))
    return fail(FDWT_ENOMEM, "injected allocation failure (FDWT_SERVER_INJECT_ENOMEM) after the spectrum step");
  void* packed = nullptr;
  if (j.holds_packed) {
    CacheEntry& pe = j.net->packed;
    packed = base + pe.off;
    if (!j.packed_hit) {
      if (!pe.ready) FDWT_HIP(hipEventCreateWithFlags(&pe.ready, hipEventDisableTiming));
      if (int rc = launch_net_packed(net, packed, st)) return rc;
      FDWT_HIP(hipEventRecord(pe.ready, st));
    } else {
      FDWT_HIP(hipStreamWaitEvent(st, pe.ready, 0));
    }
  }
  if (int rc = launch_sample(net, r.family, r.a.data(), f, st)) return rc;
  const double scale = 1.0 / (double)net.N;  // Eq. (eq_dwalshcoeff)
  int rc = net.p == 2 ? fwt_run_tmp(2, net.m, false, K_F32, f, K_F32, K_F32, ft, nullptr, 1, scale, st)
                      : fwt_run_tmp(net.p, net.m, false, K_F32, f, K_CF32, K_CF32, ft, nullptr, 1, scale, st);
  if (rc) return rc;
  if (r.kind == FDWT_JOB_INTERP) {
    if ((rc = run_spline_coef(net, sc, &kern, gk, ft, c, st))) return rc;
    if ((rc = upload(sc, r.q.data(), (size_t)r.s * r.nq * 4, qd, st))) return rc;
    if ((rc = run_spline_eval(net, sc, &kern, packed, c, r.nq, qd, sf, st))) return rc;
    if ((rc = pin_take(sc, (size_t)r.nq * 4, &j.pin_out))) return rc;
    FDWT_HIP(hipMemcpyAsync(j.pin_out, sf, (size_t)r.nq * 4, hipMemcpyDeviceToHost, st));
  } else {
    if ((rc = pin_take(sc, eff_dim_res_bytes(net), &j.pin_out))) return rc;
    if ((rc = eff_dim_enqueue(net, sc, &kern, gk, ft, j.z.chunk, (double*)j.pin_out, nullptr, st))) return rc;
  }
  return FDWT_OK;
}

// Lane `lane` has completed: collect the result and release the job's hold.
void fdwt_server::finish(int lane) {
  Lane& L = lanes[lane];
  std::shared_ptr<Job> jp = L.job;
  Job& j = *jp;
  if (j.status == FDWT_OK && j.pin_out) {
    if (j.r.kind == FDWT_JOB_INTERP) {
      j.sf.resize(j.r.nq);
      std::memcpy(j.sf.data(), j.pin_out, (size_t)j.r.nq * 4);
    } else {
      j.res.resize(2 * j.r.s + 2);
      std::memcpy(j.res.data(), j.pin_out, j.res.size() * sizeof(double));
    }
  }
  if (j.job_off != kNone) arena.release(j.job_off, j.z.job);
  j.job_off = kNone;
  if (j.spec) --j.spec->refs;
  if (j.holds_packed) --j.net->packed.refs;
  L.job.reset();
  --in_flight;
  std::lock_guard<std::mutex> g(mu);
  j.t_done = now();
  j.done = true;
  if (j.status == FDWT_OK) ++n_completed; else ++n_failed;
  cv_done.notify_all();
}

void fdwt_server::loop() {
  (void)hipSetDevice(device);
  std::vector<std::shared_ptr<Job>> order;
  for (;;) {
    bool progress = false;
    // Completions.
    for (int l = 0; l < (int)lanes.size(); ++l) {
      if (!lanes[l].job) continue;
      const hipError_t e = hipEventQuery(lanes[l].done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) {
        (void)hipGetLastError();
        Job& j = *lanes[l].job;
        j.status = FDWT_EDEVICE;
        j.err = std::string("device error: ") + hipGetErrorString(e);
      }
      finish(l);
      progress = true;
    }
    // Admissions, in arrival order with bounded overtaking.
    {
      std::unique_lock<std::mutex> g(mu);
      if (stop && pending.empty() && in_flight == 0) break;
      order.assign(pending.begin(), pending.end());
    }
    // A waiting job is overtaken each time a later one is admitted; once it
    // has been overtaken max_bypass times, nothing behind it is admitted.
    std::vector<std::shared_ptr<Job>> admitted, waiting;
    bool head_refused = false;
    for (auto& jp : order) {
      int lane = -1;
      for (int l = 0; l < (int)lanes.size(); ++l)
        if (!lanes[l].job) {
          lane = l;
          break;
        }
      if (lane < 0) break;
      bool blocked = false;
      for (auto& w : waiting) blocked |= w->bypassed >= cfg.max_bypass;
      if (blocked) break;
      if (try_admit(jp, lane)) {
        admitted.push_back(jp);
        for (auto& w : waiting) ++w->bypassed;
        if (jp->status != FDWT_OK && !lanes[lane].job) {
          // Failed before reaching the device (net generation).
          std::lock_guard<std::mutex> g(mu);
          jp->t_admit = jp->t_done = now();
          jp->done = true;
          ++n_failed;
          cv_done.notify_all();
        }
        progress = true;
      } else {
        if (waiting.empty() && admitted.empty()) head_refused = true;
        waiting.push_back(jp);
      }
    }
    if (!admitted.empty()) {
      std::lock_guard<std::mutex> g(mu);
      for (auto& jp : admitted) {
        auto pos = std::find(pending.begin(), pending.end(), jp);
        if (pos != pending.end()) pending.erase(pos);
      }
    }
    if (!progress) {
      std::unique_lock<std::mutex> g(mu);
      if (in_flight > 0)
        cv_sched.wait_for(g, std::chrono::microseconds(50));
      else
        cv_sched.wait_for(g, std::chrono::milliseconds(5), [&] { return stop || !pending.empty(); });
      if (head_refused && in_flight == 0 && arena.used() == 0 && !pending.empty() &&
          pending.front() == order.front()) {
        // The head was refused with nothing running and nothing resident (all
        // of the arena free): it can never be admitted.
        auto jp = pending.front();
        pending.pop_front();
        jp->status = FDWT_EBUDGET;
        jp->err = "request does not fit the server's memory budget";
        jp->t_admit = jp->t_done = now();
        jp->done = true;
        ++n_failed;
        cv_done.notify_all();
      }
    }
  }
}

extern "C" {

int fdwt_server_request_bytes(const fdwt_request* req, size_t effdim_chunk_bytes, size_t* job_bytes,
                              size_t* cache_bytes) {
  try {
    if (int rc = check_request(req)) return rc;
    const Request r = copy_request(req);
    const Sizes z = request_sizes(r, effdim_chunk_bytes ? effdim_chunk_bytes : ((size_t)1 << 30));
    if (job_bytes) *job_bytes = z.job;
    if (cache_bytes) *cache_bytes = align_ws(z.spectrum) + (z.packed ? align_ws(z.packed) : 0);
    return FDWT_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDWT_ENOMEM, "host allocation failed");
  }
}

int fdwt_server_create(const fdwt_server_config* cfg, fdwt_server** out) {
  if (!cfg || !out) return fail(FDWT_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->hbm_budget < ((size_t)1 << 20)) return fail(FDWT_EINVAL, "budget must be at least 1 MiB");
  if (cfg->lanes < 1 || cfg->lanes > 64) return fail(FDWT_EINVAL, "lanes must be in 1..64");
  if (cfg->max_bypass < 0) return fail(FDWT_EINVAL, "max_bypass must be >= 0");
  std::unique_ptr<fdwt_server> sv(new fdwt_server());
  sv->cfg = *cfg;
  if (!sv->cfg.effdim_chunk_bytes) sv->cfg.effdim_chunk_bytes = (size_t)1 << 30;
  FDWT_HIP(hipGetDevice(&sv->device));
  const size_t budget = align_ws(cfg->hbm_budget);
  if (hipMalloc((void**)&sv->base, budget) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FDWT_ENOMEM, "server arena of " + std::to_string(budget) + " bytes could not be allocated");
  }
  sv->arena.reset(budget);
  sv->lanes.resize(cfg->lanes);
  for (auto& L : sv->lanes) {
    if (hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      fdwt_server_free(sv.release());
      return fail(FDWT_EDEVICE, "stream creation failed");
    }
  }
  if (const char* e = getenv("FDWT_SERVER_INJECT_ENOMEM")) {
    // comma-separated job ids
    for (const char* c = e; *c;) {
      char* end = nullptr;
      const long long v = strtoll(c, &end, 10);
      if (end == c) break;
      sv->inject_enomem.insert((int64_t)v);
      c = *end == ',' ? end + 1 : end;
    }
  }
  sv->t0 = std::chrono::steady_clock::now();
  fdwt_server* raw = sv.get();
  sv->th = std::thread([raw] { raw->loop(); });
  *out = sv.release();
  return FDWT_OK;
}

int fdwt_server_submit(fdwt_server* sv, const fdwt_request* req, int64_t* id) {
  if (!sv || !id) return fail(FDWT_EINVAL, "NULL argument");
  try {
    if (int rc = check_request(req)) {
      std::lock_guard<std::mutex> g(sv->mu);
      ++sv->n_rejected;
      return rc;
    }
    auto j = std::make_shared<Job>();
    j->r = copy_request(req);
    j->z = request_sizes(j->r, sv->cfg.effdim_chunk_bytes);
    const size_t need = align_ws(j->z.job) + align_ws(j->z.spectrum) + (j->z.packed ? align_ws(j->z.packed) : 0);
    std::lock_guard<std::mutex> g(sv->mu);
    if (need > sv->arena.size()) {
      ++sv->n_rejected;
      return fail(FDWT_EBUDGET, "request needs " + std::to_string(need) + " bytes, more than the budget");
    }
    const std::string sig = sig_of(j->r.p, j->r.m, j->r.s, j->r.C);
    auto k = sv->net_keys.find(j->r.net_key);
    if (k == sv->net_keys.end()) {
      sv->net_keys[j->r.net_key] = std::vector<uint8_t>(sig.begin(), sig.end());
    } else if (std::string(k->second.begin(), k->second.end()) != sig) {
      ++sv->n_rejected;
      return fail(FDWT_EINVAL, "net_key already names a different (p, m, s, C)");
    }
    if (sv->stop) return fail(FDWT_EINVAL, "server is shutting down");
    j->id = sv->next_id++;
    j->t_submit = sv->now();
    sv->jobs[j->id] = j;
    sv->pending.push_back(j);
    ++sv->n_submitted;
    *id = j->id;
    sv->cv_sched.notify_one();
    return FDWT_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDWT_ENOMEM, "host allocation failed");
  }
}

int fdwt_server_wait(fdwt_server* sv, int64_t id, fdwt_job_info* info, float* sf_host, fdwt_effdim* eff) {
  if (!sv) return fail(FDWT_EINVAL, "NULL server");
  std::shared_ptr<Job> j;
  {
    std::unique_lock<std::mutex> g(sv->mu);
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return fail(FDWT_EINVAL, "unknown job id");
    j = it->second;
    sv->cv_done.wait(g, [&] { return j->done; });
    sv->jobs.erase(id);
  }
  if (info) {
    info->status = j->status;
    info->t_submit = j->t_submit;
    info->t_admit = j->t_admit;
    info->t_done = j->t_done;
    info->bytes = j->z.job;
    info->spectrum_hit = j->spectrum_hit;
    info->packed_hit = j->packed_hit;
  }
  if (j->status != FDWT_OK) return fail(j->status, j->err);
  if (j->r.kind == FDWT_JOB_INTERP) {
    if (sf_host) std::memcpy(sf_host, j->sf.data(), j->sf.size() * 4);
  } else if (eff) {
    if (!eff->var_trc || !eff->var_sup) return fail(FDWT_EINVAL, "eff_dim result arrays are NULL");
    eff_dim_finish(j->r.s, j->res.data(), eff);
  }
  return FDWT_OK;
}

int fdwt_server_stats(fdwt_server* sv, fdwt_server_counters* st) {
  if (!sv || !st) return fail(FDWT_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(sv->mu);
  st->submitted = sv->n_submitted;
  st->completed = sv->n_completed;
  st->failed = sv->n_failed;
  st->rejected = sv->n_rejected;
  st->pending = (int64_t)sv->pending.size();
  st->in_flight = sv->in_flight;
  st->arena_bytes = sv->arena.size();
  st->arena_used = sv->arena.used();
  st->arena_peak = sv->arena.peak();
  st->spectrum_hits = sv->spec_hits;
  st->spectrum_misses = sv->spec_misses;
  st->packed_hits = sv->packed_hits;
  st->packed_misses = sv->packed_misses;
  st->evictions = sv->evictions;
  st->nets_built = sv->nets_built;
  return FDWT_OK;
}

void fdwt_server_free(fdwt_server* sv) {
  if (!sv) return;
  if (sv->th.joinable()) {
    {
      std::lock_guard<std::mutex> g(sv->mu);
      sv->stop = true;
    }
    sv->cv_sched.notify_all();
    sv->th.join();
  }
  (void)hipSetDevice(sv->device);
  for (auto& L : sv->lanes) {
    if (L.st) (void)hipStreamSynchronize(L.st);
    if (L.st) (void)hipStreamDestroy(L.st);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.pin) (void)hipHostFree(L.pin);
  }
  for (auto& kv : sv->spectra)
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
  for (auto& kv : sv->nets) {
    if (kv.second->packed.ready) (void)hipEventDestroy(kv.second->packed.ready);
    fdwt_net_free(kv.second->h);
  }
  if (sv->base) (void)hipFree(sv->base);
  delete sv;
}

}  // extern "C"
