// Ragged batches of p = 2 forward transforms.
//
// A batch is a list of independent jobs (float data, N_j = 2^{m_j} points,
// each normalised by 2^-m_j as in Eq. (eq_dwalshcoeff)).  Every job's
// transform is split into passes (Algorithm 1's stages grouped by digit
// ranges) and every pass into tiles.  Two ways to run them:
//
//  * grouped (FDWT_PREC_F32, m >= 7): jobs of equal m form a group; pass k of
//    a group is one launch of the static-shape pass kernel over all of the
//    group's tiles, its columns read through tables of the jobs' pointers.
//    The plan of a group (how large the first, contiguous pass is) is picked
//    by fdwt_batch_autotune, which times every distinct plan on the device.
//  * generic (FDWT_PREC_BF16X2, FDWT_PREC_F32_GENERIC, and jobs with m < 7):
//    level k of the batch is the list of all tiles of pass k of every job;
//    each level is one persistent launch whose workgroups take the level's
//    tiles with a fixed stride (largest jobs first);
//  * one launch (FDWT_PREC_F32_ONE_LAUNCH): the same items, all levels, in
//    one persistent launch with a ticket counter and per-job pass counters
//    (k_batch_one below).
//
// In the first two no workgroup ever waits for another: the kernel boundary
// between passes orders pass k before pass k+1.  A first one-launch design
// (fixed-stride item order, plain counter stores and loads) did not finish on
// the device; two causes fit what was seen and neither was shown: counter
// updates and reads without device-scope release/acquire ordering (each XCD
// has its own L2), and waits on producer workgroups that were not yet
// resident (a fixed-stride order gives no forward-progress guarantee).
// k_batch_one removes both: tickets in dependency order (a wait is always on
// an item a running workgroup holds, checked by a host emulation of the
// schedule), release/acquire at device scope, and bounded waits.
//
// Precision FDWT_PREC_BF16X2: in each job's first pass the stages of index
// digits 0..3 (16-point Walsh-Hadamard blocks) run on the matrix cores as
// H16 (hi + lo), with x = hi + lo split into two bfloat16 values, H16's +-1
// entries exact in bfloat16 and float32 accumulation: one
// v_mfma_f32_16x16x32_bf16 per 16 vectors of 16 points, A = [H16 | H16],
// B = [hi ; lo].  All other stages stay in float32.
#include "p2_stages.h"
#include "pass_core.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>

namespace fdwt {

constexpr int kBThreads = 512;   // threads per workgroup
constexpr int kBLogE = 13;       // largest tile: 2^13 floats (33 KiB of LDS)
constexpr int kBMaxPass = 3;

struct BJob {
  const float* in;
  float* out;
  int m;
  int npass;
  float scale;            // 2^-m
  int d0[kBMaxPass], r[kBMaxPass], wdig[kBMaxPass], ntiles[kBMaxPass];
};

struct BItem {
  int job, pass, tile, pad_;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Stages of digits 0..3 of a contiguous float tile in LDS on the matrix
// cores.  Lane l of a wave: vector n = l % 16 of the current 256-point chunk,
// operand slice q = l / 16.  Operand layout of v_mfma_f32_16x16x32_bf16
// (checked with a probe on gfx950): A[l%16][8q+i], B[8q+i][l%16] are element i
// of the lane's A and B vectors; D[4q+i][l%16] is element i of the result.
__device__ void mfma_low4(float* lds, int E) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  bf16x8 a;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = (8 * q + i) & 15;  // A = [H16 | H16]
    a[i] = (__builtin_popcount(n & k) & 1) ? (__bf16)(-1.0f) : (__bf16)(1.0f);
  }
  for (int c = wave; c < E / 256; c += nw) {
    const int src = 256 * c + 16 * n + 8 * (q & 1);
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float x = lds[pad(src + i)];
      const __bf16 hi = (__bf16)x;
      b[i] = (q < 2) ? hi : (__bf16)(x - (float)hi);
    }
    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    const f32x4 dres = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, z, 0, 0, 0);
    const int dst = 256 * c + 16 * n + 4 * q;
#pragma unroll
    for (int i = 0; i < 4; ++i) lds[pad(dst + i)] = dres[i];
  }
}

// One tile of one pass of one job (runtime geometry): load into LDS, the
// pass's stages in register groups, store (scaled by 2^-m in the last pass).
// Ends with a workgroup barrier.  With COHERENT, a tile written by an earlier
// pass of the same launch (pass > 0) is loaded, and a tile that a later pass
// of the launch reads (not the last pass) is stored, with device-scope
// (relaxed atomic) accesses, which read and write at the point of coherence
// of all XCDs instead of through this XCD's L2.
template <bool COHERENT>
__device__ __forceinline__ void batch_tile(const BJob& J, const BItem I, int prec, float* blds) {
  const int ps = I.pass;
  PassDesc d{};
  d.r = J.r[ps];
  d.wdig = J.wdig[ps];
  d.w = 1 << d.wdig;
  d.sd0 = int64_t(1) << J.d0[ps];
  d.shi = int64_t(1) << (J.d0[ps] + d.r);
  d.nlo = 1 << (J.d0[ps] - d.wdig);
  d.E = 1 << (d.r + d.wdig);
  d.kreg = 4;
  const int lo = I.tile % d.nlo, hi = I.tile / d.nlo;
  const int64_t base = (int64_t)lo * d.w + (int64_t)hi * d.shi;
  const gptr<const float> src = to_global((ps == 0 ? J.in : J.out) + base);
  for (int e = threadIdx.x; e < d.E; e += blockDim.x) {
    const int c = e & (d.w - 1), i = e >> d.wdig;
    if (COHERENT && ps > 0)
      blds[pad(e)] = __hip_atomic_load(to_global(const_cast<float*>((ps == 0 ? J.in : J.out) + base)) + c +
                                           (int64_t)i * d.sd0,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      blds[pad(e)] = src[c + (int64_t)i * d.sd0];
  }
  __syncthreads();
  int q0 = 0;
  if (prec == FDWT_PREC_BF16X2 && ps == 0 && d.wdig == 0 && d.r >= 8) {
    mfma_low4(blds, d.E);
    __syncthreads();
    q0 = 4;
  }
  for (int q = q0; q < d.r; q += 4) {
    const int kk = min(4, d.r - q);
    if (kk == 4) run_group<2, false, float, 4>(blds, d, q);
    else if (kk == 3) run_group<2, false, float, 3>(blds, d, q);
    else if (kk == 2) run_group<2, false, float, 2>(blds, d, q);
    else run_group<2, false, float, 1>(blds, d, q);
    __syncthreads();
  }
  const float sc = (ps == J.npass - 1) ? J.scale : 1.0f;
  const gptr<float> dst = to_global(J.out + base);
  for (int e = threadIdx.x; e < d.E; e += blockDim.x) {
    const int c = e & (d.w - 1), i = e >> d.wdig;
    if (COHERENT && ps < J.npass - 1)
      __hip_atomic_store(dst + c + (int64_t)i * d.sd0, blds[pad(e)] * sc, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    else
      dst[c + (int64_t)i * d.sd0] = blds[pad(e)] * sc;
  }
  __syncthreads();
}

// Level launch of the generic path: items of one pass level, fixed stride.
__global__ void __launch_bounds__(kBThreads) k_batch_fwd(const BJob* __restrict__ jobs, const BItem* __restrict__ items,
                                                       int n_items, int prec) {
  extern __shared__ __align__(16) float blds[];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const BItem I = items[it];
    batch_tile<false>(jobs[I.job], I, prec, blds);
  }
}

// ------------------------------------------ static tile of the one launch
// A tile of 2^13 floats, rows of W = 2^WDIG contiguous elements (WDIG 0 for
// a contiguous first pass; 13 - WDIG digits transformed), 512 threads with
// 16 elements each, all offsets compile-time strides from a per-thread base:
//  1. element e = tid + 512 k: the stages of e bits [max(9, WDIG), 13) (the
//     register index k) run in registers; with WDIG >= 9 that is every digit
//     and the tile goes straight back to memory;
//  2. for WDIG < 6, the stages of e bits [WDIG, 6) through LDS (register
//     groups as fwt_p2);
//  3. read back as e = lane + 64 k + 1024 w: the stages of e bits
//     [max(6, WDIG), 9) in registers, then the store.
// coh_in: the tile was written by an earlier pass of the launch, and is read
// with device-coherent buffer loads (sc1: served at the point of coherence of
// all XCDs); coh_out: a later pass reads it, and it is stored with
// device-scope relaxed atomic stores.
template <int WDIG>
__device__ __noinline__ void tile13(const float* src, float* dst, uint32_t sd0, uint32_t nbytes, float sc, bool coh_in,
                                       bool coh_out, float* lds) {
  constexpr int TH = kBThreads, EPT = 16, W = 1 << WDIG;
  static_assert(TH * EPT == 8192, "2^13-element tiles");
  const int tid = threadIdx.x;
  // load mapping e = tid + 512 k
  // Offsets within a job's buffer fit in 32 bits (at most 2^26 elements).
  auto off1 = [&](int k) -> uint32_t {
    if constexpr (WDIG <= 9)
      return (uint32_t)(tid & (W - 1)) + ((uint32_t)(tid >> WDIG) + (uint32_t)k * (TH >> WDIG)) * sd0;
    else
      return (uint32_t)tid + TH * (k & ((W / TH) - 1)) + (uint32_t)(k >> (WDIG - 9)) * sd0;
  };
  float v[EPT];
  if (coh_in) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, (int)nbytes, 0x00020000);
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      v[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(off1(k) * 4u), 0, 16));
  } else {
    const gptr<const float> g = to_global(src);
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[k] = g[off1(k)];
  }
  reg_bfly_bits<(WDIG > 9 ? WDIG - 9 : 0), 4>(v);
  if constexpr (WDIG >= 9) {
    if (coh_out) {
#pragma unroll
      for (int k = 0; k < EPT; ++k)
        __hip_atomic_store(to_global(dst) + off1(k), v[k] * sc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) to_global(dst)[off1(k)] = v[k] * sc;
    }
    (void)lds;
  } else {
    float* lrow = lds + cpad(tid);
#pragma unroll
    for (int k = 0; k < EPT; ++k) lrow[cpad(k * TH)] = v[k];
    lds_barrier();
    if constexpr (WDIG < 6) P2Groups<13, WDIG, 0, float, 4, 6 - WDIG>::run(lds, tid);
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float* lrowS = lds + cpad(lane + 1024 * wv);
    float y[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) y[k] = lrowS[66 * k];
    reg_bfly_bits<(WDIG > 6 ? WDIG - 6 : 0), 3>(y);
    // store mapping e = lane + 64 k + 1024 wv
    auto off2 = [&](int k) -> uint32_t {
      if constexpr (WDIG <= 6)
        return (uint32_t)(lane & (W - 1)) +
               ((uint32_t)(lane >> WDIG) + (uint32_t)wv * (1024 >> WDIG) + (uint32_t)k * (64 >> WDIG)) * sd0;
      else
        return (uint32_t)lane + 64 * (k & ((W >> 6) - 1)) +
               ((uint32_t)(k >> (WDIG - 6)) + (uint32_t)wv * (1024 >> WDIG)) * sd0;
    };
    if (coh_out) {
#pragma unroll
      for (int k = 0; k < EPT; ++k)
        __hip_atomic_store(to_global(dst) + off2(k), y[k] * sc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) to_global(dst)[off2(k)] = y[k] * sc;
    }
    lds_barrier();
  }
}

// One item of the one launch: the job's pass geometry picks the tile.
__device__ __forceinline__ void one_item(const BJob& J, const BItem I, float* blds) {
  const int ps = I.pass;
  if (J.m < 13) {
    batch_tile<true>(J, I, FDWT_PREC_F32, blds);
    return;
  }
  const int wd = J.wdig[ps], d0 = J.d0[ps];
  const uint32_t sd0 = 1u << d0;
  const int nlo = 1 << (d0 - wd);
  const int lo = I.tile % nlo, hi = I.tile / nlo;
  const int64_t base = ((int64_t)lo << wd) + ((int64_t)hi << (d0 + J.r[ps]));
  const float* src = (ps == 0 ? J.in : J.out) + base;
  float* dst = J.out + base;
  const uint32_t nbytes = (uint32_t)((uint64_t(4) << J.m) - (uint64_t)base * 4);
  const float sc = (ps == J.npass - 1) ? J.scale : 1.0f;
  const bool ci = ps > 0, co = ps < J.npass - 1;
  switch (wd) {
    case 0: tile13<0>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 4: tile13<4>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 5: tile13<5>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 6: tile13<6>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 7: tile13<7>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 8: tile13<8>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 9: tile13<9>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 10: tile13<10>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 11: tile13<11>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
    case 12: tile13<12>(src, dst, sd0, nbytes, sc, ci, co, blds); break;
  }
}

// ------------------------------------------------ one launch for the batch
// FDWT_PREC_F32_ONE_LAUNCH runs every pass of every job in one persistent
// launch.  Work items (job, pass, tile) are numbered level by level (every
// job's pass 0, then every pass 1, ...), and a workgroup takes the next
// kBChunk of them from a ticket counter and runs them in order.  An item of
// pass k > 0 waits until all ntiles[k-1] tiles of its job's pass k-1 are
// done.  Those items have smaller numbers, so their tickets were taken
// before and are held by workgroups that are running (a workgroup takes a
// ticket only while it runs and keeps running until its items are done);
// by induction on the item number every wait ends, whatever the number of
// workgroups resident at once.  Each XCD has its own L2, so data must not
// pass between workgroups through it: where another pass of the launch wrote
// or reads a tile, it is loaded with device-coherent buffer loads and stored
// with device-scope relaxed atomic stores (both served at the point of
// coherence of all XCDs), every thread waits for its stores to be
// acknowledged, and only
// then, after a workgroup barrier, is the job's pass counter incremented
// (device scope); a waiting workgroup polls the counter with device-scope
// loads before it loads the tile.  A job's input is read only by its first
// pass and its last pass's output by no one in the launch: those accesses
// stay ordinary, and the last pass counts nothing.  (Release and acquire
// fences would do the same by writing back and invalidating the whole L2
// around every tile: a batch of 512 jobs took 58 ms that way.)  Waits are
// bounded: after `timeout` ticks of the wall clock, or once another
// workgroup has given up, a workgroup raises the error flag and exits, so
// the launch always ends (fdwt_batch_check then reports the failure).
constexpr int kBChunk = 4;  // items per ticket

struct BCtl {
  int next;   // next ticket (item number)
  int error;  // set when a wait gave up
};

__global__ void k_batch_reset(BCtl* ctl, int* done, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctl->next = 0;
    ctl->error = 0;
  }
  if (i < n) done[i] = 0;
}

// Thread 0 of a workgroup: spin until *cnt >= need; 1 if it gave up (after
// `timeout` wall-clock ticks, or 2^26 polls, whichever comes first).
// timeout 0 gives up at every wait (the host's test setting for the
// failure path).
__device__ int wait_count(int* cnt, int need, BCtl* ctl, uint64_t timeout) {
  if (timeout == 0) {
    __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 1;
  }
  if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return 0;
  const uint64_t t0 = wall_clock64();
  for (int polls = 0;; ++polls) {
    __builtin_amdgcn_s_sleep(2);
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return 0;
    if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 1;
    if (wall_clock64() - t0 > timeout || polls >= (1 << 26)) {
      __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 1;
    }
  }
}

__global__ void __launch_bounds__(kBThreads) k_batch_one(const BJob* __restrict__ jobs, const BItem* __restrict__ items,
                                                       int n_items, BCtl* ctl, int* done, uint64_t timeout) {
  extern __shared__ __align__(16) float blds[];
  __shared__ int s_first, s_abort;
  for (;;) {
    __syncthreads();  // every thread has read the previous ticket
    if (threadIdx.x == 0)
      s_first = __hip_atomic_fetch_add(&ctl->next, kBChunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int first = s_first;
    if (first >= n_items) return;
    const int last = min(first + kBChunk, n_items);
    for (int it = first; it < last; ++it) {
      const BItem I = items[it];
      const BJob& J = jobs[I.job];
      if (I.pass > 0) {
        if (threadIdx.x == 0)
          s_abort = wait_count(done + I.job * kBMaxPass + I.pass - 1, J.ntiles[I.pass - 1], ctl, timeout);
        __syncthreads();
        if (s_abort) return;
      }
      one_item(J, I, blds);
      if (I.pass < J.npass - 1) {  // a later pass of the job reads this tile
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores acknowledged
        __syncthreads();
        if (threadIdx.x == 0)
          __hip_atomic_fetch_add(done + I.job * kBMaxPass + I.pass, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

}  // namespace fdwt

struct fdwt_batch {
  int device = 0;
  int n_jobs = 0, prec = 0;
  // generic path
  fdwt::BJob* d_jobs = nullptr;
  fdwt::BItem* d_items = nullptr;
  int level_begin[fdwt::kBMaxPass + 1] = {0};  // items of level k: [begin[k], begin[k+1])
  int n_levels = 0;
  int grid_per_level[fdwt::kBMaxPass] = {0};
  // one-launch path: control block, per-job pass counters, grid, wait limit
  bool one_launch = false;
  fdwt::BCtl* d_ctl = nullptr;
  int* d_done = nullptr;
  int n_items = 0, one_grid = 0;
  uint64_t timeout_ticks = 0;
  // grouped path: one entry per distinct m
  struct Group {
    int m = 0, emax = 14, njobs = 0;
    bool in_place = false;
    void** d_in = nullptr;   // device array of the jobs' input pointers
    void** d_out = nullptr;  // ... and output pointers
  };
  std::vector<Group> groups;
  double alg_bytes = 0.0;
};

namespace fdwt {

// Pass split of one job with tiles of at most 2^kBLogE elements: a
// contiguous first pass, then strided passes with rows of 16 floats.
static int batch_plan_job(int m, BJob& J) {
  const int emax = kBLogE, wd = 4;
  J.m = m;
  if (m <= emax) {
    J.npass = 1;
    J.d0[0] = 0;
    J.r[0] = m;
    J.wdig[0] = 0;
  } else {
    const int rem = m - emax, cap = emax - wd;
    const int nstr = (rem + cap - 1) / cap;
    if (nstr + 1 > kBMaxPass) return -1;
    const int rd = std::max((rem + nstr - 1) / nstr, 1);
    const int first = m - nstr * rd;
    J.npass = 1 + nstr;
    J.d0[0] = 0;
    J.r[0] = first;
    J.wdig[0] = 0;
    for (int i = 0; i < nstr; ++i) {
      J.d0[1 + i] = first + i * rd;
      J.r[1 + i] = rd;
      J.wdig[1 + i] = std::min(wd, first + i * rd);
    }
  }
  for (int k = 0; k < J.npass; ++k) J.ntiles[k] = (int)((int64_t(1) << m) >> (J.r[k] + J.wdig[k]));
  J.scale = (float)std::ldexp(1.0, -m);
  return 0;
}

// Pass split of one job in the one-launch batch: m >= 13 gives tiles of
// exactly 2^13 elements in every pass (tile13): a contiguous first pass of
// 13 digits, then the other m - 13 digits split evenly into strided passes of
// at most 9 digits, each over rows of 2^(13 - r) elements; m < 13 one
// generic pass.
static int batch_plan_one(int m, BJob& J) {
  J.m = m;
  J.d0[0] = 0;
  J.wdig[0] = 0;
  if (m < 13) {
    J.npass = 1;
    J.r[0] = m;
    J.ntiles[0] = 1;
  } else {
    const int rem = m - 13, nstr = (rem + 8) / 9;
    if (1 + nstr > kBMaxPass) return -1;
    J.npass = 1 + nstr;
    J.r[0] = 13;
    int d = 13;
    for (int i = 0; i < nstr; ++i) {
      const int r = (rem - (d - 13) + (nstr - i) - 1) / (nstr - i);
      J.d0[1 + i] = d;
      J.r[1 + i] = r;
      J.wdig[1 + i] = 13 - r;
      d += r;
    }
    for (int k = 0; k < J.npass; ++k) J.ntiles[k] = (int)((int64_t(1) << m) >> 13);
  }
  J.scale = (float)std::ldexp(1.0, -m);
  return 0;
}

// Work items of the generic and one-launch paths: level k holds every tile
// of pass k of every job, jobs largest first (stable), tiles in order;
// level_begin[k] is the first item of level k (maxpass + 1 entries).  one:
// the one-launch plan (batch_plan_one) instead of batch_plan_job.
static int build_items(const std::vector<int>& ms, std::vector<BJob>& hj, std::vector<BItem>& hi,
                       int* level_begin, int& maxpass, bool one) {
  hj.assign(ms.size(), BJob{});
  hi.clear();
  maxpass = 0;
  for (size_t i = 0; i < ms.size(); ++i) {
    if (one ? batch_plan_one(ms[i], hj[i]) : batch_plan_job(ms[i], hj[i])) return -1;
    maxpass = std::max(maxpass, hj[i].npass);
  }
  std::vector<int> order(hj.size());
  for (size_t j = 0; j < hj.size(); ++j) order[j] = (int)j;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return hj[x].m > hj[y].m; });
  for (int ps = 0; ps < maxpass; ++ps) {
    level_begin[ps] = (int)hi.size();
    for (int j : order)
      if (ps < hj[j].npass)
        for (int t = 0; t < hj[j].ntiles[ps]; ++t) hi.push_back({j, ps, t, 0});
  }
  level_begin[maxpass] = (int)hi.size();
  return 0;
}

}  // namespace fdwt

using namespace fdwt;

namespace fdwt {
int p2_plan_passes(int m, int emax);
bool p2_plans_equal(int m, int e1, int e2);
int fwt_p2_group_pass(int m, int emax, int level, const void* const* in_tab, void* const* out_tab, int njobs,
                      hipStream_t st);

// Plans chosen by the tuner, per m, reused by later batches in the process.
static std::mutex g_tuned_mu;
static std::map<int, int> g_tuned_emax;

static int tuned_emax(int m) {
  std::lock_guard<std::mutex> g(g_tuned_mu);
  auto it = g_tuned_emax.find(m);
  return it == g_tuned_emax.end() ? 14 : it->second;
}

static size_t generic_lds() { return (size_t)((1 << kBLogE) + (1 << kBLogE) / 32 + 1) * sizeof(float); }

static int run_group(const fdwt_batch::Group& g, hipStream_t st) {
  const int np = p2_plan_passes(g.m, g.emax);
  for (int k = 0; k < np; ++k)
    if (int rc = fwt_p2_group_pass(g.m, g.emax, k, (const void* const*)g.d_in, g.d_out, g.njobs, st)) return rc;
  return FDWT_OK;
}
}  // namespace fdwt

extern "C" {

int fdwt_batch_create(int n_jobs, const fdwt_batch_job* jobs, int precision, fdwt_batch** out) {
  if (!out || !jobs || n_jobs < 1 || n_jobs > (1 << 20)) return fail(FDWT_EINVAL, "bad batch arguments");
  *out = nullptr;
  if (precision != FDWT_PREC_F32 && precision != FDWT_PREC_BF16X2 && precision != FDWT_PREC_F32_GENERIC &&
      precision != FDWT_PREC_F32_ONE_LAUNCH)
    return fail(FDWT_EINVAL, "unknown precision");
  for (int j = 0; j < n_jobs; ++j) {
    if (jobs[j].m < 1 || jobs[j].m > kMaxLog2N) return fail(FDWT_EINVAL, "job m must be in 1..26");
    if (!jobs[j].in_dev || !jobs[j].out_dev) return fail(FDWT_EINVAL, "NULL job buffer");
  }
  auto* b = new fdwt_batch();
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return fail(FDWT_EDEVICE, "no HIP device");
  }
  b->n_jobs = n_jobs;
  b->prec = precision;
  auto bail = [&](int code, const char* msg) {
    (void)hipGetLastError();
    fdwt_batch_free(b);
    return fail(code, msg);
  };
  // Grouped jobs (by m, largest first) and generic ones.
  std::map<int, std::vector<int>, std::greater<int>> by_m;
  std::vector<int> generic;
  for (int j = 0; j < n_jobs; ++j) {
    b->alg_bytes += 8.0 * (double)(int64_t(1) << jobs[j].m);
    if (precision == FDWT_PREC_F32 && jobs[j].m >= 7) by_m[jobs[j].m].push_back(j);
    else generic.push_back(j);
  }
  for (auto& kv : by_m) {
    fdwt_batch::Group g;
    g.m = kv.first;
    g.emax = tuned_emax(kv.first);
    g.njobs = (int)kv.second.size();
    std::vector<void*> hin, hout;
    for (int j : kv.second) {
      hin.push_back((void*)jobs[j].in_dev);
      hout.push_back((void*)jobs[j].out_dev);
      g.in_place |= jobs[j].in_dev == jobs[j].out_dev;
    }
    if (hipMalloc((void**)&g.d_in, hin.size() * sizeof(void*)) != hipSuccess ||
        hipMalloc((void**)&g.d_out, hout.size() * sizeof(void*)) != hipSuccess) {
      b->groups.push_back(g);
      return bail(FDWT_ENOMEM, "batch allocation failed");
    }
    b->groups.push_back(g);
    if (hipMemcpy(g.d_in, hin.data(), hin.size() * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g.d_out, hout.data(), hout.size() * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess)
      return bail(FDWT_EDEVICE, "batch upload failed");
  }
  if (!generic.empty()) {
    std::vector<BJob> hj;
    std::vector<BItem> hi;
    std::vector<int> ms;
    for (int j : generic) ms.push_back(jobs[j].m);
    int maxpass = 0;
    if (build_items(ms, hj, hi, b->level_begin, maxpass, precision == FDWT_PREC_F32_ONE_LAUNCH))
      return bail(FDWT_EUNSUPPORTED, "job needs too many passes");
    for (size_t i = 0; i < generic.size(); ++i) {
      hj[i].in = jobs[generic[i]].in_dev;
      hj[i].out = jobs[generic[i]].out_dev;
    }
    b->n_levels = maxpass;
    b->n_items = (int)hi.size();
    if (hi.size() > (size_t)(INT32_MAX - kBChunk)) return bail(FDWT_EINVAL, "batch too large");
    if (hipMalloc(&b->d_jobs, hj.size() * sizeof(BJob)) != hipSuccess ||
        hipMalloc(&b->d_items, hi.size() * sizeof(BItem)) != hipSuccess)
      return bail(FDWT_ENOMEM, "batch allocation failed");
    if (hipMemcpy(b->d_jobs, hj.data(), hj.size() * sizeof(BJob), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_items, hi.data(), hi.size() * sizeof(BItem), hipMemcpyHostToDevice) != hipSuccess)
      return bail(FDWT_EDEVICE, "batch upload failed");
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch_fwd, kBThreads, generic_lds()) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
      return bail(FDWT_EDEVICE, "occupancy query failed");
    for (int k = 0; k < maxpass; ++k)
      b->grid_per_level[k] =
          std::max(1, std::min(b->level_begin[k + 1] - b->level_begin[k], std::max(1, per_cu) * cus));
    if (precision == FDWT_PREC_F32_ONE_LAUNCH) {
      b->one_launch = true;
      if (hipMalloc((void**)&b->d_ctl, sizeof(BCtl)) != hipSuccess ||
          hipMalloc((void**)&b->d_done, hj.size() * kBMaxPass * sizeof(int)) != hipSuccess)
        return bail(FDWT_ENOMEM, "batch allocation failed");
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_batch_one, kBThreads, generic_lds()) !=
          hipSuccess)
        return bail(FDWT_EDEVICE, "occupancy query failed");
      const int tickets = (b->n_items + kBChunk - 1) / kBChunk;
      b->one_grid = std::max(1, std::min(tickets, std::max(1, occ) * cus));
      // Wait limit: FDWT_BATCH_WAIT_MS (default 2000) of the device wall clock
      // (kHz rate reported by HIP); 0 makes every wait give up (tests).
      int khz = 0;
      if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) != hipSuccess || khz <= 0)
        khz = 100000;
      const char* e = getenv("FDWT_BATCH_WAIT_MS");
      const long ms = e ? std::max(0L, std::min(60000L, atol(e))) : 2000L;
      b->timeout_ticks = (uint64_t)khz * (uint64_t)ms;
    }
  }
  *out = b;
  return FDWT_OK;
}

int fdwt_batch_run(fdwt_batch* b, void* stream) {
  if (!b) return fail(FDWT_EINVAL, "NULL batch");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t tb = timed_begin(st);
  for (const auto& g : b->groups)
    if (int rc = run_group(g, st)) return rc;
  if (b->one_launch) {
    const int nc = b->n_jobs * kBMaxPass;
    hipLaunchKernelGGL(k_batch_reset, dim3((nc + 255) / 256), dim3(256), 0, st, b->d_ctl, b->d_done, nc);
    hipLaunchKernelGGL(k_batch_one, dim3(b->one_grid), dim3(kBThreads), generic_lds(), st, b->d_jobs, b->d_items,
                       b->n_items, b->d_ctl, b->d_done, b->timeout_ticks);
    FDWT_HIP(hipGetLastError());
  } else {
    for (int k = 0; k < b->n_levels; ++k) {
      const int n = b->level_begin[k + 1] - b->level_begin[k];
      hipLaunchKernelGGL(k_batch_fwd, dim3(b->grid_per_level[k]), dim3(kBThreads), generic_lds(), st, b->d_jobs,
                         b->d_items + b->level_begin[k], n, b->prec);
      FDWT_HIP(hipGetLastError());
    }
  }
  timed_end(tb, st, FDWT_TC_BATCH, b->alg_bytes);
  return FDWT_OK;
}

int fdwt_batch_autotune(fdwt_batch* b, int reps, void* stream) {
  if (!b) return fail(FDWT_EINVAL, "NULL batch");
  if (reps < 1 || reps > 1000) return fail(FDWT_EINVAL, "reps must be in 1..1000");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  FDWT_HIP(hipEventCreate(&e0));
  FDWT_HIP(hipEventCreate(&e1));
  int rc = FDWT_OK;
  for (auto& g : b->groups) {
    if (g.in_place) continue;  // timing runs would overwrite the inputs
    std::vector<int> cands;
    for (int e = 14; e >= 10; --e) {
      bool dup = false;
      for (int c : cands) dup |= p2_plans_equal(g.m, c, e);
      if (!dup) cands.push_back(e);
    }
    if (cands.size() < 2) continue;
    float best = 0.0f;
    int best_e = g.emax;
    for (int e : cands) {
      fdwt_batch::Group t = g;
      t.emax = e;
      std::vector<float> ms;
      rc = run_group(t, st);  // warm-up
      for (int r = 0; r < reps && !rc; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) rc = fail(FDWT_EDEVICE, "event record failed");
        if (!rc) rc = run_group(t, st);
        if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = fail(FDWT_EDEVICE, "event record failed");
        float v = 0.0f;
        if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&v, e0, e1) != hipSuccess))
          rc = fail(FDWT_EDEVICE, "event timing failed");
        ms.push_back(v);
      }
      if (rc) break;
      std::nth_element(ms.begin(), ms.begin() + ms.size() / 2, ms.end());
      const float med = ms[ms.size() / 2];
      if (best == 0.0f || med < best) {
        best = med;
        best_e = e;
      }
    }
    if (rc) break;
    g.emax = best_e;
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned_emax[g.m] = best_e;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int fdwt_batch_describe(const fdwt_batch* b, int cap, int* m, int* emax, int* njobs, int* n_groups) {
  if (!b || !n_groups) return fail(FDWT_EINVAL, "NULL argument");
  *n_groups = (int)b->groups.size();
  for (int i = 0; i < (int)b->groups.size() && i < cap; ++i) {
    if (m) m[i] = b->groups[i].m;
    if (emax) emax[i] = b->groups[i].emax;
    if (njobs) njobs[i] = b->groups[i].njobs;
  }
  return FDWT_OK;
}

int fdwt_batch_check(fdwt_batch* b, void* stream) {
  if (!b) return fail(FDWT_EINVAL, "NULL batch");
  FDWT_HIP(hipStreamSynchronize((hipStream_t)stream));
  if (b->one_launch) {
    BCtl c{};
    FDWT_HIP(hipMemcpy(&c, b->d_ctl, sizeof(c), hipMemcpyDeviceToHost));
    if (c.error) return fail(FDWT_ETIMEOUT, "a wait of the one-launch batch gave up (outputs incomplete)");
  }
  return FDWT_OK;
}

int fdwt_batch_schedule(int n_jobs, const int* m, int cap, int* job, int* pass, int* tile, int* need, int* n_items,
                        int* chunk) {
  if (n_jobs < 1 || n_jobs > (1 << 20) || !m || !n_items || cap < 0) return fail(FDWT_EINVAL, "bad schedule arguments");
  std::vector<int> ms(m, m + n_jobs);
  for (int v : ms)
    if (v < 1 || v > kMaxLog2N) return fail(FDWT_EINVAL, "job m must be in 1..26");
  std::vector<BJob> hj;
  std::vector<BItem> hi;
  int lb[kBMaxPass + 1] = {0}, maxpass = 0;
  if (build_items(ms, hj, hi, lb, maxpass, true)) return fail(FDWT_EUNSUPPORTED, "job needs too many passes");
  *n_items = (int)hi.size();
  if (chunk) *chunk = kBChunk;
  for (int i = 0; i < cap && i < (int)hi.size(); ++i) {
    if (job) job[i] = hi[i].job;
    if (pass) pass[i] = hi[i].pass;
    if (tile) tile[i] = hi[i].tile;
    if (need) need[i] = hi[i].pass > 0 ? hj[hi[i].job].ntiles[hi[i].pass - 1] : 0;
  }
  return FDWT_OK;
}

void fdwt_batch_free(fdwt_batch* b) {
  if (!b) return;
  bool any = b->d_jobs || b->d_items || b->d_ctl || b->d_done;
  for (auto& g : b->groups) any |= g.d_in || g.d_out;
  if (any) (void)hipDeviceSynchronize();
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_ctl) (void)hipFree(b->d_ctl);
  if (b->d_done) (void)hipFree(b->d_done);
  for (auto& g : b->groups) {
    if (g.d_in) (void)hipFree(g.d_in);
    if (g.d_out) (void)hipFree(g.d_out);
  }
  delete b;
}

}  // extern "C"
