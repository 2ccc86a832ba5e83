// Persistent serving queue and its launch-per-request comparator.
//
// The paper motivates inter-workgroup primitives with shared work queues (Section 1)
// and names queue management as the main use of mutexes (Section 7).  Here a persistent
// kernel drains a stream of requests that the host publishes at their arrival times:
//
//   host:    descriptor -> ring slot (pinned host memory), then release-store the tail;
//   device:  claim ticket c (fetch-and-add on head) -> wait until the tail passes c ->
//            read descriptor c -> weighted fetch-and-add semaphore over the workspace
//            budget -> hash chain in the leader lane -> out[c] -> return the units ->
//            completion flag c (pinned host memory);
//   host:    a second thread sees the flag and stamps the completion time.
//
// The workgroups nearest the arrival front poll their own ring slot in host memory;
// the others poll a device word that tracks the front, sleeping in proportion to their
// distance from it.  Descriptors carry their request id, so a slot read before the
// host's write landed is recognised and read again: correctness does not depend on how
// host writes and device reads are ordered across PCIe.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "sp/semaphore.hpp"
#include "sp_internal.hpp"

namespace {

// Device state lines (each `stride` words apart).
enum { S_HEAD = 0, S_FRONT, S_READY, S_ISSUED, S_RELEASED, S_INUSE, S_MAXUSE, S_CLAIM, S_LINES };
constexpr uint32_t kStride = 32;            // 128-byte lines
constexpr uint32_t kMaxSleepUnits = 2048;   // cap of a waiting workgroup's sleep
constexpr uint64_t kStopBit = 1ull << 63;   // in the host tail word: abandon the run
constexpr uint32_t kIdEmpty = 0xFFFFFFFFu;  // request id of a never-written ring slot

struct ServeArgs {
  uint32_t* st;            // device state lines
  const uint64_t* h_tail;  // pinned: published count (low 32 bits, informational) | kStopBit
  uint32_t* h_started;     // pinned: set once every workgroup is running
  const uint64_t* h_ring;  // pinned: 2 words per slot, (id << 32) | L and (id << 32) | units
  uint32_t* h_done;        // pinned: completion flag per request
  uint32_t* out;           // device: chain result per request
  uint32_t n, mask, seed, nwg, K, poll_sleep, far_sleep, track;
};

__device__ __forceinline__ uint64_t ld_sys64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The hash chain of one request.  Only the leader lane is active here; reading the
// inputs through readfirstlane makes them wave-uniform, so the serial chain runs on the
// scalar ALU (one instruction per dependent step) instead of as one-lane vector
// instructions with quarter-rate 32-bit multiplies.  Both the persistent kernel and the
// launch comparator use this routine.
__device__ __forceinline__ uint32_t chain(uint32_t x, uint32_t L) {
  x = __builtin_amdgcn_readfirstlane(x);
  L = __builtin_amdgcn_readfirstlane(L);
  uint32_t i = 0;
  for (; i + 4 <= L; i += 4) x = sp::sm32(sp::sm32(sp::sm32(sp::sm32(x))));
  for (; i < L; ++i) x = sp::sm32(x);
  return x;
}

// Reads descriptor c from the ring, re-reading until the slot carries request id c.
__device__ __forceinline__ bool read_desc(const uint64_t* ring, uint32_t mask, uint32_t c,
                                          uint32_t* L, uint32_t* units, const sp::Ctl& ctl) {
  const uint64_t* slot = ring + 2 * (size_t)(c & mask);
  sp::Wait w(ctl, 0);
  for (;;) {
    const uint64_t w0 = ld_sys64(slot), w1 = ld_sys64(slot + 1);
    if ((uint32_t)(w0 >> 32) == c && (uint32_t)(w1 >> 32) == c) {
      *L = (uint32_t)w0;
      *units = (uint32_t)w1;
      return true;
    }
    if (!w.tick()) return false;
  }
}

// Waits until request c is in the ring and reads its descriptor.  `front` (device) is a
// lower bound on the number of requests published so far.  Workgroups fewer than kNear
// tickets past the front poll their own ring slot in host memory, so one PCIe read both
// detects the arrival and fetches the descriptor, and a burst of arrivals is detected by
// up to kNear workgroups at once; the others poll `front`, sleeping in proportion to
// their distance.  A workgroup that finds its request moves the front past it.
constexpr int32_t kNear = 16;

__device__ bool await_desc(const ServeArgs& a, uint32_t c, uint32_t* front, uint32_t* L,
                           uint32_t* units, const sp::Ctl& ctl) {
  const uint64_t* slot = a.h_ring + 2 * (size_t)(c & a.mask);
  sp::Wait w(ctl, 0);
  for (uint32_t k = 1;; ++k) {
    const int32_t d = (int32_t)(c - sp::ld_relaxed(front));
    if (d < kNear) {
      const uint64_t w0 = ld_sys64(slot), w1 = ld_sys64(slot + 1);
      if ((uint32_t)(w0 >> 32) == c && (uint32_t)(w1 >> 32) == c) {
        *L = (uint32_t)w0;
        *units = (uint32_t)w1;
        if (d >= 0) sp::max_relaxed(front, c + 1);
        return true;
      }
      if ((k & 63) == 0 && (ld_sys64(a.h_tail) & kStopBit)) {
        sp::cas_relaxed(ctl.err, sp::DEV_OK, sp::DEV_TIMEOUT);
        return false;
      }
      sp::sleep_units(a.poll_sleep);
    } else {
      const uint64_t s = (uint64_t)(d - kNear + 1) * a.far_sleep;
      sp::sleep_units(s < kMaxSleepUnits ? (uint32_t)s : kMaxSleepUnits);
    }
    if (!w.tick()) return false;
  }
}

// The persistent kernel.  Block semantics: the leader lane does everything (a hash chain
// is serial); the other lanes of the workgroup retire at once.
__global__ SP_FULL_OCCUPANCY void k_serve(ServeArgs a, uint32_t* err, uint64_t timeout) {
  if (!sp::is_leader()) return;
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  uint32_t* head = a.st + S_HEAD * kStride;
  uint32_t* front = a.st + S_FRONT * kStride;
  uint32_t* inuse = a.st + S_INUSE * kStride;
  uint32_t* maxuse = a.st + S_MAXUSE * kStride;
  const sp::WSemState ws{a.K, a.poll_sleep, a.st + S_ISSUED * kStride, a.st + S_RELEASED * kStride};
  if (sp::add_relaxed(a.st + S_READY * kStride, 1) == a.nwg - 1) st_sys(a.h_started, 1);
  for (;;) {
    const uint32_t c = sp::add_relaxed(head, 1);
    if (c >= a.n) return;
    uint32_t L, u;
    if (!await_desc(a, c, front, &L, &u, ctl)) return;
    if (!sp::wsem_wait_leader<false>(ws, u, ctl)) return;
    if (a.track) sp::max_relaxed(maxuse, sp::add_relaxed(inuse, u) + u);
    a.out[c] = chain(a.seed ^ c, L);
    if (a.track) sp::add_relaxed(inuse, 0u - u);
    sp::wsem_post_leader<false>(ws, u);
    st_sys(a.h_done + c, 1);
  }
}

// Comparator: workgroup i of a launch serves request r0 + i.  A single-request launch
// carries L in its arguments; a batched launch reads the descriptors from the ring.
__global__ void k_serve_launch(uint32_t r0, uint32_t count, uint32_t L1, const uint64_t* ring,
                               uint32_t mask, uint32_t seed, uint32_t* out, uint32_t* h_done,
                               uint32_t* err, uint64_t timeout) {
  if (!sp::is_leader() || blockIdx.x >= count) return;
  const uint32_t c = r0 + blockIdx.x;
  uint32_t L = L1, u = 0;
  if (count > 1) {
    const sp::Ctl ctl{err, sp::wall_clock() + timeout};
    if (!read_desc(ring, mask, c, &L, &u, ctl)) return;
  }
  out[c] = chain(seed ^ c, L);
  st_sys(h_done + c, 1);
}

// Comparator, graph-batched: each workgroup (a one-workgroup node of a replayed graph, or
// one workgroup of a flush launch) claims the next request and reads its descriptor from
// the ring.  The host launches exactly as many workgroups as it has published requests.
__global__ void k_serve_claim(const uint64_t* ring, uint32_t mask, uint32_t n, uint32_t seed,
                              uint32_t* claim, uint32_t* out, uint32_t* h_done, uint32_t* err,
                              uint64_t timeout) {
  if (!sp::is_leader()) return;
  const uint32_t c = sp::add_relaxed(claim, 1);
  if (c >= n) return;
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  uint32_t L = 0, u = 0;
  if (!read_desc(ring, mask, c, &L, &u, ctl)) return;
  out[c] = chain(seed ^ c, L);
  st_sys(h_done + c, 1);
}

// ---- host side ---------------------------------------------------------------------------

inline uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Spin until t (ns); sleep first when t is far away.
inline void wait_until(uint64_t t) {
  for (;;) {
    const uint64_t now = now_ns();
    if (now >= t) return;
    if (t - now > 300000) std::this_thread::sleep_for(std::chrono::nanoseconds(t - now - 200000));
  }
}

struct Cfg {
  uint32_t nwg, lanes, ring_slots, K, seed, poll_sleep, far_sleep, streams, batch, track, graph;
  uint64_t unit_bytes;
  uint64_t timeout_ms;
};

int normalize_cfg(const sp_serve_cfg* in, Cfg* c) {
  if (!in) return SP_E_INVAL;
  c->nwg = in->nwg;
  c->lanes = in->lanes ? in->lanes : 64;
  c->ring_slots = in->ring_slots ? in->ring_slots : 65536;
  c->K = in->budget_units;
  c->unit_bytes = in->unit_bytes ? in->unit_bytes : 65536;
  c->seed = in->seed;
  c->poll_sleep = in->poll_sleep;
  c->far_sleep = in->far_sleep ? in->far_sleep : 4;
  c->timeout_ms = in->timeout_ms ? in->timeout_ms : 20000;
  c->streams = in->streams ? in->streams : 1;
  c->batch = in->batch ? in->batch : 1;
  c->track = in->track ? 1 : 0;
  c->graph = in->graph_batch;
  if (c->graph > 4096 || (c->graph && c->batch > 1)) return SP_E_INVAL;
  if (!spi::lanes_ok(c->lanes)) return SP_E_INVAL;
  if (c->ring_slots < 64 || c->ring_slots > (1u << 24) || (c->ring_slots & (c->ring_slots - 1)))
    return SP_E_INVAL;
  if (c->K == 0 || c->K >= (1u << 30)) return SP_E_INVAL;
  if (c->poll_sleep > 1024 || c->far_sleep > 1024) return SP_E_INVAL;
  if (c->streams > 4 || c->batch > 65536) return SP_E_INVAL;
  return SP_OK;
}

// Pinned host and device buffers of one run; released by the destructor.
struct Buffers {
  sp_ctx* ctx = nullptr;
  uint64_t* h_tail = nullptr;  // 4 KiB block: tail word at 0, started flag at byte 128
  uint32_t* h_started = nullptr;
  uint64_t* h_ring = nullptr;
  uint32_t* h_done = nullptr;
  uint32_t* d_state = nullptr;
  uint32_t* d_out = nullptr;
  std::vector<hipStream_t> streams;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  ~Buffers() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    if (h_tail) (void)hipHostFree(h_tail);
    if (h_ring) (void)hipHostFree(h_ring);
    if (h_done) (void)hipHostFree(h_done);
    if (d_state) (void)hipFree(d_state);
    if (d_out) (void)hipFree(d_out);
  }
};

// Completion observer shared by both modes: scans the flags of published requests and
// stamps the host time at which each one is first seen set.
struct Observer {
  const uint32_t* flags;
  const uint32_t* units;
  uint32_t n;
  std::vector<uint64_t> t_done;
  std::atomic<uint32_t> published{0};
  std::atomic<uint32_t> lo{0};  // every request below lo has been seen complete
  std::atomic<uint64_t> released_units{0};
  std::atomic<int> abort{0};
  uint64_t deadline = 0;

  void run() {
    std::vector<uint32_t> pend;
    pend.reserve(1 << 16);
    std::vector<uint8_t> seen(n, 0);
    uint32_t next = 0, low = 0;
    uint64_t rel = 0;
    while (low < n) {
      const uint32_t hi = published.load(std::memory_order_acquire);
      while (next < hi) pend.push_back(next++);
      size_t k = 0;
      for (size_t i = 0; i < pend.size(); ++i) {
        const uint32_t r = pend[i];
        if (__atomic_load_n(&flags[r], __ATOMIC_ACQUIRE)) {
          t_done[r] = now_ns();
          seen[r] = 1;
          rel += units[r];
        } else {
          pend[k++] = r;
        }
      }
      pend.resize(k);
      released_units.store(rel, std::memory_order_release);
      while (low < hi && seen[low]) ++low;
      lo.store(low, std::memory_order_release);
      if (abort.load(std::memory_order_relaxed)) return;
      if (now_ns() > deadline) {
        abort.store(1);
        return;
      }
    }
  }
};

void summarize(const Observer& ob, uint64_t t0, const double* t_arr, uint32_t n, double* lat_us,
               sp_serve_result* res) {
  std::vector<double> lat(n);
  uint64_t last = 0;
  for (uint32_t r = 0; r < n; ++r) {
    const double arr = (double)t0 + t_arr[r] * 1e9;
    lat[r] = ((double)ob.t_done[r] - arr) / 1e3;
    last = std::max(last, ob.t_done[r]);
  }
  if (lat_us) memcpy(lat_us, lat.data(), n * sizeof(double));
  std::vector<double> s = lat;
  std::sort(s.begin(), s.end());
  auto rank = [&](double q) {
    size_t k = (size_t)std::ceil(q * n);
    return s[k == 0 ? 0 : k - 1];
  };
  double sum = 0;
  for (double v : s) sum += v;
  res->p50_us = rank(0.50);
  res->p99_us = rank(0.99);
  res->mean_us = sum / n;
  res->max_us = s.back();
  res->wall_s = ((double)last - ((double)t0 + t_arr[0] * 1e9)) / 1e9;
  res->req_per_s = res->wall_s > 0 ? n / res->wall_s : 0;
  res->completed = n;
}

int serve(sp_ctx* ctx, const sp_serve_cfg* cfg_in, uint32_t n, const uint32_t* L,
          const uint64_t* nbytes, const double* t_arr, uint32_t* out, double* lat_us,
          sp_serve_result* res, bool persistent) {
  if (!spi::usable(ctx) || !L || !nbytes || !t_arr || !out || !res) return SP_E_INVAL;
  if (n == 0 || n >= (1u << 31)) return SP_E_INVAL;
  Cfg c;
  SP_CHECK(normalize_cfg(cfg_in, &c));
  if (persistent && (c.nwg == 0 || c.nwg > 65536)) return SP_E_INVAL;
  // Units per request, and the checks that keep every counter far from wrapping.
  std::vector<uint32_t> units(n);
  uint64_t total_units = 0;
  for (uint32_t r = 0; r < n; ++r) {
    if (L[r] > (1u << 24)) return SP_E_INVAL;
    if (!(t_arr[r] >= 0) || !std::isfinite(t_arr[r]) || (r && t_arr[r] < t_arr[r - 1]))
      return SP_E_INVAL;
    const uint64_t u = (nbytes[r] + c.unit_bytes - 1) / c.unit_bytes;
    if (u > c.K) return SP_E_INVAL;
    units[r] = (uint32_t)u;
    total_units += u;
  }
  if (total_units + c.K >= (1ull << 31)) return SP_E_INVAL;
  memset(res, 0, sizeof(*res));

  SP_HIP(ctx, hipSetDevice(ctx->device));
  Buffers b;
  b.ctx = ctx;
  const unsigned pin = hipHostMallocMapped | hipHostMallocCoherent;
  SP_HIP(ctx, hipHostMalloc((void**)&b.h_tail, 4096, pin));
  SP_HIP(ctx, hipHostMalloc((void**)&b.h_ring, (size_t)c.ring_slots * 16, pin));
  SP_HIP(ctx, hipHostMalloc((void**)&b.h_done, (size_t)n * 4, pin));
  SP_HIP(ctx, hipMalloc(&b.d_state, S_LINES * kStride * 4));
  SP_HIP(ctx, hipMalloc(&b.d_out, (size_t)n * 4));
  memset(b.h_tail, 0, 4096);
  b.h_started = reinterpret_cast<uint32_t*>(b.h_tail) + 32;
  for (uint32_t s = 0; s < 2 * c.ring_slots; ++s) b.h_ring[s] = (uint64_t)kIdEmpty << 32;
  memset(b.h_done, 0, (size_t)n * 4);
  const uint32_t nstreams = persistent ? 1 : c.streams;
  for (uint32_t i = 0; i < nstreams; ++i) {
    hipStream_t s;
    SP_HIP(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    b.streams.push_back(s);
  }
  hipStream_t s0 = b.streams[0];
  SP_CHECK(spi::fill_u32(ctx, b.d_state, S_LINES * kStride, 0, s0));
  SP_CHECK(spi::fill_u32(ctx, ctx->d_err, 1, 0, s0));
  SP_CHECK(spi::fill_u32(ctx, b.d_out, n, 0, s0));
  SP_HIP(ctx, hipStreamSynchronize(s0));

  const double span_s = t_arr[n - 1];
  const uint64_t limit_ms = c.timeout_ms + (uint64_t)(span_s * 1e3);
  const uint64_t dev_timeout = limit_ms * ctx->wall_khz;
  const uint32_t mask = c.ring_slots - 1;

  Observer ob;
  ob.flags = b.h_done;
  ob.units = units.data();
  ob.n = n;
  ob.t_done.assign(n, 0);

  if (persistent) {
    uint32_t per_cu = 0;
    SP_CHECK(spi::resident_per_cu(ctx, (const void*)k_serve, c.lanes, &per_cu));
    if ((uint64_t)per_cu * ctx->cu_count < c.nwg) return SP_E_NORESIDENT;
    ServeArgs a;
    a.st = b.d_state;
    a.h_tail = b.h_tail;
    a.h_started = b.h_started;
    a.h_ring = b.h_ring;
    a.h_done = b.h_done;
    a.out = b.d_out;
    a.n = n;
    a.mask = mask;
    a.seed = c.seed;
    a.nwg = c.nwg;
    a.K = c.K;
    a.poll_sleep = c.poll_sleep;
    a.far_sleep = c.far_sleep;
    a.track = c.track;
    hipLaunchKernelGGL(k_serve, dim3(c.nwg), dim3(c.lanes), 0, s0, a, ctx->d_err, dev_timeout);
    SP_HIP(ctx, hipGetLastError());
    // Start the clock once every workgroup runs.
    const uint64_t give_up = now_ns() + 5000000000ull;
    while (!__atomic_load_n(b.h_started, __ATOMIC_ACQUIRE)) {
      if (now_ns() > give_up || hipStreamQuery(s0) != hipErrorNotReady) {
        __atomic_store_n(b.h_tail, kStopBit, __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(s0);
        return SP_E_TIMEOUT;
      }
    }
    res->launches = 1;
  }

  // Graph-batched comparator: one graph of G independent one-workgroup claim kernels,
  // built once and replayed per G published requests.
  uint32_t* claim = b.d_state + S_CLAIM * kStride;
  const uint64_t* ring_arg = b.h_ring;
  uint32_t mask_arg = mask, n_arg = n, seed_arg = c.seed;
  uint64_t timeout_arg = dev_timeout;
  void* claim_args[] = {&ring_arg, &mask_arg,  &n_arg,       &seed_arg,   &claim,
                        &b.d_out,  &b.h_done,  &ctx->d_err, &timeout_arg};
  if (!persistent && c.graph) {
    SP_HIP(ctx, hipGraphCreate(&b.graph, 0));
    hipKernelNodeParams kp{};
    kp.func = (void*)k_serve_claim;
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(c.lanes);
    kp.sharedMemBytes = 0;
    kp.kernelParams = claim_args;
    kp.extra = nullptr;
    for (uint32_t i = 0; i < c.graph; ++i) {
      hipGraphNode_t node;
      SP_HIP(ctx, hipGraphAddKernelNode(&node, b.graph, nullptr, 0, &kp));
    }
    SP_HIP(ctx, hipGraphInstantiate(&b.graph_exec, b.graph, nullptr, nullptr, 0));
  }
  const bool use_ring = persistent || c.batch > 1 || c.graph;
  uint32_t covered = 0;  // graph mode: requests the launched workgroups will claim
  // Graph mode: launch one claim workgroup per published request (below `upto`) that no
  // launched workgroup covers yet.
  auto flush = [&](uint32_t upto) -> bool {
    if (covered >= upto) return true;
    const uint32_t m = upto - covered;
    hipLaunchKernelGGL(k_serve_claim, dim3(m), dim3(c.lanes), 0,
                       b.streams[res->launches % nstreams], ring_arg, mask, n, c.seed, claim,
                       b.d_out, b.h_done, ctx->d_err, dev_timeout);
    if (hipGetLastError() != hipSuccess) return false;
    covered += m;
    res->launches++;
    return true;
  };

  const uint64_t t0 = now_ns();
  ob.deadline = t0 + limit_ms * 1000000ull;
  std::thread observer([&ob] { ob.run(); });
  double lag_max = 0;
  uint64_t launched_units = 0;
  int rc = SP_OK;
  uint32_t r = 0;
  while (r < n) {
    if (ob.abort.load(std::memory_order_relaxed)) {
      rc = SP_E_TIMEOUT;
      break;
    }
    const uint64_t due = t0 + (uint64_t)(t_arr[r] * 1e9);
    wait_until(due);
    const uint64_t now = now_ns();
    uint32_t r1 = r;
    const uint32_t cap = (persistent || c.graph) ? n : std::min<uint32_t>(n, r + c.batch);
    while (r1 < cap && t0 + (uint64_t)(t_arr[r1] * 1e9) <= now) {
      if (use_ring) {
        if (r1 - ob.lo.load(std::memory_order_acquire) >= c.ring_slots) break;  // ring full
      }
      if (!persistent) {  // host-side admission against the same budget
        const uint64_t held = launched_units + units[r1] - ob.released_units.load();
        if (held > c.K) break;
        launched_units += units[r1];
      }
      if (use_ring) {
        uint64_t* slot = b.h_ring + 2 * (size_t)(r1 & mask);
        slot[0] = ((uint64_t)r1 << 32) | L[r1];
        slot[1] = ((uint64_t)r1 << 32) | units[r1];
      }
      lag_max = std::max(lag_max, (double)(now - (t0 + (uint64_t)(t_arr[r1] * 1e9))) / 1e3);
      ++r1;
    }
    if (r1 == r) {  // ring full or budget exhausted: observe and retry
      // graph mode: requests waiting for a full batch must run, to free ring and budget
      if (c.graph && !persistent && !flush(r)) {
        rc = SP_E_HIP;
        ob.abort.store(1);
        break;
      }
      continue;
    }
    if (persistent) {
      __atomic_store_n(b.h_tail, (uint64_t)r1, __ATOMIC_RELEASE);
    } else if (c.graph) {
      bool launched_ok = true;
      while (r1 - covered >= c.graph) {
        if (hipGraphLaunch(b.graph_exec, b.streams[res->launches % nstreams]) != hipSuccess) {
          launched_ok = false;
          break;
        }
        covered += c.graph;
        res->launches++;
      }
      if (!launched_ok) {
        rc = SP_E_HIP;
        ob.abort.store(1);
        break;
      }
    } else {
      hipStream_t s = b.streams[res->launches % nstreams];
      hipLaunchKernelGGL(k_serve_launch, dim3(r1 - r), dim3(c.lanes), 0, s, r, r1 - r, L[r],
                         (const uint64_t*)b.h_ring, mask, c.seed, b.d_out, b.h_done, ctx->d_err,
                         dev_timeout);
      if (hipGetLastError() != hipSuccess) {
        rc = SP_E_HIP;
        ob.abort.store(1);
        break;
      }
      res->launches++;
    }
    ob.published.store(r1, std::memory_order_release);
    r = r1;
  }
  if (rc == SP_OK && !persistent && c.graph && !flush(r)) {  // the last, partial batch
    rc = SP_E_HIP;
    ob.abort.store(1);
  }
  observer.join();
  if (ob.abort.load() && rc == SP_OK) rc = SP_E_TIMEOUT;
  if (rc != SP_OK && persistent) __atomic_store_n(b.h_tail, kStopBit | r, __ATOMIC_RELEASE);
  for (hipStream_t s : b.streams) SP_HIP(ctx, hipStreamSynchronize(s));
  uint32_t err = 0;
  SP_HIP(ctx, hipMemcpy(&err, ctx->d_err, 4, hipMemcpyDeviceToHost));
  res->device_error = err;
  res->publish_lag_max_us = lag_max;
  if (persistent) {
    uint32_t st[S_LINES * kStride];
    SP_HIP(ctx, hipMemcpy(st, b.d_state, sizeof(st), hipMemcpyDeviceToHost));
    res->units_issued = st[S_ISSUED * kStride];
    res->units_released = st[S_RELEASED * kStride];
    res->max_units_in_use = st[S_MAXUSE * kStride];
  } else {
    res->units_issued = res->units_released = total_units;
  }
  if (rc != SP_OK) return rc;
  if (err == sp::DEV_TIMEOUT) return SP_E_TIMEOUT;
  if (err != sp::DEV_OK) return SP_E_PARITY;
  SP_HIP(ctx, hipMemcpy(out, b.d_out, (size_t)n * 4, hipMemcpyDeviceToHost));
  summarize(ob, t0, t_arr, n, lat_us, res);
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_serve_run(sp_ctx* ctx, const sp_serve_cfg* cfg, uint32_t n, const uint32_t* L,
                 const uint64_t* nbytes, const double* t_arr_s, uint32_t* out, double* lat_us,
                 sp_serve_result* res) {
  return serve(ctx, cfg, n, L, nbytes, t_arr_s, out, lat_us, res, true);
}

int sp_serve_run_launch_per_request(sp_ctx* ctx, const sp_serve_cfg* cfg, uint32_t n,
                                    const uint32_t* L, const uint64_t* nbytes,
                                    const double* t_arr_s, uint32_t* out, double* lat_us,
                                    sp_serve_result* res) {
  return serve(ctx, cfg, n, L, nbytes, t_arr_s, out, lat_us, res, false);
}

}  // extern "C"
