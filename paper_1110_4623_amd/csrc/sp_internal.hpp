// Host-side internals of libsp.so shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sp.h"
#include "sp/atomics.hpp"

struct sp_default_entry {
  uint32_t kind;
  sp_params p;
};

struct sp_ctx {
  // Objects created from the context (barriers, mutexes, semaphores, graphs) hold a
  // reference: sp_fini releases the context's device resources at once, but the struct
  // itself lives until the last object is destroyed, so an object destroyed after
  // sp_fini (as a garbage-collecting caller may do at exit) touches no freed memory.
  int refs = 0;
  bool closed = false;
  int device = 0;
  hipDeviceProp_t prop{};
  int last_hip = 0;
  uint32_t cu_count = 0;
  uint32_t xcd_count = 0;
  uint32_t xcc_mask = 0;  // XCC ids seen at sp_init (bit i = id i)
  uint32_t wall_khz = 100000;
  uint32_t* d_err = nullptr;   // watchdog word, own 256-byte block
  uint32_t* d_scratch = nullptr;  // small staging area (4 KiB) for state readback
  // the allocation-free entry point's fixed workspace on this device (a file-scope device
  // array; its address is looked up once per device at sp_init)
  uint32_t* static_scratch = nullptr;
  uint64_t static_scratch_words = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipStream_t capture_stream = nullptr;
  hipStream_t setup_stream = nullptr;  // work done while creating objects (not the caller's)
  sp_default_entry defaults[3][2];
};

namespace spi {

// Looks up (once per device) the address of the allocation-free entry point's fixed
// workspace and records it in the context.  The context's device must be current.
int static_scratch_setup(sp_ctx* ctx);


// Records a failing HIP call in the context and returns SP_E_HIP from the caller.
#define SP_HIP(ctx, call)                                      \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) {                                    \
      if (ctx) (ctx)->last_hip = (int)e_;                      \
      return SP_E_HIP;                                         \
    }                                                          \
  } while (0)

#define SP_CHECK(expr)                  \
  do {                                  \
    int rc_ = (expr);                   \
    if (rc_ != SP_OK) return rc_;       \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// A context that can still run work (not NULL, not finalized).
inline bool usable(const sp_ctx* ctx) { return ctx && !ctx->closed; }
// Object lifetime: every create that succeeds takes a reference, every destroy drops it;
// the last drop after sp_fini deletes the context.
inline void ctx_ref(sp_ctx* ctx) { ++ctx->refs; }
inline void ctx_unref(sp_ctx* ctx) {
  if (--ctx->refs == 0 && ctx->closed) delete ctx;
}

// Normalized parameters (defaults filled, ranges clamped); returns SP_E_INVAL on bad
// values.
int normalize(const sp_ctx* ctx, const sp_params* in, sp_params* out);

inline uint32_t stride_words(const sp_params& p) { return std::max<uint32_t>(1, p.pad_bytes / 4); }

inline uint64_t timeout_ticks(const sp_ctx* ctx, const sp_params& p) {
  return (uint64_t)p.timeout_ms * ctx->wall_khz;
}

inline sp::BackoffCfg backoff_cfg(const sp_params& p, uint32_t* private_word) {
  sp::BackoffCfg c;
  c.kind = p.backoff;
  c.imin = p.backoff_min;
  c.imax = p.backoff_max;
  c.unit = p.backoff_unit;
  c.private_word = private_word;
  return c;
}

// Zero `words` uint32 at d with a kernel (no memset nodes, so launches stay capturable).
int fill_u32(sp_ctx* ctx, uint32_t* d, uint64_t words, uint32_t value, hipStream_t s);

// True while `s` is being captured into a HIP graph (sp_graph_begin): run calls then
// record their kernels and skip timing, host waits and host readbacks.
bool capturing(hipStream_t s);
// hipStreamSynchronize(s), or nothing while `s` is being captured.
int sync_unless_capturing(sp_ctx* ctx, hipStream_t s);

// Clears the watchdog word, records ev0 (nothing under capture).
int begin_timed(sp_ctx* ctx, hipStream_t s);
// Records ev1, waits for the stream, reads the watchdog word, fills st (under capture:
// zeroes st and returns SP_OK).
int end_timed(sp_ctx* ctx, hipStream_t s, sp_stats* st, uint32_t nwg, uint32_t lanes,
              uint32_t resident_per_cu, uint64_t ops);

// Workgroups of `kern` (launched with `lanes` threads) that fit on one CU at once: the
// runtime's occupancy figure checked against the kernel's own VGPR and LDS use
// (sp_resident_per_cu).
int resident_per_cu(sp_ctx* ctx, const void* kern, uint32_t lanes, uint32_t* per_cu);

inline bool lanes_ok(uint32_t lanes) { return lanes >= 64 && lanes <= 1024 && lanes % 64 == 0; }

// Device memory owned for the duration of one call; the caller synchronizes the stream
// before it goes out of scope.
struct DeviceScratch {
  void* p = nullptr;
  DeviceScratch() = default;
  DeviceScratch(const DeviceScratch&) = delete;
  DeviceScratch& operator=(const DeviceScratch&) = delete;
  ~DeviceScratch() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

inline uint32_t bucket_of(uint32_t contenders) { return contenders >= 64 ? 1u : 0u; }
// Barriers: every workgroup is a contender.  The central counter is the faster default up
// to 32 workgroups and the per-XCD barrier from 48 on (1.75 / 2.39 / 3.88 against 2.72 /
// 2.72 / 2.85 us per round at 16 / 32 / 48, 256 lanes), so the high bucket starts at 40.
inline uint32_t barrier_bucket_of(uint32_t nwg) { return nwg >= 40 ? 1u : 0u; }
// A default mutex whose bucket names the CU-cohort lock runs it only where a lock has at
// least two contenders per CU on average; below that few hand-overs stay within a CU and
// the XCD-cohort lock is faster (one lock, 16 words, M acquisitions/s, XCD-cohort
// against CU-cohort: 256 workgroups 0.78 / 0.71, 512 0.78 / 0.93, 1024 0.77 / 1.18, 2048
// 0.74 / 1.13; 2048 workgroups on 8 locks 6.58 / 6.91, on 16 locks 13.1 / 12.7).
inline bool cu_cohort_pays(uint64_t nwg, uint64_t nlocks, uint64_t cu_count) {
  return nwg >= 2 * nlocks * cu_count;
}

}  // namespace spi
