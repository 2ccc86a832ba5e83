// Device-side building blocks of the synchronization primitives on gfx950.
//
// Memory model.  One gfx950 agent spans eight XCDs, each with its own L2; ordinary
// loads and stores are cached per XCD and are not coherent across XCDs.  Every word a
// primitive polls or updates is therefore accessed with agent-scope atomics, which the
// compiler emits with the coherence bits that bypass the per-XCD caches, and data that
// a primitive protects (critical sections, barrier-exchanged values) is published with
// an agent-scope release fence (write back dirty L2 lines) and consumed after an
// agent-scope acquire fence (invalidate stale L1/L2 lines).  The paper's "volatile"
// access (Section 3) maps to an agent-scope relaxed atomic load or store: a C volatile
// access may be served from the XCD's own L2 and never see another XCD's update.
//
// Block semantics (Section 3): the whole workgroup calls a primitive; thread 0 of the
// workgroup (the leader) performs every atomic; the other lanes wait at the workgroup
// barrier.  Before the leader publishes, every wavefront waits until its own stores
// have completed, so the leader's release covers stores made by other wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../sp.h"

// Kernels whose workgroups must all be resident at once are compiled for eight waves per
// SIMD (the gfx950 maximum), so that the register budget the compiler picks matches the
// occupancy the runtime reports for a cooperative launch.
#define SP_FULL_OCCUPANCY __attribute__((amdgpu_waves_per_eu(8)))

namespace sp {

// ---- agent-scope atomics ------------------------------------------------------------
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Workgroup-scope load and store: they may hit the CU's L1, which every wavefront on the
// CU shares, so a store by one workgroup reaches another on the same CU without a trip to
// memory (another CU's store is not seen until the L1 line is invalidated).
__device__ __forceinline__ uint32_t ld_cu(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_cu(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t ld_relaxed64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_relaxed(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t exch_relaxed(uint32_t* p, uint32_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t max_relaxed(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Compare-and-swap; returns the value seen (== expected on success).
__device__ __forceinline__ uint32_t cas_relaxed(uint32_t* p, uint32_t expected, uint32_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;
}

// Wait until this wavefront's outstanding vector-memory operations have completed
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their maxima).
__device__ __forceinline__ void wave_stores_complete() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Agent-scope fences.  The release fence writes back the XCD's dirty L2 lines and the
// acquire fence invalidates stale L1/L2 lines; both are asynchronous cache operations.
// An explicit vmcnt(0) wait follows each one so that the writeback has finished before
// the flag store that publishes it, and the invalidation has finished before the
// workgroup barrier lets other wavefronts load (the compiler's own wait after the
// writeback is elided when no other memory operation is outstanding).
__device__ __forceinline__ void fence_acquire() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  wave_stores_complete();
}
__device__ __forceinline__ void fence_release() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  wave_stores_complete();
}

// A workgroup-scope invalidate (buffer_inv sc0).  It costs ~310 shader clocks and is not
// serialized at the L2, unlike the agent-scope one; but it does not make another XCD's
// written-back data visible: after it, a plain load returned the old value in 28 % of
// 4.1 M message-passing trials, as many as with no invalidate at all.  Measurements only
// (sp_bench_fence kind 2, litmus variant 4); no primitive relies on it.
__device__ __forceinline__ void invalidate_workgroup_scope() {
  __asm__ __volatile__("buffer_inv sc0" ::: "memory");
  wave_stores_complete();
}

// Release store / release add: publish everything this wavefront wrote, then the flag.
__device__ __forceinline__ void st_release(uint32_t* p, uint32_t v) {
  fence_release();
  st_relaxed(p, v);
}
__device__ __forceinline__ uint32_t add_release(uint32_t* p, uint32_t v) {
  fence_release();
  return add_relaxed(p, v);
}

// Wrap-safe "monotone counter a has reached b".
__device__ __forceinline__ bool reached(uint32_t a, uint32_t b) { return (int32_t)(a - b) >= 0; }

__device__ __forceinline__ bool is_leader() { return threadIdx.x == 0; }

// ---- clocks ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t shader_clock() { return __builtin_amdgcn_s_memtime(); }
__device__ __forceinline__ uint64_t wall_clock() { return __builtin_amdgcn_s_memrealtime(); }
__device__ __forceinline__ uint32_t xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xF;  // HW_REG_XCC_ID[3:0]
}
// Identity of the CU within its XCD: HW_REG_HW_ID bits [15:8] (CU, SH and SE ids).
__device__ __forceinline__ uint32_t cu_in_xcc() {
  return (__builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4) >> 8) & 0xFF;
}

// Busy-wait `cycles` shader clocks (non-critical delays and critical-section holds).
__device__ __forceinline__ void spin_cycles(uint32_t cycles) {
  if (cycles == 0) return;
  const uint64_t t0 = shader_clock();
  while (shader_clock() - t0 < cycles) {
  }
}

__device__ __forceinline__ void sleep_units(uint32_t n) {
  for (uint32_t k = 0; k < n; ++k) __builtin_amdgcn_s_sleep(1);
}

// ---- workload hash ------------------------------------------------------------------
// splitmix32: golden-ratio increment, then the MurmurHash3 32-bit finalizer.
__device__ __forceinline__ uint32_t sm32(uint32_t x) {
  uint32_t z = x + 0x9E3779B9u;
  z = (z ^ (z >> 16)) * 0x85EBCA6Bu;
  z = (z ^ (z >> 13)) * 0xC2B2AE35u;
  return z ^ (z >> 16);
}
// Schedule key of operation j of workgroup w in stream s.
__device__ __forceinline__ uint32_t sched_key(uint32_t seed, uint32_t w, uint32_t j, uint32_t s) {
  return sm32(sm32(sm32(seed ^ s) ^ w) ^ j);
}

// ---- watchdog ---------------------------------------------------------------------------
enum : uint32_t { DEV_OK = 0, DEV_TIMEOUT = 1, DEV_PARITY = 2 };

// Per-launch control block: the device error word and the wall-clock deadline.  Every
// wait loop of every primitive checks it, so a kernel always drains in bounded time.
struct Ctl {
  uint32_t* err;
  uint64_t deadline;
};

struct Wait {
  Ctl ctl;
  uint32_t poll_sleep;
  uint32_t n;
  __device__ explicit Wait(const Ctl& c, uint32_t ps) : ctl(c), poll_sleep(ps), n(0) {}
  // One unsuccessful poll: sleep poll_sleep units; every 64 polls check the error word
  // and the deadline.  Returns false when the wait must be abandoned.
  __device__ __forceinline__ bool tick() {
    sleep_units(poll_sleep);
    if ((++n & 63) != 0) return true;
    if (ld_relaxed(ctl.err) != DEV_OK) return false;
    if (wall_clock() > ctl.deadline) {
      cas_relaxed(ctl.err, DEV_OK, DEV_TIMEOUT);
      return false;
    }
    return true;
  }
};

// ---- backoff (Section 5, Mutex) -----------------------------------------------------
struct BackoffCfg {
  uint32_t kind, imin, imax, unit;
  uint32_t* private_word;  // an uncontended word for SP_UNIT_LOAD
};

struct Backoff {
  uint32_t i;
  __device__ explicit Backoff(const BackoffCfg& c) : i(c.imin) {}
  __device__ __forceinline__ void pause(const BackoffCfg& c, uint32_t units) {
    if (c.unit == SP_UNIT_LOAD) {
      uint32_t acc = 0;
      for (uint32_t k = 0; k < units; ++k) acc += ld_relaxed(c.private_word);
      __asm__ volatile("" ::"v"(acc));
    } else {
      sleep_units(units);
    }
  }
  // Called after every failed attempt.
  __device__ __forceinline__ void operator()(const BackoffCfg& c) {
    if (c.kind == SP_BACKOFF_NONE) return;
    pause(c, i);
    if (c.kind == SP_BACKOFF_PAPER) {
      i += 1;
      if (i > c.imax) i = c.imin;
    } else {
      i = (2 * i > c.imax) ? c.imax : 2 * i;
    }
  }
};

}  // namespace sp
