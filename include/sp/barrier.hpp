// Device-side global barriers (Section 5, Barrier; Table 4 Barrier()).
//
// Every barrier here is monotone: round r (0-based, counted by the caller) waits for
// stamp r + 1, and counters and flags are never reset inside a run, so no reset race
// exists and a 32-bit wrap is handled by signed differences.  The whole workgroup calls
// barrier_wait(); the leader (and, for the flag barriers, the master workgroup's lanes)
// do the inter-workgroup work; the call returns false if the watchdog abandoned the
// wait, and the kernel must then return.
//
// All workgroups taking part must be co-resident (Section 5: the barrier is the
// primitive that needs "persistent threads").
#pragma once

#include "atomics.hpp"

namespace sp {

struct BarrierState {
  uint32_t nwg;         // workgroups taking part
  uint32_t stride;      // uint32 words between padded state words
  uint32_t groups;      // tree: number of groups (<= nwg); xcd: number of XCDs
  uint32_t flag_stride; // flag barrier: uint32 words between flags (1 = packed)
  uint32_t poll_sleep;  // s_sleep units between polls
  uint32_t xblock;      // xcd: uint32 words of each XCD's block of local arrival flags
  uint32_t* cnt;        // centralized counter
  uint32_t* gen;        // centralized split: release word
  uint32_t* gcnt;       // tree: per-group counters (groups lines)
  uint32_t* ggen;       // tree: per-group release words (groups lines)
  uint32_t* top;        // tree: top counter
  uint32_t* topgen;     // tree: top release word
  uint32_t* arrive;     // flag barrier: arrival flags (nwg)
  uint32_t* release;    // flag barrier: release flags (nwg)
  uint32_t* mismatch;   // xcd: set when a workgroup is not on XCD (id mod groups)
  uint32_t* xarrive;    // xcd: per-XCD arrival stamps (groups lines)
  uint32_t* lrelease;   // xcd: per-workgroup release flags (nwg lines), XCD-major
  uint32_t* larrive;    // xcd: packed arrival flags, XCD-major blocks of xblock words
};

namespace detail {

__device__ __forceinline__ bool poll_until(const uint32_t* p, uint32_t stamp, Wait& w) {
  while (!reached(ld_relaxed(p), stamp))
    if (!w.tick()) return false;
  return true;
}

// Leader part of the counter-based barriers.  Each leader publishes its workgroup's
// stores with a release fence before arriving and acquires after the wait.
template <int KIND>
__device__ __forceinline__ bool counter_arrive_wait(const BarrierState& s, uint32_t stamp,
                                                    const Ctl& ctl) {
  Wait w(ctl, s.poll_sleep);
  if constexpr (KIND == SP_BARRIER_CENTRAL) {
    // Two-stage atomic barrier: one increment per workgroup, then poll the counter.
    add_release(s.cnt, 1);
    return poll_until(s.cnt, s.nwg * stamp, w);
  } else if constexpr (KIND == SP_BARRIER_CENTRAL_SPLIT) {
    // Same counter; the last arriver publishes a separate release word, so pollers
    // read a line that receives no read-modify-writes.
    const uint32_t old = add_release(s.cnt, 1);
    if (old == s.nwg * stamp - 1) {
      fence_acquire();
      st_release(s.gen, stamp);
      return true;
    }
    return poll_until(s.gen, stamp, w);
  } else {
    // Tree of depth two (Section 2's hierarchical barrier): workgroup w joins group
    // w mod G; the last arriver of a group arrives at the top counter; the last group
    // publishes the top release word, which each group's last arriver copies into its
    // group's release word.
    const uint32_t G = s.groups;
    const uint32_t g = blockIdx.x % G;
    const uint32_t members = (s.nwg - g + G - 1) / G;
    uint32_t* gc = s.gcnt + (size_t)g * s.stride;
    uint32_t* gg = s.ggen + (size_t)g * s.stride;
    const uint32_t old = add_release(gc, 1);
    if (old != members * stamp - 1) return poll_until(gg, stamp, w);
    fence_acquire();
    const uint32_t t = add_release(s.top, 1);
    if (t == G * stamp - 1) {
      fence_acquire();
      st_release(s.topgen, stamp);
    } else {
      if (!poll_until(s.topgen, stamp, w)) return false;
      fence_acquire();
    }
    st_release(gg, stamp);
    return true;
  }
}

// Master side of a flag scan: every lane checks flags i = lane, lane + lanes, ... of
// `n` flags (skipping index `skip`) and all of a lane's flags are loaded together each
// poll, so a scan costs one memory round trip rather than one per flag.
__device__ __forceinline__ int scan_flags(const uint32_t* flags, uint32_t fs, uint32_t n,
                                          uint32_t skip, uint32_t stamp, Wait& w) {
  for (uint32_t base = threadIdx.x; base < n; base += 8 * blockDim.x) {
    for (;;) {
      bool all = true;
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t i = base + k * blockDim.x;
        if (i < n && i != skip) all &= reached(ld_relaxed(flags + (size_t)i * fs), stamp);
      }
      if (all) break;
      if (!w.tick()) return 0;
    }
  }
  return 1;
}

// Decentralized flag barrier (the "XF" barrier of Section 5): no read-modify-writes.
__device__ __forceinline__ bool flag_wait(const BarrierState& s, uint32_t stamp,
                                          const Ctl& ctl) {
  __shared__ uint32_t s_ok;
  const uint32_t fs = s.flag_stride;
  if (blockIdx.x == 0) {
    __syncthreads();
    Wait w(ctl, s.poll_sleep);
    int ok = scan_flags(s.arrive, fs, s.nwg, 0, stamp, w);
    fence_acquire();
    ok = __syncthreads_and(ok);
    if (ok) {
      fence_release();
      for (uint32_t i = threadIdx.x; i < s.nwg; i += blockDim.x)
        if (i != 0) st_relaxed(s.release + (size_t)i * fs, stamp);
    }
    return ok;
  }
  __syncthreads();
  if (is_leader()) {
    Wait w(ctl, s.poll_sleep);
    st_release(s.arrive + (size_t)blockIdx.x * fs, stamp);
    const bool ok = poll_until(s.release + (size_t)blockIdx.x * fs, stamp, w);
    fence_acquire();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

// Per-XCD barrier.  Workgroup w runs on XCD w mod X (X = s.groups; checked in round 0)
// and is member k = w / X of its XCD; member 0 is the XCD's master.
//   1. Each member waits for its own stores to complete (they are then in the XCD's L2)
//      and stores its arrival stamp into its XCD's packed block of arrival flags; the
//      master's lanes scan the block.
//   2. The master writes back the XCD's dirty L2 lines once for all its members (agent
//      release), publishes the XCD's stamp, and polls the other XCDs' stamps
//      (all-to-all between at most eight masters).
//   3. The master acquires (agent scope) and its lanes store the members' release
//      flags, one line each; each released member acquires as well.
// Only the masters issue the L2 writeback; writebacks serialize at each XCD's L2
// controller, so issuing one per workgroup per round would dominate the round.  The
// acquire cannot be shared the same way: on gfx950 the only cache invalidation that
// reaches a CU's L1 is the agent-scope one (a workgroup-scope invalidate leaves stale
// L1 lines in place), so every workgroup invalidates for its own CU.
// All flags are accessed with agent-scope atomics.
__device__ __forceinline__ bool xcd_wait(const BarrierState& s, uint32_t stamp, const Ctl& ctl) {
  __shared__ uint32_t s_ok;
  const uint32_t X = s.groups;
  const uint32_t x = blockIdx.x % X, k = blockIdx.x / X;
  const uint32_t members = (s.nwg - x + X - 1) / X;
  uint32_t* block = s.larrive + (size_t)x * s.xblock;
  uint32_t* rel = s.lrelease + (size_t)x * s.xblock * s.stride;  // member i: rel + i*stride
  __syncthreads();
  if (k == 0) {
    Wait w(ctl, s.poll_sleep);
    int ok = scan_flags(block, 1, members, 0, stamp, w);
    ok = __syncthreads_and(ok);
    if (!ok) return false;
    if (threadIdx.x < X) {
      if (is_leader()) st_release(s.xarrive + (size_t)x * s.stride, stamp);
      // all-to-all between the XCD masters: lane i waits for XCD i
      ok = poll_until(s.xarrive + (size_t)threadIdx.x * s.stride, stamp, w);
    }
    ok = __syncthreads_and(ok);
    if (!ok) return false;
    if (is_leader()) fence_acquire();
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < members; i += blockDim.x)
      if (i != 0) st_relaxed(rel + (size_t)i * s.stride, stamp);
    return true;
  }
  if (is_leader()) {
    Wait w(ctl, s.poll_sleep);
    st_relaxed(block + k, stamp);
    const bool ok = poll_until(rel + (size_t)k * s.stride, stamp, w);
    fence_acquire();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

}  // namespace detail

// Global barrier, round `round` (0-based) of the current run.
template <int KIND>
__device__ bool barrier_wait(const BarrierState& s, uint32_t round, const Ctl& ctl) {
  __shared__ uint32_t s_ok;
  const uint32_t stamp = round + 1;
  wave_stores_complete();
  if constexpr (KIND == SP_BARRIER_FLAG) {
    return detail::flag_wait(s, stamp, ctl);
  } else if constexpr (KIND == SP_BARRIER_XCD) {
    // Round 0 runs the tree barrier with per-workgroup fences and, on the way, checks
    // that every workgroup sits on XCD (id mod X); later rounds use the per-XCD
    // protocol only if no workgroup reported a mismatch.
    __shared__ uint32_t s_local;
    if (round == 0) {
      if (is_leader() && xcc_id() != blockIdx.x % s.groups) add_relaxed(s.mismatch, 1);
      __syncthreads();
      if (is_leader()) {
        const bool ok = detail::counter_arrive_wait<SP_BARRIER_TREE>(s, stamp, ctl);
        fence_acquire();
        s_local = ld_relaxed(s.mismatch) == 0;
        s_ok = ok;
      }
      __syncthreads();
      return s_ok;
    }
    if (s_local) return detail::xcd_wait(s, stamp, ctl);
    __syncthreads();
    if (is_leader()) {
      const bool ok = detail::counter_arrive_wait<SP_BARRIER_TREE>(s, stamp, ctl);
      fence_acquire();
      s_ok = ok;
    }
    __syncthreads();
    return s_ok;
  } else {
    __syncthreads();
    if (is_leader()) {
      const bool ok = detail::counter_arrive_wait<KIND>(s, stamp, ctl);
      fence_acquire();
      s_ok = ok;
    }
    __syncthreads();
    return s_ok;
  }
}

}  // namespace sp
