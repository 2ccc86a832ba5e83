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
  uint32_t tgroups;     // groups of the counter tree (tree, xcd round 0 and fallback), <= nwg
  uint32_t flag_stride; // flag barrier: uint32 words between flags (1 = packed)
  uint32_t poll_sleep;  // s_sleep units between polls
  uint32_t xblock;      // xcd: uint32 words of each XCD's block of local arrival flags
  uint32_t fenced;      // 1: order plain memory (release / acquire fences); 0: the data
                        // exchanged across the barrier is accessed with agent-scope
                        // loads and stores, so the barrier does no cache maintenance
  uint32_t xcopies;     // xcd: copies of the XCD stamps (0 = xarrive, one line per XCD)
  uint32_t xmstride;    // xcd: words between two copies (>= groups, whole lines)
  // xcd: where each XCD's flags live.  XCD x's block of arrival flags starts xoff[x]
  // words into larrive, its per-CU release lines roff[x] words into lrelease (the CU of
  // rank r at + r * stride); copy c of the stamps starts moff[c mod groups] + (c / groups)
  // * xmstep words into xmail (with xcopies a multiple of groups, only XCD c mod groups
  // polls copy c, so each XCD's copies can sit in memory close to it).
  uint32_t xmstep;
  uint32_t xoff[16];
  uint32_t moff[16];
  uint32_t roff[16];
  uint32_t* cnt;        // centralized counter
  uint32_t* gen;        // centralized split: release word
  uint32_t* gcnt;       // tree: per-group counters (groups lines)
  uint32_t* ggen;       // tree: per-group release words (groups lines)
  uint32_t* top;        // tree: top counter
  uint32_t* topgen;     // tree: top release word
  uint32_t* arrive;     // flag barrier: arrival flags (nwg)
  uint32_t* release;    // flag barrier: release flags (nwg)
  uint32_t* mismatch;   // xcd: workgroups not on XCD (id mod groups), informational
  uint32_t* overflow;   // xcd: registrations that did not fit (nonzero = tree fallback)
  uint32_t* xarrive;    // xcd: per-XCD arrival stamps (groups lines)
  uint32_t* lrelease;   // xcd: per-CU release lines (kCuLines per XCD)
  uint32_t* larrive;    // xcd: arrival flags kArriveWords apart, XCD-major blocks of
                        // xblock flags
  uint32_t* cu_count;   // xcd: workgroups registered per CU key (groups * 256 words)
  uint32_t* xcount;     // xcd: members registered per XCD (groups words)
  uint32_t* xcu;        // xcd: CU leaders registered per XCD (groups words)
  uint32_t* cu_rank;    // xcd: rank of each CU key within its XCD (groups * 256 words)
  uint32_t* xmail;      // xcd: xcopies copies, each holding every XCD's stamp packed
};

// CUs with members per XCD that the per-XCD barrier takes (gfx950 has 32 per XCD).
constexpr uint32_t kCuLines = 64;
// Words between two arrival flags of an XCD's block: 16 bytes, eight flags per 128-byte
// line.  Packed flags put 32 concurrent writers on every line and one line per flag
// makes the master's scan touch a line per member; eight per line measured fastest.
constexpr uint32_t kArriveWords = 4;

namespace detail {

__device__ __forceinline__ bool poll_until(const uint32_t* p, uint32_t stamp, Wait& w) {
  while (!reached(ld_relaxed(p), stamp))
    if (!w.tick()) return false;
  return true;
}
__device__ __forceinline__ bool poll_until_cu(const uint32_t* p, uint32_t stamp, Wait& w) {
  while (!reached(ld_cu(p), stamp))
    if (!w.tick()) return false;
  return true;
}

// Leader part of the counter-based barriers.  Each leader publishes its workgroup's
// stores with a release fence before arriving and acquires after the wait.
template <int KIND>
__device__ __forceinline__ bool counter_arrive_wait(const BarrierState& s, uint32_t stamp,
                                                    const Ctl& ctl) {
  Wait w(ctl, s.poll_sleep);
  const bool f = s.fenced;
  if constexpr (KIND == SP_BARRIER_CENTRAL) {
    // Two-stage atomic barrier: one increment per workgroup, then poll the counter.
    if (f) fence_release();
    add_relaxed(s.cnt, 1);
    return poll_until(s.cnt, s.nwg * stamp, w);
  } else if constexpr (KIND == SP_BARRIER_CENTRAL_SPLIT) {
    // Same counter; the last arriver publishes a separate release word, so pollers
    // read a line that receives no read-modify-writes.
    if (f) fence_release();
    const uint32_t old = add_relaxed(s.cnt, 1);
    if (old == s.nwg * stamp - 1) {
      if (f) {
        fence_acquire();
        fence_release();
      }
      st_relaxed(s.gen, stamp);
      return true;
    }
    return poll_until(s.gen, stamp, w);
  } else {
    // Tree of depth two (Section 2's hierarchical barrier): workgroup w joins group
    // w mod G; the last arriver of a group arrives at the top counter; the last group
    // publishes the top release word, which each group's last arriver copies into its
    // group's release word.
    const uint32_t G = s.tgroups;
    const uint32_t g = blockIdx.x % G;
    const uint32_t members = (s.nwg - g + G - 1) / G;
    uint32_t* gc = s.gcnt + (size_t)g * s.stride;
    uint32_t* gg = s.ggen + (size_t)g * s.stride;
    if (f) fence_release();
    const uint32_t old = add_relaxed(gc, 1);
    if (old != members * stamp - 1) return poll_until(gg, stamp, w);
    if (f) {
      fence_acquire();
      fence_release();
    }
    const uint32_t t = add_relaxed(s.top, 1);
    if (t == G * stamp - 1) {
      if (f) {
        fence_acquire();
        fence_release();
      }
      st_relaxed(s.topgen, stamp);
    } else {
      if (!poll_until(s.topgen, stamp, w)) return false;
      if (f) {
        fence_acquire();
        fence_release();
      }
    }
    st_relaxed(gg, stamp);
    return true;
  }
}

// Master side of a flag scan: every lane checks flags i = lane, lane + lanes, ... of
// `n` flags (skipping index `skip`) and all of a lane's flags are loaded together each
// poll, so a scan costs one memory round trip rather than one per flag.  `lanes` is the
// workgroup size (the per-XCD barrier passes the value it saved in round 0: reading
// blockDim.x is a load from the dispatch packet).
__device__ __forceinline__ int scan_flags(const uint32_t* flags, uint32_t fs, uint32_t n,
                                          uint32_t skip, uint32_t stamp, Wait& w,
                                          uint32_t lanes) {
  for (uint32_t base = threadIdx.x; base < n; base += 8 * lanes) {
    for (;;) {
      bool all = true;
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t i = base + k * lanes;
        if (i < n && i != skip) all &= reached(ld_relaxed(flags + (size_t)i * fs), stamp);
      }
      if (all) break;
      if (!w.tick()) return 0;
    }
  }
  return 1;
}

// Workgroup AND of `ok` with one workgroup barrier, for the rounds of the flag and
// per-XCD barriers.  HIP's __syncthreads_and loads the workgroup size from the kernel's
// arguments (a memory round trip) and runs three barriers around an LDS reduction; here
// a wavefront writes only when one of its lanes failed (the watchdog fired).
// fail[stamp & 1] is zero on entry: the caller cleared it at least one workgroup barrier
// earlier, after every thread had read it two rounds before.  Every thread of the
// workgroup calls.
__device__ __forceinline__ int and_sync(int ok, uint32_t stamp, uint32_t* fail) {
  if (__builtin_amdgcn_ballot_w64(!ok) != 0 && (threadIdx.x & 63) == 0) fail[stamp & 1] = 1;
  __syncthreads();
  return fail[stamp & 1] == 0;
}

// Decentralized flag barrier (the "XF" barrier of Section 5): no read-modify-writes.
__device__ __forceinline__ bool flag_wait(const BarrierState& s, uint32_t stamp,
                                          const Ctl& ctl) {
  __shared__ uint32_t s_ok;
  __shared__ uint32_t s_fail[2];
  const uint32_t fs = s.flag_stride;
  if (blockIdx.x == 0) {
    // this round's entry; the other one may still be read for the previous round
    if (threadIdx.x == 0) s_fail[stamp & 1] = 0;
    __syncthreads();
    Wait w(ctl, s.poll_sleep);
    int ok = scan_flags(s.arrive, fs, s.nwg, 0, stamp, w, blockDim.x);
    if (s.fenced) fence_acquire();
    ok = and_sync(ok, stamp, s_fail);
    if (ok) {
      if (s.fenced) fence_release();
      for (uint32_t i = threadIdx.x; i < s.nwg; i += blockDim.x)
        if (i != 0) st_relaxed(s.release + (size_t)i * fs, stamp);
    }
    return ok;
  }
  __syncthreads();
  if (is_leader()) {
    Wait w(ctl, s.poll_sleep);
    if (s.fenced) fence_release();
    st_relaxed(s.arrive + (size_t)blockIdx.x * fs, stamp);
    const bool ok = poll_until(s.release + (size_t)blockIdx.x * fs, stamp, w);
    if (s.fenced) fence_acquire();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

// Per-XCD barrier.  In round 0 every workgroup registers under the XCD it runs on (the
// XCC id register), which makes it member k of that XCD in registration order (member 0
// is the XCD's master), and under the id of its CU, where the first workgroup to register
// becomes the CU's leader.  The placement is read, not assumed: the dispatcher normally
// sends workgroup w to XCD w mod 8, but not always (after a cooperative launch, for
// example, later dispatches have been measured to start one XCD further on).  Later rounds:
//   1. Each member waits for its own stores to complete (they are then in the XCD's L2)
//      and stores its arrival stamp into its XCD's block of arrival flags (16 bytes
//      apart); the master's lanes scan the block.
//   2. The master writes back the XCD's dirty L2 lines once for all its members (agent
//      release) and publishes the XCD's stamp.
//   3. Each CU leader polls the stamps of every XCD that has members; once all are
//      published it acquires (agent scope) and releases the other workgroups of its CU
//      with one store to the CU's release line, which they poll.  That line is stored and
//      polled at workgroup scope: the CU's workgroups share its L1, and a store by one
//      wavefront is seen by the CU's other wavefronts there (what makes workgroup scope
//      coherent without cache maintenance), so the signal stays within the CU instead of
//      taking a memory round trip.  With xcopies = C > 0
//      the masters write their stamps into C lines that each hold all of them packed,
//      and the CUs spread their polls over the copies by their rank in their XCD (fewer
//      pollers per line).
// Writebacks and invalidations both serialize at each XCD's L2 controller.  The
// writeback is shared by the whole XCD.  The invalidation has to reach each CU's L1, and
// on gfx950 only the agent-scope invalidate does (a workgroup-scope one leaves stale L1
// lines), so it is shared by the workgroups of one CU: all of them are waiting when
// their leader invalidates, so nothing stale can re-enter the L1 before they read.
// If an XCD holds more members than its flag block or more than kCuLines CUs, every
// workgroup falls back to the counter tree.  All other flags are agent-scope atomics.
struct XcdLocal {
  uint32_t x;        // the XCD this workgroup runs on
  uint32_t k;        // member index within the XCD (0 = master)
  uint32_t members;  // members of this XCD
  uint32_t xmask;    // XCDs that have members (bit i = XCD i)
  uint32_t key;      // CU key: XCD * 256 + CU id
  uint32_t slot;     // registration order on the CU (0 = CU leader)
  uint32_t rank;     // rank of the CU among its XCD's CUs with members
  uint32_t mail;     // the copy of the XCD stamps this workgroup polls (xcopies > 0)
  // Resolved once in round 0 from the barrier's state and its placement tables, so that
  // later rounds read nothing from the kernel's arguments (reloading those fields inside
  // the round, or indexing the tables there, was measured to cost ~10 % of a round):
  uint32_t* block;         // this XCD's block of arrival flags
  const uint32_t* stamps;  // the stamps this workgroup polls: its copy, or xarrive
  uint32_t* rel;           // this CU's release line
  uint32_t* mail_x;        // xmail + x: the master stores copy c at mail_x + pub[c]
  uint32_t* xarrive_x;     // the XCD's stamp line when there are no copies
  uint32_t groups, copies, sstride, fenced, poll_sleep, lanes;
};

// A pointer that is the same for the whole workgroup, in scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// The master's stores of its stamp: copy c at pub[c] + the XCD's index in xmail.
constexpr uint32_t kMaxCopies = 256;

__device__ __forceinline__ bool xcd_wait(uint32_t stamp, const Ctl& ctl, const XcdLocal& L,
                                         const uint32_t* pub, uint32_t* fail) {
  __shared__ uint32_t s_ok;
  // The registration is the same for the whole workgroup: keep it in scalar registers.
  const uint32_t X = __builtin_amdgcn_readfirstlane(L.groups);
  const uint32_t k = __builtin_amdgcn_readfirstlane(L.k);
  const uint32_t members = __builtin_amdgcn_readfirstlane(L.members);
  const uint32_t xmask = __builtin_amdgcn_readfirstlane(L.xmask);
  const uint32_t slot = __builtin_amdgcn_readfirstlane(L.slot);
  const uint32_t fenced = __builtin_amdgcn_readfirstlane(L.fenced);
  uint32_t* block = uniform_ptr(L.block);
  Wait w(ctl, __builtin_amdgcn_readfirstlane(L.poll_sleep));
  int ok = 1;
  __syncthreads();
  if (threadIdx.x == 0) fail[(stamp + 1) & 1] = 0;  // for the next round's and_sync
  const uint32_t C = __builtin_amdgcn_readfirstlane(L.copies);
  if (k == 0) {
    // XCD master: gather the XCD's arrivals, write the XCD's L2 back once, publish (in
    // every copy of the stamps, by the first wavefront after its writeback).
    ok = scan_flags(block, kArriveWords, members, 0, stamp, w,
                    __builtin_amdgcn_readfirstlane(L.lanes));
    ok = and_sync(ok, stamp, fail);
    if (!ok) return false;
    if (C == 0) {
      if (is_leader()) {
        if (fenced) fence_release();
        st_relaxed(uniform_ptr(L.xarrive_x), stamp);
      }
    } else if (threadIdx.x < 64) {
      if (fenced) fence_release();
      uint32_t* mail_x = uniform_ptr(L.mail_x);
      for (uint32_t c = threadIdx.x; c < C; c += 64) st_relaxed(mail_x + pub[c], stamp);
    }
  } else if (is_leader()) {
    st_relaxed(block + (size_t)k * kArriveWords, stamp);
  }
  // The populated XCDs' stamps: one line each, or packed in this CU's copy.
  const uint32_t* stamps = uniform_ptr(L.stamps);
  const uint32_t sstride = __builtin_amdgcn_readfirstlane(L.sstride);
  if (!fenced) {
    // Coherent data: no cache maintenance, so nothing is shared per CU; every workgroup
    // polls the populated XCDs' stamps itself (two flag hops per round).
    if (threadIdx.x < X && ((xmask >> threadIdx.x) & 1))
      ok = poll_until(stamps + (size_t)threadIdx.x * sstride, stamp, w);
    return and_sync(ok, stamp, fail);
  }
  // this CU's release line
  uint32_t* rel = uniform_ptr(L.rel);
  if (slot == 0) {
    // CU leader: once every populated XCD has published, invalidate for the CU and
    // release it.  The invalidation has to follow the last XCD's writeback: a line that
    // a kernel on another stream reads on this XCD before then (say, other words of a
    // line that participants elsewhere write) would otherwise stay stale in the L2.
    if (threadIdx.x < X && ((xmask >> threadIdx.x) & 1))
      ok = poll_until(stamps + (size_t)threadIdx.x * sstride, stamp, w);
    ok = and_sync(ok, stamp, fail);
    if (!ok) return false;
    if (is_leader()) {
      fence_acquire();  // completes before the release store is issued
      st_cu(rel, stamp);  // only this CU's workgroups poll the line
    }
    __syncthreads();
    return true;
  }
  if (is_leader()) {
    ok = poll_until_cu(rel, stamp, w);
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

// Round 0 of the per-XCD barrier: register per XCD and per CU, run the counter tree
// with per-workgroup fences, then load what the later rounds use.
__device__ __forceinline__ bool xcd_setup(const BarrierState& s, const Ctl& ctl, XcdLocal& L,
                                          uint32_t* pub, uint32_t* fail, uint32_t* use_xcd) {
  __shared__ uint32_t s_ok;
  const uint32_t X = s.groups;
  __syncthreads();  // every wavefront's stores have completed (barrier_wait's entry wait)
  if (is_leader()) {
    // XCDs are told apart by their XCC id modulo the XCD count.  An id at or above the
    // count would share a group, and its one writeback, with another XCD: fall back.
    const uint32_t raw = xcc_id();
    const uint32_t xcc = raw % X;
    if (raw >= X) add_relaxed(s.overflow, 1);
    if (xcc != blockIdx.x % X) add_relaxed(s.mismatch, 1);
    L.x = xcc;
    L.k = add_relaxed(s.xcount + xcc, 1);
    if (L.k >= s.xblock) add_relaxed(s.overflow, 1);
    L.key = xcc * 256 + cu_in_xcc();
    L.slot = add_relaxed(s.cu_count + L.key, 1);
    if (L.slot == 0) {
      const uint32_t r = add_relaxed(s.xcu + xcc, 1);
      st_relaxed(s.cu_rank + L.key, r);
      if (r >= kCuLines) add_relaxed(s.overflow, 1);
    }
    // the registration stores are complete before the arrival (with or without fences)
    wave_stores_complete();
    const bool ok = counter_arrive_wait<SP_BARRIER_TREE>(s, 1, ctl);
    fence_acquire();  // round 0 only: always, so the registrations below read fresh
    *use_xcd = ld_relaxed(s.overflow) == 0;
    L.rank = ld_relaxed(s.cu_rank + L.key);
    L.members = ld_relaxed(s.xcount + xcc);
    uint32_t mask = 0;
    for (uint32_t i = 0; i < X; ++i)
      if (ld_relaxed(s.xcount + i) != 0) mask |= 1u << i;
    L.xmask = mask;
    L.mail = s.xcopies ? (xcc + X * L.rank) % s.xcopies : 0;
    L.block = s.larrive + s.xoff[xcc];
    L.stamps = s.xcopies ? s.xmail + s.moff[L.mail % X] + (size_t)(L.mail / X) * s.xmstep
                         : s.xarrive;
    L.sstride = s.xcopies ? 1 : s.stride;
    L.rel = s.lrelease + s.roff[xcc] + (size_t)L.rank * s.stride;
    L.mail_x = s.xmail + xcc;
    L.xarrive_x = s.xarrive + (size_t)xcc * s.stride;
    L.groups = X;
    L.copies = s.xcopies;
    L.fenced = s.fenced;
    L.poll_sleep = s.poll_sleep;
    L.lanes = blockDim.x;
    fail[0] = fail[1] = 0;
    s_ok = ok;
  }
  for (uint32_t c = threadIdx.x; c < s.xcopies && c < kMaxCopies; c += blockDim.x)
    pub[c] = s.moff[c % X] + (c / X) * s.xmstep;
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
    // Round 0 registers every workgroup by XCD and CU; later rounds use the per-XCD
    // protocol unless a registration did not fit, the counter tree otherwise.
    __shared__ detail::XcdLocal s_local;
    __shared__ uint32_t s_use;
    __shared__ uint32_t s_pub[detail::kMaxCopies];
    __shared__ uint32_t s_fail[2];
    if (round == 0) return detail::xcd_setup(s, ctl, s_local, s_pub, s_fail, &s_use);
    if (s_use) return detail::xcd_wait(stamp, ctl, s_local, s_pub, s_fail);
    __syncthreads();
    if (is_leader()) {
      const bool ok = detail::counter_arrive_wait<SP_BARRIER_TREE>(s, stamp, ctl);
      if (s.fenced) fence_acquire();
      s_ok = ok;
    }
    __syncthreads();
    return s_ok;
  } else {
    __syncthreads();
    if (is_leader()) {
      const bool ok = detail::counter_arrive_wait<KIND>(s, stamp, ctl);
      if (s.fenced) fence_acquire();
      s_ok = ok;
    }
    __syncthreads();
    return s_ok;
  }
}

}  // namespace sp
