// Device-side mutexes (Section 5, Mutex; Algorithms 1-3; Table 4 Lock()/Unlock()).
//
// Block semantics: every thread of the workgroup calls mutex_lock / mutex_unlock; the
// leader performs the atomics; a workgroup may hold several different locks.
#pragma once

#include "atomics.hpp"

namespace sp {

struct MutexState {
  uint32_t stride;      // uint32 words between per-lock state lines
  uint32_t poll_sleep;  // SP_MUTEX_SLEEP: s_sleep units between polls
  uint32_t* lockw;      // lock words (0 free, 1 held), one line per lock
  uint32_t* ticket;     // ticket mutex: next ticket, one line per lock
  uint32_t* turn;       // ticket mutex: ticket being served; ring: head; one line per lock
  uint32_t* queue;      // ring / array: qlen slots per lock, qstride words apart;
                        // cohort: per lock and XCC id, kCohortLines lines (local ticket,
                        // 64-bit grant slots), qstride (even) words apart
  uint32_t qlen;        // slots per lock (power of two; the ring needs >= contenders)
  uint32_t qstride;     // words between slots
  uint32_t cohort_bound;  // cohort: holders of one XCD in a row, at most; CU cohort: also
                          // holders of one CU in a row
  BackoffCfg bo;        // backoff between failed attempts
  uint32_t* cuq;        // CU cohort: per lock, XCC id and CU id, kCuLines lines (CU ticket,
                        // CU grant, session record), qstride (>= 4) words apart
};

// What the leader remembers about a lock it holds: for the ticket mutex, the ticket it
// was served with.  Only the holder writes `turn`, and it entered when turn == ticket, so
// unlock can publish ticket + 1 without loading turn first (one memory round trip fewer
// on every hand-over).
struct MutexHold {
  uint32_t ticket;
  uint32_t handoff;  // SP_MUTEX_ADAPTIVE: learned wall-clock ticks per hand-over (0 = none yet)
  uint32_t session;  // SP_MUTEX_COHORT: holders of this XCD before this one since the
                     // cohort took the global lock (0 = this holder took it)
  uint32_t global;   // SP_MUTEX_COHORT: the global ticket the cohort holds
  uint32_t cu_ticket;   // SP_MUTEX_CU_COHORT: the ticket drawn on this CU
  uint32_t cu_session;  // SP_MUTEX_CU_COHORT: holders of this CU before this one since the
                        // CU's cohort took the XCD lock (0 = this holder took it)
};

// Cohort lock state of `lock` for the XCD with XCC id x (kXccSlots per lock: the XCC id
// register has four bits, so every XCD has its own cohort whatever the count):
// kCohortLines lines, line 0 the local ticket counter, then kCohortGrants 64-bit grant
// slots.  Local ticket t polls slot t mod kCohortGrants (a few waiters per line instead
// of the XCD's whole queue on one), which holds local turn (bits 0-23, modulo 2^24) |
// session (bits 24-31) | global ticket of the session (bits 32-63); the holder of local
// ticket t writes slot t + 1, so one store hands over turn, session and global ticket at
// once.  A slot is rewritten (for ticket t + kCohortGrants) only after ticket t entered.
constexpr uint32_t kXccSlots = 16;
constexpr uint32_t kCohortGrants = 32;
constexpr uint32_t kCohortLines = 1 + kCohortGrants;
constexpr uint32_t kTurnMask = 0xFFFFFFu;
__device__ __forceinline__ uint32_t* cohort_ticket(const MutexState& s, uint32_t lock, uint32_t x) {
  return s.queue + ((size_t)lock * kXccSlots + x) * kCohortLines * s.qstride;
}
__device__ __forceinline__ uint64_t* cohort_grant(const MutexState& s, uint32_t lock, uint32_t x,
                                                  uint32_t t) {
  const size_t line =
      ((size_t)lock * kXccSlots + x) * kCohortLines + 1 + (t & (kCohortGrants - 1));
  return reinterpret_cast<uint64_t*>(s.queue + line * s.qstride);
}

// CU cohort state of `lock` for the CU with id c (HW_ID bits [15:8], kCuIds values) on the
// XCD with XCC id x: line 0 the CU's ticket counter, line 1 its grant word (CU turn, bits
// 0-23, modulo 2^24 | CU session, bits 24-31), line 2 the record of the XCD cohort lock
// the CU's session holds (words 0-2: local ticket, session, global ticket) and in word 3
// the count of CU tickets drawn as some waiter last announced it (a lower bound: racing
// announcements may land out of order).  Grant, record and announcement are stored and
// loaded at workgroup scope: only workgroups of that CU touch them, and they share the
// CU's L1, in which a store by one wavefront is seen by the others.
constexpr uint32_t kCuIds = 256;
constexpr uint32_t kCuLines = 3;
__device__ __forceinline__ uint32_t* cu_line(const MutexState& s, uint32_t lock, uint32_t x,
                                             uint32_t c, uint32_t i) {
  return s.cuq + ((((size_t)lock * kXccSlots + x) * kCuIds + c) * kCuLines + i) * s.qstride;
}

namespace detail {

// The XCD cohort lock's two levels, shared by SP_MUTEX_COHORT and SP_MUTEX_CU_COHORT:
// take XCD x's local ticket, wait for its grant, and queue for the global lock when the
// grant says the XCD's cohort does not hold it.  Leader only.
__device__ __forceinline__ bool cohort_acquire(const MutexState& s, uint32_t lock, uint32_t x,
                                               Wait& w, uint32_t* t, uint32_t* k,
                                               uint32_t* g) {
  bool ok = true;
  *t = add_relaxed(cohort_ticket(s, lock, x), 1);
  const uint64_t* grant = cohort_grant(s, lock, x, *t);
  uint64_t v;
  for (;;) {
    v = ld_relaxed64(grant);
    if (((uint32_t)v & kTurnMask) == (*t & kTurnMask)) break;
    if (!(ok = w.tick())) break;
  }
  *k = ((uint32_t)v >> 24) & 0xFF;
  *g = (uint32_t)(v >> 32);
  if (ok && *k == 0) {  // the cohort does not hold the global lock: queue for it
    *g = add_relaxed(s.ticket + (size_t)lock * s.stride, 1);
    const uint32_t* turn = s.turn + (size_t)lock * s.stride;
    while (ld_relaxed(turn) != *g)
      if (!(ok = w.tick())) break;
  }
  return ok;
}

// Hands the XCD cohort lock held with local ticket t (session k - 1, global ticket g) on:
// within the XCD when a later local ticket was drawn (`drawn`, loaded by the caller) and
// the session may grow, else back to the global queue.  Leader only, after the critical
// section's stores have completed.
template <bool FENCED>
__device__ __forceinline__ void cohort_release(const MutexState& s, uint32_t lock, uint32_t x,
                                               uint32_t drawn, uint32_t t, uint32_t k,
                                               uint32_t g) {
  uint64_t* grant = cohort_grant(s, lock, x, t + 1);  // the next local ticket's slot
  const uint64_t next_turn = (t + 1) & kTurnMask;
  if ((int32_t)(drawn - (t + 1)) > 0 && k < s.cohort_bound) {
    // The next holder runs on this XCD: pass the global lock with the local one.  The
    // critical section's stores have completed into this XCD's L2, which the next holder
    // reads through after its own acquire: no writeback.
    st_relaxed64(grant, ((uint64_t)g << 32) | ((uint64_t)k << 24) | next_turn);
  } else {
    uint32_t* turn = s.turn + (size_t)lock * s.stride;
    if constexpr (FENCED) st_release(turn, g + 1);  // writes back every local holder's stores
    else st_relaxed(turn, g + 1);
    st_relaxed64(grant, next_turn);  // session 0: the next local holder queues globally
  }
}

}  // namespace detail

// MCS lock node of workgroup w for `lock`: word 0 = next (workgroup + 1, 0 = none), word 1
// = locked; qlen nodes per lock (one per workgroup of the launch), qstride words apart.
__device__ __forceinline__ uint32_t* mcs_node(const MutexState& s, uint32_t lock, uint32_t w) {
  return s.queue + ((size_t)lock * s.qlen + w) * s.qstride;
}

// KIND:
//   SP_MUTEX_SPIN_CAS     compare-and-swap 0 -> 1 until it succeeds (backoff if configured)
//   SP_MUTEX_SPIN_EXCH    exchange with 1 until the old value is 0 (Algorithm 1; with a
//                         configured backoff, Algorithm 2)
//   SP_MUTEX_SPIN_BACKOFF compare-and-swap with backoff after each failure
//   SP_MUTEX_TICKET       fetch-and-add a ticket, poll turn with backoff (Algorithm 3);
//                         unlock adds one to turn with a plain load and a release store
//   SP_MUTEX_SLEEP        poll the lock word with loads and s_sleep until it reads free,
//                         then one compare-and-swap (waiting by polling, Section 5's GPU
//                         sleeping)
//   SP_MUTEX_RING         Section 5's ring-buffer mutex: draw ticket t, write the arrival's
//                         id (t + 1) into slot t of the ring, then poll the head and the
//                         slot it points at until that slot holds one's own id; unlock
//                         advances the head.  Two reads per poll.
//   SP_MUTEX_ARRAY        array queue lock: draw ticket t and poll only slot t (its own
//                         line) until it holds t; unlock writes t + 1 into slot t + 1.  A
//                         grant is overwritten only after its owner entered and left, so
//                         any number of slots is correct; more slots spread the polling.
//   SP_MUTEX_COHORT       XCD-cohort lock (lock cohorting, made for per-XCD L2s): a ticket
//                         lock per XCD in front of a global ticket lock.  The grant a
//                         local waiter polls (in its ticket's slot, a line shared by few
//                         waiters) carries the session (0 = the XCD does not hold the
//                         global lock; k > 0 = it does, k holders of this XCD took it in
//                         a row) and the session's global ticket.  A local holder that
//                         reads session 0 takes the global lock.  Unlock passes the
//                         global lock with the local one (one store into the next local
//                         ticket's slot: turn + 1, session k + 1) when a local ticket beyond
//                         one's own was drawn and k + 1 < cohort_bound; that hand-over
//                         needs no L2 writeback, since both holders use this XCD's L2
//                         (the critical section's stores have completed into it).
//                         Otherwise it releases the global lock (with the writeback), then
//                         grants the local turn with session 0.  Cohorts are the actual
//                         XCDs (XCC id), never merged: the local hand-over relies on the
//                         shared L2.
//   SP_MUTEX_CU_COHORT    CU-cohort lock: SP_MUTEX_COHORT behind a ticket lock per CU.  A
//                         waiter draws a CU ticket, announces it in the CU's record line
//                         and polls the CU's grant word at workgroup scope (in the CU's
//                         L1).  Session k > 0: the CU's cohort holds the XCD lock (the
//                         record says how), enter with no cache maintenance, since the
//                         previous holder's stores went through this L1.  Session 0: take
//                         the XCD-cohort lock, acquire, write the record.  Unlock passes
//                         within the CU (session k + 1) when a later CU ticket was
//                         announced and k + 1 < cohort_bound, else hands the XCD lock on
//                         and grants session 0.
//   SP_MUTEX_MCS          MCS queue lock: each workgroup has a node per lock (next, locked)
//                         in its own line; lock stores next = none and locked = 1, then
//                         exchanges the lock word (the queue's tail) with its node id;
//                         behind a predecessor it links in (predecessor.next = me) and
//                         polls only its own locked word.  Unlock hands the lock to the
//                         successor (its locked = 0), or, when none has linked in,
//                         swings the tail back to free with a compare-and-swap (waiting
//                         for a successor whose exchange came first to link in).
//   SP_MUTEX_ADAPTIVE     ticket mutex with proportional waiting tuned online (Section 5's
//                         aggressive lock that reverts to backoff): a waiter d tickets from
//                         the head sleeps about (d - 1) / 4 hand-over times before polling
//                         again, the one next in line polls without sleeping; each
//                         workgroup keeps a running average of the hand-over time in its
//                         MutexHold (which must then persist across acquisitions), measured
//                         as the rate at which the head advanced between its first and last
//                         polls that saw the head short of its ticket -- not its own
//                         elapsed wait, which would include its own lag in noticing its
//                         turn and feed oversleeping back into the estimate.
// FENCED = false: the caller's critical sections touch the protected data only with
// agent-scope (coherent) loads and stores, so the lock needs no acquire fence and the
// unlock no release fence; the unlock still waits until the section's stores completed.
template <int KIND, bool FENCED = true>
__device__ bool mutex_lock(const MutexState& s, uint32_t lock, const Ctl& ctl,
                           MutexHold* hold = nullptr) {
  __shared__ uint32_t s_ok;
  if (is_leader()) {
    uint32_t* m = s.lockw + (size_t)lock * s.stride;
    Wait w(ctl, (KIND == SP_MUTEX_SLEEP || KIND == SP_MUTEX_RING || KIND == SP_MUTEX_ARRAY ||
                 KIND == SP_MUTEX_COHORT || KIND == SP_MUTEX_CU_COHORT ||
                 KIND == SP_MUTEX_MCS)
                    ? s.poll_sleep : 0);
    Backoff bo(s.bo);
    bool ok = true;
    if constexpr (KIND == SP_MUTEX_SPIN_CAS || KIND == SP_MUTEX_SPIN_BACKOFF) {
      while (cas_relaxed(m, 0, 1) != 0) {
        bo(s.bo);
        if (!(ok = w.tick())) break;
      }
    } else if constexpr (KIND == SP_MUTEX_SPIN_EXCH) {
      while (exch_relaxed(m, 1) != 0) {
        bo(s.bo);
        if (!(ok = w.tick())) break;
      }
    } else if constexpr (KIND == SP_MUTEX_TICKET) {
      const uint32_t my = add_relaxed(s.ticket + (size_t)lock * s.stride, 1);
      const uint32_t* turn = s.turn + (size_t)lock * s.stride;
      while (ld_relaxed(turn) != my) {
        bo(s.bo);
        if (!(ok = w.tick())) break;
      }
      if (hold) hold->ticket = my;
    } else if constexpr (KIND == SP_MUTEX_ADAPTIVE) {
      const uint32_t my = add_relaxed(s.ticket + (size_t)lock * s.stride, 1);
      const uint32_t* turn = s.turn + (size_t)lock * s.stride;
      const uint32_t learned = hold ? hold->handoff : 0;
      uint64_t t_first = 0, t_last = 0;
      uint32_t c_first = 0, c_last = 0;
      bool seen = false;
      for (;;) {
        const uint32_t cur = ld_relaxed(turn);
        const uint64_t now = wall_clock();
        if (cur == my) break;
        if (!seen) {
          seen = true;
          t_first = now;
          c_first = cur;
        }
        t_last = now;
        c_last = cur;
        const uint32_t d = my - cur;
        if (d > 1 && learned) {
          // (d - 1) / 4 hand-overs; one wall tick (10 ns) is ~0.375 s_sleep units at 2.4 GHz
          const uint64_t units = ((uint64_t)(d - 1) * learned * 3) / 32;
          sleep_units(units < 4096 ? (uint32_t)units : 4096u);
        }
        if (!(ok = w.tick())) break;
      }
      if (hold) {
        hold->ticket = my;
        const uint32_t moved = c_last - c_first;
        if (seen && moved > 0) {
          const uint32_t sample = (uint32_t)((t_last - t_first) / moved);
          const uint32_t avg = learned ? (7 * learned + sample) / 8 : sample;
          hold->handoff = avg < 100000 ? avg : 100000;  // at most 1 ms of wall clock
        }
      }
    } else if constexpr (KIND == SP_MUTEX_RING) {
      const uint32_t t = add_relaxed(s.ticket + (size_t)lock * s.stride, 1);
      uint32_t* q = s.queue + (size_t)lock * s.qlen * s.qstride;
      const uint32_t mask = s.qlen - 1;
      st_relaxed(q + (size_t)(t & mask) * s.qstride, t + 1);
      const uint32_t* head = s.turn + (size_t)lock * s.stride;
      for (;;) {
        const uint32_t h = ld_relaxed(head);
        if (ld_relaxed(q + (size_t)(h & mask) * s.qstride) == t + 1) break;
        if (!(ok = w.tick())) break;
      }
      if (hold) hold->ticket = t;
    } else if constexpr (KIND == SP_MUTEX_COHORT) {
      uint32_t t, k, g;
      ok = detail::cohort_acquire(s, lock, xcc_id(), w, &t, &k, &g);
      if (hold) {
        hold->ticket = t;
        hold->session = k;
        hold->global = g;
      }
    } else if constexpr (KIND == SP_MUTEX_CU_COHORT) {
      const uint32_t x = xcc_id(), c = cu_in_xcc();
      const uint32_t tc = add_relaxed(cu_line(s, lock, x, c, 0), 1);
      const uint32_t* cgrant = cu_line(s, lock, x, c, 1);
      uint32_t* rec = cu_line(s, lock, x, c, 2);
      st_cu(rec + 3, tc + 1);  // tell the holder that a later CU ticket was drawn
      uint32_t v;
      for (;;) {
        v = ld_cu(cgrant);
        if ((v & kTurnMask) == (tc & kTurnMask)) break;
        if (!(ok = w.tick())) break;
      }
      const uint32_t kc = v >> 24;
      uint32_t t = 0, k = 0, g = 0;
      if (ok && kc > 0) {
        // This CU's cohort holds the XCD lock: its record says how, and the previous
        // holder ran on this CU, whose L1 its stores went through (no acquire).
        t = ld_cu(rec);
        k = ld_cu(rec + 1);
        g = ld_cu(rec + 2);
      } else if (ok) {
        ok = detail::cohort_acquire(s, lock, x, w, &t, &k, &g);
        if constexpr (FENCED) fence_acquire();
        // for the CU's later holders of this session (complete before the first CU grant)
        st_cu(rec, t);
        st_cu(rec + 1, k);
        st_cu(rec + 2, g);
      }
      hold->ticket = t;
      hold->session = k;
      hold->global = g;
      hold->cu_ticket = tc;
      hold->cu_session = kc;
    } else if constexpr (KIND == SP_MUTEX_MCS) {
      uint32_t* node = mcs_node(s, lock, blockIdx.x);
      st_relaxed(node, 0);      // next: none
      st_relaxed(node + 1, 1);  // locked
      wave_stores_complete();   // both land before the exchange makes the node reachable
      const uint32_t prev = exch_relaxed(m, blockIdx.x + 1);
      if (prev != 0) {
        st_relaxed(mcs_node(s, lock, prev - 1), blockIdx.x + 1);  // predecessor.next = me
        while (ld_relaxed(node + 1) != 0)
          if (!(ok = w.tick())) break;
      }
    } else if constexpr (KIND == SP_MUTEX_ARRAY) {
      const uint32_t t = add_relaxed(s.ticket + (size_t)lock * s.stride, 1);
      const uint32_t* slot =
          s.queue + ((size_t)lock * s.qlen + (t & (s.qlen - 1))) * s.qstride;
      while (ld_relaxed(slot) != t)
        if (!(ok = w.tick())) break;
      if (hold) hold->ticket = t;
    } else {
      for (;;) {
        while (ld_relaxed(m) != 0)
          if (!(ok = w.tick())) break;
        if (!ok || cas_relaxed(m, 0, 1) == 0) break;
      }
    }
    if constexpr (FENCED && KIND != SP_MUTEX_CU_COHORT) fence_acquire();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

// `hold`: the record mutex_lock filled in (leader's copy).  It may be nullptr except for
// SP_MUTEX_ARRAY, SP_MUTEX_COHORT and SP_MUTEX_CU_COHORT (whose mutex_lock needs it too):
// the ticket and ring mutexes then load turn / head to find the value to publish.  `ctl` bounds SP_MUTEX_MCS's wait for a successor that
// has taken the tail but not linked in yet (no other kind waits in unlock).
template <int KIND, bool FENCED = true>
__device__ void mutex_unlock(const MutexState& s, uint32_t lock, const MutexHold* hold = nullptr,
                             const Ctl* ctl = nullptr) {
  if constexpr (KIND == SP_MUTEX_MCS) {
    wave_stores_complete();
    __syncthreads();
    if (!is_leader()) return;
    uint32_t* node = mcs_node(s, lock, blockIdx.x);
    uint32_t* tail = s.lockw + (size_t)lock * s.stride;
    if constexpr (FENCED) fence_release();  // before either hand-over
    uint32_t next = ld_relaxed(node);
    if (next == 0) {
      if (cas_relaxed(tail, blockIdx.x + 1, 0) == blockIdx.x + 1) return;  // nobody queued
      // a successor took the tail after us: it links in within a round trip
      Wait w(ctl ? *ctl : Ctl{nullptr, 0}, 0);
      while ((next = ld_relaxed(node)) == 0)
        if (ctl && !w.tick()) return;
    }
    st_relaxed(mcs_node(s, lock, next - 1) + 1, 0);  // successor.locked = 0
    return;
  }
  if constexpr (KIND == SP_MUTEX_COHORT) {
    // The local ticket count is loaded first so that its round trip overlaps the wait
    // for the critical section's stores.
    const uint32_t x = xcc_id();
    const uint32_t drawn = is_leader() ? ld_relaxed(cohort_ticket(s, lock, x)) : 0;
    wave_stores_complete();
    __syncthreads();
    if (!is_leader()) return;
    detail::cohort_release<FENCED>(s, lock, x, drawn, hold->ticket, hold->session + 1,
                                   hold->global);
    return;
  }
  if constexpr (KIND == SP_MUTEX_CU_COHORT) {
    // Whether a later CU ticket was drawn comes from the waiters' announcement in the
    // CU's L1, not from the ticket counter at memory: no round trip on a CU hand-over (a
    // stale announcement only ends the CU's session early).
    const uint32_t x = xcc_id(), c = cu_in_xcc();
    const uint32_t drawn_c = is_leader() ? ld_cu(cu_line(s, lock, x, c, 2) + 3) : 0;
    wave_stores_complete();
    __syncthreads();
    if (!is_leader()) return;
    uint32_t* cgrant = cu_line(s, lock, x, c, 1);
    const uint32_t tc = hold->cu_ticket, kc = hold->cu_session + 1;
    const uint32_t next_turn = (tc + 1) & kTurnMask;
    if ((int32_t)(drawn_c - (tc + 1)) > 0 && kc < s.cohort_bound) {
      // The next holder runs on this CU: it keeps the XCD lock and reads the critical
      // section's stores through this CU's L1 (they have completed): no cache maintenance.
      st_cu(cgrant, (kc << 24) | next_turn);
    } else {
      const uint32_t drawn = ld_relaxed(cohort_ticket(s, lock, x));
      detail::cohort_release<FENCED>(s, lock, x, drawn, hold->ticket, hold->session + 1,
                                     hold->global);
      st_cu(cgrant, next_turn);  // session 0: the CU's next holder takes the XCD lock
    }
    return;
  }
  wave_stores_complete();
  __syncthreads();
  if (is_leader()) {
    uint32_t* w;
    uint32_t v;
    if constexpr (KIND == SP_MUTEX_TICKET || KIND == SP_MUTEX_RING || KIND == SP_MUTEX_ADAPTIVE) {
      // only the holder writes turn / head, so it can publish its own ticket + 1
      w = s.turn + (size_t)lock * s.stride;
      v = (hold ? hold->ticket : ld_relaxed(w)) + 1;
    } else if constexpr (KIND == SP_MUTEX_ARRAY) {
      // the holder's ticket is needed: nothing else records it
      v = hold->ticket + 1;
      w = s.queue + ((size_t)lock * s.qlen + (v & (s.qlen - 1))) * s.qstride;
    } else {
      w = s.lockw + (size_t)lock * s.stride;
      v = 0;
    }
    if constexpr (FENCED) st_release(w, v);
    else st_relaxed(w, v);
  }
}

}  // namespace sp
