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
  uint32_t* turn;       // ticket mutex: ticket being served, one line per lock
  BackoffCfg bo;        // backoff between failed attempts
};

// What the leader remembers about a lock it holds: for the ticket mutex, the ticket it
// was served with.  Only the holder writes `turn`, and it entered when turn == ticket, so
// unlock can publish ticket + 1 without loading turn first (one memory round trip fewer
// on every hand-over).
struct MutexHold {
  uint32_t ticket;
};

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
// FENCED = false: the caller's critical sections touch the protected data only with
// agent-scope (coherent) loads and stores, so the lock needs no acquire fence and the
// unlock no release fence; the unlock still waits until the section's stores completed.
template <int KIND, bool FENCED = true>
__device__ bool mutex_lock(const MutexState& s, uint32_t lock, const Ctl& ctl,
                           MutexHold* hold = nullptr) {
  __shared__ uint32_t s_ok;
  if (is_leader()) {
    uint32_t* m = s.lockw + (size_t)lock * s.stride;
    Wait w(ctl, KIND == SP_MUTEX_SLEEP ? s.poll_sleep : 0);
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
    } else {
      for (;;) {
        while (ld_relaxed(m) != 0)
          if (!(ok = w.tick())) break;
        if (!ok || cas_relaxed(m, 0, 1) == 0) break;
      }
    }
    if constexpr (FENCED) fence_acquire();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

// `hold`: the record mutex_lock filled in (leader's copy), or nullptr, in which case the
// ticket mutex loads turn to find the value to publish.
template <int KIND, bool FENCED = true>
__device__ void mutex_unlock(const MutexState& s, uint32_t lock, const MutexHold* hold = nullptr) {
  wave_stores_complete();
  __syncthreads();
  if (is_leader()) {
    uint32_t* w = KIND == SP_MUTEX_TICKET ? s.turn + (size_t)lock * s.stride
                                          : s.lockw + (size_t)lock * s.stride;
    // ticket: only the holder writes turn, so it can publish its own ticket + 1
    const uint32_t v = KIND != SP_MUTEX_TICKET ? 0u : (hold ? hold->ticket : ld_relaxed(w)) + 1;
    if constexpr (FENCED) st_release(w, v);
    else st_relaxed(w, v);
  }
}

}  // namespace sp
