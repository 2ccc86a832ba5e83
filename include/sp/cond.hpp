// Device-side condition variables (the future-work item of Section 7: semaphores are
// easy to misuse, condition variables over a mutex are the safer way to wait for a
// predicate).  Mesa semantics: a woken workgroup re-acquires the mutex and must re-test
// its predicate.  Block semantics as for the mutexes.
//
// A condition variable is two monotone counters on their own lines:
//   waiters  tickets drawn by workgroups that started waiting;
//   signals  tickets released by signal / broadcast.
// wait:      draw ticket t while still holding the mutex, unlock, poll until
//            signals > t, lock again.  Registering before the unlock is what rules out
//            lost wakeups: a signaller that holds the mutex afterwards sees the waiter.
// signal:    if some drawn ticket is not yet released (signals < waiters), release the
//            next one with a compare-and-swap; a signal with nobody waiting has no effect.
// broadcast: release every drawn ticket (signals = waiters).
// Waiters wake in ticket order.  Counters wrap; comparisons are signed differences.
#pragma once

#include "mutex.hpp"

namespace sp {

struct CondState {
  uint32_t* waiters;
  uint32_t* signals;
  uint32_t poll_sleep;  // s_sleep units between polls
};

// Called by the whole workgroup while it holds mutex `lock` (acquired with `hold`);
// returns holding it again, or false if the watchdog fired (the mutex is then not held).
template <int MKIND, bool FENCED = true>
__device__ bool cond_wait(const CondState& cv, const MutexState& m, uint32_t lock,
                          MutexHold* hold, const Ctl& ctl) {
  __shared__ uint32_t s_ok;
  __shared__ uint32_t s_ticket;
  if (is_leader()) s_ticket = add_relaxed(cv.waiters, 1);
  mutex_unlock<MKIND, FENCED>(m, lock, hold);
  if (is_leader()) {
    Wait w(ctl, cv.poll_sleep);
    bool ok = true;
    while (!((int32_t)(ld_relaxed(cv.signals) - s_ticket) > 0))
      if (!(ok = w.tick())) break;
    s_ok = ok;
  }
  __syncthreads();
  if (!s_ok) return false;
  return mutex_lock<MKIND, FENCED>(m, lock, ctl, hold);
}

// Leader-side helpers (called by the leader, normally while holding the mutex).
__device__ __forceinline__ void cond_signal_leader(const CondState& cv) {
  uint32_t s = ld_relaxed(cv.signals);
  for (;;) {
    const uint32_t w = ld_relaxed(cv.waiters);
    if ((int32_t)(w - s) <= 0) return;  // nobody waiting without a signal
    const uint32_t seen = cas_relaxed(cv.signals, s, s + 1);
    if (seen == s) return;
    s = seen;
  }
}

__device__ __forceinline__ void cond_broadcast_leader(const CondState& cv) {
  uint32_t s = ld_relaxed(cv.signals);
  for (;;) {
    const uint32_t w = ld_relaxed(cv.waiters);
    if ((int32_t)(w - s) <= 0) return;
    const uint32_t seen = cas_relaxed(cv.signals, s, w);
    if (seen == s) return;
    s = seen;
  }
}

}  // namespace sp
