// Device-side counting semaphores (Section 5, Semaphore; Algorithms 4-5; Table 4
// Wait()/Post()).  Block semantics as for the mutexes.
#pragma once

#include "atomics.hpp"

namespace sp {

struct SemState {
  uint32_t K;           // initial value: at most K workgroups inside
  uint32_t poll_sleep;  // SP_SEM_SLEEP: s_sleep units between polls
  uint32_t* S;          // Algorithm 4: S = K + 1 at rest, 0 while being updated
  uint32_t* count;      // Algorithm 5: workgroups inside or queued
  uint32_t* ticket;     // Algorithm 5: next queue ticket; counters: tickets drawn
  uint32_t* turn;       // Algorithm 5: number of queued workgroups admitted; counters:
                        // posts made
  BackoffCfg bo;        // SP_SEM_SPIN_BACKOFF
  uint32_t post_backoff;  // SP_SEM_SPIN_BACKOFF: 1 = post backs off too (Algorithm 4's
                          // listing); 0 = post retries at once (Section 5's prose)
};

// Per-workgroup waiting state that persists across waits (SP_SEM_ADAPTIVE).
struct SemHold {
  uint32_t interval;  // learned wall-clock ticks between two posts (0 = none yet)
};

// KIND: SP_SEM_SPIN / SP_SEM_SPIN_BACKOFF (Algorithm 4), SP_SEM_TICKET / SP_SEM_SLEEP
// (Algorithm 5, the queued waiter proceeds once turn is strictly greater than the
// 0-based ticket it drew), SP_SEM_COUNTERS (every waiter draws ticket t from one monotone
// counter and enters once the posts counter plus K exceeds t: the unit case of the
// weighted semaphore below, with Algorithm 5's FIFO order but one atomic per wait and
// one per post instead of Algorithm 5's two dependent ones on a queued post).
// SP_SEM_ADAPTIVE has SP_SEM_COUNTERS' admission rule and only waits differently: a
// waiter d posts short of admission sleeps about (d - 1) / 4 post intervals before it
// polls again, the next in line polls at the base rate.  The interval is a running
// average, kept in the workgroup's SemHold (which must persist across waits), of the rate
// at which the posts counter advanced between the waiter's first and last polls.  With
// 2048 workgroups queued on K = 32 the polling of one line otherwise slows the posts'
// atomics on that line (measured: a uniform s_sleep of 64 units between polls alone
// gives +47 %).
// FENCED = false: the data the semaphore guards is accessed with agent-scope loads and
// stores, which every XCD sees without cache maintenance, so wait skips the acquire
// invalidation and post the release writeback.
template <int KIND, bool FENCED = true>
__device__ bool sem_wait(const SemState& s, const Ctl& ctl, SemHold* hold = nullptr) {
  __shared__ uint32_t s_ok;
  if (is_leader()) {
    bool ok = true;
    if constexpr (KIND == SP_SEM_SPIN || KIND == SP_SEM_SPIN_BACKOFF) {
      Wait w(ctl, 0);
      Backoff bo(s.bo);
      for (;;) {
        const uint32_t v = exch_relaxed(s.S, 0);
        if (v > 1) {  // below capacity: take one unit
          exch_relaxed(s.S, v - 1);
          break;
        }
        if (v == 1) exch_relaxed(s.S, 1);  // at capacity: put the value back
        if constexpr (KIND == SP_SEM_SPIN_BACKOFF) bo(s.bo);
        if (!(ok = w.tick())) break;
      }
    } else if constexpr (KIND == SP_SEM_ADAPTIVE) {
      Wait w(ctl, s.poll_sleep);
      const uint32_t t = add_relaxed(s.ticket, 1);
      const uint32_t learned = hold ? hold->interval : 0;
      uint64_t t_first = 0, t_last = 0;
      uint32_t c_first = 0, c_last = 0;
      bool seen = false;
      for (;;) {
        const uint32_t posts = ld_relaxed(s.turn);
        const uint64_t now = wall_clock();
        if ((int32_t)(posts + s.K - t) > 0) break;
        if (!seen) {
          seen = true;
          t_first = now;
          c_first = posts;
        }
        t_last = now;
        c_last = posts;
        const uint32_t d = t - (posts + s.K) + 1;  // posts still needed, >= 1
        if (d > 1 && learned) {
          // (d - 1) / 4 intervals; one wall tick (10 ns) is ~0.375 s_sleep units
          const uint64_t units = ((uint64_t)(d - 1) * learned * 3) / 32;
          sleep_units(units < 4096 ? (uint32_t)units : 4096u);
        }
        if (!(ok = w.tick())) break;
      }
      if (hold) {
        const uint32_t moved = c_last - c_first;
        if (seen && moved > 0) {
          const uint32_t sample = (uint32_t)((t_last - t_first) / moved);
          const uint32_t avg = learned ? (7 * learned + sample) / 8 : sample;
          hold->interval = avg < 100000 ? avg : 100000;  // at most 1 ms of wall clock
        }
      }
    } else if constexpr (KIND == SP_SEM_COUNTERS) {
      Wait w(ctl, s.poll_sleep);
      const uint32_t t = add_relaxed(s.ticket, 1);
      uint32_t posts = ld_relaxed(s.turn);  // in flight with the ticket; a lower bound
      while (!((int32_t)(posts + s.K - t) > 0)) {
        if (!(ok = w.tick())) break;
        posts = ld_relaxed(s.turn);
      }
    } else {
      Wait w(ctl, KIND == SP_SEM_SLEEP ? s.poll_sleep : 0);
      const uint32_t old = add_relaxed(s.count, 1);
      if (old >= s.K) {  // at capacity: queue
        const uint32_t idx = add_relaxed(s.ticket, 1);
        while (!((int32_t)(ld_relaxed(s.turn) - idx) > 0))
          if (!(ok = w.tick())) break;
      }
    }
    if constexpr (FENCED) fence_acquire();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

template <int KIND, bool FENCED = true>
__device__ bool sem_post(const SemState& s, const Ctl& ctl) {
  __shared__ uint32_t s_ok;
  wave_stores_complete();
  __syncthreads();
  if (is_leader()) {
    bool ok = true;
    if constexpr (FENCED) fence_release();
    if constexpr (KIND == SP_SEM_SPIN || KIND == SP_SEM_SPIN_BACKOFF) {
      Wait w(ctl, 0);
      Backoff bo(s.bo);
      for (;;) {
        const uint32_t v = exch_relaxed(s.S, 0);
        if (v > 0) {
          exch_relaxed(s.S, v + 1);
          break;
        }
        if constexpr (KIND == SP_SEM_SPIN_BACKOFF)
          if (s.post_backoff) bo(s.bo);
        if (!(ok = w.tick())) break;
      }
    } else if constexpr (KIND == SP_SEM_COUNTERS || KIND == SP_SEM_ADAPTIVE) {
      add_relaxed(s.turn, 1);
    } else {
      const uint32_t old = add_relaxed(s.count, 0xFFFFFFFFu);  // count -= 1
      if (old > s.K) add_relaxed(s.turn, 1);                   // admit one queued waiter
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok;
}

// ---- weighted fetch-and-add semaphore --------------------------------------------------
// Algorithm 5 admits one unit per ticket.  A request that needs u units of a budget of K
// draws u consecutive tickets with one fetch-and-add, [t, t + u), and is admitted once the
// units ever returned plus K cover its last ticket: released + K >= t + u.  Returned units
// only grow, so admitted requests hold at most K units at any time whatever order the
// tickets were drawn in (every admitted range lies below the largest admitted end T, and
// released >= T - K held when that request was admitted).  Admission is FIFO in ticket
// order, and a request with u <= K always gets in once the ranges below it are returned.
// Waiting costs one atomic plus polling loads; posting one atomic.  The budget guards
// capacity, not data, so FENCE = false skips the acquire/release fences.
struct WSemState {
  uint32_t K;
  uint32_t poll_sleep;
  uint32_t* issued;    // tickets drawn so far (units)
  uint32_t* released;  // units returned so far
};

// Leader-only (no workgroup barrier): returns false when the watchdog fired.
template <bool FENCE>
__device__ __forceinline__ bool wsem_wait_leader(const WSemState& s, uint32_t u, const Ctl& ctl) {
  // The first load of `released` does not depend on the fetch-and-add, so both are in
  // flight together; a value older than the ticket is a lower bound and only delays.
  const uint32_t end = add_relaxed(s.issued, u) + u;
  uint32_t rel = ld_relaxed(s.released);
  Wait w(ctl, s.poll_sleep);
  while (!reached(rel + s.K, end)) {
    if (!w.tick()) return false;
    rel = ld_relaxed(s.released);
  }
  if constexpr (FENCE) fence_acquire();
  return true;
}

template <bool FENCE>
__device__ __forceinline__ void wsem_post_leader(const WSemState& s, uint32_t u) {
  if constexpr (FENCE) fence_release();
  add_relaxed(s.released, u);
}

}  // namespace sp
