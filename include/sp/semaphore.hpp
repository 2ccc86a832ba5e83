// Device-side counting semaphores (Section 5, Semaphore; Algorithms 4-5; Table 4
// Wait()/Post()).  Block semantics as for the mutexes.
#pragma once

#include "atomics.hpp"
#include "mutex.hpp"

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
  // SP_SEM_COHORT: per XCD (cq_n of them; a workgroup queues on XCC id mod cq_n) a queue
  // of cq_len 64-bit grant slots, after two lines (local tickets drawn, local tickets
  // served); lines cq_stride words apart (even, so the 64-bit slots are aligned)
  uint32_t* cq;
  uint32_t cq_n;         // queues in use, 1..kXccQueues
  uint32_t cq_local;     // 1: every XCC id is below cq_n, so queue x holds XCD x's
                         // workgroups only (the cohort kind's K = 1 writeback skip and
                         // the per-XCD chains' skip rely on it)
  uint32_t cq_stride;
  uint32_t cq_len;       // power of two
  uint32_t cohort_bound; // local hand-overs of one unit in a row, at most
  // SP_SEM_ARRAY and SP_SEM_CHAIN use queue 0's memory: line 0 the tickets drawn, line 1
  // the posts made (64-bit counters), then the cq_len 64-bit grant slots; SP_SEM_XCD_CHAIN
  // lays out every queue in use that way.
  uint32_t chain_len;    // SP_SEM_CHAIN: slots in use, the largest multiple of K <= cq_len
};

// Per-workgroup waiting state that persists across waits (SP_SEM_ADAPTIVE), or from a
// wait to its post (SP_SEM_COHORT, SP_SEM_CHAIN, SP_SEM_XCD_CHAIN).
struct SemHold {
  uint32_t interval;  // learned wall-clock ticks between two posts (0 = none yet)
  uint32_t pass;      // SP_SEM_COHORT: local hand-overs of the unit held, in a row;
                      // SP_SEM_XCD_CHAIN: the queue the unit belongs to
  uint64_t ticket;    // SP_SEM_CHAIN, SP_SEM_XCD_CHAIN: the ticket the unit was taken with
  MutexHold lock;     // SP_SEM_CU_LOCK: what the lock's unlock needs
};

// SP_SEM_CU_LOCK: K = 1 makes the semaphore a binary one, i.e. a lock, run here as the
// CU-cohort lock.  Its state sits in the semaphore's memory: the global ticket and turn on
// the ticket / turn lines, the XCD cohorts' lines and then the CU cohorts' lines in the
// queue memory, cq_stride (>= 4) words apart.
__device__ __forceinline__ MutexState cu_lock_state(const SemState& s) {
  MutexState m{};
  m.stride = 0;  // one lock
  m.poll_sleep = s.poll_sleep;
  m.ticket = s.ticket;
  m.turn = s.turn;
  m.queue = s.cq;
  m.qlen = 1;
  m.qstride = s.cq_stride;
  m.cohort_bound = s.cohort_bound;
  m.bo = s.bo;
  m.cuq = s.cq + (size_t)kXccSlots * kCohortLines * s.cq_stride;
  return m;
}

// ---- cohort semaphore queues -------------------------------------------------------------
constexpr uint32_t kXccQueues = 16;  // the XCC id register has four bits
__device__ __forceinline__ uint32_t* cq_base(const SemState& s, uint32_t x) {
  return s.cq + (size_t)x * (2 + s.cq_len) * s.cq_stride;
}
__device__ __forceinline__ uint32_t* cq_drawn(const SemState& s, uint32_t x) { return cq_base(s, x); }
__device__ __forceinline__ uint32_t* cq_served(const SemState& s, uint32_t x) {
  return cq_base(s, x) + s.cq_stride;
}
__device__ __forceinline__ uint64_t* cq_slot(const SemState& s, uint32_t x, uint32_t t) {
  return reinterpret_cast<uint64_t*>(cq_base(s, x) +
                                     (size_t)(2 + (t & (s.cq_len - 1))) * s.cq_stride);
}

// ---- per-XCD chains ----------------------------------------------------------------------
// Units of queue x; at least one, since K >= cq_n for this kind (sp_sem_create refuses a
// smaller K, and a default semaphore runs the one-chain kind there).
__device__ __forceinline__ uint32_t xchain_units(const SemState& s, uint32_t x) {
  return s.K / s.cq_n + (x < s.K % s.cq_n ? 1u : 0u);
}
__device__ __forceinline__ uint64_t* xchain_slot(const SemState& s, uint32_t x, uint32_t kx,
                                                 uint64_t t) {
  const uint32_t m = s.cq_len / kx * kx;
  return reinterpret_cast<uint64_t*>(cq_base(s, x) + (size_t)(2 + t % m) * s.cq_stride);
}

// ---- array semaphore (ticket-indexed grant slots); 64-bit counters of the slot kinds ----
__device__ __forceinline__ uint64_t add_relaxed64(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t max_relaxed64(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t* as_tickets(const SemState& s) {
  return reinterpret_cast<uint64_t*>(cq_base(s, 0));
}
__device__ __forceinline__ uint64_t* as_posts(const SemState& s) {
  return reinterpret_cast<uint64_t*>(cq_base(s, 0) + s.cq_stride);
}
__device__ __forceinline__ uint64_t* as_slot(const SemState& s, uint64_t t) {
  return reinterpret_cast<uint64_t*>(cq_base(s, 0) +
                                     (size_t)(2 + (t & (s.cq_len - 1))) * s.cq_stride);
}
__device__ __forceinline__ uint64_t* chain_slot(const SemState& s, uint64_t t) {
  return reinterpret_cast<uint64_t*>(cq_base(s, 0) + (size_t)(2 + t % s.chain_len) * s.cq_stride);
}

namespace detail {

__device__ __forceinline__ uint64_t cas_relaxed64(uint64_t* p, uint64_t expected,
                                                  uint64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found
}

// Claims XCD x's oldest unserved local ticket (compare-and-swap on its served counter),
// starting from the counters `served` and `drawn` already loaded; false when every ticket
// drawn so far is served.
__device__ __forceinline__ bool cq_claim_at(const SemState& s, uint32_t x, uint32_t served,
                                            uint32_t drawn, uint32_t* t) {
  uint32_t* sp = cq_served(s, x);
  uint32_t v = served;
  while ((int32_t)(drawn - v) > 0) {
    const uint32_t seen = cas_relaxed(sp, v, v + 1);
    if (seen == v) {
      *t = v;
      return true;
    }
    v = seen;
    drawn = ld_relaxed(cq_drawn(s, x));
  }
  return false;
}

__device__ __forceinline__ bool cq_claim(const SemState& s, uint32_t x, uint32_t* t) {
  const uint32_t served = ld_relaxed(cq_served(s, x));
  const uint32_t drawn = ld_relaxed(cq_drawn(s, x));
  return cq_claim_at(s, x, served, drawn, t);
}

// Claims a ticket on the first XCD (in the order first, first + 1, ...) that has one;
// retries until one is found (a waiter counted in `count` draws its ticket within a round
// trip).  One round trip per queue tried: the preferred queue usually has a waiter, and
// loading every queue's counters first was measured slower (an extra round trip before
// every claim).  Returns false when the watchdog fired.
__device__ __forceinline__ bool cq_claim_from(const SemState& s, uint32_t first, uint32_t* y,
                                              uint32_t* t, Wait& w) {
  const uint32_t n = s.cq_n;
  if (first >= n) first -= n;
  for (;;) {
    uint32_t x = first;
    for (uint32_t d = 0; d < n; ++d) {
      if (cq_claim(s, x, t)) {
        *y = x;
        return true;
      }
      if (++x == n) x = 0;
    }
    if (!w.tick()) return false;
  }
}

// Grants ticket t of XCD y with pass count k, once the slot's previous ticket (t - cq_len)
// has taken its grant.  A compare-and-swap from empty, not a check then a store: the
// previous ticket's own grant may still be on its way from another poster, and a store
// after a check could overwrite it.
__device__ __forceinline__ bool cq_grant(const SemState& s, uint32_t y, uint32_t t, uint32_t k,
                                         Wait& w) {
  uint64_t* slot = cq_slot(s, y, t);
  const uint64_t g = ((uint64_t)k << 32) | (uint64_t)(t + 1);
  while (cas_relaxed64(slot, 0, g) != 0)
    if (!w.tick()) return false;
  return true;
}

}  // namespace detail

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
// SP_SEM_ARRAY has SP_SEM_COUNTERS' admission rule with the admitting post telling the
// waiter directly: the post that draws p (0-based, from the posts counter) raises grant
// slot (p + K) mod len to p + K + 1 with an atomic max, and ticket t >= K waits until its
// slot holds at least t + 1.  Each waiter polls a line of its own, so the posts counter's
// line carries only the posts' atomics (with ~2000 waiters on the counter's line the
// polling, not the cache maintenance, limits the other two-counter kinds).
//   At most K inside: a slot value v >= t + 1 is some post's p + K + 1 with p + K >= t,
//   so that post has drawn p >= t - K, and posts > t - K when t enters -- the
//   two-counter rule; every entered ticket is below posts + K, so at most posts + K
//   tickets have entered and at most K of them have not posted.
//   Every waiter enters: tickets below t enter and post (induction), the post that draws
//   t - K then raises slot t mod len to at least t + 1, and a maximum never decreases.
//   The slots may be reused in any order (len any power of two): a grant for a later
//   ticket of the same slot is larger, so it admits the earlier one too, which the rule
//   already allows; an earlier grant landing late cannot lower it.  64-bit counters and
//   slots do not wrap.
// SP_SEM_CHAIN ties each unit to a chain of tickets instead: ticket t >= K enters once
// the holder of ticket t - K has posted, and that post stores t + 1 into slot t mod M
// itself, with no atomic to wait for (M = chain_len, a multiple of K).  The post needs
// the ticket its own workgroup's wait drew (SemHold::ticket), so it must follow that
// wait; the posts counter is only counted, for the state at rest.
//   At most K inside: entering ticket t >= K needs a post by the holder of t - K, so the
//   tickets at or above K that have entered map one to one onto tickets that have
//   posted, and at most K + posts tickets have entered.
//   Every waiter enters: by induction, ticket t - K enters and posts.
//   Slots: t and t + M (M a multiple of K) lie on one chain, t first, so the store for
//   t + M comes after t has entered (the holder of t + M - K entered after t posted) and
//   the store for t - M landed before t - K could enter; while t waits its slot holds
//   t + 1 or an older ticket's value.  With M not a multiple of K a later chain's store
//   could admit t early (the model checker finds the bound broken).
// SP_SEM_XCD_CHAIN runs the chain rule once per XCD: queue x (XCC id mod cq_n) owns
// K_x = K / cq_n units (the first K mod cq_n queues one more, every queue at least one)
// and its own tickets, posts and chain_slots (in queue x's memory, the largest multiple
// of K_x up to cq_len).  Each queue is a chain semaphore of K_x units, so at most
// sum K_x = K inside, and every waiter enters (its queue has a unit).  When every XCC id
// is below cq_n (cq_local), a queue's workgroups share one L2: the next holder of a chain
// reads the critical section's stores (completed into that L2 before the post) after its
// own acquire, so the post skips the writeback.  Data shared with other XCDs needs a
// synchronization that writes this L2 back anyway.  Otherwise the post writes back.
// FENCED = false: the data the semaphore guards is accessed with agent-scope loads and
// stores, which every XCD sees without cache maintenance, so wait skips the acquire
// invalidation and post the release writeback.
template <int KIND, bool FENCED = true>
__device__ bool sem_wait(const SemState& s, const Ctl& ctl, SemHold* hold = nullptr) {
  if constexpr (KIND == SP_SEM_CU_LOCK)
    return mutex_lock<SP_MUTEX_CU_COHORT, FENCED>(cu_lock_state(s), 0, ctl, &hold->lock);
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
    } else if constexpr (KIND == SP_SEM_COHORT) {
      // Algorithm 5's count; a waiter beyond capacity queues on its own XCD and takes the
      // unit a poster grants it (with the unit's count of local hand-overs in a row)
      Wait w(ctl, s.poll_sleep);
      uint32_t k = 0;
      const uint32_t old = add_relaxed(s.count, 1);
      if (old >= s.K) {
        const uint32_t x = xcc_id() % s.cq_n;
        const uint32_t t = add_relaxed(cq_drawn(s, x), 1);
        uint64_t* slot = cq_slot(s, x, t);
        uint64_t v = 0;
        for (;;) {
          v = ld_relaxed64(slot);
          if ((uint32_t)v == t + 1) break;
          if (!(ok = w.tick())) break;
        }
        if (ok) {
          k = (uint32_t)(v >> 32);
          st_relaxed64(slot, 0);  // taken: the slot may carry the grant of ticket t + len
        }
      }
      if (hold) hold->pass = k;
    } else if constexpr (KIND == SP_SEM_XCD_CHAIN) {
      Wait w(ctl, s.poll_sleep);
      const uint32_t x = xcc_id() % s.cq_n, kx = xchain_units(s, x);
      const uint64_t t = add_relaxed64(reinterpret_cast<uint64_t*>(cq_base(s, x)), 1);
      hold->ticket = t;
      hold->pass = x;  // the queue, for the post
      if (t >= kx) {
        const uint64_t* g = xchain_slot(s, x, kx, t);
        while (ld_relaxed64(g) <= t)
          if (!(ok = w.tick())) break;
      }
    } else if constexpr (KIND == SP_SEM_CHAIN) {
      Wait w(ctl, s.poll_sleep);
      const uint64_t t = add_relaxed64(as_tickets(s), 1);
      hold->ticket = t;
      if (t >= s.K) {
        const uint64_t* g = chain_slot(s, t);
        while (ld_relaxed64(g) <= t)
          if (!(ok = w.tick())) break;
      }
    } else if constexpr (KIND == SP_SEM_ARRAY) {
      Wait w(ctl, s.poll_sleep);
      const uint64_t t = add_relaxed64(as_tickets(s), 1);
      if (t >= s.K) {
        const uint64_t* g = as_slot(s, t);
        while (ld_relaxed64(g) <= t)
          if (!(ok = w.tick())) break;
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

// `hold`: SP_SEM_COHORT needs the record its sem_wait filled in (the unit's local
// hand-overs), SP_SEM_CHAIN and SP_SEM_XCD_CHAIN require it (the ticket and queue, so not
// null); other kinds ignore it.
template <int KIND, bool FENCED = true>
__device__ bool sem_post(const SemState& s, const Ctl& ctl, const SemHold* hold = nullptr) {
  if constexpr (KIND == SP_SEM_CU_LOCK) {
    mutex_unlock<SP_MUTEX_CU_COHORT, FENCED>(cu_lock_state(s), 0, &hold->lock, &ctl);
    return true;
  }
  __shared__ uint32_t s_ok;
  wave_stores_complete();
  __syncthreads();
  if constexpr (KIND == SP_SEM_COHORT) {
    // Hand the unit on.  Algorithm 5's post: write back, then decrement count; if a waiter
    // is beyond capacity the unit goes to the oldest waiter of this XCD while the unit has
    // passed fewer than cohort_bound times in a row here, else to the first other XCD with
    // a waiter.  K = 1, one XCD per queue (cq_local) and count > 1 (loaded): the poster
    // holds the only unit, so no other post can lower count before its own decrement,
    // which therefore returns more than 1: a waiter exists, and one of this XCD's (it
    // reads through the same L2) takes the unit without the writeback.  The decrement has
    // completed before the grant is written, so the next holder's load of count already
    // includes it.  For K >= 2 a loaded count proves nothing -- the other K - 1 units can
    // change hands any number of times before the decrement lands -- so every post writes
    // back first.
    if (is_leader()) {
      bool ok = true;
      Wait w(ctl, 0);
      const uint32_t x = xcc_id() % s.cq_n;
      const uint32_t k = hold ? hold->pass : s.cohort_bound;
      const bool stay = k + 1 < s.cohort_bound;
      uint32_t y = 0, t = 0, kk = 0;
      bool grant = true;
      // one round trip: the count and this XCD's queue counters, loaded together
      const uint32_t c = ld_relaxed(s.count);
      const uint32_t served = ld_relaxed(cq_served(s, x));
      const uint32_t drawn = ld_relaxed(cq_drawn(s, x));
      if (s.K == 1 && s.cq_local && c > 1) {
        add_relaxed(s.count, 0xFFFFFFFFu);
        if (stay && detail::cq_claim_at(s, x, served, drawn, &t)) {
          wave_stores_complete();  // the decrement is done before the grant store
          y = x;
          kk = k + 1;
        } else {
          if constexpr (FENCED) fence_release();
          ok = detail::cq_claim_from(s, x + 1, &y, &t, w);
        }
      } else {
        if constexpr (FENCED) fence_release();
        const uint32_t old = add_relaxed(s.count, 0xFFFFFFFFu);
        grant = old > s.K;
        if (grant) {
          // first with the counters loaded beside count: while they are current, one
          // compare-and-swap claims this XCD's oldest waiter
          if (stay && detail::cq_claim_at(s, x, served, drawn, &t))
            y = x;
          else
            ok = detail::cq_claim_from(s, stay ? x : x + 1, &y, &t, w);
          kk = y == x ? k + 1 : 0;
        }
      }
      if (ok && grant) ok = detail::cq_grant(s, y, t, kk, w);
      s_ok = ok;
    }
    __syncthreads();
    return s_ok;
  }
  if (is_leader()) {
    bool ok = true;
    if constexpr (FENCED) {
      if (KIND != SP_SEM_XCD_CHAIN || !s.cq_local) fence_release();
    }
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
    } else if constexpr (KIND == SP_SEM_ARRAY) {
      const uint64_t q = add_relaxed64(as_posts(s), 1) + s.K;  // the ticket this post admits
      max_relaxed64(as_slot(s, q), q + 1);
    } else if constexpr (KIND == SP_SEM_CHAIN) {
      const uint64_t q = hold->ticket + s.K;  // the next ticket of this unit's chain
      st_relaxed64(chain_slot(s, q), q + 1);
      add_relaxed64(as_posts(s), 1);
    } else if constexpr (KIND == SP_SEM_XCD_CHAIN) {
      const uint32_t x = hold->pass, kx = xchain_units(s, x);
      const uint64_t q = hold->ticket + kx;
      st_relaxed64(xchain_slot(s, x, kx, q), q + 1);
      add_relaxed64(reinterpret_cast<uint64_t*>(cq_base(s, x) + s.cq_stride), 1);
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
