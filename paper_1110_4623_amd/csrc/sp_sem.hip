// Counting semaphores: state objects and the wait/hold/post workload (Section 5,
// Semaphore; Section 6's wait-then-post loop, here with a tracked occupancy and holds).
#include <string.h>

#include "sp/semaphore.hpp"
#include "sp_internal.hpp"

struct sp_sem {
  sp_ctx* ctx = nullptr;
  uint32_t kind = 0;  // SP_SEM_* or SP_SEM_DEFAULT (resolved per run)
  uint32_t K = 0;
  sp_params p{};
  uint32_t* d_state = nullptr;
  uint64_t state_words = 0;
  uint32_t* d_owner = nullptr;  // K <= kMaxPool: owner word of each pool slot, kOwnerWords apart
  uint32_t* d_cq = nullptr;     // SP_SEM_COHORT, SP_SEM_ARRAY (and DEFAULT): the queues
  uint64_t cq_words = 0;
  uint32_t cq_stride = 0;
};

namespace {

// Line indices of the semaphore state (each line `stride` words).
enum { L_S = 0, L_COUNT, L_TICKET, L_TURN, L_OCC, L_MAXOCC, L_ADM, L_PRIVATE, L_LINES };
// Guarded data: a pool of K slots for K <= kMaxPool, owner words 32 bytes apart.
constexpr uint32_t kMaxPool = 4096;
constexpr uint32_t kOwnerWords = 8;
// Algorithm 4's waiter backoff cap when the caller names no backoff policy (s_sleep units).
constexpr uint32_t kAlg4BackoffCap = 8192;
// Grant slots of each XCD's queue (cohort kind; the array and chain kinds use the first
// queue's).  Any number is correct for the first two: a cohort post waits for a slot's
// previous ticket to take its grant before it writes the next one, an array post's grant
// is a maximum.  The chain kind uses the largest multiple of K that fits.
constexpr uint32_t kCohortSlots = 4096;

// The wait/hold/post workload.  With `data` (K uint32 words, packed, plain memory) every
// holder also updates guarded data: for K = 1 the semaphore is a mutex and the data is
// the one word, ordered by the semaphore's own acquire and release; for K > 1 the holder
// claims a free slot of a pool of K (compare-and-swap on the slot's owner word, then the
// acquire the hand-over of the slot needs), and returns it with a release before it posts.
// The update is a plain load and store by the workgroup's last thread (another wavefront
// than the leader's when lanes > 64), so the totals are exact only if the fences order it.
template <int KIND, bool FENCED>
__global__ SP_FULL_OCCUPANCY void k_sem(sp::SemState s, uint32_t stride, uint32_t* state, uint32_t nwg,
                      uint64_t total, uint32_t max_hold, uint32_t seed, uint32_t track,
                      uint32_t* chk, uint32_t* data, uint32_t* owner, uint32_t* err,
                      uint64_t timeout) {
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  __shared__ uint32_t s_slot;
  const uint32_t b = blockIdx.x;
  const uint64_t A = total / nwg + (b < total % nwg ? 1 : 0);
  uint32_t* occ = state + L_OCC * stride;
  uint32_t* maxocc = state + L_MAXOCC * stride;
  const bool pool = data && s.K > 1;
  uint32_t c = 0;
  sp::SemHold sh{0};  // the adaptive kind's learned post interval, kept across waits
  for (uint64_t j = 0; j < A; ++j) {
    const uint32_t hold = sp::sched_key(seed, b, (uint32_t)j, 3) % (max_hold + 1);
    if (!sp::sem_wait<KIND, FENCED>(s, ctl, &sh)) return;
    if (sp::is_leader()) {
      if (track) sp::max_relaxed(maxocc, sp::add_relaxed(occ, 1) + 1);
      c ^= sp::sm32(seed ^ (b << 16) ^ (uint32_t)j);
      uint32_t slot = 0;
      if (pool) {
        // at most K holders, so some slot is free; start where the schedule says
        sp::Wait w(ctl, 0);
        slot = sp::sched_key(seed, b, (uint32_t)j, 4) % s.K;
        while (sp::cas_relaxed(owner + (size_t)slot * kOwnerWords, 0, b + 1) != 0) {
          slot = slot + 1 == s.K ? 0 : slot + 1;
          if (!w.tick()) {
            slot = s.K;
            break;
          }
        }
        if constexpr (FENCED) sp::fence_acquire();
      }
      s_slot = slot;
    }
    __syncthreads();
    const uint32_t slot = s_slot;
    if (slot >= s.K) return;  // the watchdog ended the run
    if (data && threadIdx.x == blockDim.x - 1) {
      if constexpr (FENCED) data[slot] = data[slot] + 1;
      else sp::st_relaxed(data + slot, sp::ld_relaxed(data + slot) + 1);
    }
    if (sp::is_leader()) {
      sp::spin_cycles(hold);
      if (track) sp::add_relaxed(occ, 0xFFFFFFFFu);
    }
    if (pool) {
      sp::wave_stores_complete();
      __syncthreads();
      if (sp::is_leader()) {
        if constexpr (FENCED) sp::st_release(owner + (size_t)slot * kOwnerWords, 0);
        else sp::st_relaxed(owner + (size_t)slot * kOwnerWords, 0);
      }
    }
    if (!sp::sem_post<KIND, FENCED>(s, ctl, &sh)) return;
  }
  if (sp::is_leader()) {
    chk[b] = c;
    sp::add_relaxed(state + L_ADM * stride, (uint32_t)A);
  }
}

__global__ void k_sem_state(const uint32_t* state, uint32_t stride, uint32_t alg4,
                            const uint32_t* cq, uint32_t cq_stride, uint32_t cq_len,
                            const uint32_t* arr, uint32_t nq, uint32_t* out) {
  if (threadIdx.x == 0) {
    // cohort kind: local tickets drawn but never served, over the queues in use (0 at rest)
    uint32_t unserved = 0;
    if (cq)
      for (uint32_t x = 0; x < nq; ++x) {
        const uint32_t* b = cq + (size_t)x * (2 + cq_len) * cq_stride;
        unserved += b[0] - b[cq_stride];
      }
    out[0] = state[L_MAXOCC * stride];
    out[1] = alg4 ? state[L_S * stride] : state[L_COUNT * stride];
    // array and chain kinds: the low halves of their 64-bit tickets and posts counters,
    // summed over the queues that hold them
    uint32_t tickets = 0, posts = 0;
    for (uint32_t x = 0; arr && x < nq; ++x) {
      const uint32_t* b = arr + (size_t)x * (2 + cq_len) * cq_stride;
      tickets += b[0];
      posts += b[cq_stride];
    }
    out[2] = arr ? tickets : state[L_TICKET * stride];
    out[3] = arr ? posts : state[L_TURN * stride];
    out[4] = state[L_ADM * stride];
    out[5] = state[L_COUNT * stride];
    out[6] = state[L_OCC * stride];
    out[7] = unserved;
  }
}

// FENCED = false is the variant for critical sections that access their data coherently
// (agent-scope loads and stores of the guarded data).
template <bool FENCED>
const void* sem_kernel_f(uint32_t kind) {
  switch (kind) {
    case SP_SEM_SPIN: return (const void*)k_sem<SP_SEM_SPIN, FENCED>;
    case SP_SEM_SPIN_BACKOFF: return (const void*)k_sem<SP_SEM_SPIN_BACKOFF, FENCED>;
    case SP_SEM_TICKET: return (const void*)k_sem<SP_SEM_TICKET, FENCED>;
    case SP_SEM_SLEEP: return (const void*)k_sem<SP_SEM_SLEEP, FENCED>;
    case SP_SEM_COUNTERS: return (const void*)k_sem<SP_SEM_COUNTERS, FENCED>;
    case SP_SEM_ADAPTIVE: return (const void*)k_sem<SP_SEM_ADAPTIVE, FENCED>;
    case SP_SEM_COHORT: return (const void*)k_sem<SP_SEM_COHORT, FENCED>;
    case SP_SEM_ARRAY: return (const void*)k_sem<SP_SEM_ARRAY, FENCED>;
    case SP_SEM_CHAIN: return (const void*)k_sem<SP_SEM_CHAIN, FENCED>;
    case SP_SEM_XCD_CHAIN: return (const void*)k_sem<SP_SEM_XCD_CHAIN, FENCED>;
    case SP_SEM_CU_LOCK: return (const void*)k_sem<SP_SEM_CU_LOCK, FENCED>;
    default: return nullptr;
  }
}

// SP_SEM_XCD_CHAIN: a unit for every XCD's queue and at most a slot per chain in each.
bool xchain_fits(const sp_ctx* ctx, uint32_t K) {
  const uint32_t n = std::min<uint32_t>(std::max<uint32_t>(ctx->xcd_count, 1), sp::kXccQueues);
  return K >= n && K / n + (K % n ? 1u : 0u) <= kCohortSlots;
}

const void* sem_kernel(uint32_t kind, bool coherent_cs) {
  return coherent_cs ? sem_kernel_f<false>(kind) : sem_kernel_f<true>(kind);
}

}  // namespace

extern "C" {

int sp_sem_create(sp_ctx* ctx, uint32_t kind, uint32_t K, const sp_params* p, sp_sem** out) {
  if (!spi::usable(ctx) || !out || K == 0 || K >= (1u << 30)) return SP_E_INVAL;
  if (kind > SP_SEM_CU_LOCK && kind != SP_SEM_DEFAULT) return SP_E_INVAL;
  if (kind == SP_SEM_CU_LOCK && K != 1) return SP_E_INVAL;  // a binary semaphore
  if (kind == SP_SEM_CHAIN && K > kCohortSlots) return SP_E_INVAL;  // a slot per chain at least
  if (kind == SP_SEM_XCD_CHAIN && !xchain_fits(ctx, K)) return SP_E_INVAL;
  *out = nullptr;
  sp_params q;
  SP_CHECK(spi::normalize(ctx, p, &q));
  SP_HIP(ctx, hipSetDevice(ctx->device));
  sp_sem* s = new sp_sem();
  s->ctx = ctx;
  s->kind = kind;
  s->K = K;
  s->p = q;
  s->state_words = (uint64_t)L_LINES * 1024;  // room for the widest padding
  hipError_t e = hipMalloc(&s->d_state, s->state_words * sizeof(uint32_t));
  if (e == hipSuccess && K <= kMaxPool)
    e = hipMalloc(&s->d_owner, (size_t)K * kOwnerWords * sizeof(uint32_t));
  if (e == hipSuccess && (kind == SP_SEM_COHORT || kind == SP_SEM_ARRAY ||
                          kind == SP_SEM_CHAIN || kind == SP_SEM_XCD_CHAIN ||
                          kind == SP_SEM_CU_LOCK || kind == SP_SEM_DEFAULT)) {
    // queues for the cohort, array and chain kinds (a DEFAULT semaphore may resolve to
    // any of them): allocated now, so that every run can be recorded into a graph
    // even, for the 64-bit slots; at least 4 for the CU-cohort lock's session record
    s->cq_stride = std::max<uint32_t>(4, spi::stride_words(q));
    s->cq_words = (uint64_t)sp::kXccQueues * (2 + kCohortSlots) * s->cq_stride;
    e = hipMalloc(&s->d_cq, s->cq_words * sizeof(uint32_t));
  }
  if (e != hipSuccess) {
    ctx->last_hip = (int)e;
    (void)hipFree(s->d_state);
    (void)hipFree(s->d_owner);
    delete s;
    return SP_E_HIP;
  }
  spi::ctx_ref(ctx);
  *out = s;
  return SP_OK;
}

int sp_sem_destroy(sp_sem* s) {
  if (!s) return SP_E_INVAL;
  sp_ctx* ctx = s->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipFree(s->d_state);
  if (s->d_owner) (void)hipFree(s->d_owner);
  if (s->d_cq) (void)hipFree(s->d_cq);
  delete s;
  spi::ctx_unref(ctx);
  return SP_OK;
}

int sp_sem_run(sp_sem* sem, uint32_t nwg, uint32_t lanes, uint64_t total_pairs,
               uint32_t max_hold_cyc, uint32_t seed, uint32_t track, uint32_t* out_chk,
               uint32_t* out_state, uint32_t* out_data, sp_stats* st, void* stream) {
  if (!sem || !out_chk || !out_state || nwg == 0 || !spi::lanes_ok(lanes) ||
      max_hold_cyc == 0xFFFFFFFFu || total_pairs >= (1ull << 32))
    return SP_E_INVAL;
  if (out_data && sem->K > kMaxPool) return SP_E_INVAL;
  sp_ctx* ctx = sem->ctx;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  uint32_t kind = sem->kind;
  sp_params q = sem->p;
  if (kind == SP_SEM_DEFAULT) {
    const sp_default_entry& d = ctx->defaults[2][spi::bucket_of(nwg / sem->K)];
    kind = d.kind;
    const uint32_t t = q.timeout_ms;
    const uint32_t coherent = q.coherent_cs;  // a property of the caller's critical sections
    q = d.p;
    q.timeout_ms = t;
    q.coherent_cs = coherent;
    // the chain kinds need at least a unit per queue and a slot per chain: outside their
    // range the next kind (per-XCD chains, one set of chains, the array kind)
    if (kind == SP_SEM_XCD_CHAIN && !xchain_fits(ctx, sem->K)) kind = SP_SEM_CHAIN;
    if (kind == SP_SEM_CHAIN && sem->K > kCohortSlots) kind = SP_SEM_ARRAY;
    // K = 1 with at least two workgroups per CU: the CU-cohort lock (2048 workgroups,
    // holds U[0, 2000] clocks: 0.76 against 0.59 M pairs/s for one chain, fenced)
    if (kind == SP_SEM_CHAIN && sem->K == 1 && spi::cu_cohort_pays(nwg, 1, ctx->cu_count))
      kind = SP_SEM_CU_LOCK;
  }
  if (kind == SP_SEM_SPIN_BACKOFF && q.backoff == SP_BACKOFF_NONE) {
    // No policy chosen: exponential, capped at 8192 units.  With posts retrying at once,
    // a 32-unit cap lets 256-2048 waiters keep S busy until the watchdog (measured).
    q.backoff = SP_BACKOFF_EXP;
    q.backoff_max = std::max<uint32_t>(q.backoff_max, kAlg4BackoffCap);
  }
  if (kind != SP_SEM_SPIN_BACKOFF) q.backoff = SP_BACKOFF_NONE;
  const void* kern = sem_kernel(kind, q.coherent_cs != 0);
  if (!kern) return SP_E_INVAL;
  const uint32_t sw = spi::stride_words(q);
  uint32_t* base = sem->d_state;
  sp::SemState ss;
  ss.K = sem->K;
  ss.poll_sleep = q.poll_sleep;
  ss.S = base + L_S * sw;
  ss.count = base + L_COUNT * sw;
  ss.ticket = base + L_TICKET * sw;
  ss.turn = base + L_TURN * sw;
  ss.bo = spi::backoff_cfg(q, base + L_PRIVATE * sw);
  ss.post_backoff = q.post_backoff;
  ss.cq = sem->d_cq;
  // one queue per XCD (every XCC id the dispatcher uses lands in one of them)
  ss.cq_n = std::min<uint32_t>(std::max<uint32_t>(ctx->xcd_count, 1), sp::kXccQueues);
  ss.cq_local = ctx->xcc_mask == (1u << ss.cq_n) - 1;
  ss.cq_stride = sem->cq_stride;
  ss.cq_len = kCohortSlots;
  ss.cohort_bound = q.cohort_passes;
  ss.chain_len = sem->K <= kCohortSlots ? kCohortSlots / sem->K * sem->K : kCohortSlots;
  const bool queued = kind == SP_SEM_COHORT || kind == SP_SEM_ARRAY || kind == SP_SEM_CHAIN ||
                      kind == SP_SEM_XCD_CHAIN || kind == SP_SEM_CU_LOCK;
  if (queued && !sem->d_cq) return SP_E_INVAL;
  SP_CHECK(spi::fill_u32(ctx, base, sem->state_words, 0, s));
  // the queues a run uses: one per XCD (cohort, per-XCD chains) or queue 0 (array, chain)
  const uint32_t nq = kind == SP_SEM_ARRAY || kind == SP_SEM_CHAIN ? 1u : ss.cq_n;
  const uint64_t cu_lock_lines =
      (uint64_t)sp::kXccSlots * (sp::kCohortLines + sp::kCuIds * sp::kCuLines);
  const uint64_t qwords = kind == SP_SEM_CU_LOCK ? cu_lock_lines * sem->cq_stride
                                                 : (uint64_t)nq * (2 + kCohortSlots) * sem->cq_stride;
  if (queued) SP_CHECK(spi::fill_u32(ctx, sem->d_cq, qwords, 0, s));
  if (out_data) {
    SP_CHECK(spi::fill_u32(ctx, out_data, sem->K, 0, s));
    if (sem->K > 1) SP_CHECK(spi::fill_u32(ctx, sem->d_owner, (uint64_t)sem->K * kOwnerWords, 0, s));
  }
  uint32_t* owner = sem->d_owner;
  if (kind == SP_SEM_SPIN || kind == SP_SEM_SPIN_BACKOFF)
    SP_CHECK(spi::fill_u32(ctx, ss.S, 1, sem->K + 1, s));  // Algorithm 4: S = K + 1
  uint32_t per_cu = 0;
  SP_CHECK(spi::resident_per_cu(ctx, kern, lanes, &per_cu));
  SP_CHECK(spi::begin_timed(ctx, s));
  uint64_t timeout = spi::timeout_ticks(ctx, q);
  uint32_t stride = sw;
  void* args[] = {&ss, &stride, &base, &nwg, &total_pairs, &max_hold_cyc, &seed, &track,
                  &out_chk, &out_data, &owner, &ctx->d_err, &timeout};
  SP_HIP(ctx, hipLaunchKernel(kern, dim3(nwg), dim3(lanes), args, 0, s));
  int rc = spi::end_timed(ctx, s, st, nwg, lanes, (uint32_t)per_cu, total_pairs);
  const uint32_t alg4 = kind == SP_SEM_SPIN || kind == SP_SEM_SPIN_BACKOFF;
  const uint32_t* cq = kind == SP_SEM_COHORT ? sem->d_cq : nullptr;
  const uint32_t* arr = kind == SP_SEM_ARRAY || kind == SP_SEM_CHAIN || kind == SP_SEM_XCD_CHAIN
                            ? sem->d_cq : nullptr;
  hipLaunchKernelGGL(k_sem_state, dim3(1), dim3(64), 0, s, base, sw, alg4, cq, sem->cq_stride,
                     kCohortSlots, arr, queued ? nq : 0u, out_state);
  SP_HIP(ctx, hipGetLastError());
  SP_CHECK(spi::sync_unless_capturing(ctx, s));
  return rc;
}

}  // extern "C"
