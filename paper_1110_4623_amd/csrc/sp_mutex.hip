// Mutexes: state objects and the contention workload (Section 5, Mutex; Section 6's
// lock-then-unlock loop, here with a non-empty critical section and random delays).
#include <string.h>

#include "sp/mutex.hpp"
#include "sp_internal.hpp"

struct sp_mutex {
  sp_ctx* ctx = nullptr;
  uint32_t kind = 0;      // SP_MUTEX_* or SP_MUTEX_DEFAULT (resolved per run)
  uint32_t nlocks = 0;
  uint32_t W = 0;         // words per lock
  uint32_t wstride = 0;   // uint32 words between two locks' word blocks (line multiple)
  sp_params p{};
  uint32_t* d_state = nullptr;  // lock, ticket and turn lines + one private line
  uint64_t state_words = 0;
  uint32_t* d_words = nullptr;  // critical-section words, nlocks x wstride
  uint32_t* d_queue = nullptr;  // ring / array: slots, sized per run; cohort: at creation
  uint64_t queue_words = 0;
};

namespace {

// The cohort locks' state: lines per lock (each XCC id's ticket and grant slots, and for
// the CU cohort lock each CU's ticket, grant and session record), and the words between
// lines (64-bit grant words need two, the CU cohort's three-word record four).
uint32_t cohort_lines(uint32_t kind) {
  const uint32_t xcd = sp::kCohortLines * sp::kXccSlots;
  return kind == SP_MUTEX_CU_COHORT ? xcd + sp::kXccSlots * sp::kCuIds * sp::kCuLines : xcd;
}
uint32_t cohort_stride(uint32_t kind, uint32_t sw) {
  return std::max<uint32_t>(sw, kind == SP_MUTEX_CU_COHORT ? 4 : 2);
}
uint64_t cohort_words(uint32_t kind, uint32_t nlocks, uint32_t sw) {
  return (uint64_t)nlocks * cohort_lines(kind) * cohort_stride(kind, sw);
}

// With `owner` set, the leader swaps its id into the lock's owner word on entry and
// back out on exit; any other value seen means two workgroups were inside at once.
template <int KIND, bool FENCED>
__global__ SP_FULL_OCCUPANCY void k_mutex(sp::MutexState s, uint32_t nlocks, uint32_t W, uint32_t wstride,
                        uint32_t* words, uint32_t nwg, uint64_t total, uint32_t max_delay,
                        uint32_t seed, uint64_t* finish, uint32_t* owner, uint32_t* err,
                        uint64_t timeout) {
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  const uint32_t b = blockIdx.x;
  const uint64_t A = total / nwg + (b < total % nwg ? 1 : 0);
  sp::MutexHold hold{0, 0};  // persists: the adaptive mutex learns across acquisitions
  for (uint64_t j = 0; j < A; ++j) {
    const uint32_t lock = sp::sched_key(seed, b, (uint32_t)j, 1) % nlocks;
    if (sp::is_leader()) sp::spin_cycles(sp::sched_key(seed, b, (uint32_t)j, 2) % (max_delay + 1));
    if (!sp::mutex_lock<KIND, FENCED>(s, lock, ctl, &hold)) return;
    uint32_t* own = owner ? owner + (size_t)lock * s.stride : nullptr;
    if (own && sp::is_leader() && sp::exch_relaxed(own, b + 1) != 0)
      sp::cas_relaxed(err, sp::DEV_OK, sp::DEV_PARITY);
    uint32_t* wp = words + (size_t)lock * wstride;
    if constexpr (FENCED) {
      for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) wp[w] = wp[w] + 1;
    } else {  // coherent critical section: agent-scope loads and stores
      for (uint32_t w = threadIdx.x; w < W; w += blockDim.x)
        sp::st_relaxed(wp + w, sp::ld_relaxed(wp + w) + 1);
    }
    if (own && sp::is_leader() && sp::exch_relaxed(own, 0) != b + 1)
      sp::cas_relaxed(err, sp::DEV_OK, sp::DEV_PARITY);
    sp::mutex_unlock<KIND, FENCED>(s, lock, &hold, &ctl);
  }
  if (sp::is_leader() && finish) finish[b] = sp::wall_clock();
}

__global__ void k_gather_words(const uint32_t* words, uint32_t nlocks, uint32_t W,
                               uint32_t wstride, uint32_t* out) {
  const uint64_t n = (uint64_t)nlocks * W;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = words[(i / W) * wstride + i % W];
}

template <bool FENCED>
const void* mutex_kernel_f(uint32_t kind) {
  switch (kind) {
    case SP_MUTEX_SPIN_CAS: return (const void*)k_mutex<SP_MUTEX_SPIN_CAS, FENCED>;
    case SP_MUTEX_SPIN_EXCH: return (const void*)k_mutex<SP_MUTEX_SPIN_EXCH, FENCED>;
    case SP_MUTEX_SPIN_BACKOFF: return (const void*)k_mutex<SP_MUTEX_SPIN_BACKOFF, FENCED>;
    case SP_MUTEX_TICKET: return (const void*)k_mutex<SP_MUTEX_TICKET, FENCED>;
    case SP_MUTEX_SLEEP: return (const void*)k_mutex<SP_MUTEX_SLEEP, FENCED>;
    case SP_MUTEX_RING: return (const void*)k_mutex<SP_MUTEX_RING, FENCED>;
    case SP_MUTEX_ARRAY: return (const void*)k_mutex<SP_MUTEX_ARRAY, FENCED>;
    case SP_MUTEX_ADAPTIVE: return (const void*)k_mutex<SP_MUTEX_ADAPTIVE, FENCED>;
    case SP_MUTEX_COHORT: return (const void*)k_mutex<SP_MUTEX_COHORT, FENCED>;
    case SP_MUTEX_MCS: return (const void*)k_mutex<SP_MUTEX_MCS, FENCED>;
    case SP_MUTEX_CU_COHORT: return (const void*)k_mutex<SP_MUTEX_CU_COHORT, FENCED>;
    default: return nullptr;
  }
}

const void* mutex_kernel(uint32_t kind, bool coherent_cs) {
  return coherent_cs ? mutex_kernel_f<false>(kind) : mutex_kernel_f<true>(kind);
}

}  // namespace

extern "C" {

int sp_mutex_create(sp_ctx* ctx, uint32_t kind, uint32_t nlocks, uint32_t words_per_lock,
                    const sp_params* p, sp_mutex** out) {
  if (!spi::usable(ctx) || !out || nlocks == 0 || words_per_lock == 0 || nlocks > (1u << 20) ||
      words_per_lock > (1u << 16))
    return SP_E_INVAL;
  if (kind > SP_MUTEX_CU_COHORT && kind != SP_MUTEX_DEFAULT) return SP_E_INVAL;
  *out = nullptr;
  sp_params q;
  SP_CHECK(spi::normalize(ctx, p, &q));
  SP_HIP(ctx, hipSetDevice(ctx->device));
  sp_mutex* m = new sp_mutex();
  m->ctx = ctx;
  m->kind = kind;
  m->nlocks = nlocks;
  m->W = words_per_lock;
  m->p = q;
  // A DEFAULT mutex may resolve to any layout, so size for the widest padding.
  const uint32_t sw = kind == SP_MUTEX_DEFAULT ? 1024 : spi::stride_words(q);
  m->state_words = (4ull * nlocks + 1) * sw;  // lock, ticket, turn, owner lines + private
  const uint32_t line_words = 32;  // 128-byte lines for the critical-section words
  m->wstride = (words_per_lock + line_words - 1) / line_words * line_words;
  hipError_t e = hipMalloc(&m->d_state, m->state_words * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&m->d_words, (uint64_t)nlocks * m->wstride * sizeof(uint32_t));
  // The cohort lock's state depends only on the lock count and padding: allocate it now
  // (for a DEFAULT mutex when a built-in default is the cohort lock), so that even the
  // first run can be recorded into a graph.
  uint64_t words = 0;
  if (kind == SP_MUTEX_COHORT || kind == SP_MUTEX_CU_COHORT)
    words = cohort_words(kind, nlocks, spi::stride_words(q));
  for (int b = 0; b < 2 && kind == SP_MUTEX_DEFAULT; ++b) {
    const sp_default_entry& d = ctx->defaults[1][b];
    uint32_t dk = d.kind;
    // the CU-cohort lock runs only with two contenders per CU and lock, which a grid of
    // at most maxThreadsPerMultiProcessor / 64 workgroups per CU may not reach
    const uint64_t max_wg = (uint64_t)ctx->cu_count * (ctx->prop.maxThreadsPerMultiProcessor / 64);
    if (dk == SP_MUTEX_CU_COHORT && !spi::cu_cohort_pays(max_wg, nlocks, ctx->cu_count))
      dk = SP_MUTEX_COHORT;
    if (dk == SP_MUTEX_COHORT || dk == SP_MUTEX_CU_COHORT)
      words = std::max(words, cohort_words(dk, nlocks, spi::stride_words(d.p)));
  }
  if (words) {
    if (e == hipSuccess && words <= (1ull << 28)) {
      e = hipMalloc(&m->d_queue, words * sizeof(uint32_t));
      if (e == hipSuccess) m->queue_words = words;
    }
  }
  if (e != hipSuccess) {
    ctx->last_hip = (int)e;
    hipFree(m->d_state);
    hipFree(m->d_words);
    hipFree(m->d_queue);
    delete m;
    return SP_E_HIP;
  }
  spi::ctx_ref(ctx);
  *out = m;
  return SP_OK;
}

int sp_mutex_destroy(sp_mutex* m) {
  if (!m) return SP_E_INVAL;
  sp_ctx* ctx = m->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipFree(m->d_state);
  (void)hipFree(m->d_words);
  if (m->d_queue) (void)hipFree(m->d_queue);
  delete m;
  spi::ctx_unref(ctx);
  return SP_OK;
}

int sp_mutex_run(sp_mutex* m, uint32_t nwg, uint32_t lanes, uint64_t total_acq,
                 uint32_t max_delay_cyc, uint32_t seed, uint32_t* out_words,
                 uint64_t* out_finish, sp_stats* st, void* stream) {
  if (!m || !out_words || nwg == 0 || !spi::lanes_ok(lanes) || max_delay_cyc == 0xFFFFFFFFu)
    return SP_E_INVAL;
  sp_ctx* ctx = m->ctx;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  uint32_t kind = m->kind;
  sp_params q = m->p;
  if (kind == SP_MUTEX_DEFAULT) {
    const sp_default_entry& d = ctx->defaults[1][spi::bucket_of(nwg / m->nlocks)];
    kind = d.kind;
    const uint32_t t = q.timeout_ms;
    q = d.p;
    q.timeout_ms = t;
    q.coherent_cs = m->p.coherent_cs;  // a property of the caller's critical sections
    if (kind == SP_MUTEX_CU_COHORT && !spi::cu_cohort_pays(nwg, m->nlocks, ctx->cu_count))
      kind = SP_MUTEX_COHORT;
  }
  if (kind == SP_MUTEX_SPIN_BACKOFF && q.backoff == SP_BACKOFF_NONE) q.backoff = SP_BACKOFF_EXP;
  if (kind == SP_MUTEX_SPIN_CAS || kind == SP_MUTEX_SLEEP || kind == SP_MUTEX_ADAPTIVE ||
      kind == SP_MUTEX_MCS || kind == SP_MUTEX_CU_COHORT)
    q.backoff = SP_BACKOFF_NONE;
  const void* kern = mutex_kernel(kind, q.coherent_cs != 0);
  if (!kern) return SP_E_INVAL;
  const uint32_t sw = spi::stride_words(q);
  uint32_t* base = m->d_state;
  sp::MutexState ms;
  ms.stride = sw;
  ms.poll_sleep = q.poll_sleep;
  ms.lockw = base;
  ms.ticket = base + (uint64_t)m->nlocks * sw;
  ms.turn = base + 2ull * m->nlocks * sw;
  ms.bo = spi::backoff_cfg(q, base + 4ull * m->nlocks * sw);
  uint32_t* owner = q.verify ? base + 3ull * m->nlocks * sw : nullptr;
  ms.queue = nullptr;
  ms.qlen = 1;
  ms.qstride = 1;
  ms.cohort_bound = q.cohort_passes;
  ms.cuq = nullptr;
  if (kind == SP_MUTEX_RING || kind == SP_MUTEX_ARRAY || kind == SP_MUTEX_COHORT ||
      kind == SP_MUTEX_MCS || kind == SP_MUTEX_CU_COHORT) {
    // The ring needs a slot per contender (each workgroup has at most one arrival
    // outstanding); the array lock is correct with any number and polls one line each;
    // the cohort lock keeps kCohortLines lines per lock and XCC id (ticket, 64-bit grant
    // slots);
    // the MCS lock one node (next, locked) per lock and workgroup.
    uint32_t Q = 64;
    while (Q < nwg) Q <<= 1;
    if (kind == SP_MUTEX_COHORT) Q = sp::kCohortLines * sp::kXccSlots;
    if (kind == SP_MUTEX_CU_COHORT) Q = cohort_lines(kind);
    if (kind == SP_MUTEX_MCS) Q = nwg;
    ms.qlen = Q;
    ms.qstride = kind == SP_MUTEX_RING ? 1 : sw;  // ring entries packed, others padded
    if ((kind == SP_MUTEX_COHORT || kind == SP_MUTEX_MCS) && ms.qstride < 2)
      ms.qstride = 2;  // 64-bit grant words; an MCS node's two words
    if (kind == SP_MUTEX_CU_COHORT) ms.qstride = cohort_stride(kind, sw);
    const uint64_t words = (uint64_t)m->nlocks * Q * ms.qstride;
    if (words > (1ull << 28)) return SP_E_INVAL;  // 1 GiB of slots at most
    if (words > m->queue_words) {
      if (spi::capturing(s)) return SP_E_INVAL;  // no allocation while recording
      SP_HIP(ctx, hipStreamSynchronize(s));
      if (m->d_queue) SP_HIP(ctx, hipFree(m->d_queue));
      m->d_queue = nullptr;
      m->queue_words = 0;
      SP_HIP(ctx, hipMalloc(&m->d_queue, words * sizeof(uint32_t)));
      m->queue_words = words;
    }
    ms.queue = m->d_queue;
    if (kind == SP_MUTEX_CU_COHORT)  // the CU cohorts' lines follow the XCD cohorts'
      ms.cuq = ms.queue + (uint64_t)m->nlocks * sp::kCohortLines * sp::kXccSlots * ms.qstride;
    SP_CHECK(spi::fill_u32(ctx, m->d_queue, words, 0, s));
  }
  SP_CHECK(spi::fill_u32(ctx, m->d_state, m->state_words, 0, s));
  SP_CHECK(spi::fill_u32(ctx, m->d_words, (uint64_t)m->nlocks * m->wstride, 0, s));
  uint32_t per_cu = 0;
  SP_CHECK(spi::resident_per_cu(ctx, kern, lanes, &per_cu));
  SP_CHECK(spi::begin_timed(ctx, s));
  uint64_t timeout = spi::timeout_ticks(ctx, q);
  uint32_t nlocks = m->nlocks, W = m->W, wstride = m->wstride;
  void* args[] = {&ms, &nlocks, &W, &wstride, &m->d_words, &nwg, &total_acq, &max_delay_cyc,
                  &seed, &out_finish, &owner, &ctx->d_err, &timeout};
  SP_HIP(ctx, hipLaunchKernel(kern, dim3(nwg), dim3(lanes), args, 0, s));
  int rc = spi::end_timed(ctx, s, st, nwg, lanes, (uint32_t)per_cu, total_acq);
  if (rc != SP_OK && rc != SP_E_TIMEOUT && rc != SP_E_PARITY) return rc;
  hipLaunchKernelGGL(k_gather_words, dim3(256), dim3(256), 0, s, m->d_words, nlocks, W, wstride,
                     out_words);
  SP_HIP(ctx, hipGetLastError());
  SP_CHECK(spi::sync_unless_capturing(ctx, s));
  return rc;
}

}  // extern "C"
