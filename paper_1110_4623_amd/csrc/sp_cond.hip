// Condition variables: the bounded-buffer workload (a mutex and two condition variables,
// the classic use; Section 7 names condition variables as the safer alternative to
// semaphores for waiting on a predicate).
#include <string.h>

#include <mutex>

#include "sp/cond.hpp"
#include "sp_internal.hpp"

namespace {

// Buffer state words (each on its own line), protected by the mutex.
enum { B_COUNT = 0, B_HEAD, B_TAIL, B_MAX, B_LINES };
// Condition-variable counters (each on its own line).
enum { C_NF_WAITERS = 0, C_NF_SIGNALS, C_NE_WAITERS, C_NE_SIGNALS, C_LINES };
constexpr uint32_t kLine = 32;  // words per 128-byte line

// Workgroups [0, producers) put their share of `items` values sm32(seed ^ (w << 16) ^ j)
// into a ring of `capacity` words; the others take their share.  Only the leader touches
// the buffer (plain loads and stores, ordered by the mutex); the whole workgroup takes
// part in every mutex and condition-variable call.  res: 4 uint64 per workgroup = {xor of
// values taken, sum of values taken, values taken or put, 0}.  taken (optional): consumer
// i's j-th value goes to taken[first_i + j], first_i the start of its share.
template <int MKIND>
__global__ SP_FULL_OCCUPANCY void k_bounded_buffer(sp::MutexState m, sp::CondState not_full,
                                                   sp::CondState not_empty, uint32_t* bstate,
                                                   uint32_t* buf, uint32_t capacity,
                                                   uint32_t producers, uint64_t items,
                                                   uint32_t seed, unsigned long long* res,
                                                   uint32_t* taken, uint32_t* err,
                                                   uint64_t timeout) {
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  __shared__ uint32_t s_blocked;
  const uint32_t b = blockIdx.x;
  const bool prod = b < producers;
  const uint32_t consumers = gridDim.x - producers;
  const uint32_t parts = prod ? producers : consumers;
  const uint32_t idx = prod ? b : b - producers;
  const uint64_t A = items / parts + (idx < items % parts ? 1 : 0);
  // where this consumer records the values it takes: its share's place in [0, items)
  const uint64_t first = (uint64_t)idx * (items / parts) + (idx < items % parts ? idx : items % parts);
  uint32_t* count = bstate + B_COUNT * kLine;
  uint32_t* head = bstate + B_HEAD * kLine;
  uint32_t* tail = bstate + B_TAIL * kLine;
  uint32_t* maxc = bstate + B_MAX * kLine;
  const sp::CondState& mine = prod ? not_full : not_empty;
  const sp::CondState& other = prod ? not_empty : not_full;
  uint32_t x = 0;
  unsigned long long sum = 0;
  uint64_t done = 0;
  for (uint64_t j = 0; j < A; ++j) {
    sp::MutexHold hold{0, 0};
    if (!sp::mutex_lock<MKIND>(m, 0, ctl, &hold)) return;
    for (;;) {
      if (sp::is_leader()) s_blocked = prod ? (*count == capacity) : (*count == 0);
      __syncthreads();
      const bool blocked = s_blocked;
      __syncthreads();
      if (!blocked) break;
      if (!sp::cond_wait<MKIND>(mine, m, 0, &hold, ctl)) return;
    }
    if (sp::is_leader()) {
      if (prod) {
        const uint32_t v = sp::sm32(seed ^ (b << 16) ^ (uint32_t)j);
        const uint32_t t = *tail;
        buf[t % capacity] = v;
        *tail = t + 1;
        const uint32_t c = *count + 1;
        *count = c;
        if (c > *maxc) *maxc = c;
      } else {
        const uint32_t h = *head;
        const uint32_t v = buf[h % capacity];
        *head = h + 1;
        *count = *count - 1;
        x ^= v;
        sum += v;
        if (taken) taken[first + j] = v;
      }
      sp::cond_signal_leader(other);
    }
    sp::mutex_unlock<MKIND>(m, 0, &hold);
    ++done;
  }
  if (sp::is_leader()) {
    res[4 * (size_t)b + 0] = x;
    res[4 * (size_t)b + 1] = sum;
    res[4 * (size_t)b + 2] = done;
    res[4 * (size_t)b + 3] = 0;
  }
}

// out[0] = xor of taken values, out[1] = sum, out[2] = values taken, out[3] = values put,
// out[4] = most values ever in the buffer, out[5] = values left in it.
__global__ void k_bb_reduce(const unsigned long long* res, uint32_t nwg, uint32_t producers,
                            const uint32_t* bstate, unsigned long long* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long x = 0, s = 0, taken = 0, put = 0;
  for (uint32_t b = 0; b < nwg; ++b) {
    if (b < producers) {
      put += res[4 * (size_t)b + 2];
    } else {
      x ^= res[4 * (size_t)b + 0];
      s += res[4 * (size_t)b + 1];
      taken += res[4 * (size_t)b + 2];
    }
  }
  out[0] = x;
  out[1] = s;
  out[2] = taken;
  out[3] = put;
  out[4] = bstate[B_MAX * kLine];
  out[5] = bstate[B_COUNT * kLine];
}

const void* bb_kernel(uint32_t kind) {
  switch (kind) {
    case SP_MUTEX_SPIN_CAS: return (const void*)k_bounded_buffer<SP_MUTEX_SPIN_CAS>;
    case SP_MUTEX_TICKET: return (const void*)k_bounded_buffer<SP_MUTEX_TICKET>;
    case SP_MUTEX_SLEEP: return (const void*)k_bounded_buffer<SP_MUTEX_SLEEP>;
    case SP_MUTEX_ARRAY: return (const void*)k_bounded_buffer<SP_MUTEX_ARRAY>;
    case SP_MUTEX_COHORT: return (const void*)k_bounded_buffer<SP_MUTEX_COHORT>;
    default: return nullptr;
  }
}

}  // namespace

// ---- allocation-free variant -------------------------------------------------------
// A fixed workspace in device memory, one copy per GPU the library runs on, for callers
// that cannot allocate (code under graph capture, tight serving loops).  Host code never
// passes the array's name to a kernel: it is a host-side stand-in, not a device address.
// sp_init looks the address up once per device (with the device current) and every
// later call uses that pointer.
constexpr uint64_t kStaticWords = 256 * 1024;  // 1 MiB
static __device__ __align__(256) uint32_t scratch[kStaticWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

// Workspace words the bounded buffer needs: the mutex's state (lock, ticket, turn and
// private lines, then the array lock's slots or the cohort lock's lines), both condition
// variables, the buffer's state, the ring, per-workgroup results.
struct BBLayout {
  uint32_t sw, Q, qstride;
  uint64_t qoff, mutex_words, cond_words, bstate_words, total;
};

BBLayout bb_layout(uint32_t mutex_kind, uint32_t nwg, uint32_t capacity, const sp_params& q) {
  BBLayout L{};
  L.sw = spi::stride_words(q);
  L.Q = 64;
  while (L.Q < nwg) L.Q <<= 1;
  // the array lock's slots, or the cohort lock's lines per XCC id (64-bit grant slots)
  L.qstride = mutex_kind == SP_MUTEX_COHORT ? std::max<uint32_t>(L.sw, 2) : L.sw;
  const uint64_t qwords = mutex_kind == SP_MUTEX_ARRAY    ? (uint64_t)L.Q * L.sw
                          : mutex_kind == SP_MUTEX_COHORT ? (uint64_t)sp::kCohortLines * sp::kXccSlots * L.qstride
                                                          : 0;
  L.qoff = (5ull * L.sw + 1) & ~1ull;  // 8-byte aligned for the grant words
  L.mutex_words = L.qoff + qwords;
  L.cond_words = (uint64_t)C_LINES * kLine;
  L.bstate_words = (uint64_t)B_LINES * kLine;
  const uint64_t res_words = 8ull * nwg;  // 4 uint64 per workgroup
  L.total = L.mutex_words + L.cond_words + L.bstate_words + capacity + res_words + 64;
  return L;
}

int bb_check_args(sp_ctx* ctx, uint32_t mutex_kind, uint32_t nwg, uint32_t producers,
                  uint32_t lanes, uint32_t capacity, uint64_t items, uint64_t* out) {
  if (!spi::usable(ctx) || !out || nwg < 2 || producers == 0 || producers >= nwg ||
      !spi::lanes_ok(lanes) || capacity == 0 || capacity > (1u << 24) || items == 0 ||
      items >= (1ull << 32))
    return SP_E_INVAL;
  if (!bb_kernel(mutex_kind)) return SP_E_INVAL;
  return SP_OK;
}

// Runs the workload in `base` (L.total words of device memory); clears what must start
// at zero, launches, reduces into `out`.
int bb_run(sp_ctx* ctx, uint32_t mutex_kind, uint32_t nwg, uint32_t producers, uint32_t lanes,
           uint32_t capacity, uint64_t items, uint32_t seed, const sp_params& q,
           const BBLayout& L, uint32_t* base, uint64_t* out, uint32_t* out_taken, sp_stats* st,
           hipStream_t s) {
  const void* kern = bb_kernel(mutex_kind);
  // Producers and consumers wait for each other: all must be resident at once.
  uint32_t per_cu = 0;
  SP_CHECK(spi::resident_per_cu(ctx, kern, lanes, &per_cu));
  if ((uint64_t)per_cu * ctx->cu_count < nwg) return SP_E_NORESIDENT;
  const uint32_t sw = L.sw;
  sp::MutexState ms;
  ms.stride = sw;
  ms.poll_sleep = q.poll_sleep;
  ms.lockw = base;
  ms.ticket = base + sw;
  ms.turn = base + 2ull * sw;
  ms.bo = spi::backoff_cfg(q, base + 3ull * sw);
  ms.queue = base + L.qoff;
  ms.qlen = L.Q;
  ms.qstride = L.qstride;
  ms.cohort_bound = q.cohort_passes;
  ms.cuq = nullptr;
  uint32_t* cond = base + L.mutex_words;
  sp::CondState nf{cond + C_NF_WAITERS * kLine, cond + C_NF_SIGNALS * kLine, q.poll_sleep};
  sp::CondState ne{cond + C_NE_WAITERS * kLine, cond + C_NE_SIGNALS * kLine, q.poll_sleep};
  uint32_t* bstate = cond + L.cond_words;
  uint32_t* buf = bstate + L.bstate_words;
  // 8-byte aligned per-workgroup results, then the 6 reduced values
  uint64_t off = (uint64_t)(buf + capacity - base);
  off = (off + 1) & ~1ull;
  unsigned long long* res = reinterpret_cast<unsigned long long*>(base + off);
  SP_CHECK(spi::fill_u32(ctx, base, L.total, 0, s));
  SP_CHECK(spi::begin_timed(ctx, s));
  uint64_t timeout = spi::timeout_ticks(ctx, q);
  unsigned long long* resp = res;
  void* args[] = {&ms, &nf, &ne, &bstate, &buf, &capacity, &producers, &items, &seed, &resp,
                  &out_taken, &ctx->d_err, &timeout};
  SP_HIP(ctx, hipLaunchKernel(kern, dim3(nwg), dim3(lanes), args, 0, s));
  int rc = spi::end_timed(ctx, s, st, nwg, lanes, per_cu, items);
  hipLaunchKernelGGL(k_bb_reduce, dim3(1), dim3(64), 0, s, res, nwg, producers, bstate,
                     reinterpret_cast<unsigned long long*>(out));
  const hipError_t launch = hipGetLastError();
  SP_CHECK(spi::sync_unless_capturing(ctx, s));
  SP_HIP(ctx, launch);
  return rc;
}

}  // namespace

namespace spi {

int static_scratch_setup(sp_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return SP_E_INVAL;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    SP_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[ctx->device] = static_cast<uint32_t*>(p);
  }
  ctx->static_scratch = g_scratch_ptr[ctx->device];
  ctx->static_scratch_words = kStaticWords;
  return SP_OK;
}

}  // namespace spi

extern "C" {

int sp_cond_run_bounded_buffer(sp_ctx* ctx, uint32_t mutex_kind, uint32_t nwg, uint32_t producers,
                               uint32_t lanes, uint32_t capacity, uint64_t items, uint32_t seed,
                               const sp_params* p, uint64_t* out, uint32_t* out_taken,
                               sp_stats* st, void* stream) {
  SP_CHECK(bb_check_args(ctx, mutex_kind, nwg, producers, lanes, capacity, items, out));
  sp_params q;
  SP_CHECK(spi::normalize(ctx, p, &q));
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  if (spi::capturing(s)) return SP_E_INVAL;  // allocates its buffers
  const BBLayout L = bb_layout(mutex_kind, nwg, capacity, q);
  spi::DeviceScratch mem;
  SP_HIP(ctx, hipMalloc(&mem.p, L.total * sizeof(uint32_t)));
  const int rc = bb_run(ctx, mutex_kind, nwg, producers, lanes, capacity, items, seed, q, L,
                        mem.as<uint32_t>(), out, out_taken, st, s);
  (void)hipStreamSynchronize(s);  // before the buffer is freed, whatever happened
  return rc;
}

int sp_cond_run_bounded_buffer_noalloc(sp_ctx* ctx, uint32_t mutex_kind, uint32_t nwg,
                                       uint32_t producers, uint32_t lanes, uint32_t capacity,
                                       uint64_t items, uint32_t seed, const sp_params* p,
                                       uint64_t* out, uint32_t* out_taken, sp_stats* st,
                                       void* stream) {
  SP_CHECK(bb_check_args(ctx, mutex_kind, nwg, producers, lanes, capacity, items, out));
  sp_params q;
  SP_CHECK(spi::normalize(ctx, p, &q));
  const BBLayout L = bb_layout(mutex_kind, nwg, capacity, q);
  if (!ctx->static_scratch || L.total > ctx->static_scratch_words) return SP_E_RANGE;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  return bb_run(ctx, mutex_kind, nwg, producers, lanes, capacity, items, seed, q, L,
                ctx->static_scratch, out, out_taken, st, s);
}

}  // extern "C"
