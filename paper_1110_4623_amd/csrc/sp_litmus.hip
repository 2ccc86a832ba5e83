// Memory-model litmus kernels: the orderings the primitives rely on, measured on pairs of
// workgroups that run on different XCDs (each XCD has its own L2).
//
//   MP (message passing): the writer stores data = i with a plain store, then publishes
//      flag = i; the reader polls the flag until it reads i, then loads the data with a
//      plain load.  Forbidden: data < i.  Variants: 0 release fence before the flag and
//      acquire fence after it (the primitives' idiom), 1 no acquire, 2 no release,
//      3 neither, 4 release fence and a workgroup-scope invalidate instead of the
//      acquire.  The reader loads the data every iteration, so a stale copy sits in its
//      caches unless the acquire invalidates it; the writer's store sits in its own XCD's
//      L2 unless the release writes it back.  Variant 4 asks whether the cheaper
//      invalidate is enough (measured: no, as many stale reads as variant 1).
//   SB (store buffering): in iteration i each side stores i + 1 into its own word, then
//      loads the other's (agent-scope relaxed accesses).  Forbidden: both see the old
//      value i.  Variants: 0 an agent-scope sequentially consistent fence between the
//      store and the load, 1 none.
// Both sides of a pair meet every iteration through handshake flags, so every iteration
// is one trial.  Every wait is bounded by the watchdog.
#include <string.h>

#include "sp_internal.hpp"

namespace {

constexpr uint32_t kLine = 32;  // words per 128-byte line
// Per pair, one line each: data, flag, ack (MP) or x, y and two arrival records per side,
// by iteration parity (SB).
constexpr uint32_t kPairLines = 6;

// Keeps the compiler from moving plain accesses across this point; emits no instruction
// (a C volatile access is not used: on gfx950 it bypasses the caches under test).
__device__ __forceinline__ void compiler_barrier() { __asm__ __volatile__("" ::: "memory"); }

__global__ void k_litmus_mp(uint32_t* mem, uint32_t iters, uint32_t variant,
                            unsigned long long* bad, uint32_t* err, uint64_t timeout) {
  if (!sp::is_leader()) return;
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  const uint32_t pair = blockIdx.x / 2;
  uint32_t* base = mem + (size_t)pair * kPairLines * kLine;
  uint32_t* data = base;
  uint32_t* flag = base + kLine;
  uint32_t* ack = base + 2 * kLine;
  const bool rel = variant == 0 || variant == 1 || variant == 4;
  const bool acq = variant == 0 || variant == 2, l1 = variant == 4;
  sp::Wait w(ctl, 0);
  if (blockIdx.x % 2 == 0) {  // writer
    for (uint32_t i = 1; i <= iters; ++i) {
      *data = i;  // plain store: cached in the writer's XCD
      compiler_barrier();
      if (rel) sp::fence_release();
      sp::st_relaxed(flag, i);
      while (sp::ld_relaxed(ack) != i)
        if (!w.tick()) return;
    }
  } else {  // reader
    unsigned long long n = 0;
    for (uint32_t i = 1; i <= iters; ++i) {
      while (sp::ld_relaxed(flag) != i)
        if (!w.tick()) return;
      if (acq) sp::fence_acquire();
      if (l1) sp::invalidate_workgroup_scope();
      compiler_barrier();
      const uint32_t v = *data;  // plain load: may hit a copy cached in an earlier iteration
      compiler_barrier();
      if (v < i) ++n;
      sp::st_relaxed(ack, i);
    }
    bad[pair] = n;
  }
}

__global__ void k_litmus_sb(uint32_t* mem, uint32_t iters, uint32_t variant,
                            unsigned long long* bad, uint32_t* err, uint64_t timeout) {
  if (!sp::is_leader()) return;
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  const uint32_t pair = blockIdx.x / 2, side = blockIdx.x % 2;
  uint32_t* base = mem + (size_t)pair * kPairLines * kLine;
  uint32_t* mine = base + side * kLine;         // x for side 0, y for side 1
  uint32_t* other = base + (1 - side) * kLine;
  // arrival records: lines 2, 3 for side 0 and 4, 5 for side 1, by iteration parity.  A
  // side overwrites its record of iteration i only in iteration i + 2, which it reaches
  // after the other side published i + 1, i.e. after that side read the record of i.
  uint32_t* my_arrive = base + (2 + 2 * side) * kLine;
  uint32_t* their_arrive = base + (2 + 2 * (1 - side)) * kLine;
  sp::Wait w(ctl, 0);
  unsigned long long n = 0;
  for (uint32_t i = 0; i < iters; ++i) {
    sp::st_relaxed(mine, i + 1);
    if (variant == 0) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    const uint32_t seen = sp::ld_relaxed(other);
    const uint32_t old = seen == i ? 1u : 0u;  // the other side's store not yet visible
    // publish (iteration, saw-old) and wait for the other side's record of iteration i
    sp::st_relaxed(my_arrive + (i & 1) * kLine, ((i + 1) << 1) | old);
    uint32_t t;
    for (;;) {
      t = sp::ld_relaxed(their_arrive + (i & 1) * kLine);
      if ((t >> 1) == i + 1) break;
      if (!w.tick()) return;
    }
    if (side == 0 && old && (t & 1)) ++n;  // both saw the old value: forbidden under SC
  }
  if (side == 0) bad[pair] = n;
}

__global__ void k_litmus_sum(const unsigned long long* bad, uint32_t pairs,
                             unsigned long long* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long s = 0;
  for (uint32_t p = 0; p < pairs; ++p) s += bad[p];
  out[0] = s;
}

}  // namespace

extern "C" {

int sp_bench_litmus(sp_ctx* ctx, uint32_t test, uint32_t variant, uint32_t pairs, uint32_t iters,
                    uint64_t* out, sp_stats* st, void* stream) {
  if (!spi::usable(ctx) || !out || test > 1 || pairs == 0 || pairs > 1024 || iters == 0 ||
      iters >= (1u << 30) || (test == 0 && variant > 4) || (test == 1 && variant > 1))
    return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  if (spi::capturing(s)) return SP_E_INVAL;
  const uint64_t mem_words = (uint64_t)pairs * kPairLines * kLine;
  spi::DeviceScratch mem, bad;
  SP_HIP(ctx, hipMalloc(&mem.p, mem_words * sizeof(uint32_t)));
  SP_HIP(ctx, hipMalloc(&bad.p, (size_t)pairs * sizeof(unsigned long long)));
  SP_CHECK(spi::fill_u32(ctx, mem.as<uint32_t>(), mem_words, 0, s));
  SP_CHECK(spi::fill_u32(ctx, bad.as<uint32_t>(), 2ull * pairs, 0, s));
  SP_CHECK(spi::begin_timed(ctx, s));
  sp_params q;
  sp_params_default(&q);
  const uint64_t timeout = spi::timeout_ticks(ctx, q);
  const uint32_t nwg = 2 * pairs;  // both sides of every pair resident: 2048 at most
  auto* badp = bad.as<unsigned long long>();
  auto* memp = mem.as<uint32_t>();
  if (test == 0)
    hipLaunchKernelGGL(k_litmus_mp, dim3(nwg), dim3(64), 0, s, memp, iters, variant, badp,
                       ctx->d_err, timeout);
  else
    hipLaunchKernelGGL(k_litmus_sb, dim3(nwg), dim3(64), 0, s, memp, iters, variant, badp,
                       ctx->d_err, timeout);
  int rc = spi::end_timed(ctx, s, st, nwg, 64, 0, (uint64_t)pairs * iters);
  hipLaunchKernelGGL(k_litmus_sum, dim3(1), dim3(64), 0, s, badp, pairs,
                     reinterpret_cast<unsigned long long*>(out));
  const hipError_t launch = hipGetLastError();
  SP_HIP(ctx, hipStreamSynchronize(s));  // before the buffers are freed
  SP_HIP(ctx, launch);
  return rc;
}

}  // extern "C"
