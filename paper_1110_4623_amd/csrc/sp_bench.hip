// Memory-system microbenchmarks (Section 3; Table 1) and the ceilings they measure:
// contended and distributed atomic throughput, streaming bandwidth, and the one-way
// coherence latency between two workgroups.
#include <string.h>

#include "sp/atomics.hpp"
#include "sp_internal.hpp"

namespace {

// Block-wide sum of a per-thread uint64 followed by one atomic per workgroup.
__device__ void block_sum_to(unsigned long long v, unsigned long long* out) {
  __shared__ unsigned long long part[16];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (uint32_t w = 0; w < (blockDim.x + 63) / 64; ++w) s += part[w];
    atomicAdd(out, s);
  }
}

__global__ void k_prefill(uint32_t* buf, uint32_t T, uint32_t stride_words, uint32_t seed,
                          uint32_t hashed) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x)
    buf[(size_t)t * stride_words] = hashed ? sp::sm32(seed ^ t) : 0u;
}

// Issuer u performs n operations; the i-th targets word perm[(u + i) mod T].
// A compare-and-swap loop can starve under contention, so its retries are bounded by
// the watchdog like every other wait.
template <int OP, int MODE>
__global__ SP_FULL_OCCUPANCY void k_bench_atomic(uint32_t T, uint32_t stride_words, uint64_t n, uint32_t seed,
                               const uint32_t* __restrict__ perm, uint32_t* buf,
                               unsigned long long* out_sum, uint32_t* err, uint64_t timeout) {
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t waves = blockDim.x >> 6;
  unsigned long long sum = 0;
  const bool issues = MODE == SP_ISSUE_PER_LANE || lane == 0;
  if (issues) {
    const uint32_t u = MODE == SP_ISSUE_PER_LANE ? blockIdx.x * blockDim.x + threadIdx.x
                                                 : blockIdx.x * waves + wave;
    const uint32_t hu = sp::sm32(seed ^ u);
    uint32_t pos = u % T;
    for (uint64_t i = 0; i < n; ++i) {
      const uint32_t t = perm[pos];
      uint32_t* p = buf + (size_t)t * stride_words;
      if constexpr (OP == SP_OP_ADD) {
        sum += sp::add_relaxed(p, 1);
      } else if constexpr (OP == SP_OP_CAS) {
        uint32_t o = sp::ld_relaxed(p);
        sp::Wait w(ctl, 0);
        bool ok = true;
        for (;;) {
          const uint32_t seen = sp::cas_relaxed(p, o, o + 1);
          if (seen == o) break;
          o = seen;
          if (!(ok = w.tick())) break;
        }
        if (!ok) break;
        sum += o;
      } else if constexpr (OP == SP_OP_EXCH) {
        sum += sp::exch_relaxed(p, sp::sm32(hu ^ (uint32_t)i));
      } else if constexpr (OP == SP_OP_LD) {
        sum += sp::ld_relaxed(p);
      } else {
        sp::st_relaxed(p, sp::sm32(seed ^ t));
      }
      pos = pos + 1 == T ? 0 : pos + 1;
    }
  }
  block_sum_to(sum, out_sum);
}

// Adds the final word values (for the exchange conservation sum).
__global__ void k_sum_words(const uint32_t* buf, uint32_t T, uint32_t stride_words,
                            unsigned long long* out_sum) {
  unsigned long long s = 0;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x)
    s += buf[(size_t)t * stride_words];
  block_sum_to(s, out_sum);
}

// The twelve tests of Section 3: the leader of each workgroup performs n accesses.
__global__ void k_paper12(uint32_t test, uint32_t n, uint32_t stride_words, uint32_t zero,
                          uint32_t* buf, unsigned long long* out_sum) {
  if (threadIdx.x != 0) return;
  const bool cont = test == SP_P12_CONT_VOL_READ || test == SP_P12_CONT_VOL_WRITE ||
                    test == SP_P12_CONT_ATOM_READ || test == SP_P12_CONT_ATOM_WRITE ||
                    test == SP_P12_CONT_VOL_READ_AFTER_ATOM ||
                    test == SP_P12_CONT_VOL_WRITE_AFTER_ATOM;
  uint32_t* p = buf + (cont ? 0 : (size_t)blockIdx.x * stride_words);
  unsigned long long s = 0;
  switch (test) {
    case SP_P12_CONT_VOL_READ_AFTER_ATOM:
    case SP_P12_NONCONT_VOL_READ_AFTER_ATOM:
      s += sp::add_relaxed(p, zero);
      [[fallthrough]];
    case SP_P12_CONT_VOL_READ:
    case SP_P12_NONCONT_VOL_READ:
      for (uint32_t i = 0; i < n; ++i) s += sp::ld_relaxed(p);
      break;
    case SP_P12_CONT_VOL_WRITE_AFTER_ATOM:
    case SP_P12_NONCONT_VOL_WRITE_AFTER_ATOM:
      sp::exch_relaxed(p, zero);
      [[fallthrough]];
    case SP_P12_CONT_VOL_WRITE:
    case SP_P12_NONCONT_VOL_WRITE:
      for (uint32_t i = 0; i < n; ++i) sp::st_relaxed(p, zero);
      break;
    case SP_P12_CONT_ATOM_READ:
    case SP_P12_NONCONT_ATOM_READ:
      for (uint32_t i = 0; i < n; ++i) s += sp::add_relaxed(p, zero);
      break;
    default:
      for (uint32_t i = 0; i < n; ++i) s += sp::exch_relaxed(p, zero);
      break;
  }
  atomicAdd(out_sum, s);
}

// Streaming read: 16-byte loads, grid-stride, uint32 words summed.
// Four independent 16-byte loads per lane in flight per step (each one coalesced across
// the wavefront), then the grid-stride tail one at a time; the sum is exact in any order.
__global__ void k_stream(const uint4* __restrict__ buf, uint64_t n16, uint32_t reps,
                         unsigned long long* out_sum) {
  unsigned long long s = 0;
  const uint64_t g = (uint64_t)gridDim.x * blockDim.x;
  for (uint32_t r = 0; r < reps; ++r) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * g < n16; i += 4 * g) {
      const uint4 a = buf[i], b = buf[i + g], c = buf[i + 2 * g], d = buf[i + 3 * g];
      s += (unsigned long long)a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w;
      s += (unsigned long long)c.x + c.y + c.z + c.w + d.x + d.y + d.z + d.w;
    }
    for (; i < n16; i += g) {
      const uint4 v = buf[i];
      s += (unsigned long long)v.x + v.y + v.z + v.w;
    }
  }
  block_sum_to(s, out_sum);
}

// Clock probe: one lane spins for `wall_ticks` ticks of the constant-rate wall clock and
// counts the shader clock meanwhile.
__global__ void k_clock(uint64_t wall_ticks, unsigned long long* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t w0 = sp::wall_clock(), c0 = sp::shader_clock();
  uint64_t w = w0;
  while (w - w0 < wall_ticks) w = sp::wall_clock();
  out[0] = sp::shader_clock() - c0;
  out[1] = w - w0;
}

// Fence cost: each workgroup's leader makes `lines` of its own 128-byte lines dirty (plain
// stores, completed into its XCD's L2), meets the others at a start counter, then times
// `reps` fences of one kind: 0 = agent-scope release (write back the XCD's dirty L2 lines),
// 1 = agent-scope acquire (invalidate the CU's L1 and the XCD's stale L2 lines),
// 2 = workgroup-scope invalidate.  out[4 w + 0] =
// shader clocks for the reps, out[4 w + 1] / [4 w + 2] = wall clock at start / end.
__global__ SP_FULL_OCCUPANCY void k_fence(uint32_t kind, uint32_t reps, uint32_t lines,
                                          uint32_t* scratch, uint32_t* start, uint32_t nwg,
                                          unsigned long long* out, uint32_t* err,
                                          uint64_t timeout) {
  if (!sp::is_leader()) return;
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  const uint32_t b = blockIdx.x;
  for (uint32_t i = 0; i < lines; ++i) scratch[((size_t)b * lines + i) * 32] = b + i + 1;
  sp::wave_stores_complete();
  sp::add_relaxed(start, 1);
  sp::Wait w(ctl, 0);
  while (sp::ld_relaxed(start) < nwg)
    if (!w.tick()) return;
  const uint64_t w0 = sp::wall_clock(), c0 = sp::shader_clock();
  for (uint32_t r = 0; r < reps; ++r) {
    if (kind == 0) sp::fence_release();
    else if (kind == 1) sp::fence_acquire();
    else sp::invalidate_workgroup_scope();
    __asm__ __volatile__("" ::: "memory");
  }
  const uint64_t c1 = sp::shader_clock(), w1 = sp::wall_clock();
  out[4 * (size_t)b + 0] = c1 - c0;
  out[4 * (size_t)b + 1] = w0;
  out[4 * (size_t)b + 2] = w1;
  out[4 * (size_t)b + 3] = 0;
}

// Streaming copy: 16-byte loads and stores, grid-stride.
__global__ void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, uint64_t n16) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n16;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Token passing between workgroup 0 and a partner workgroup through two words 1 KiB
// apart.  FENCED: release store and acquire fence per hand-over; otherwise relaxed
// agent-scope accesses only.  Workgroups other than 0 and the partner leave at once.
template <bool FENCED>
__global__ SP_FULL_OCCUPANCY void k_pingpong(uint32_t rounds, uint32_t partner, uint32_t* words,
                                             uint32_t* out, uint32_t* err, uint64_t timeout) {
  if (threadIdx.x != 0 || (blockIdx.x != 0 && blockIdx.x != partner)) return;
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  sp::Wait w(ctl, 0);
  uint32_t* from1 = words;        // written by the partner
  uint32_t* from0 = words + 256;  // written by workgroup 0
  if (blockIdx.x == 0) {
    for (uint32_t r = 0; r < rounds; ++r) {
      if constexpr (FENCED) sp::st_release(from0, 2 * r + 1);
      else sp::st_relaxed(from0, 2 * r + 1);
      while (!sp::reached(sp::ld_relaxed(from1), 2 * r + 2))
        if (!w.tick()) return;
      if constexpr (FENCED) sp::fence_acquire();
    }
  } else {
    for (uint32_t r = 0; r < rounds; ++r) {
      while (!sp::reached(sp::ld_relaxed(from0), 2 * r + 1))
        if (!w.tick()) return;
      if constexpr (FENCED) {
        sp::fence_acquire();
        sp::st_release(from1, 2 * r + 2);
      } else {
        sp::st_relaxed(from1, 2 * r + 2);
      }
    }
  }
  out[blockIdx.x == 0 ? 2 : 3] = sp::xcc_id();
  if (blockIdx.x == 0) {
    out[0] = sp::ld_relaxed(from1);
    out[1] = sp::ld_relaxed(from0);
  }
}

template <int OP>
const void* bench_kernel_mode(uint32_t mode) {
  return mode == SP_ISSUE_PER_LANE ? (const void*)k_bench_atomic<OP, SP_ISSUE_PER_LANE>
                                   : (const void*)k_bench_atomic<OP, SP_ISSUE_WAVE_LEADER>;
}

const void* bench_kernel(uint32_t op, uint32_t mode) {
  switch (op) {
    case SP_OP_ADD: return bench_kernel_mode<SP_OP_ADD>(mode);
    case SP_OP_CAS: return bench_kernel_mode<SP_OP_CAS>(mode);
    case SP_OP_EXCH: return bench_kernel_mode<SP_OP_EXCH>(mode);
    case SP_OP_LD: return bench_kernel_mode<SP_OP_LD>(mode);
    case SP_OP_ST: return bench_kernel_mode<SP_OP_ST>(mode);
    default: return nullptr;
  }
}

}  // namespace

extern "C" {

int sp_bench_atomic(sp_ctx* ctx, uint32_t op, uint32_t nwg, uint32_t lanes, uint32_t T,
                    uint32_t stride_bytes, uint32_t mode, uint64_t ops_per_issuer,
                    uint32_t seed, const uint32_t* perm, uint32_t* buf, uint64_t* out_sum,
                    sp_stats* st, void* stream) {
  if (!spi::usable(ctx) || !perm || !buf || !out_sum || nwg == 0 || T == 0 || !spi::lanes_ok(lanes) ||
      stride_bytes == 0 || stride_bytes % 4 || op > SP_OP_ST || mode > SP_ISSUE_WAVE_LEADER)
    return SP_E_INVAL;
  if ((uint64_t)nwg * lanes > 0xFFFFFFFFull) return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  const uint32_t sw = stride_bytes / 4;
  const uint32_t hashed = op == SP_OP_EXCH || op == SP_OP_LD;
  hipLaunchKernelGGL(k_prefill, dim3(std::min<uint32_t>((T + 255) / 256, 4096)), dim3(256), 0, s,
                     buf, T, sw, seed, hashed);
  SP_CHECK(spi::fill_u32(ctx, reinterpret_cast<uint32_t*>(out_sum), 2, 0, s));
  const void* kern = bench_kernel(op, mode);
  uint32_t per_cu = 0;
  SP_CHECK(spi::resident_per_cu(ctx, kern, lanes, &per_cu));
  SP_CHECK(spi::begin_timed(ctx, s));
  uint64_t n = ops_per_issuer;
  unsigned long long* sum = reinterpret_cast<unsigned long long*>(out_sum);
  sp_params q;
  sp_params_default(&q);
  uint64_t timeout = spi::timeout_ticks(ctx, q);
  void* args[] = {&T, (void*)&sw, &n, &seed, (void*)&perm, &buf, &sum, &ctx->d_err, &timeout};
  SP_HIP(ctx, hipLaunchKernel(kern, dim3(nwg), dim3(lanes), args, 0, s));
  const uint64_t issuers =
      mode == SP_ISSUE_PER_LANE ? (uint64_t)nwg * lanes : (uint64_t)nwg * (lanes / 64);
  SP_CHECK(spi::end_timed(ctx, s, st, nwg, lanes, (uint32_t)per_cu, issuers * n));
  if (op == SP_OP_EXCH) {
    hipLaunchKernelGGL(k_sum_words, dim3(std::min<uint32_t>((T + 255) / 256, 4096)), dim3(256), 0,
                       s, buf, T, sw, sum);
    SP_HIP(ctx, hipGetLastError());
    SP_CHECK(spi::sync_unless_capturing(ctx, s));
  }
  return SP_OK;
}

int sp_bench_paper12(sp_ctx* ctx, uint32_t test, uint32_t nwg, uint32_t lanes, uint32_t n_ops,
                     uint32_t stride_bytes, uint32_t* buf, uint64_t* out_sum, sp_stats* st,
                     void* stream) {
  if (!spi::usable(ctx) || !buf || !out_sum || nwg == 0 || test > SP_P12_NONCONT_VOL_WRITE_AFTER_ATOM ||
      !spi::lanes_ok(lanes) || stride_bytes == 0 || stride_bytes % 4)
    return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  const uint32_t sw = stride_bytes / 4;
  SP_CHECK(spi::fill_u32(ctx, buf, (uint64_t)nwg * sw, 0, s));
  SP_CHECK(spi::fill_u32(ctx, reinterpret_cast<uint32_t*>(out_sum), 2, 0, s));
  uint32_t per_cu = 0;
  SP_CHECK(spi::resident_per_cu(ctx, (const void*)k_paper12, lanes, &per_cu));
  SP_CHECK(spi::begin_timed(ctx, s));
  hipLaunchKernelGGL(k_paper12, dim3(nwg), dim3(lanes), 0, s, test, n_ops, sw, 0u, buf,
                     reinterpret_cast<unsigned long long*>(out_sum));
  return spi::end_timed(ctx, s, st, nwg, lanes, (uint32_t)per_cu, (uint64_t)nwg * n_ops);
}

int sp_bench_stream(sp_ctx* ctx, const void* buf, uint64_t bytes, uint32_t nwg, uint32_t reps,
                    uint64_t* out_sum, sp_stats* st, void* stream) {
  if (!spi::usable(ctx) || !buf || !out_sum || bytes == 0 || bytes % 16 || reps == 0) return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  // 32 per CU: with four loads in flight per lane, 8192 workgroups read 1 GiB at 7.1-7.3
  // TB/s on an MI355X against 5.4 with 8 per CU (and 6.6 for one load per lane at best)
  if (nwg == 0) nwg = ctx->cu_count * 32;
  SP_CHECK(spi::fill_u32(ctx, reinterpret_cast<uint32_t*>(out_sum), 2, 0, s));
  SP_CHECK(spi::begin_timed(ctx, s));
  hipLaunchKernelGGL(k_stream, dim3(nwg), dim3(256), 0, s, (const uint4*)buf, bytes / 16, reps,
                     reinterpret_cast<unsigned long long*>(out_sum));
  return spi::end_timed(ctx, s, st, nwg, 256, 0, bytes * reps);
}

int sp_bench_clock(sp_ctx* ctx, uint32_t ms, uint64_t* out, double* mhz, void* stream) {
  if (!spi::usable(ctx) || !out || !mhz || ms == 0 || ms > 10000) return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  if (spi::capturing(s)) return SP_E_INVAL;  // waits and reads the result back
  const uint64_t ticks = (uint64_t)ms * ctx->wall_khz;
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, s, ticks,
                     reinterpret_cast<unsigned long long*>(out));
  SP_HIP(ctx, hipGetLastError());
  SP_HIP(ctx, hipStreamSynchronize(s));
  uint64_t h[2];
  SP_HIP(ctx, hipMemcpy(h, out, sizeof(h), hipMemcpyDeviceToHost));
  *mhz = h[1] ? (double)h[0] / (double)h[1] * ctx->wall_khz / 1e3 : 0.0;
  return SP_OK;
}

int sp_bench_fence(sp_ctx* ctx, uint32_t kind, uint32_t nwg, uint32_t lanes, uint32_t reps,
                   uint32_t lines, uint64_t* out, sp_stats* st, void* stream) {
  if (!spi::usable(ctx) || !out || kind > 2 || nwg == 0 || nwg > 65536 || !spi::lanes_ok(lanes) ||
      reps == 0 || reps > 1000 || lines > 1024)
    return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  if (spi::capturing(s)) return SP_E_INVAL;  // allocates its buffers
  // every workgroup waits for all others at the start counter: all must be resident
  uint32_t per_cu = 0;
  SP_CHECK(spi::resident_per_cu(ctx, (const void*)k_fence, lanes, &per_cu));
  if ((uint64_t)per_cu * ctx->cu_count < nwg) return SP_E_NORESIDENT;
  const uint64_t scratch_words = (uint64_t)nwg * (lines ? lines : 1) * 32;
  spi::DeviceScratch scratch, start;
  SP_HIP(ctx, hipMalloc(&scratch.p, scratch_words * sizeof(uint32_t)));
  SP_HIP(ctx, hipMalloc(&start.p, 64 * sizeof(uint32_t)));
  SP_CHECK(spi::fill_u32(ctx, start.as<uint32_t>(), 64, 0, s));
  sp_params q;
  sp_params_default(&q);
  const uint64_t timeout = spi::timeout_ticks(ctx, q);
  SP_CHECK(spi::begin_timed(ctx, s));
  hipLaunchKernelGGL(k_fence, dim3(nwg), dim3(lanes), 0, s, kind, reps, lines,
                     scratch.as<uint32_t>(), start.as<uint32_t>(), nwg,
                     reinterpret_cast<unsigned long long*>(out), ctx->d_err, timeout);
  const int rc = spi::end_timed(ctx, s, st, nwg, lanes, (uint32_t)per_cu, (uint64_t)nwg * reps);
  SP_HIP(ctx, hipStreamSynchronize(s));  // before the buffers are freed
  return rc;
}

int sp_bench_copy(sp_ctx* ctx, void* dst, const void* src, uint64_t bytes, uint32_t reps,
                  sp_stats* st, void* stream) {
  if (!spi::usable(ctx) || !dst || !src || bytes == 0 || bytes % 16 || reps == 0) return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  const uint32_t nwg = ctx->cu_count * 8;
  SP_CHECK(spi::begin_timed(ctx, s));
  for (uint32_t r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_copy, dim3(nwg), dim3(256), 0, s, (uint4*)dst, (const uint4*)src,
                       bytes / 16);
  return spi::end_timed(ctx, s, st, nwg, 256, 0, 2 * bytes * reps);
}

int sp_bench_pingpong(sp_ctx* ctx, uint32_t rounds, uint32_t mode, uint32_t* words,
                      uint32_t* out, sp_stats* st, void* stream) {
  if (!spi::usable(ctx) || !words || !out || rounds == 0 ||
      (mode & ~(SP_PINGPONG_FENCED | SP_PINGPONG_SAME_XCD)) != 0)
    return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  SP_CHECK(spi::fill_u32(ctx, words, 512, 0, s));
  SP_CHECK(spi::fill_u32(ctx, out, 4, 0, s));
  sp_params q;
  sp_params_default(&q);
  uint64_t timeout = spi::timeout_ticks(ctx, q);
  // Workgroup b goes to XCD b mod xcd_count, so workgroup xcd_count shares workgroup 0's.
  uint32_t partner = (mode & SP_PINGPONG_SAME_XCD) ? std::max<uint32_t>(1, ctx->xcd_count) : 1;
  const void* kern = (mode & SP_PINGPONG_FENCED) ? (const void*)k_pingpong<true>
                                                 : (const void*)k_pingpong<false>;
  SP_CHECK(spi::begin_timed(ctx, s));
  // Both workgroups must run at once: at most 17 one-wave workgroups always fit.
  void* args[] = {&rounds, &partner, &words, &out, &ctx->d_err, &timeout};
  SP_HIP(ctx, hipLaunchKernel(kern, dim3(partner + 1), dim3(64), args, 0, s));
  return spi::end_timed(ctx, s, st, 2, 64, 0, 2ull * rounds);
}

}  // extern "C"
