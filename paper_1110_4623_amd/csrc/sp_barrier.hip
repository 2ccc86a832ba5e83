// Global barriers: state objects, the hash-exchange workload and its comparators
// (Section 5, Barrier; Section 2 on kernel launches as the global synchronization).
#include <hip/hip_cooperative_groups.h>
#include <string.h>

#include <vector>

#include "sp/barrier.hpp"
#include "sp_internal.hpp"

struct sp_barrier {
  sp_ctx* ctx = nullptr;
  uint32_t kind = 0;
  uint32_t nwg = 0;
  sp_params p{};
  uint32_t* d_state = nullptr;  // counters and flags
  uint64_t state_words = 0;
  uint32_t* d_slots = nullptr;  // 2 x nwg exchanged values
  uint32_t* d_near = nullptr;   // per-XCD blocks in measured chunks (flag_placement 0)
  uint64_t near_words = 0;
  uint32_t near_placed = 0;     // bits: 1 arrival blocks, 2 stamp copies, 4 release lines
  bool counted = false;         // holds a reference on ctx (set once creation succeeded)
  sp::BarrierState st{};
};

namespace {

// Hash-exchange workload: the slot is written by the workgroup's last thread and read
// by thread 64 (a different wavefront when the workgroup has more than one), with plain
// stores and loads, so only the barrier orders them -- or, for a barrier created with
// coherent_cs, with agent-scope stores and loads (the paper's volatile accesses), which
// the barrier then orders without cache maintenance.
template <int KIND, bool COHERENT>
__global__ SP_FULL_OCCUPANCY void k_barrier_hash(sp::BarrierState s, uint32_t rounds, uint32_t seed,
                               uint32_t* slots, uint32_t* out, uint32_t* err,
                               uint64_t timeout) {
  const sp::Ctl ctl{err, sp::wall_clock() + timeout};
  const uint32_t b = blockIdx.x, N = s.nwg;
  const uint32_t writer = blockDim.x - 1, reader = 64 % blockDim.x;
  uint32_t chk = 0;
  for (uint32_t r = 0; r < rounds; ++r) {
    if (threadIdx.x == writer) {
      uint32_t* p = slots + (r & 1) * N + b;
      const uint32_t v = sp::sm32(seed ^ (b << 16) ^ r);
      if constexpr (COHERENT) sp::st_relaxed(p, v);
      else *p = v;
    }
    if (!sp::barrier_wait<KIND>(s, r, ctl)) return;
    if (threadIdx.x == reader) {
      const uint32_t* p = slots + (r & 1) * N + (uint32_t)(((uint64_t)b + r) % N);
      if constexpr (COHERENT) chk ^= sp::ld_relaxed(p);
      else chk ^= *p;
    }
  }
  if (threadIdx.x == reader) out[b] = chk;
}

// Comparator: HIP cooperative groups' grid-wide barrier.
__global__ SP_FULL_OCCUPANCY void k_barrier_hash_gridsync(uint32_t N, uint32_t rounds, uint32_t seed,
                                        uint32_t* slots, uint32_t* out) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const uint32_t b = blockIdx.x;
  const uint32_t writer = blockDim.x - 1, reader = 64 % blockDim.x;
  uint32_t chk = 0;
  for (uint32_t r = 0; r < rounds; ++r) {
    if (threadIdx.x == writer) slots[(r & 1) * N + b] = sp::sm32(seed ^ (b << 16) ^ r);
    grid.sync();
    if (threadIdx.x == reader) chk ^= slots[(r & 1) * N + (uint32_t)(((uint64_t)b + r) % N)];
  }
  if (threadIdx.x == reader) out[b] = chk;
}

// Comparator: kernel boundaries as the barrier.  Launch r (0 <= r <= rounds) first
// consumes round r - 1, then publishes round r.
__global__ void k_barrier_round(uint32_t N, uint32_t r, uint32_t rounds, uint32_t seed,
                                uint32_t* slots, uint32_t* out) {
  const uint32_t b = blockIdx.x;
  if (threadIdx.x != 0) return;
  if (r > 0) {
    const uint32_t q = r - 1;
    out[b] ^= slots[(q & 1) * N + (uint32_t)(((uint64_t)b + q) % N)];
  }
  if (r < rounds) slots[(r & 1) * N + b] = sp::sm32(seed ^ (b << 16) ^ r);
}

// The coherent-data variant is its own instantiation (its slot accesses differ, and a
// kernel trace then tells the two apart); the barrier protocol reads s.fenced.
template <bool COHERENT>
const void* barrier_kernel_c(uint32_t kind) {
  switch (kind) {
    case SP_BARRIER_CENTRAL: return (const void*)k_barrier_hash<SP_BARRIER_CENTRAL, COHERENT>;
    case SP_BARRIER_CENTRAL_SPLIT:
      return (const void*)k_barrier_hash<SP_BARRIER_CENTRAL_SPLIT, COHERENT>;
    case SP_BARRIER_TREE: return (const void*)k_barrier_hash<SP_BARRIER_TREE, COHERENT>;
    case SP_BARRIER_XCD: return (const void*)k_barrier_hash<SP_BARRIER_XCD, COHERENT>;
    case SP_BARRIER_FLAG: return (const void*)k_barrier_hash<SP_BARRIER_FLAG, COHERENT>;
    case SP_BARRIER_GRID_SYNC: return (const void*)k_barrier_hash_gridsync;
    default: return nullptr;
  }
}

const void* barrier_kernel(uint32_t kind, bool coherent) {
  return coherent ? barrier_kernel_c<true>(kind) : barrier_kernel_c<false>(kind);
}

// Flag placement.  A signal between two workgroups of one XCD takes 640-720 shader clocks
// one way when its line lives in a chunk of memory close to that XCD and 950-1080 when it
// does not; which 8 KiB chunks are close changes with the XCD.  The probe measures it:
// the first two one-wave workgroups that register on an XCD hand a token back and forth
// `rounds` times through two lines of every chunk in turn (XCD x starting at chunk
// x * nchunks / groups, so that the pairs work on different chunks), and the first of
// them stores the mean one-way time per chunk in lat[x * nchunks + chunk].  Every wait
// ends at the wall-clock deadline; a chunk not measured keeps 0.
constexpr uint32_t kChunkWords = 2048;  // 8 KiB
constexpr uint32_t kNearChunks = 64;    // 512 KiB
constexpr uint32_t kProbeWorkgroups = 64;

__global__ void k_near_probe(uint32_t* area, uint32_t nchunks, uint32_t groups,
                             uint32_t rounds, uint32_t* claims, uint32_t* lat,
                             uint64_t deadline_ticks) {
  if (threadIdx.x != 0) return;
  const uint64_t end = sp::wall_clock() + deadline_ticks;
  const uint32_t x = sp::xcc_id() % groups;
  const uint32_t role = sp::add_relaxed(claims + x, 1);
  if (role > 1) return;
  for (uint32_t i = 0; i < nchunks; ++i) {
    const uint32_t j = (i + x * (nchunks / groups)) % nchunks;
    uint32_t* ping = area + (size_t)j * kChunkWords + x * 64;  // two lines per XCD
    uint32_t* pong = ping + 32;
    const uint64_t t0 = sp::shader_clock();
    for (uint32_t r = 0; r < rounds; ++r) {
      if (role == 0) {
        sp::st_relaxed(ping, 2 * r + 1);
        while (sp::ld_relaxed(pong) < 2 * r + 2)
          if (sp::wall_clock() > end) return;
      } else {
        while (sp::ld_relaxed(ping) < 2 * r + 1)
          if (sp::wall_clock() > end) return;
        sp::st_relaxed(pong, 2 * r + 2);
      }
    }
    if (role == 0) {
      const uint64_t t = (sp::shader_clock() - t0) / (2ull * rounds);
      sp::st_relaxed(lat + (size_t)x * nchunks + j, (uint32_t)std::max<uint64_t>(1, t));
    }
  }
}

// Measures the chunks of b->d_near and gives each XCD its fastest free chunk for its
// arrival block, then (`mail`) for its stamp copies and (`rel`) for its per-CU release
// lines.  Leaves the fixed layout in place (returns SP_OK) when any XCD could not be
// measured.
int place_near(sp_barrier* b, uint32_t G, bool mail, bool rel) {
  sp_ctx* ctx = b->ctx;
  spi::DeviceScratch scratch;
  const uint64_t words = G + (uint64_t)G * kNearChunks;
  SP_HIP(ctx, hipMalloc(&scratch.p, words * sizeof(uint32_t)));
  uint32_t* claims = scratch.as<uint32_t>();
  uint32_t* lat = claims + G;
  // the library's own stream: the probe neither joins nor waits for the caller's work
  hipStream_t s = ctx->setup_stream;
  SP_CHECK(spi::fill_u32(ctx, claims, words, 0, s));
  SP_CHECK(spi::fill_u32(ctx, b->d_near, b->near_words, 0, s));
  const uint64_t deadline = (uint64_t)ctx->wall_khz * 50;  // 50 ms
  hipLaunchKernelGGL(k_near_probe, dim3(kProbeWorkgroups), dim3(64), 0, s, b->d_near,
                     kNearChunks, G, 32u, claims, lat, deadline);
  SP_HIP(ctx, hipGetLastError());
  SP_HIP(ctx, hipStreamSynchronize(s));
  std::vector<uint32_t> h((size_t)G * kNearChunks);
  SP_HIP(ctx, hipMemcpyAsync(h.data(), lat, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  SP_HIP(ctx, hipStreamSynchronize(s));
  for (uint32_t v : h)
    if (v == 0) return SP_OK;
  std::vector<bool> used(kNearChunks, false);
  auto take = [&](uint32_t x) {
    uint32_t best = kNearChunks;
    for (uint32_t j = 0; j < kNearChunks; ++j)
      if (!used[j] && (best == kNearChunks || h[(size_t)x * kNearChunks + j] <
                                                   h[(size_t)x * kNearChunks + best]))
        best = j;
    used[best] = true;
    return best * kChunkWords;
  };
  sp::BarrierState& st = b->st;
  for (uint32_t x = 0; x < G; ++x) st.xoff[x] = take(x);
  st.larrive = b->d_near;
  b->near_placed = 1;
  if (mail) {
    for (uint32_t x = 0; x < G; ++x) st.moff[x] = take(x);
    st.xmail = b->d_near;
    st.xmstep = st.xmstride;
    b->near_placed |= 2;
  }
  if (rel) {
    for (uint32_t x = 0; x < G; ++x) st.roff[x] = take(x);
    st.lrelease = b->d_near;
    b->near_placed |= 4;
  }
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_barrier_create(sp_ctx* ctx, uint32_t kind, uint32_t nwg, const sp_params* p,
                      sp_barrier** out) {
  if (!spi::usable(ctx) || !out || nwg == 0 || nwg > (1u << 16)) return SP_E_INVAL;
  *out = nullptr;
  sp_params q;
  if (kind == SP_BARRIER_DEFAULT) {
    const sp_default_entry& d = ctx->defaults[0][spi::barrier_bucket_of(nwg)];
    kind = d.kind;
    sp_params dp = d.p;
    if (p && p->timeout_ms) dp.timeout_ms = p->timeout_ms;  // an explicit timeout applies
    if (p) dp.coherent_cs = p->coherent_cs;  // a property of the caller's data accesses
    if (p) dp.flag_placement = p->flag_placement;
    SP_CHECK(spi::normalize(ctx, &dp, &q));  // fills fan_in and the other "auto" fields
  } else {
    if (kind > SP_BARRIER_XCD) return SP_E_INVAL;
    SP_CHECK(spi::normalize(ctx, p, &q));
  }
  SP_HIP(ctx, hipSetDevice(ctx->device));
  sp_barrier* b = new sp_barrier();
  b->ctx = ctx;
  b->kind = kind;
  b->nwg = nwg;
  b->p = q;
  const uint32_t sw = spi::stride_words(q);
  // the per-XCD barrier groups by XCD; the tree by fan_in
  const uint32_t X = std::max<uint32_t>(1, ctx->xcd_count);
  // (the per-XCD barrier keeps a group for every XCD: the placement decides which are used)
  const uint32_t G = kind == SP_BARRIER_XCD ? X : std::min(q.fan_in, nwg);
  const uint32_t fs = q.flags_packed ? 1u : sw;
  // per-XCD blocks of packed local arrival flags, each a whole number of 128-byte lines
  const uint32_t xblock = (uint32_t)(((nwg + G - 1) / G + 31) / 32 * 32);
  // layout, in lines of sw words: cnt, gen, top, topgen, mismatch, gcnt[G], ggen[G],
  // xarrive[G], then the flag barrier's arrive and release arrays, the per-XCD
  // arrival blocks and the per-XCD blocks of release flags (one line per member)
  const uint64_t flag_lines = ((uint64_t)nwg * fs + sw - 1) / sw;
  const uint64_t local_lines = ((uint64_t)G * xblock * sp::kArriveWords + sw - 1) / sw;
  const uint64_t lrel_lines = (uint64_t)G * sp::kCuLines;
  // per-CU and per-XCD registration (per-XCD barrier): counts and ranks per CU key,
  // member and CU counts per XCD, the overflow word
  const uint64_t cu_words = (uint64_t)G * 256 * 2 + 2ull * G + 1;
  // copies of the XCD stamps, each one word per XCD, padded to at least a line
  const uint32_t copies = kind == SP_BARRIER_XCD ? q.xcd_copies : 0;
  const uint32_t mstride = (std::max(sw, G) + sw - 1) / sw * sw;
  const uint64_t mail_lines = (uint64_t)copies * (mstride / sw);
  const uint64_t cu_lines = (cu_words + sw - 1) / sw;
  const uint64_t lines =
      5 + 3ull * G + 2 * flag_lines + local_lines + lrel_lines + cu_lines + mail_lines;
  b->state_words = lines * sw;
  hipError_t e = hipMalloc(&b->d_state, b->state_words * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&b->d_slots, 2ull * nwg * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(b->d_state, 0, b->state_words * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(b->d_slots, 0, 2ull * nwg * sizeof(uint32_t));
  if (e != hipSuccess) {
    ctx->last_hip = (int)e;
    (void)hipFree(b->d_state);
    (void)hipFree(b->d_slots);
    delete b;
    return SP_E_HIP;
  }
  uint32_t* base = b->d_state;
  sp::BarrierState& s = b->st;
  s.nwg = nwg;
  s.stride = sw;
  s.groups = G;
  s.tgroups = std::min(G, nwg);
  s.fenced = q.coherent_cs ? 0u : 1u;
  s.xcopies = copies;
  s.xmstride = mstride;
  s.flag_stride = fs;
  s.poll_sleep = q.poll_sleep;
  s.xblock = xblock;
  s.cnt = base + 0 * sw;
  s.gen = base + 1 * sw;
  s.top = base + 2 * sw;
  s.topgen = base + 3 * sw;
  s.mismatch = base + 4 * sw;
  s.gcnt = base + 5ull * sw;
  s.ggen = base + (5ull + G) * sw;
  s.xarrive = base + (5ull + 2 * G) * sw;
  s.arrive = base + (5ull + 3 * G) * sw;
  s.release = s.arrive + flag_lines * sw;
  s.larrive = s.release + flag_lines * sw;
  s.lrelease = s.larrive + local_lines * sw;
  s.cu_count = s.lrelease + lrel_lines * sw;           // G * 256 words
  s.xcount = s.cu_count + (uint64_t)G * 256;           // G words
  s.overflow = s.xcount + G;                                   // 1 word
  s.xcu = s.overflow + 1;                                      // G words
  s.cu_rank = s.xcu + G;                                       // G * 256 words
  s.xmail = s.cu_count + cu_lines * sw;  // xcopies copies of xmstride words
  // Fixed layout: XCD-major blocks of arrival flags and release lines, copies in order.
  for (uint32_t x = 0; x < G && x < 16; ++x) {
    s.xoff[x] = x * xblock * sp::kArriveWords;
    s.roff[x] = x * sp::kCuLines * sw;
    s.moff[x] = x * mstride;
  }
  s.xmstep = G * mstride;
  if (kind == SP_BARRIER_XCD && q.flag_placement == 0 && G >= 2 && G <= 16 &&
      xblock * sp::kArriveWords <= kChunkWords) {
    const bool mail = copies >= G && copies % G == 0 && (copies / G) * mstride <= kChunkWords;
    const bool rel = sp::kCuLines * sw <= kChunkWords;
    b->near_words = (uint64_t)kNearChunks * kChunkWords;
    int rc = SP_OK;
    e = hipMalloc(&b->d_near, b->near_words * sizeof(uint32_t));
    if (e != hipSuccess) {
      ctx->last_hip = (int)e;
      rc = SP_E_HIP;
    } else {
      rc = place_near(b, G, mail, rel);
    }
    if (rc != SP_OK) {
      sp_barrier_destroy(b);
      return rc;
    }
    if (b->near_placed == 0) {  // not measured: keep the fixed layout, drop the area
      (void)hipFree(b->d_near);
      b->d_near = nullptr;
      b->near_words = 0;
    }
  }
  spi::ctx_ref(ctx);
  b->counted = true;
  *out = b;
  return SP_OK;
}

int sp_barrier_destroy(sp_barrier* b) {
  if (!b) return SP_E_INVAL;
  sp_ctx* ctx = b->ctx;
  const bool counted = b->counted;
  (void)hipSetDevice(ctx->device);
  (void)hipFree(b->d_state);
  (void)hipFree(b->d_slots);
  if (b->d_near) (void)hipFree(b->d_near);
  delete b;
  if (counted) spi::ctx_unref(ctx);
  return SP_OK;
}

int sp_barrier_info_get(sp_barrier* b, sp_barrier_info* out) {
  if (!b || !out || !spi::usable(b->ctx)) return SP_E_INVAL;
  sp_ctx* ctx = b->ctx;
  SP_HIP(ctx, hipSetDevice(ctx->device));
  memset(out, 0, sizeof(*out));
  out->kind = b->kind;
  out->nwg = b->nwg;
  if (b->kind == SP_BARRIER_XCD) {
    uint32_t w[2] = {0, 0};
    SP_HIP(ctx, hipMemcpy(&w[0], b->st.mismatch, sizeof(uint32_t), hipMemcpyDeviceToHost));
    SP_HIP(ctx, hipMemcpy(&w[1], b->st.overflow, sizeof(uint32_t), hipMemcpyDeviceToHost));
    out->misplaced = w[0];
    out->cu_overflow = w[1];
    out->xcd_path = w[1] == 0;
    out->near_placed = b->near_placed;
  }
  return SP_OK;
}

int sp_barrier_run_hash(sp_barrier* b, uint32_t lanes, uint32_t rounds, uint32_t seed,
                        uint32_t* out_checksums, sp_stats* st, void* stream) {
  if (!b || !out_checksums || !spi::lanes_ok(lanes)) return SP_E_INVAL;
  sp_ctx* ctx = b->ctx;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  const void* kern = barrier_kernel(b->kind, b->st.fenced == 0);
  if (!kern) return SP_E_INVAL;
  // Every workgroup must be resident at once (the barrier's persistent-threads
  // requirement, Section 5); refuse instead of hanging.
  uint32_t per_cu = 0;
  SP_CHECK(spi::resident_per_cu(ctx, kern, lanes, &per_cu));
  if ((uint64_t)per_cu * ctx->cu_count < b->nwg) return SP_E_NORESIDENT;
  // cooperative launches are not recorded: refuse before anything joins the capture
  const bool coop = b->kind == SP_BARRIER_GRID_SYNC || b->p.cooperative;
  if (coop && spi::capturing(s)) return SP_E_INVAL;
  SP_CHECK(spi::fill_u32(ctx, b->d_state, b->state_words, 0, s));
  SP_CHECK(spi::fill_u32(ctx, b->d_slots, 2ull * b->nwg, 0, s));
  if (b->d_near) SP_CHECK(spi::fill_u32(ctx, b->d_near, b->near_words, 0, s));
  SP_CHECK(spi::begin_timed(ctx, s));
  uint64_t timeout = spi::timeout_ticks(ctx, b->p);
  uint32_t N = b->nwg;
  if (b->kind == SP_BARRIER_GRID_SYNC) {  // grid.sync() requires a cooperative launch
    void* args[] = {&N, &rounds, &seed, &b->d_slots, &out_checksums};
    SP_HIP(ctx, hipLaunchCooperativeKernel(kern, dim3(N), dim3(lanes), args, 0, s));
  } else {
    sp::BarrierState state = b->st;
    void* args[] = {&state, &rounds, &seed, &b->d_slots, &out_checksums, &ctx->d_err, &timeout};
    if (b->p.cooperative)
      SP_HIP(ctx, hipLaunchCooperativeKernel(kern, dim3(N), dim3(lanes), args, 0, s));
    else
      SP_HIP(ctx, hipLaunchKernel(kern, dim3(N), dim3(lanes), args, 0, s));
  }
  return spi::end_timed(ctx, s, st, N, lanes, (uint32_t)per_cu, rounds);
}

int sp_barrier_run_hash_launches(sp_ctx* ctx, uint32_t nwg, uint32_t lanes, uint32_t rounds,
                                 uint32_t seed, uint32_t graph, uint32_t* slots,
                                 uint32_t* out_checksums, sp_stats* st, void* stream) {
  if (!spi::usable(ctx) || !slots || !out_checksums || nwg == 0 || nwg > (1u << 16) ||
      !spi::lanes_ok(lanes))
    return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  if (graph && spi::capturing(s)) return SP_E_INVAL;
  SP_CHECK(spi::fill_u32(ctx, out_checksums, nwg, 0, s));
  SP_CHECK(spi::fill_u32(ctx, slots, 2ull * nwg, 0, s));
  if (!graph) {
    SP_CHECK(spi::begin_timed(ctx, s));
    for (uint32_t r = 0; r <= rounds; ++r)
      hipLaunchKernelGGL(k_barrier_round, dim3(nwg), dim3(lanes), 0, s, nwg, r, rounds, seed,
                         slots, out_checksums);
    return spi::end_timed(ctx, s, st, nwg, lanes, 0, rounds);
  }
  // Capture the rounds + 1 launches once, then time one replay of the graph.
  hipStream_t cs = ctx->capture_stream;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  SP_HIP(ctx, hipStreamSynchronize(s));
  SP_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  for (uint32_t r = 0; r <= rounds; ++r)
    hipLaunchKernelGGL(k_barrier_round, dim3(nwg), dim3(lanes), 0, cs, nwg, r, rounds, seed,
                       slots, out_checksums);
  hipError_t e = hipStreamEndCapture(cs, &g);
  if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    ctx->last_hip = (int)e;
    if (g) (void)hipGraphDestroy(g);
    return SP_E_HIP;
  }
  int rc = spi::begin_timed(ctx, s);
  if (rc == SP_OK) {
    e = hipGraphLaunch(ge, s);
    if (e != hipSuccess) {
      ctx->last_hip = (int)e;
      rc = SP_E_HIP;
    } else {
      rc = spi::end_timed(ctx, s, st, nwg, lanes, 0, rounds);
    }
  }
  (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  return rc;
}

}  // extern "C"
