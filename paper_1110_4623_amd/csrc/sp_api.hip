// Context, parameters, errors and shared launch helpers of libsp.so.
#include <string.h>

#include "sp_internal.hpp"

namespace {

__global__ void k_fill_u32(uint32_t* d, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    d[i] = v;
}

__global__ void k_probe_xcc(uint32_t* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = sp::xcc_id();
}

}  // namespace

namespace spi {

int normalize(const sp_ctx* ctx, const sp_params* in, sp_params* out) {
  sp_params p;
  if (in) p = *in; else sp_params_default(&p);
  if (p.backoff > SP_BACKOFF_EXP || p.backoff_unit > SP_UNIT_LOAD) return SP_E_INVAL;
  if (p.backoff_min == 0) p.backoff_min = 1;
  if (p.backoff_max < p.backoff_min) p.backoff_max = p.backoff_min;
  if (p.backoff_max > 1u << 16) return SP_E_INVAL;
  if (p.poll_sleep > 1024) return SP_E_INVAL;
  if (p.pad_bytes == 0) p.pad_bytes = 128;
  if (p.pad_bytes < 4 || p.pad_bytes > 4096 || (p.pad_bytes & (p.pad_bytes - 1))) return SP_E_INVAL;
  if (p.fan_in == 0) p.fan_in = ctx && ctx->xcd_count ? ctx->xcd_count : 8;
  if (p.timeout_ms == 0) p.timeout_ms = 20000;
  if (p.xcd_copies > 256 || (p.xcd_copies & (p.xcd_copies - 1))) return SP_E_INVAL;
  if (p.cohort_passes == 0) p.cohort_passes = 64;
  if (p.cohort_passes > 255) return SP_E_INVAL;  // the grant word's session field
  if (p.flag_placement > 1) return SP_E_INVAL;
  if (p.post_backoff > 1) return SP_E_INVAL;
  *out = p;
  return SP_OK;
}

int fill_u32(sp_ctx* ctx, uint32_t* d, uint64_t words, uint32_t value, hipStream_t s) {
  if (words == 0) return SP_OK;
  uint64_t blocks = std::min<uint64_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, d, words, value);
  SP_HIP(ctx, hipGetLastError());
  return SP_OK;
}

int resident_per_cu(sp_ctx* ctx, const void* kern, uint32_t lanes, uint32_t* per_cu) {
  int rt = 0;
  SP_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&rt, kern, (int)lanes, 0));
  hipFuncAttributes fa{};
  SP_HIP(ctx, hipFuncGetAttributes(&fa, kern));
  sp_occupancy occ{};
  occ.runtime_per_cu = rt > 0 ? (uint32_t)rt : 0u;
  occ.vgprs = fa.numRegs > 0 ? (uint32_t)fa.numRegs : 0u;
  occ.lds_bytes = (uint32_t)fa.sharedSizeBytes;
  occ.lanes = lanes;
  *per_cu = sp_resident_per_cu(&occ);
  return SP_OK;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus c = hipStreamCaptureStatusNone;
  return s && hipStreamIsCapturing(s, &c) == hipSuccess && c == hipStreamCaptureStatusActive;
}

int sync_unless_capturing(sp_ctx* ctx, hipStream_t s) {
  if (capturing(s)) return SP_OK;
  SP_HIP(ctx, hipStreamSynchronize(s));
  return SP_OK;
}

int begin_timed(sp_ctx* ctx, hipStream_t s) {
  if (!usable(ctx)) return SP_E_INVAL;
  // Under capture the graph's launcher clears the watchdog word once per replay and
  // times the replays; the recorded call adds only its own kernels.
  if (capturing(s)) return SP_OK;
  SP_CHECK(fill_u32(ctx, ctx->d_err, 1, 0, s));
  SP_HIP(ctx, hipEventRecord(ctx->ev0, s));
  return SP_OK;
}

int end_timed(sp_ctx* ctx, hipStream_t s, sp_stats* st, uint32_t nwg, uint32_t lanes,
              uint32_t resident_per_cu, uint64_t ops) {
  SP_HIP(ctx, hipGetLastError());
  if (capturing(s)) {
    if (st) memset(st, 0, sizeof(*st));
    return SP_OK;
  }
  SP_HIP(ctx, hipEventRecord(ctx->ev1, s));
  SP_HIP(ctx, hipStreamSynchronize(s));
  float ms = 0.f;
  SP_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  uint32_t err = 0;
  SP_HIP(ctx, hipMemcpy(&err, ctx->d_err, sizeof(err), hipMemcpyDeviceToHost));
  if (st) {
    memset(st, 0, sizeof(*st));
    st->kernel_ms = ms;
    st->nwg = nwg;
    st->lanes = lanes;
    st->resident_per_cu = resident_per_cu;
    st->device_error = err;
    st->ops = ops;
  }
  if (err == sp::DEV_TIMEOUT) return SP_E_TIMEOUT;
  if (err != sp::DEV_OK) return SP_E_PARITY;
  return SP_OK;
}

}  // namespace spi

using spi::usable;

extern "C" {

void sp_params_default(sp_params* p) {
  memset(p, 0, sizeof(*p));
  p->backoff = SP_BACKOFF_NONE;
  p->backoff_min = 1;
  p->backoff_max = 32;
  p->backoff_unit = SP_UNIT_SLEEP;
  p->poll_sleep = 1;
  p->fan_in = 0;
  p->pad_bytes = 128;
  p->flags_packed = 0;
  p->timeout_ms = 20000;
  p->xcd_copies = 64;
}

uint32_t sp_resident_per_cu(const sp_occupancy* occ) {
  if (!occ || occ->lanes == 0) return 0;
  constexpr uint32_t kSimds = 4, kWavesPerSimd = 8, kVgprsPerSimd = 512, kVgprGranule = 8;
  constexpr uint32_t kLdsBytes = 160 * 1024, kLdsGranule = 512;
  const uint32_t waves = (occ->lanes + 63) / 64;
  uint32_t per_simd = kWavesPerSimd;
  if (occ->vgprs > 0) {
    const uint32_t v = (occ->vgprs + kVgprGranule - 1) / kVgprGranule * kVgprGranule;
    per_simd = std::min(per_simd, kVgprsPerSimd / v);
  }
  uint32_t wgs = kSimds * per_simd / waves;
  if (occ->lds_bytes > 0) {
    const uint32_t l = (occ->lds_bytes + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
    wgs = std::min(wgs, kLdsBytes / l);
  }
  return std::min(wgs, occ->runtime_per_cu);
}

const char* sp_strerror(int code) {
  switch (code) {
    case SP_OK: return "ok";
    case SP_E_INVAL: return "invalid argument";
    case SP_E_HIP: return "HIP runtime error";
    case SP_E_NORESIDENT: return "not enough co-resident workgroups for a global barrier";
    case SP_E_TIMEOUT: return "device watchdog expired";
    case SP_E_PARITY: return "device consistency check failed";
    case SP_E_RANGE: return "request exceeds the fixed workspace of an allocation-free call";
    default: return "unknown error";
  }
}

int sp_last_hip_error(const sp_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

int sp_init(int device, sp_ctx** out) {
  if (!out) return SP_E_INVAL;
  *out = nullptr;
  sp_ctx* ctx = new sp_ctx();
  auto fail = [&](hipError_t e) {
    (void)e;
    delete ctx;
    return SP_E_HIP;
  };
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return fail(e);
  ctx->device = device;
  if ((e = hipGetDeviceProperties(&ctx->prop, device)) != hipSuccess) return fail(e);
  ctx->cu_count = (uint32_t)ctx->prop.multiProcessorCount;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    ctx->wall_khz = (uint32_t)khz;
  if ((e = hipMalloc(&ctx->d_err, 256)) != hipSuccess) return fail(e);
  if ((e = hipMalloc(&ctx->d_scratch, 4096)) != hipSuccess) return fail(e);
  if ((e = hipEventCreate(&ctx->ev0)) != hipSuccess) return fail(e);
  if ((e = hipEventCreate(&ctx->ev1)) != hipSuccess) return fail(e);
  if ((e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking)) != hipSuccess)
    return fail(e);
  if ((e = hipStreamCreateWithFlags(&ctx->setup_stream, hipStreamNonBlocking)) != hipSuccess)
    return fail(e);
  if (spi::static_scratch_setup(ctx) != SP_OK) return fail(hipErrorInvalidSymbol);
  // Count XCDs: launch 8 workgroups per CU and collect the distinct XCC ids.
  {
    uint32_t n = ctx->cu_count * 8;
    uint32_t* d = nullptr;
    if ((e = hipMalloc(&d, n * sizeof(uint32_t))) != hipSuccess) return fail(e);
    hipLaunchKernelGGL(k_probe_xcc, dim3(n), dim3(64), 0, 0, d);
    uint32_t* h = new uint32_t[n];
    e = hipMemcpy(h, d, n * sizeof(uint32_t), hipMemcpyDeviceToHost);
    hipFree(d);
    if (e != hipSuccess) {
      delete[] h;
      return fail(e);
    }
    uint32_t seen = 0;
    for (uint32_t i = 0; i < n; ++i) seen |= 1u << (h[i] & 15);
    delete[] h;
    ctx->xcd_count = (uint32_t)__builtin_popcount(seen);
    ctx->xcc_mask = seen;
  }
  // Built-in defaults: the winners of a full tuning pass on an MI355X (fewer than 64 /
  // at least 64 workgroups per resource); a tuner run installs its own with
  // sp_set_default.
  for (int prim = 0; prim < 3; ++prim)
    for (int b = 0; b < 2; ++b) {
      sp_params_default(&ctx->defaults[prim][b].p);
      ctx->defaults[prim][b].kind = 0;
    }
  ctx->defaults[0][0].kind = SP_BARRIER_CENTRAL;  // 1.7 us/round at 16 workgroups
  ctx->defaults[0][0].p.poll_sleep = 0;
  ctx->defaults[0][1].kind = SP_BARRIER_XCD;      // 6.1 us/round at 1024, 64 stamp copies
  ctx->defaults[0][1].p.poll_sleep = 0;
  // paper's linear backoff, I_max 8: 0.62 / 0.74 M/s at 4 / 32 workgroups on one lock
  // (cohort lock 0.52 / 0.84, ticket 0.57 / 0.68)
  ctx->defaults[1][0].kind = SP_MUTEX_SPIN_BACKOFF;
  ctx->defaults[1][0].p.backoff = SP_BACKOFF_PAPER;
  ctx->defaults[1][0].p.backoff_max = 8;
  // CU-cohort lock (the XCD-cohort lock below two contenders per CU and lock): one lock
  // 1.13 M/s at 2048 workgroups, 1.18 at 1024 (XCD-cohort lock 0.74 / 0.77, ticket 0.65);
  // 16 locks at 2048 run the XCD-cohort lock, 13.1 M/s (array 9.2)
  ctx->defaults[1][1].kind = SP_MUTEX_CU_COHORT;
  ctx->defaults[1][1].p.poll_sleep = 0;
  ctx->defaults[1][1].p.cohort_passes = 64;
  // per-XCD chains (K below the XCD count: one set of chains; K above 4096 per XCD: the
  // array kind): 20.8 M pairs/s K = 32 at 256, 126 M K = 256 at 2048 (one set of chains
  // 18.6 / 57.7); 20.3 M K = 32 at 2048, 2.31 M K = 4 (chains 17.9 / 2.31, adaptive
  // 6.3 / 1.55)
  ctx->defaults[2][0].kind = SP_SEM_XCD_CHAIN;
  ctx->defaults[2][0].p.poll_sleep = 0;
  ctx->defaults[2][1].kind = SP_SEM_XCD_CHAIN;
  ctx->defaults[2][1].p.poll_sleep = 0;
  // resolve the "auto" fields (fan_in = XCD count, ...) as sp_set_default does
  for (int prim = 0; prim < 3; ++prim)
    for (int b = 0; b < 2; ++b)
      if (spi::normalize(ctx, &ctx->defaults[prim][b].p, &ctx->defaults[prim][b].p) != SP_OK)
        return fail(hipErrorInvalidValue);
  *out = ctx;
  return SP_OK;
}

int sp_fini(sp_ctx* ctx) {
  if (!usable(ctx)) return SP_E_INVAL;
  // Nothing of this context may still run when its memory goes: wait for the device,
  // then release in the reverse order of sp_init.
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipStreamDestroy(ctx->setup_stream);
  (void)hipStreamDestroy(ctx->capture_stream);
  (void)hipEventDestroy(ctx->ev1);
  (void)hipEventDestroy(ctx->ev0);
  (void)hipFree(ctx->d_scratch);
  (void)hipFree(ctx->d_err);
  ctx->capture_stream = ctx->setup_stream = nullptr;
  ctx->ev0 = ctx->ev1 = nullptr;
  ctx->d_err = ctx->d_scratch = nullptr;
  ctx->closed = true;
  if (ctx->refs == 0) delete ctx;
  return SP_OK;
}

int sp_device_info_get(const sp_ctx* ctx, sp_device_info* out) {
  if (!usable(ctx) || !out) return SP_E_INVAL;
  memset(out, 0, sizeof(*out));
  strncpy(out->name, ctx->prop.name, sizeof(out->name) - 1);
  strncpy(out->arch, ctx->prop.gcnArchName, sizeof(out->arch) - 1);
  out->cu_count = ctx->cu_count;
  out->xcd_count = ctx->xcd_count;
  out->wall_clock_khz = ctx->wall_khz;
  out->clock_khz = (uint32_t)ctx->prop.clockRate;
  out->hbm_bytes = (uint64_t)ctx->prop.totalGlobalMem;
  out->max_threads_per_cu = (uint32_t)ctx->prop.maxThreadsPerMultiProcessor;
  return SP_OK;
}

int sp_set_default(sp_ctx* ctx, uint32_t primitive, uint32_t bucket, uint32_t kind,
                   const sp_params* p) {
  if (!usable(ctx) || primitive > 2 || bucket > 1) return SP_E_INVAL;
  const uint32_t max_kind[3] = {SP_BARRIER_XCD, SP_MUTEX_CU_COHORT, SP_SEM_CU_LOCK};
  if (kind > max_kind[primitive]) return SP_E_INVAL;
  sp_params q;
  SP_CHECK(spi::normalize(ctx, p, &q));
  ctx->defaults[primitive][bucket].kind = kind;
  ctx->defaults[primitive][bucket].p = q;
  return SP_OK;
}

int sp_get_default(const sp_ctx* ctx, uint32_t primitive, uint32_t bucket, uint32_t* kind,
                   sp_params* p) {
  if (!usable(ctx) || primitive > 2 || bucket > 1 || !kind) return SP_E_INVAL;
  *kind = ctx->defaults[primitive][bucket].kind;
  if (p) *p = ctx->defaults[primitive][bucket].p;
  return SP_OK;
}

int sp_probe_xcc(sp_ctx* ctx, uint32_t nwg, uint32_t lanes, uint32_t* out, void* stream) {
  if (!usable(ctx) || !out || nwg == 0 || !spi::lanes_ok(lanes)) return SP_E_INVAL;
  hipStream_t s = spi::as_stream(stream);
  hipLaunchKernelGGL(k_probe_xcc, dim3(nwg), dim3(lanes), 0, s, out);
  SP_HIP(ctx, hipGetLastError());
  SP_HIP(ctx, hipStreamSynchronize(s));
  return SP_OK;
}

int sp_buffer_alloc(sp_ctx* ctx, uint64_t bytes, void** out) {
  if (!usable(ctx) || !out || bytes == 0) return SP_E_INVAL;
  *out = nullptr;
  SP_HIP(ctx, hipSetDevice(ctx->device));
  void* p = nullptr;
  SP_HIP(ctx, hipMalloc(&p, bytes));
  hipError_t e = hipMemset(p, 0, bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    ctx->last_hip = (int)e;
    (void)hipFree(p);
    return SP_E_HIP;
  }
  *out = p;
  return SP_OK;
}

int sp_buffer_free(sp_ctx* ctx, void* p) {
  if (!usable(ctx) || !p) return SP_E_INVAL;
  SP_HIP(ctx, hipSetDevice(ctx->device));
  SP_HIP(ctx, hipFree(p));
  return SP_OK;
}

int sp_buffer_read(sp_ctx* ctx, void* host_dst, const void* dev_src, uint64_t bytes) {
  if (!usable(ctx) || !host_dst || !dev_src) return SP_E_INVAL;
  SP_HIP(ctx, hipSetDevice(ctx->device));
  SP_HIP(ctx, hipMemcpy(host_dst, dev_src, bytes, hipMemcpyDeviceToHost));
  return SP_OK;
}

int sp_buffer_write(sp_ctx* ctx, void* dev_dst, const void* host_src, uint64_t bytes) {
  if (!usable(ctx) || !dev_dst || !host_src) return SP_E_INVAL;
  SP_HIP(ctx, hipSetDevice(ctx->device));
  SP_HIP(ctx, hipMemcpy(dev_dst, host_src, bytes, hipMemcpyHostToDevice));
  return SP_OK;
}

// ---- recorded batches (HIP graphs) ---------------------------------------------------

struct sp_graph {
  sp_ctx* ctx = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
};

int sp_graph_begin(sp_ctx* ctx, void* stream, void** capture_stream) {
  if (!usable(ctx) || !capture_stream) return SP_E_INVAL;
  SP_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = stream ? spi::as_stream(stream) : ctx->capture_stream;
  if (spi::capturing(s)) return SP_E_INVAL;
  SP_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  *capture_stream = s;
  return SP_OK;
}

int sp_graph_end(sp_ctx* ctx, void* capture_stream, sp_graph** out) {
  if (!usable(ctx) || !capture_stream || !out) return SP_E_INVAL;
  *out = nullptr;
  hipStream_t s = spi::as_stream(capture_stream);
  hipGraph_t g = nullptr;
  SP_HIP(ctx, hipStreamEndCapture(s, &g));
  hipGraphExec_t ge = nullptr;
  hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    ctx->last_hip = (int)e;
    (void)hipGraphDestroy(g);
    return SP_E_HIP;
  }
  sp_graph* gr = new sp_graph();
  gr->ctx = ctx;
  spi::ctx_ref(ctx);
  gr->g = g;
  gr->ge = ge;
  *out = gr;
  return SP_OK;
}

int sp_graph_launch(sp_graph* gr, uint32_t replays, sp_stats* st, void* stream) {
  if (!gr || replays == 0) return SP_E_INVAL;
  sp_ctx* ctx = gr->ctx;
  hipStream_t s = spi::as_stream(stream);
  SP_HIP(ctx, hipSetDevice(ctx->device));
  if (spi::capturing(s)) return SP_E_INVAL;
  SP_CHECK(spi::begin_timed(ctx, s));
  for (uint32_t i = 0; i < replays; ++i) SP_HIP(ctx, hipGraphLaunch(gr->ge, s));
  return spi::end_timed(ctx, s, st, 0, 0, 0, replays);
}

int sp_graph_destroy(sp_graph* gr) {
  if (!gr) return SP_E_INVAL;
  sp_ctx* ctx = gr->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipGraphExecDestroy(gr->ge);
  (void)hipGraphDestroy(gr->g);
  delete gr;
  spi::ctx_unref(ctx);
  return SP_OK;
}

}  // extern "C"
