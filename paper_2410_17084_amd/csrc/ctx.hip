// Context, workspace, error reporting and launch timing of the Voxel-GPR library.
#include <cmath>
#include <cstdio>
#include <mutex>

#include "vgpr_internal.h"

namespace vgpr {

// Fixed device scratch of vgpr_fit_predict_noalloc: a file-scope device array,
// one copy per GPU, held until the process ends. Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): vgpr_create looks up each device's address once, with that device
// current, and every use goes through that address.
static __device__ __align__(256) char scratch[kFixedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

// Address of this device's fixed scratch (the current device must be `device`).
static hipError_t fixed_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    g_scratch_done[device] = true;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

vgpr_status fail(vgpr_ctx* ctx, vgpr_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

vgpr_status hip_fail(vgpr_ctx* ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? VGPR_E_NOMEM : VGPR_E_DEVICE, m);
}

namespace {
vgpr_status reserve_buffer(vgpr_ctx* ctx, DeviceBuffer& buf, size_t bytes, const char* what) {
  if (bytes <= buf.bytes) return VGPR_OK;
  size_t want = bytes + bytes / 4;
  size_t others = ctx->held - buf.bytes;
  if (ctx->budget && others + want > ctx->budget) {
    want = bytes;
    if (others + want > ctx->budget)
      return fail(ctx, VGPR_E_BUDGET,
                  std::string(what) + " of " + std::to_string(bytes) + " bytes exceeds the HBM budget");
  }
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (buf.ptr) VGPR_HIP(ctx, hipFree(buf.ptr));
  ctx->held -= buf.bytes;
  buf = DeviceBuffer{};
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) return hip_fail(ctx, e, &buf == &ctx->stage ? "hipMalloc(map staging)" : "hipMalloc(workspace)");
  buf.ptr = p;
  buf.bytes = want;
  ctx->held += want;
  return VGPR_OK;
}
}  // namespace

vgpr_status reserve_work(vgpr_ctx* ctx, size_t bytes) { return reserve_buffer(ctx, ctx->work, bytes, "scratch"); }

vgpr_status reserve_stage(vgpr_ctx* ctx, size_t bytes) {
  return reserve_buffer(ctx, ctx->stage, bytes, "map staging");
}

vgpr_status reserve_pinned(vgpr_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->pinned_bytes) return VGPR_OK;
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->pinned) VGPR_HIP(ctx, hipHostFree(ctx->pinned));
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  size_t want = bytes < 4096 ? 4096 : bytes * 2;
  VGPR_HIP(ctx, hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
  ctx->pinned_bytes = want;
  return VGPR_OK;
}

vgpr_status alloc_owned(vgpr_ctx* ctx, void** p, size_t bytes) {
  if (ctx->budget && ctx->held + bytes > ctx->budget)
    return fail(ctx, VGPR_E_BUDGET, "allocation of " + std::to_string(bytes) + " bytes exceeds the HBM budget");
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc");
  ctx->held += bytes;
  return VGPR_OK;
}

void free_owned(vgpr_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->held -= bytes;
}

static hipEvent_t take_event(vgpr_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(vgpr_ctx* ctx, const char* family, hipStream_t stream, hipEvent_t* start) {
  (void)family;
  *start = nullptr;
  if (!ctx->profiling) return;
  hipEvent_t e = take_event(ctx);
  if (e && hipEventRecord(e, stream) == hipSuccess) *start = e;
}

void prof_end(vgpr_ctx* ctx, const char* family, hipStream_t stream, hipEvent_t start) {
  if (!ctx->profiling || !start) return;
  hipEvent_t e = take_event(ctx);
  if (!e || hipEventRecord(e, stream) != hipSuccess) return;
  ctx->prof[family].pending.emplace_back(start, e);
}

vgpr_status ensure_aux(vgpr_ctx* ctx) {
  if (ctx->aux[0]) return VGPR_OK;
  // default priority on purpose: every stream of the library runs at the same priority
  for (int i = 0; i < vgpr_ctx::kAux; ++i) {
    VGPR_HIP(ctx, hipStreamCreateWithFlags(&ctx->aux[i], hipStreamNonBlocking));
    VGPR_HIP(ctx, hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming));
  }
  VGPR_HIP(ctx, hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  return VGPR_OK;
}

vgpr_status check_params(vgpr_ctx* ctx, const vgpr_params* p) {
  if (!p) return fail(ctx, VGPR_E_INVALID, "params is NULL");
  if (!(p->voxel_size > 0.f) || !std::isfinite(p->voxel_size))
    return fail(ctx, VGPR_E_INVALID, "voxel_size must be a positive finite number");
  if (p->max_pts < 1) return fail(ctx, VGPR_E_INVALID, "max_pts must be >= 1");
  if (p->max_pts > kMaxPtsLimit)
    return fail(ctx, VGPR_E_UNSUPPORTED, "max_pts above 512 is not supported by the library");
  if (p->min_pts < 1) return fail(ctx, VGPR_E_INVALID, "min_pts must be >= 1");
  if (p->grid_side < 1) return fail(ctx, VGPR_E_INVALID, "grid_side must be >= 1");
  if (p->grid_side > kMaxGridSide)
    return fail(ctx, VGPR_E_UNSUPPORTED, "grid_side above 16 is not supported by the library");
  if (!(p->signal_var > 0.f) || !(p->length_scale > 0.f) || !(p->noise_var >= 0.f))
    return fail(ctx, VGPR_E_INVALID, "signal_var and length_scale must be > 0, noise_var >= 0");
  if (p->ls_mode != 0 && p->ls_mode != 1) return fail(ctx, VGPR_E_INVALID, "ls_mode must be 0 or 1");
  if (p->frame_mode != 0 && p->frame_mode != 1) return fail(ctx, VGPR_E_INVALID, "frame_mode must be 0 or 1");
  if (p->precision != VGPR_PREC_FP32 && p->precision != VGPR_PREC_FP64 && p->precision != VGPR_PREC_MIXED)
    return fail(ctx, VGPR_E_INVALID, "unknown precision");
  if (p->precision != VGPR_PREC_FP64 && !(p->cond_threshold > 0.f))
    return fail(ctx, VGPR_E_INVALID, "cond_threshold must be > 0");
  return VGPR_OK;
}

}  // namespace vgpr

using namespace vgpr;

extern "C" {

void vgpr_params_default(vgpr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->voxel_size = 0.2f;
  p->max_pts = 128;
  p->min_pts = 10;
  p->grid_side = 9;
  p->signal_var = 1.0f;
  p->length_scale = 0.70710678f;
  p->noise_var = 1e-3f;
  p->ls_mode = 0;
  p->frame_mode = 0;
  p->precision = VGPR_PREC_FP32;
  p->refine_threshold = 40.0f;
  p->converge_var = 0.3f;
  p->cond_threshold = 1e4f;
}

const char* vgpr_status_str(vgpr_status s) {
  switch (s) {
    case VGPR_OK: return "VGPR_OK";
    case VGPR_E_INVALID: return "VGPR_E_INVALID";
    case VGPR_E_NOMEM: return "VGPR_E_NOMEM";
    case VGPR_E_CAPACITY: return "VGPR_E_CAPACITY";
    case VGPR_E_RANGE: return "VGPR_E_RANGE";
    case VGPR_E_BUDGET: return "VGPR_E_BUDGET";
    case VGPR_E_DEVICE: return "VGPR_E_DEVICE";
    case VGPR_E_UNSUPPORTED: return "VGPR_E_UNSUPPORTED";
  }
  return "VGPR_E_UNKNOWN";
}

// Why the calling thread's last vgpr_create failed (no context exists to hold it).
static thread_local std::string create_error;

static vgpr_status create_fail(vgpr_status st, const char* what, hipError_t e) {
  create_error = std::string(what) + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
  return st;
}

vgpr_status vgpr_create(int device, void* hip_stream, size_t hbm_budget_bytes, vgpr_ctx** out) {
  if (!out) return create_fail(VGPR_E_INVALID, "out is NULL", hipSuccess);
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return create_fail(VGPR_E_DEVICE, "hipGetDeviceCount", e);
  if (device < 0 || device >= n) return create_fail(VGPR_E_DEVICE, "device index out of range", hipSuccess);
  e = hipSetDevice(device);
  if (e != hipSuccess) return create_fail(VGPR_E_DEVICE, "hipSetDevice", e);
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return create_fail(VGPR_E_DEVICE, "hipDeviceGetAttribute(multiprocessor count)", e);
  void* fixed = nullptr;
  e = fixed_scratch_address(device, &fixed);
  if (e != hipSuccess) return create_fail(VGPR_E_DEVICE, "hipGetSymbolAddress(fixed scratch)", e);
  vgpr_ctx* c = new (std::nothrow) vgpr_ctx();
  if (!c) return create_fail(VGPR_E_NOMEM, "out of host memory", hipSuccess);
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->budget = hbm_budget_bytes;
  c->cu_count = cus;
  c->fixed_scratch = fixed;
  // the side streams exist from the start, so that a call of the no-allocation
  // entry point never creates them
  if (ensure_aux(c) != VGPR_OK) {
    const std::string msg = c->last_error;
    vgpr_destroy(c);
    create_error = msg;
    return VGPR_E_DEVICE;
  }
  *out = c;
  return VGPR_OK;
}

vgpr_status vgpr_destroy(vgpr_ctx* ctx) {
  if (!ctx) return VGPR_E_INVALID;
  if (ctx->live_maps > 0) return fail(ctx, VGPR_E_INVALID, "destroy the context's maps first");
  if (ctx->live_graphs > 0) return fail(ctx, VGPR_E_INVALID, "destroy the context's graphs first");
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->work.ptr) (void)hipFree(ctx->work.ptr);
  if (ctx->stage.ptr) (void)hipFree(ctx->stage.ptr);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (auto& kv : ctx->prof)
    for (auto& pr : kv.second.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < vgpr_ctx::kAux; ++i) {
    if (ctx->aux[i]) {
      (void)hipStreamSynchronize(ctx->aux[i]);
      (void)hipStreamDestroy(ctx->aux[i]);
    }
    if (ctx->join_ev[i]) (void)hipEventDestroy(ctx->join_ev[i]);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  delete ctx;
  return VGPR_OK;
}

vgpr_status vgpr_set_stream(vgpr_ctx* ctx, void* hip_stream) {
  if (!ctx) return VGPR_E_INVALID;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return VGPR_OK;
}

const char* vgpr_last_error(const vgpr_ctx* ctx) { return ctx ? ctx->last_error.c_str() : create_error.c_str(); }

size_t vgpr_workspace_bytes(const vgpr_ctx* ctx) { return ctx ? ctx->held : 0; }

vgpr_status vgpr_set_tuning(vgpr_ctx* ctx, const vgpr_tuning* t) {
  if (!ctx || !t) return VGPR_E_INVALID;
  if (t->fp32_last_bucket < -1 || t->fp32_last_bucket > kNumBuckets - 1)
    return fail(ctx, VGPR_E_INVALID, "fp32_last_bucket must be in [-1, 6]");
  if (t->wave_last_bucket < -1 || t->wave_last_bucket > 2)
    return fail(ctx, VGPR_E_INVALID, "wave_last_bucket must be in [-1, 2]");
  if (t->streams != 1 && t->streams != 3) return fail(ctx, VGPR_E_INVALID, "streams must be 1 or 3");
  for (int b = 0; b < kNumBuckets; ++b)
    if (t->grid_scale[b] < 1 || t->grid_scale[b] > 64) return fail(ctx, VGPR_E_INVALID, "grid_scale must be in [1, 64]");
  if (t->tile_first_bucket < 2 || t->tile_first_bucket > 5)
    return fail(ctx, VGPR_E_INVALID, "tile_first_bucket must be in [2, 5]");
  if (t->tiled_first != 0 && t->tiled_first != 1) return fail(ctx, VGPR_E_INVALID, "tiled_first must be 0 or 1");
  for (int b = 0; b < kNumBuckets; ++b)
    if (t->bucket_stream[b] < 0 || t->bucket_stream[b] > vgpr_ctx::kAux)
      return fail(ctx, VGPR_E_INVALID, "bucket_stream entries must be in [0, 3]");
  if (t->tiled_merge != 0 && t->tiled_merge != 1) return fail(ctx, VGPR_E_INVALID, "tiled_merge must be 0 or 1");
  ctx->tune = *t;
  return VGPR_OK;
}

vgpr_status vgpr_get_tuning(const vgpr_ctx* ctx, vgpr_tuning* t) {
  if (!ctx || !t) return VGPR_E_INVALID;
  *t = ctx->tune;
  return VGPR_OK;
}

vgpr_status vgpr_profile_enable(vgpr_ctx* ctx, int on) {
  if (!ctx) return VGPR_E_INVALID;
  ctx->profiling = on != 0;
  return VGPR_OK;
}

vgpr_status vgpr_profile_read(vgpr_ctx* ctx, const char* name, double* h_total_ms, int64_t* h_launches) {
  if (!ctx || !name) return VGPR_E_INVALID;
  (void)hipSetDevice(ctx->device);
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < vgpr_ctx::kAux; ++i)
    if (ctx->aux[i]) VGPR_HIP(ctx, hipStreamSynchronize(ctx->aux[i]));
  double total = 0.0;
  int64_t count = 0;
  auto it = ctx->prof.find(name);
  if (it != ctx->prof.end()) {
    for (auto& pr : it->second.pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        total += ms;
        ++count;
      }
      ctx->event_pool.push_back(pr.first);
      ctx->event_pool.push_back(pr.second);
    }
    it->second.pending.clear();
  }
  if (h_total_ms) *h_total_ms = total;
  if (h_launches) *h_launches = count;
  return VGPR_OK;
}

}  // extern "C"
