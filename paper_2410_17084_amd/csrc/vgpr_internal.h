// Internal declarations of the Voxel-GPR HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "vgpr.h"

namespace vgpr {

constexpr int kKeyFieldBits = 21;
constexpr int64_t kKeyBias = int64_t(1) << 20;
constexpr int64_t kKeyAxisLimit = (int64_t(1) << 20) - 1;
constexpr uint64_t kKeySentinel = ~uint64_t(0);
constexpr int kMaxPtsLimit = 512;   // largest cap the tiled solver supports
// Size of the fixed device scratch of vgpr_fit_predict_noalloc (one array per GPU).
constexpr size_t kFixedScratchBytes = size_t(64) << 20;
constexpr int kMaxGridSide = 16;

// Size buckets of the per-voxel solver: a voxel with n kept points runs in the
// smallest bucket whose capacity is >= n.
constexpr int kNumBuckets = 7;
constexpr int kBucketCap[kNumBuckets] = {16, 32, 64, 96, 128, 256, 512};


// Hash of a 64-bit voxel key for open-addressing tables (the splitmix64
// finaliser, a published 64-bit mixing function).
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// One named family of kernel launches timed with event pairs.
struct ProfFamily {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

}  // namespace vgpr

struct vgpr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;          // 0 = unlimited
  size_t held = 0;            // workspace + staging + maps
  vgpr::DeviceBuffer work;    // per-call scratch, grown on demand
  vgpr::DeviceBuffer stage;   // map updates' solve inputs and scratch, grown on demand (shared by the
                              // context's maps: their updates are ordered on `stream`)
  void* pinned = nullptr;     // small pinned host staging area
  size_t pinned_bytes = 0;
  std::string last_error;
  int cu_count = 0;
  int live_maps = 0;          // maps created on this context and not yet destroyed
  int live_graphs = 0;        // captured graphs created on this context and not yet destroyed
  vgpr_tuning tune{0, 2, 3, {4, 4, 4, 4, 4, 4, 4}, 5, 0, {0, 2, 2, 1, 1, 3, 3}, 0};
  static constexpr int kAux = 3;
  hipStream_t aux[kAux] = {nullptr, nullptr, nullptr};  // side streams the solver buckets fork onto
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kAux] = {nullptr, nullptr, nullptr};
  bool profiling = false;
  void* fixed_scratch = nullptr;  // this device's copy of the fixed scratch array (kFixedScratchBytes)
  std::map<std::string, vgpr::ProfFamily> prof;
  std::vector<hipEvent_t> event_pool;
};

namespace vgpr {

// Error helpers: record a message on the context and return a status.
vgpr_status fail(vgpr_ctx* ctx, vgpr_status s, const std::string& msg);
vgpr_status hip_fail(vgpr_ctx* ctx, hipError_t e, const char* what);

#define VGPR_HIP(ctx, call)                                  \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return ::vgpr::hip_fail(ctx, e_, #call); \
  } while (0)

// Make sure ctx->work holds at least `bytes`; may synchronise the stream.
vgpr_status reserve_work(vgpr_ctx* ctx, size_t bytes);
// Make sure ctx->stage holds at least `bytes`; may synchronise the stream.
vgpr_status reserve_stage(vgpr_ctx* ctx, size_t bytes);
// Pinned host staging of at least `bytes`.
vgpr_status reserve_pinned(vgpr_ctx* ctx, size_t bytes);
// Device memory owned by something other than the workspace (maps).
vgpr_status alloc_owned(vgpr_ctx* ctx, void** p, size_t bytes);
void free_owned(vgpr_ctx* ctx, void* p, size_t bytes);

// Carve aligned sub-buffers out of the workspace.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
};

// Launch timing (no-ops unless profiling is on); events go on the launch's stream.
void prof_begin(vgpr_ctx* ctx, const char* family, hipStream_t stream, hipEvent_t* start);
void prof_end(vgpr_ctx* ctx, const char* family, hipStream_t stream, hipEvent_t start);

struct ProfScope {
  vgpr_ctx* ctx;
  const char* family;
  hipStream_t stream;
  hipEvent_t start = nullptr;
  ProfScope(vgpr_ctx* c, const char* f) : ctx(c), family(f), stream(c->stream) {
    prof_begin(ctx, family, stream, &start);
  }
  ProfScope(vgpr_ctx* c, const char* f, hipStream_t s) : ctx(c), family(f), stream(s) {
    prof_begin(ctx, family, stream, &start);
  }
  ~ProfScope() { prof_end(ctx, family, stream, start); }
};

// Side streams and fork/join events of a context (created on first use).
vgpr_status ensure_aux(vgpr_ctx* ctx);

vgpr_status check_params(vgpr_ctx* ctx, const vgpr_params* p);

// Voxelize into caller buffers; also used by the map and the structure loss.
// On success *n_vox holds the voxel count (host). Voxels come out in x-major
// order of their indices, or with `morton` in Morton order (index bits
// interleaved), where each run of consecutive voxels covers a compact region.
vgpr_status voxelize_impl(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts, const int64_t* h_frame_offsets,
                          int32_t n_frames, float voxel_size, uint64_t* d_keys, int32_t* d_offsets,
                          int32_t* d_counts, int32_t* d_perm, int64_t cap_vox, int64_t* h_n_vox,
                          int64_t* h_frame_vox, int64_t* h_n_invalid, size_t work_offset,
                          bool morton = false);

// Solve the voxels of a list. `d_list` (nullable) maps output slot -> voxel
// index into keys/offsets/counts; with NULL the slots are 0..n_vox-1.
// `work_offset` is where in ctx->work this call may start carving scratch.
struct FitArgs {
  const float* xyz;
  int64_t n_pts;             // points d_xyz holds (and d_perm indexes)
  const uint64_t* keys;
  const int32_t* offsets;
  const int32_t* counts;
  const int32_t* perm;       // nullable: points are contiguous from offsets
  const float* noise;        // nullable: per input point noise variance
  int64_t n_vox;
  float* out;
  int8_t* axis;
  uint8_t* status;
};
size_t fit_work_bytes(const vgpr_ctx* ctx, int64_t n_vox, int64_t n_pts, const vgpr_params* p);
// fixed_work: scratch the caller owns (at least fit_work_bytes); when null the
// context workspace from work_offset on is used (and grown if needed).
vgpr_status fit_predict_impl(vgpr_ctx* ctx, const FitArgs& a, const vgpr_params* p, size_t work_offset,
                             char* fixed_work = nullptr);

}  // namespace vgpr
