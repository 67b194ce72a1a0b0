// vgpr_map_*: the global voxel map C of Alg. S1 with the voxel states of
// Sec. 3.3 (paper), resident in HBM.
//
// Layout: an open-addressing hash table of 64-bit voxel keys (linear probing,
// 2x the voxel capacity, the all-ones sentinel marks an empty slot) pointing
// at dense voxel records: key, stored point count, total arrived count and a
// converged flag, plus a point pool with max_pts float3 slots per voxel.
//
// One frame: voxelize (Alg. S1) -> when the frame's voxels could overflow the
// map, probe the table to count the new ones (the frame is rejected when they
// would) -> insert and append
// points in arrival order up to the cap -> collect the touched voxels that
// hold >= tau points and are not converged (types (b), (c)) in ascending key
// order -> solve them from the pool with the per-voxel solver -> mark those
// whose max variance <= eta as converged (type (d)).
//
// Feedback maps (update mode 1, the covariance-centred update of Sec. 3.3 and
// Fig. 4) also keep each solved voxel's predicted grid (m float4 rows). Once a
// voxel holds a prediction its pool stops growing: a frame that touches it
// stacks the m carried rows (noise variance = their posterior variance,
// raised to kPredNoiseFloor s_f^2) with the frame's first max_pts new points
// (sensor noise) in a staging area of m + max_pts slots per voxel, re-solves
// Alg. 1 on that set, and the new rows replace the carried ones.
#include <algorithm>
#include <vector>

#include "scan.h"
#include "vgpr_internal.h"

struct vgpr_map {
  vgpr_ctx* ctx = nullptr;
  vgpr_params params{};
  int64_t max_voxels = 0;
  int64_t nslots = 0;
  uint64_t* slot_key = nullptr;
  int32_t* slot_id = nullptr;
  uint64_t* vkey = nullptr;
  int32_t* vstored = nullptr;
  int32_t* vtotal = nullptr;
  uint8_t* vconv = nullptr;
  float* pool = nullptr;
  unsigned long long* counters = nullptr;  // [0] voxels, [1] new this frame, [2] updates
  size_t bytes = 0;
  void* block = nullptr;
  int mode = 0;              // 0: re-solve on the stored points; 1: covariance feedback
  float4* pred = nullptr;    // mode 1: m predicted rows (x, y, z, var) per voxel
  uint8_t* vpred = nullptr;  // mode 1: the voxel holds a prediction (it is in the map)
  int64_t host_voxels = 0;   // voxels held, as read back after the last update (host copy)
};

namespace vgpr {
namespace {

// Smallest noise variance, relative to s_f^2, that a carried prediction takes
// into a re-solve (a posterior variance can round to 0).
constexpr float kPredNoiseFloor = 1e-6f;

__device__ __forceinline__ int64_t find_slot(const uint64_t* slot_key, int64_t nslots, uint64_t key, bool* found) {
  int64_t s = (int64_t)(mix64(key) & (uint64_t)(nslots - 1));
  for (int64_t probe = 0; probe < nslots; ++probe) {
    const uint64_t k = slot_key[s];
    if (k == key) { *found = true; return s; }
    if (k == kKeySentinel) { *found = false; return s; }
    s = (s + 1) & (nslots - 1);
  }
  *found = false;
  return -1;
}

__global__ void __launch_bounds__(256) probe_kernel(const uint64_t* __restrict__ keys, int64_t nv,
                                                    const uint64_t* __restrict__ slot_key, int64_t nslots,
                                                    unsigned long long* __restrict__ counters) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool is_new = false;
  if (v < nv) {
    bool found;
    find_slot(slot_key, nslots, keys[v], &found);
    is_new = !found;
  }
  const unsigned long long m = __ballot(is_new);
  if (lane_id() == 0 && m) atomicAdd(&counters[1], (unsigned long long)__popcll(m));
}

// One wave per frame voxel: insert or find, append points, flag for solving.
__global__ void __launch_bounds__(256) insert_kernel(vgpr_map M, const float* __restrict__ xyz,
                                                     const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ offs, const int32_t* __restrict__ cnts,
                                                     const int32_t* __restrict__ perm, int64_t nv, int cap, int tau,
                                                     uint32_t* __restrict__ flag, int32_t* __restrict__ ids) {
  const int64_t v = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = lane_id();
  if (v >= nv) return;
  const uint64_t key = keys[v];
  int id = -1;
  int stored = 0;
  int inmap = 0;
  if (lane == 0) {
    int64_t s = (int64_t)(mix64(key) & (uint64_t)(M.nslots - 1));
    for (int64_t probe = 0; probe < M.nslots; ++probe) {
      const unsigned long long prev =
          atomicCAS(reinterpret_cast<unsigned long long*>(&M.slot_key[s]), (unsigned long long)kKeySentinel,
                    (unsigned long long)key);
      if (prev == kKeySentinel) {
        // new voxel: keys are unique within a frame, so no other lane races on it
        id = (int)atomicAdd(&M.counters[0], 1ull);
        if (id >= M.max_voxels) {  // the host checks capacity first; never index past the records
          M.slot_id[s] = -1;
          id = -1;
          break;
        }
        M.slot_id[s] = id;
        M.vkey[id] = key;
        M.vstored[id] = 0;
        M.vtotal[id] = 0;
        M.vconv[id] = 0;
        if (M.vpred) M.vpred[id] = 0;
        break;
      }
      if (prev == key) {
        id = M.slot_id[s];
        if (id >= 0) {
          stored = M.vstored[id];
          inmap = M.vpred ? M.vpred[id] : 0;
        }
        break;
      }
      s = (s + 1) & (M.nslots - 1);
    }
  }
  // the record is read and written by lane 0 only; other lanes get it by shuffle
  id = __shfl(id, 0, 64);
  stored = __shfl(stored, 0, 64);
  inmap = __shfl(inmap, 0, 64);
  if (id < 0) {
    if (lane == 0) {
      flag[v] = 0u;
      ids[v] = 0;
    }
    return;
  }
  const int c = cnts[v];
  if (inmap) {  // feedback map, voxel already solved: its new points go to the re-solve, not the pool
    if (lane == 0) {
      M.vtotal[id] += c;
      ids[v] = id;
      flag[v] = M.vconv[id] ? 0u : 1u;
    }
    return;
  }
  const int take = min(c, cap - stored);
  const int o = offs[v];
  for (int i = lane; i < take; i += 64) {
    const int src = perm[o + i];
    float* dst = M.pool + ((size_t)id * cap + stored + i) * 3;
    dst[0] = xyz[3 * (size_t)src + 0];
    dst[1] = xyz[3 * (size_t)src + 1];
    dst[2] = xyz[3 * (size_t)src + 2];
  }
  if (lane == 0) {
    const int now = stored + (take > 0 ? take : 0);
    M.vstored[id] = now;
    M.vtotal[id] += c;
    ids[v] = id;
    flag[v] = (now >= tau && !M.vconv[id]) ? 1u : 0u;
  }
}

constexpr int kCompactTile = 1024;

// The update list: flagged frame voxels in frame order. Besides each entry's
// slot, the scan gives each entry's first point in a back-to-back staging of
// the voxels' pooled points (update mode 0 solves from that staging).
__device__ __forceinline__ uint32_t pooled_of(const vgpr_map& M, const int32_t* ids, const uint32_t* flag,
                                              int64_t i, int64_t n) {
  return (i < n && flag[i]) ? (uint32_t)M.vstored[ids[i]] : 0u;
}

__global__ void __launch_bounds__(1024) compact_reduce(vgpr_map M, const uint32_t* __restrict__ flag,
                                                       const int32_t* __restrict__ ids, int64_t n,
                                                       uint32_t* __restrict__ block_sums,
                                                       uint32_t* __restrict__ block_pts) {
  const int64_t i = (int64_t)blockIdx.x * kCompactTile + threadIdx.x;
  const uint32_t c = wave_sum(i < n ? flag[i] : 0u);
  const uint32_t q = wave_sum(pooled_of(M, ids, flag, i, n));
  __shared__ uint32_t s[16], sq[16];
  if (lane_id() == 0) s[threadIdx.x >> 6] = c, sq[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0, tq = 0;
    for (int w = 0; w < 16; ++w) t += s[w], tq += sq[w];
    block_sums[blockIdx.x] = t;
    block_pts[blockIdx.x] = tq;
  }
}

// One workgroup: exclusive scans of both per-block sums; total[0] = entries,
// total[1] = their pooled points.
__global__ void __launch_bounds__(1024) compact_scan(uint32_t* __restrict__ block_sums,
                                                     uint32_t* __restrict__ block_pts, int nblocks,
                                                     unsigned long long* __restrict__ total) {
  __shared__ uint32_t smem[17];
  uint32_t carry = 0, carry_q = 0;
  for (int s = 0; s < nblocks; s += 1024) {
    const int i = s + threadIdx.x;
    const uint32_t v = i < nblocks ? block_sums[i] : 0u;
    const uint32_t q = i < nblocks ? block_pts[i] : 0u;
    uint32_t tot, tot_q;
    const uint32_t ex = block_exclusive_sum<1024>(v, smem, &tot);
    const uint32_t ex_q = block_exclusive_sum<1024>(q, smem, &tot_q);
    if (i < nblocks) {
      block_sums[i] = carry + ex;
      block_pts[i] = carry_q + ex_q;
    }
    carry += tot;
    carry_q += tot_q;
  }
  if (threadIdx.x == 0) {
    total[0] = carry;
    total[1] = carry_q;
  }
}

__global__ void __launch_bounds__(1024) compact_scatter(vgpr_map M, const uint32_t* __restrict__ flag,
                                                        const int32_t* __restrict__ ids, int64_t n,
                                                        const uint32_t* __restrict__ block_base,
                                                        const uint32_t* __restrict__ block_pts,
                                                        uint64_t* __restrict__ ukey, int32_t* __restrict__ uoff,
                                                        int32_t* __restrict__ ucnt, int32_t* __restrict__ uid,
                                                        int32_t* __restrict__ ufv, int32_t* __restrict__ upts) {
  __shared__ uint32_t smem[17];
  const int64_t i = (int64_t)blockIdx.x * kCompactTile + threadIdx.x;
  const uint32_t f = i < n ? flag[i] : 0u;
  uint32_t tot;
  const uint32_t ex = block_exclusive_sum<1024>(f, smem, &tot);
  const uint32_t ex_q = block_exclusive_sum<1024>(pooled_of(M, ids, flag, i, n), smem, &tot);
  if (f) {
    const uint32_t slot = block_base[blockIdx.x] + ex;
    const int id = ids[i];
    ukey[slot] = M.vkey[id];
    uoff[slot] = id * M.params.max_pts;
    ucnt[slot] = M.vtotal[id];
    uid[slot] = id;
    ufv[slot] = (int32_t)i;
    upts[slot] = (int32_t)(block_pts[blockIdx.x] + ex_q);
  }
}

// Update mode 0: one wavefront per re-solved voxel u copies its pooled points
// to [upts[u], upts[u] + stored) of the staging area, back to back, so that the
// solve's point scratch scales with the update, not with the map's capacity.
__global__ void __launch_bounds__(256) gather_pool_kernel(vgpr_map M, const int32_t* __restrict__ uid,
                                                          const int32_t* __restrict__ upts, int64_t nu,
                                                          float* __restrict__ sxyz, int32_t* __restrict__ soff) {
  const int64_t u = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (u >= nu) return;
  const int lane = lane_id();
  const int id = uid[u];
  const int k = M.vstored[id];
  const int64_t o = upts[u];
  const float* src = M.pool + (size_t)id * M.params.max_pts * 3;
  for (int t = lane; t < 3 * k; t += 64) sxyz[3 * o + t] = src[t];
  if (lane == 0) soff[u] = (int32_t)o;
}

__global__ void __launch_bounds__(256) state_kernel(vgpr_map M, const int32_t* __restrict__ uid,
                                                    const uint8_t* __restrict__ status, int64_t nu) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < nu && (status[u] & VGPR_ST_CONVERGED)) M.vconv[uid[u]] = 1;
}

// Feedback maps: one wavefront per re-solved voxel u writes its training set to
// slots [u * per, u * per + n) of the staging area. A voxel in the map: the m
// carried rows, then the frame's first max_pts new points; otherwise (first
// solve): its pooled points. CAPPED is decided here (frame points beyond
// max_pts, or pooled arrivals beyond max_pts) since the solve sees only the
// kept points.
__global__ void __launch_bounds__(256) stack_kernel(vgpr_map M, const float* __restrict__ xyz,
                                                    const int32_t* __restrict__ foff, const int32_t* __restrict__ fcnt,
                                                    const int32_t* __restrict__ fperm, const int32_t* __restrict__ uid,
                                                    const int32_t* __restrict__ ufv, int64_t nu, int m, int per,
                                                    float* __restrict__ sxyz, float* __restrict__ snoise,
                                                    int32_t* __restrict__ soff, int32_t* __restrict__ scnt,
                                                    uint8_t* __restrict__ scap) {
  const int64_t u = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = lane_id();
  if (u >= nu) return;
  const int id = uid[u];
  const int cap = M.params.max_pts;
  const float sn = M.params.noise_var;
  const int64_t base = u * (int64_t)per;
  int n;
  bool capped;
  if (M.vpred[id]) {
    const float floor_var = kPredNoiseFloor * M.params.signal_var;
    const float4* rows = M.pred + (size_t)id * m;
    for (int q = lane; q < m; q += 64) {
      const float4 r = rows[q];
      float* d = sxyz + 3 * (base + q);
      d[0] = r.x;
      d[1] = r.y;
      d[2] = r.z;
      snoise[base + q] = fmaxf(r.w, floor_var);
    }
    const int fv = ufv[u];
    const int c = fcnt[fv];
    const int take = min(c, cap);
    const int o = foff[fv];
    for (int k = lane; k < take; k += 64) {
      const int src = fperm[o + k];
      float* d = sxyz + 3 * (base + m + k);
      d[0] = xyz[3 * (size_t)src + 0];
      d[1] = xyz[3 * (size_t)src + 1];
      d[2] = xyz[3 * (size_t)src + 2];
      snoise[base + m + k] = sn;
    }
    n = m + take;
    capped = c > cap;
  } else {
    const int st = M.vstored[id];
    const float* src = M.pool + (size_t)id * cap * 3;
    for (int k = lane; k < st; k += 64) {
      float* d = sxyz + 3 * (base + k);
      d[0] = src[3 * k + 0];
      d[1] = src[3 * k + 1];
      d[2] = src[3 * k + 2];
      snoise[base + k] = sn;
    }
    n = st;
    capped = M.vtotal[id] > cap;
  }
  if (lane == 0) {
    soff[u] = (int32_t)base;
    scnt[u] = n;
    scap[u] = capped ? 1 : 0;
  }
}

// Feedback maps: one thread per predicted row; a solved voxel's rows replace
// its carried prediction; the row-0 thread sets the voxel's flags and adds
// CAPPED to its status (the SOLVED and CONVERGED bits it reads are not
// changed by that write).
__global__ void __launch_bounds__(256) feedback_state_kernel(vgpr_map M, const int32_t* __restrict__ uid,
                                                             const uint8_t* __restrict__ scap,
                                                             const float4* __restrict__ out,
                                                             uint8_t* __restrict__ status, int64_t nu, int m) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nu * m) return;
  const int64_t u = t / m;
  const int q = (int)(t - u * m);
  const int id = uid[u];
  const uint8_t st = status[u];
  if (st & VGPR_ST_SOLVED) M.pred[(size_t)id * m + q] = out[t];
  if (q == 0) {
    if (st & VGPR_ST_SOLVED) M.vpred[id] = 1;
    if (st & VGPR_ST_CONVERGED) M.vconv[id] = 1;
    if (scap[u]) status[u] = st | VGPR_ST_CAPPED;
  }
}

__global__ void __launch_bounds__(256) stats_kernel(vgpr_map M, unsigned long long* __restrict__ out) {
  const int64_t nv = (int64_t)M.counters[0];
  unsigned long long pts = 0, conv = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    pts += (unsigned long long)M.vstored[v];
    conv += M.vconv[v] ? 1ull : 0ull;
  }
  atomicAdd(&out[0], pts);
  atomicAdd(&out[1], conv);
}

// Map import: the hash table from the voxel records (keys are unique).
__global__ void __launch_bounds__(256) rebuild_kernel(vgpr_map M, int64_t nv) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nv) return;
  const uint64_t key = M.vkey[id];
  int64_t s = (int64_t)(mix64(key) & (uint64_t)(M.nslots - 1));
  for (int64_t probe = 0; probe < M.nslots; ++probe) {
    const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(&M.slot_key[s]),
                                              (unsigned long long)kKeySentinel, (unsigned long long)key);
    if (prev == kKeySentinel) {
      M.slot_id[s] = (int32_t)id;
      return;
    }
    s = (s + 1) & (M.nslots - 1);
  }
}

// Serialised map: a fixed header, then the per-voxel arrays in this order.
constexpr char kMapMagic[8] = {'V', 'G', 'P', 'R', 'M', 'A', 'P', '1'};
constexpr uint32_t kMapVersion = 1;
struct MapHeader {
  char magic[8];
  uint32_t version;
  int32_t update_mode;
  int64_t n_voxels;
  vgpr_params params;
};

struct MapLayout {
  size_t keys, stored, total, conv, vpred, pool, pred, end;
};

MapLayout map_layout(int mode, int64_t nv, int cap, int m) {
  MapLayout L{};
  size_t o = sizeof(MapHeader);
  L.keys = o;
  o += 8 * (size_t)nv;
  L.stored = o;
  o += 4 * (size_t)nv;
  L.total = o;
  o += 4 * (size_t)nv;
  L.conv = o;
  o += (size_t)nv;
  L.vpred = o;
  o += mode == 1 ? (size_t)nv : 0;
  L.pool = o;
  o += 12 * (size_t)cap * (size_t)nv;
  L.pred = o;
  o += mode == 1 ? 16 * (size_t)m * (size_t)nv : 0;
  L.end = o;
  return L;
}

}  // namespace
}  // namespace vgpr

using namespace vgpr;

extern "C" {

vgpr_status vgpr_map_create_ex(vgpr_ctx* ctx, const vgpr_params* params, int64_t max_voxels, int update_mode,
                               vgpr_map** out) {
  if (!ctx || !out) return VGPR_E_INVALID;
  *out = nullptr;
  vgpr_status st = check_params(ctx, params);
  if (st != VGPR_OK) return st;
  if (update_mode != 0 && update_mode != 1) return fail(ctx, VGPR_E_INVALID, "update_mode must be 0 or 1");
  const int64_t m = (int64_t)params->grid_side * params->grid_side;
  if (max_voxels < 1 || max_voxels * (int64_t)params->max_pts >= (int64_t(1) << 31))
    return fail(ctx, VGPR_E_INVALID, "max_voxels * max_pts must be in [1, 2^31)");
  if (update_mode == 1 && m + params->max_pts > kMaxPtsLimit)
    return fail(ctx, VGPR_E_INVALID, "update_mode 1 needs grid_side^2 + max_pts <= 512");
  if (update_mode == 1 && max_voxels * m >= (int64_t(1) << 31))
    return fail(ctx, VGPR_E_INVALID, "max_voxels * grid_side^2 must be below 2^31");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  vgpr_map* M = new (std::nothrow) vgpr_map();
  if (!M) return VGPR_E_NOMEM;
  M->ctx = ctx;
  M->params = *params;
  M->max_voxels = max_voxels;
  int64_t ns = 1;
  while (ns < 2 * max_voxels) ns <<= 1;
  M->nslots = ns;
  const size_t cap = (size_t)params->max_pts;
  size_t off = 0;
  auto sub = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    size_t r = off;
    off += bytes;
    return r;
  };
  const size_t o_sk = sub(sizeof(uint64_t) * ns), o_si = sub(sizeof(int32_t) * ns);
  const size_t o_vk = sub(sizeof(uint64_t) * max_voxels), o_vs = sub(sizeof(int32_t) * max_voxels);
  const size_t o_vt = sub(sizeof(int32_t) * max_voxels), o_vc = sub(max_voxels);
  const size_t o_pool = sub(sizeof(float) * 3 * cap * max_voxels), o_ctr = sub(sizeof(unsigned long long) * 8);
  const size_t o_pred = update_mode == 1 ? sub(sizeof(float4) * (size_t)m * max_voxels) : 0;
  const size_t o_vp = update_mode == 1 ? sub(max_voxels) : 0;
  const size_t total = (off + 255) & ~size_t(255);
  void* blk = nullptr;
  st = alloc_owned(ctx, &blk, total);
  if (st != VGPR_OK) {
    delete M;
    return st;
  }
  char* b = static_cast<char*>(blk);
  M->block = blk;
  M->bytes = total;
  M->slot_key = reinterpret_cast<uint64_t*>(b + o_sk);
  M->slot_id = reinterpret_cast<int32_t*>(b + o_si);
  M->vkey = reinterpret_cast<uint64_t*>(b + o_vk);
  M->vstored = reinterpret_cast<int32_t*>(b + o_vs);
  M->vtotal = reinterpret_cast<int32_t*>(b + o_vt);
  M->vconv = reinterpret_cast<uint8_t*>(b + o_vc);
  M->pool = reinterpret_cast<float*>(b + o_pool);
  M->counters = reinterpret_cast<unsigned long long*>(b + o_ctr);
  M->mode = update_mode;
  if (update_mode == 1) {
    M->pred = reinterpret_cast<float4*>(b + o_pred);
    M->vpred = reinterpret_cast<uint8_t*>(b + o_vp);
  }
  if (hipMemsetAsync(M->slot_key, 0xFF, sizeof(uint64_t) * ns, ctx->stream) != hipSuccess ||
      hipMemsetAsync(M->counters, 0, sizeof(unsigned long long) * 8, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    free_owned(ctx, blk, total);
    delete M;
    return fail(ctx, VGPR_E_DEVICE, "map initialisation failed");
  }
  ctx->live_maps += 1;
  *out = M;
  return VGPR_OK;
}

vgpr_status vgpr_map_create(vgpr_ctx* ctx, const vgpr_params* params, int64_t max_voxels, vgpr_map** out) {
  return vgpr_map_create_ex(ctx, params, max_voxels, 0, out);
}

vgpr_status vgpr_map_destroy(vgpr_map* M) {
  if (!M) return VGPR_E_INVALID;
  vgpr_ctx* ctx = M->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_owned(ctx, M->block, M->bytes);
  ctx->live_maps -= 1;
  delete M;
  return VGPR_OK;
}

vgpr_status vgpr_map_update(vgpr_map* M, const float* d_xyz, int64_t n_pts, uint64_t* d_upd_keys, float* d_out,
                            int8_t* d_axis, uint8_t* d_status, int64_t cap_upd, int64_t* h_n_upd) {
  if (!M || !h_n_upd) return VGPR_E_INVALID;
  vgpr_ctx* ctx = M->ctx;
  *h_n_upd = 0;
  if (n_pts < 0 || n_pts >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_INVALID, "n_pts out of range");
  if (n_pts > 0 && !d_xyz) return fail(ctx, VGPR_E_INVALID, "d_xyz is NULL");
  if (cap_upd < 0) return fail(ctx, VGPR_E_INVALID, "cap_upd < 0");
  if (cap_upd > 0 && (!d_upd_keys || !d_out || !d_axis || !d_status))
    return fail(ctx, VGPR_E_INVALID, "output buffer is NULL");
  if (n_pts == 0) return VGPR_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  const vgpr_params& p = M->params;
  const int64_t n = n_pts;
  const int64_t nblk = (n + kCompactTile - 1) / kCompactTile;
  // scratch: frame voxels (<= n) and the update list, then voxelize / fit scratch
  size_t head = 0;
  auto sub = [&](size_t bytes) {
    head = (head + 255) & ~size_t(255);
    size_t r = head;
    head += bytes;
    return r;
  };
  const size_t o_k = sub(8 * n), o_o = sub(4 * n), o_c = sub(4 * n), o_p = sub(4 * n), o_f = sub(4 * n),
               o_id = sub(4 * n), o_bs = sub(4 * nblk + 64), o_bq = sub(4 * nblk + 64), o_uk = sub(8 * n),
               o_uo = sub(4 * n), o_uc = sub(4 * n), o_ui = sub(4 * n), o_fv = sub(4 * n), o_up = sub(4 * n),
               o_tot = sub(64);
  head = (head + 255) & ~size_t(255);
  // the solve runs from the context's staging area, sized once the update is known
  vgpr_status st = reserve_work(ctx, head + 24 * (size_t)n + 4096 * 16 + (1 << 20));
  if (st != VGPR_OK) return st;
  char* w = static_cast<char*>(ctx->work.ptr);
  uint64_t* fkeys = reinterpret_cast<uint64_t*>(w + o_k);
  int32_t* foff = reinterpret_cast<int32_t*>(w + o_o);
  int32_t* fcnt = reinterpret_cast<int32_t*>(w + o_c);
  int32_t* fperm = reinterpret_cast<int32_t*>(w + o_p);
  uint32_t* flag = reinterpret_cast<uint32_t*>(w + o_f);
  int32_t* ids = reinterpret_cast<int32_t*>(w + o_id);
  uint32_t* bsum = reinterpret_cast<uint32_t*>(w + o_bs);
  uint32_t* bpts = reinterpret_cast<uint32_t*>(w + o_bq);
  uint64_t* ukey = reinterpret_cast<uint64_t*>(w + o_uk);
  int32_t* uoff = reinterpret_cast<int32_t*>(w + o_uo);
  int32_t* ucnt = reinterpret_cast<int32_t*>(w + o_uc);
  int32_t* uid = reinterpret_cast<int32_t*>(w + o_ui);
  int32_t* ufv = reinterpret_cast<int32_t*>(w + o_fv);
  int32_t* upts = reinterpret_cast<int32_t*>(w + o_up);
  unsigned long long* dtot = reinterpret_cast<unsigned long long*>(w + o_tot);

  int64_t nv = 0;
  st = voxelize_impl(ctx, d_xyz, n, nullptr, 1, p.voxel_size, fkeys, foff, fcnt, fperm, n, &nv, nullptr, nullptr,
                     head);
  if (st != VGPR_OK) return st;
  if (nv == 0) return VGPR_OK;
  if (ctx->work.ptr != static_cast<void*>(w)) return fail(ctx, VGPR_E_DEVICE, "workspace moved during map update");

  st = reserve_pinned(ctx, 64);
  if (st != VGPR_OK) return st;
  unsigned long long* hc = static_cast<unsigned long long*>(ctx->pinned);
  if (M->host_voxels + nv > M->max_voxels) {
    // the frame might overflow the map: count its new voxels and reject it if they would
    // (otherwise even all nv voxels being new fits, and the count is not needed)
    VGPR_HIP(ctx, hipMemsetAsync(M->counters + 1, 0, sizeof(unsigned long long), ctx->stream));
    hipLaunchKernelGGL(probe_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, ctx->stream, fkeys, nv,
                       M->slot_key, M->nslots, M->counters);
    VGPR_HIP(ctx, hipGetLastError());
    VGPR_HIP(ctx, hipMemcpyAsync(hc, M->counters, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 ctx->stream));
    VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if ((int64_t)(hc[0] + hc[1]) > M->max_voxels)
      return fail(ctx, VGPR_E_CAPACITY, "frame would exceed the map's voxel capacity");
  }

  const int64_t nvb = (nv + kCompactTile - 1) / kCompactTile;
  hipLaunchKernelGGL(insert_kernel, dim3((unsigned)((nv + 3) / 4)), dim3(256), 0, ctx->stream, *M, d_xyz, fkeys,
                     foff, fcnt, fperm, nv, p.max_pts, p.min_pts, flag, ids);
  hipLaunchKernelGGL(compact_reduce, dim3((unsigned)nvb), dim3(1024), 0, ctx->stream, *M, flag, ids, nv, bsum, bpts);
  hipLaunchKernelGGL(compact_scan, dim3(1), dim3(1024), 0, ctx->stream, bsum, bpts, (int)nvb, dtot);
  hipLaunchKernelGGL(compact_scatter, dim3((unsigned)nvb), dim3(1024), 0, ctx->stream, *M, flag, ids, nv, bsum, bpts,
                     ukey, uoff, ucnt, uid, ufv, upts);
  VGPR_HIP(ctx, hipGetLastError());
  VGPR_HIP(ctx, hipMemcpyAsync(hc, dtot, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
  VGPR_HIP(ctx, hipMemcpyAsync(hc + 2, M->counters, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  M->host_voxels = (int64_t)hc[2];
  const int64_t nu = (int64_t)hc[0];
  const int64_t pooled = (int64_t)hc[1];  // pooled points of all nu entries (an upper bound for the first nout)
  *h_n_upd = nu;
  if (nu == 0) return VGPR_OK;
  const int64_t nout = nu < cap_upd ? nu : cap_upd;
  if (nout > 0 && M->mode == 1) {
    VGPR_HIP(ctx, hipMemcpyAsync(d_upd_keys, ukey, sizeof(uint64_t) * nout, hipMemcpyDeviceToDevice, ctx->stream));
    const int m = p.grid_side * p.grid_side;
    const int per = m + p.max_pts;
    const int64_t npts = nout * (int64_t)per;
    if (npts >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_CAPACITY, "too many re-solved voxels in one frame");
    vgpr_params pf = p;  // the stacked set holds up to m + max_pts points; CAPPED is set by stack_kernel
    pf.max_pts = per;
    size_t so = 0;
    auto take = [&](size_t bytes) {
      so = (so + 255) & ~size_t(255);
      size_t r = so;
      so += bytes;
      return r;
    };
    const size_t s_xyz = take(12 * (size_t)npts), s_nz = take(4 * (size_t)npts), s_off = take(4 * (size_t)nout),
                 s_cnt = take(4 * (size_t)nout), s_cap = take((size_t)nout), s_fit = take(fit_work_bytes(ctx, nout, npts, &pf));
    st = reserve_stage(ctx, (so + 255) & ~size_t(255));
    if (st != VGPR_OK) return st;
    char* sb = static_cast<char*>(ctx->stage.ptr);
    float* sxyz = reinterpret_cast<float*>(sb + s_xyz);
    float* snz = reinterpret_cast<float*>(sb + s_nz);
    int32_t* soff = reinterpret_cast<int32_t*>(sb + s_off);
    int32_t* scnt = reinterpret_cast<int32_t*>(sb + s_cnt);
    uint8_t* scap = reinterpret_cast<uint8_t*>(sb + s_cap);
    hipLaunchKernelGGL(stack_kernel, dim3((unsigned)((nout + 3) / 4)), dim3(256), 0, ctx->stream, *M, d_xyz, foff,
                       fcnt, fperm, uid, ufv, nout, m, per, sxyz, snz, soff, scnt, scap);
    VGPR_HIP(ctx, hipGetLastError());
    FitArgs a{sxyz, npts, ukey, soff, scnt, nullptr, snz, nout, d_out, d_axis, d_status};
    st = fit_predict_impl(ctx, a, &pf, 0, sb + s_fit);
    if (st != VGPR_OK) return st;
    hipLaunchKernelGGL(feedback_state_kernel, dim3((unsigned)((nout * m + 255) / 256)), dim3(256), 0, ctx->stream,
                       *M, uid, scap, reinterpret_cast<const float4*>(d_out), d_status, nout, m);
    VGPR_HIP(ctx, hipGetLastError());
  } else if (nout > 0) {
    VGPR_HIP(ctx, hipMemcpyAsync(d_upd_keys, ukey, sizeof(uint64_t) * nout, hipMemcpyDeviceToDevice, ctx->stream));
    // the re-solved voxels' pooled points back to back (counts stay the totals, for CAPPED)
    const int64_t npts = pooled > 0 ? pooled : 1;
    size_t so = 0;
    auto take = [&](size_t bytes) {
      so = (so + 255) & ~size_t(255);
      size_t r = so;
      so += bytes;
      return r;
    };
    const size_t s_xyz = take(12 * (size_t)npts), s_off = take(4 * (size_t)nout),
                 s_fit = take(fit_work_bytes(ctx, nout, npts, &p));
    st = reserve_stage(ctx, (so + 255) & ~size_t(255));
    if (st != VGPR_OK) return st;
    char* sb = static_cast<char*>(ctx->stage.ptr);
    float* sxyz = reinterpret_cast<float*>(sb + s_xyz);
    int32_t* soff = reinterpret_cast<int32_t*>(sb + s_off);
    hipLaunchKernelGGL(gather_pool_kernel, dim3((unsigned)((nout + 3) / 4)), dim3(256), 0, ctx->stream, *M, uid, upts,
                       nout, sxyz, soff);
    VGPR_HIP(ctx, hipGetLastError());
    FitArgs a{sxyz, npts, ukey, soff, ucnt, nullptr, nullptr, nout, d_out, d_axis, d_status};
    st = fit_predict_impl(ctx, a, &p, 0, sb + s_fit);
    if (st != VGPR_OK) return st;
    hipLaunchKernelGGL(state_kernel, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, ctx->stream, *M, uid,
                       d_status, nout);
    VGPR_HIP(ctx, hipGetLastError());
  }
  if (nu > cap_upd) return fail(ctx, VGPR_E_CAPACITY, "more re-solved voxels than cap_upd");
  return VGPR_OK;
}

vgpr_status vgpr_map_stats(vgpr_map* M, int64_t* h_n_voxels, int64_t* h_n_points, int64_t* h_n_converged) {
  if (!M) return VGPR_E_INVALID;
  vgpr_ctx* ctx = M->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  vgpr_status st = reserve_work(ctx, 4096);
  if (st != VGPR_OK) return st;
  st = reserve_pinned(ctx, 64);
  if (st != VGPR_OK) return st;
  unsigned long long* d = static_cast<unsigned long long*>(ctx->work.ptr);
  unsigned long long* h = static_cast<unsigned long long*>(ctx->pinned);
  VGPR_HIP(ctx, hipMemsetAsync(d, 0, 2 * sizeof(unsigned long long), ctx->stream));
  hipLaunchKernelGGL(stats_kernel, dim3(256), dim3(256), 0, ctx->stream, *M, d);
  VGPR_HIP(ctx, hipGetLastError());
  VGPR_HIP(ctx, hipMemcpyAsync(h, d, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
  VGPR_HIP(ctx, hipMemcpyAsync(h + 2, M->counters, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h_n_voxels) *h_n_voxels = (int64_t)h[2];
  if (h_n_points) *h_n_points = (int64_t)h[0];
  if (h_n_converged) *h_n_converged = (int64_t)h[1];
  return VGPR_OK;
}

vgpr_status vgpr_map_export(vgpr_map* M, void* h_buf, size_t buf_bytes, size_t* h_needed) {
  if (!M || !h_needed) return VGPR_E_INVALID;
  vgpr_ctx* ctx = M->ctx;
  *h_needed = 0;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  unsigned long long nv_u = 0;
  VGPR_HIP(ctx, hipMemcpy(&nv_u, M->counters, sizeof(nv_u), hipMemcpyDeviceToHost));
  const int64_t nv = (int64_t)nv_u < M->max_voxels ? (int64_t)nv_u : M->max_voxels;
  const int cap = M->params.max_pts, m = M->params.grid_side * M->params.grid_side;
  const MapLayout L = map_layout(M->mode, nv, cap, m);
  *h_needed = L.end;
  if (!h_buf) return VGPR_OK;
  if (buf_bytes < L.end) return fail(ctx, VGPR_E_CAPACITY, "export buffer smaller than *h_needed");
  char* b = static_cast<char*>(h_buf);
  MapHeader h{};
  std::memcpy(h.magic, kMapMagic, sizeof(kMapMagic));
  h.version = kMapVersion;
  h.update_mode = M->mode;
  h.n_voxels = nv;
  h.params = M->params;
  std::memcpy(b, &h, sizeof(h));
  if (nv > 0) {
    VGPR_HIP(ctx, hipMemcpy(b + L.keys, M->vkey, 8 * (size_t)nv, hipMemcpyDeviceToHost));
    VGPR_HIP(ctx, hipMemcpy(b + L.stored, M->vstored, 4 * (size_t)nv, hipMemcpyDeviceToHost));
    VGPR_HIP(ctx, hipMemcpy(b + L.total, M->vtotal, 4 * (size_t)nv, hipMemcpyDeviceToHost));
    VGPR_HIP(ctx, hipMemcpy(b + L.conv, M->vconv, (size_t)nv, hipMemcpyDeviceToHost));
    VGPR_HIP(ctx, hipMemcpy(b + L.pool, M->pool, 12 * (size_t)cap * (size_t)nv, hipMemcpyDeviceToHost));
    if (M->mode == 1) {
      VGPR_HIP(ctx, hipMemcpy(b + L.vpred, M->vpred, (size_t)nv, hipMemcpyDeviceToHost));
      VGPR_HIP(ctx, hipMemcpy(b + L.pred, M->pred, 16 * (size_t)m * (size_t)nv, hipMemcpyDeviceToHost));
    }
  }
  return VGPR_OK;
}

vgpr_status vgpr_map_import(vgpr_ctx* ctx, const void* h_buf, size_t buf_bytes, int64_t max_voxels, vgpr_map** out) {
  if (!ctx || !out) return VGPR_E_INVALID;
  *out = nullptr;
  if (!h_buf || buf_bytes < sizeof(MapHeader)) return fail(ctx, VGPR_E_INVALID, "buffer too short for a map header");
  MapHeader h;
  std::memcpy(&h, h_buf, sizeof(h));
  if (std::memcmp(h.magic, kMapMagic, sizeof(kMapMagic)) != 0 || h.version != kMapVersion)
    return fail(ctx, VGPR_E_INVALID, "not a serialised map of this version");
  if (h.n_voxels < 0 || h.n_voxels > max_voxels)
    return fail(ctx, VGPR_E_INVALID, "max_voxels is below the serialised voxel count");
  vgpr_map* M = nullptr;
  vgpr_status st = vgpr_map_create_ex(ctx, &h.params, max_voxels, h.update_mode, &M);
  if (st != VGPR_OK) return st;
  const int64_t nv = h.n_voxels;
  const int cap = M->params.max_pts, m = M->params.grid_side * M->params.grid_side;
  const MapLayout L = map_layout(M->mode, nv, cap, m);
  const char* b = static_cast<const char*>(h_buf);
  auto bad = [&](const char* msg) {
    vgpr_map_destroy(M);
    return fail(ctx, VGPR_E_INVALID, msg);
  };
  if (buf_bytes < L.end) return bad("buffer shorter than the serialised map");
  for (int64_t v = 0; v < nv; ++v) {
    int32_t stored;
    std::memcpy(&stored, b + L.stored + 4 * (size_t)v, 4);
    if (stored < 0 || stored > cap) return bad("a stored point count is outside [0, max_pts]");
  }
  {  // the hash table is rebuilt from the keys: they must be distinct and not the empty-slot sentinel
    std::vector<uint64_t> k((size_t)nv);
    if (nv > 0) std::memcpy(k.data(), b + L.keys, 8 * (size_t)nv);
    std::sort(k.begin(), k.end());
    for (size_t v = 0; v < k.size(); ++v)
      if (k[v] == kKeySentinel || (v > 0 && k[v] == k[v - 1])) return bad("voxel keys are repeated or invalid");
  }
  auto copy_in = [&](void* dst, size_t off, size_t bytes) {
    return hipMemcpy(dst, b + off, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool ok = true;
  if (nv > 0) {
    ok = copy_in(M->vkey, L.keys, 8 * (size_t)nv) && copy_in(M->vstored, L.stored, 4 * (size_t)nv) &&
         copy_in(M->vtotal, L.total, 4 * (size_t)nv) && copy_in(M->vconv, L.conv, (size_t)nv) &&
         copy_in(M->pool, L.pool, 12 * (size_t)cap * (size_t)nv);
    if (ok && M->mode == 1)
      ok = copy_in(M->vpred, L.vpred, (size_t)nv) && copy_in(M->pred, L.pred, 16 * (size_t)m * (size_t)nv);
    if (ok) {
      hipLaunchKernelGGL(rebuild_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, ctx->stream, *M, nv);
      ok = hipGetLastError() == hipSuccess;
    }
  }
  const unsigned long long nv_u = (unsigned long long)nv;
  ok = ok && hipMemcpyAsync(M->counters, &nv_u, sizeof(nv_u), hipMemcpyHostToDevice, ctx->stream) == hipSuccess &&
       hipStreamSynchronize(ctx->stream) == hipSuccess;
  if (!ok) {
    vgpr_map_destroy(M);
    return fail(ctx, VGPR_E_DEVICE, "copying the serialised map to the device failed");
  }
  M->host_voxels = nv;
  *out = M;
  return VGPR_OK;
}

}  // extern "C"
