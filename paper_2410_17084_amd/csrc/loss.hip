// vgpr_structure_loss: the structure similarity loss L_p of Eq. (9) (paper
// Sec. 3.3). For every scan point P_j the value min_k (|P_j - p_k| - S_k) over
// the Gaussians k (S_k the mean of Gaussian k's three scales) and the k that
// attains it (the lowest k among equal values); L_p is their mean over the
// frame's finite points.
//
// Exact search on a uniform grid of cell size h. The candidates' centres
// (compacted: rows of unsolved voxels are NaN) are sorted into cells with the
// voxelizer (Alg. S1's keys, cells in Morton order so that consecutive
// Gaussians stay close in space), each cell's range goes into an
// open-addressing table behind an occupancy filter, and each point visits the
// cells of growing cubes around its own cell (the cube of radius 1, then the
// shells r = 2, 3, sixteen lanes per point sharing out each pass's cells). Every Gaussian
// outside the cube of radius r lies at least lb_r (the distance from P_j to the
// cube's faces) away, so its value is at least lb_r - max_k S_k; once that
// bound exceeds the best value by a rounding margin no unvisited Gaussian can
// win. Points still open after kRingMax rings (far from the map) are resolved
// by an exhaustive pass over chunks of consecutive Gaussians: one wavefront per
// point visits the chunks nearest box first, starting from what the rings
// found, and skips every chunk whose bounding box rules it out against the
// best so far (the minimum of (ordered value bits, index)). Both passes
// take the minimum of the same float values with the same tie rule (lowest
// value, then lowest index), so the result does not depend on h, which only
// sets the speed.
#include <cfloat>
#include <climits>
#include <cmath>

#include "scan.h"
#include "vgpr_internal.h"

namespace vgpr {
namespace {

constexpr int kRingMax = 3;
constexpr int kReduceTile = 1024;
constexpr int kBruteChunk = 1024;  // consecutive Gaussians (cell order) under one bounding box

__device__ __forceinline__ uint32_t float_order(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float float_unorder(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ unsigned long long pack_best(float v, int k) {
  return ((unsigned long long)float_order(v) << 32) | (unsigned long long)(uint32_t)k;
}

// Value of Gaussian g (centre, mean scale in w) for point (x, y, z); every
// pass evaluates it through this one function.
__device__ __forceinline__ float gauss_value(float x, float y, float z, float4 g) {
  const float dx = x - g.x, dy = y - g.y, dz = z - g.z;
  const float v = __fsub_rn(__fsqrt_rn(__fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz))), g.w);
  return __fadd_rn(v, 0.0f);  // -0 -> +0: equal values compare equal in the packed order too
}

__device__ __forceinline__ void take_min(float v, int k, float* best, int* bk) {
  if (v < *best || (v == *best && k < *bk)) {
    *best = v;
    *bk = k;
  }
}

// Mean scale of a Gaussian row pair and whether it is a candidate (finite
// centre and scale); the counting and the compacting kernel both call it.
__device__ __forceinline__ bool row_scale(float4 a, float4 b, int scale_mode, float* s) {
  if (scale_mode == 1)
    *s = __fdiv_rn(__fadd_rn(__fadd_rn(__fsqrt_rn(b.x), __fsqrt_rn(b.y)), __fsqrt_rn(b.z)), 3.0f);
  else
    *s = __fdiv_rn(__fadd_rn(__fadd_rn(b.x, b.y), b.z), 3.0f);
  return isfinite(a.x) && isfinite(a.y) && isfinite(a.z) && isfinite(*s);
}

// Per-workgroup candidate count and largest mean scale (ordered bits).
__global__ void __launch_bounds__(256) prepare_kernel(const float4* __restrict__ rows, int64_t ng, int scale_mode,
                                                      uint32_t* __restrict__ bcnt, uint32_t* __restrict__ bmax) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t m = 0u, c = 0u;
  if (k < ng) {
    float s;
    if (row_scale(rows[2 * k], rows[2 * k + 1], scale_mode, &s)) {
      m = float_order(s);
      c = 1u;
    }
  }
  // per-workgroup slots rather than device-wide atomics (one address per wavefront serialised)
  for (int o = 32; o > 0; o >>= 1) {
    m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    c += (uint32_t)__shfl_xor((int)c, o, 64);
  }
  __shared__ uint32_t wm[4], wc[4];
  if (lane_id() == 0) wm[threadIdx.x >> 6] = m, wc[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    bmax[blockIdx.x] = max(max(wm[0], wm[1]), max(wm[2], wm[3]));
    bcnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
  }
}

// One workgroup: the largest mean scale over the workgroup maxima into smax[0],
// the exclusive scan of the workgroup counts into boff and the candidate count
// into smax[2].
constexpr int kScanThreads = 1024;
__global__ void __launch_bounds__(kScanThreads) scan_kernel(const uint32_t* __restrict__ bmax,
                                                            const uint32_t* __restrict__ bcnt, int64_t nb,
                                                            uint32_t* __restrict__ boff,
                                                            uint32_t* __restrict__ smax) {
  __shared__ uint32_t sm[kScanThreads / 64 + 1];
  uint32_t m = 0u, run = 0u;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t c = b < nb ? bcnt[b] : 0u;
    if (b < nb) m = max(m, bmax[b]);
    uint32_t tot;
    const uint32_t ex = block_exclusive_sum<kScanThreads>(c, sm, &tot);
    if (b < nb) boff[b] = run + ex;
    run += tot;
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
  __shared__ uint32_t wm[kScanThreads / 64];
  if (lane_id() == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kScanThreads / 64; ++w) m = max(m, wm[w]);
    smax[0] = m;
    smax[2] = run;
  }
}

// The candidates' centres and mean scales, compacted in row order, with their
// row indices (the voxelizer then sorts only candidates).
__global__ void __launch_bounds__(256) compact_kernel(const float4* __restrict__ rows, int64_t ng, int scale_mode,
                                                      const uint32_t* __restrict__ boff, float* __restrict__ cen,
                                                      float* __restrict__ sb, int32_t* __restrict__ orig) {
  __shared__ uint32_t sm[256 / 64 + 1];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
  float s = 0.f;
  bool ok = false;
  if (k < ng) {
    a = rows[2 * k];
    ok = row_scale(a, rows[2 * k + 1], scale_mode, &s);
  }
  uint32_t tot;
  const uint32_t pos = boff[blockIdx.x] + block_exclusive_sum<256>(ok ? 1u : 0u, sm, &tot);
  if (ok) {
    cen[3 * (size_t)pos + 0] = a.x;
    cen[3 * (size_t)pos + 1] = a.y;
    cen[3 * (size_t)pos + 2] = a.z;
    sb[pos] = s;
    orig[pos] = (int32_t)k;
  }
}

// Gaussians in cell order as (x, y, z, S) with their row index, and the cell
// table (cell key -> (key, first Gaussian, count) in one 16-byte slot, so that
// a lookup touches one cache line) behind an occupancy filter: one bit per
// hash value, set for every occupied cell, at least 64 bits per cell, so that
// most empty cells of a ring are rejected by one load from a small array.
__global__ void __launch_bounds__(256) gather_kernel(const float* __restrict__ cen, const float* __restrict__ sb,
                                                     const int32_t* __restrict__ orig,
                                                     const int32_t* __restrict__ perm, int64_t nvalid,
                                                     float4* __restrict__ G, int32_t* __restrict__ gi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvalid) return;
  const int k = perm[i];
  G[i] = make_float4(cen[3 * (size_t)k], cen[3 * (size_t)k + 1], cen[3 * (size_t)k + 2], sb[k]);
  gi[i] = orig[k];
}

struct alignas(16) Slot {
  uint64_t key;  // cell key, or the sentinel for an empty slot
  int32_t off;   // first Gaussian of the cell (cell order)
  int32_t cnt;   // Gaussians in the cell
};

__global__ void __launch_bounds__(256) table_kernel(const uint64_t* __restrict__ ckeys, const int32_t* __restrict__ coff,
                                                    const int32_t* __restrict__ ccnt, int64_t nc,
                                                    Slot* __restrict__ table, int64_t nslots,
                                                    uint32_t* __restrict__ filter, int fshift) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const uint64_t key = ckeys[c];
  const uint64_t hk = mix64(key);
  const uint64_t fi = hk >> fshift;  // top bits: independent of the slot's low bits
  atomicOr(&filter[fi >> 5], 1u << (fi & 31));
  int64_t s = (int64_t)(hk & (uint64_t)(nslots - 1));
  for (int64_t probe = 0; probe < nslots; ++probe) {
    const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(&table[s].key),
                                              (unsigned long long)kKeySentinel, (unsigned long long)key);
    if (prev == kKeySentinel) {  // cell keys are unique: no two threads insert the same key
      table[s].off = coff[c];
      table[s].cnt = ccnt[c];
      return;
    }
    s = (s + 1) & (nslots - 1);
  }
}

// The Gaussians of cell `key` (hash hk), or false if the cell holds none.
__device__ __forceinline__ bool lookup(const Slot* __restrict__ table, int64_t nslots, uint64_t key, uint64_t hk,
                                       int* off, int* cnt) {
  int64_t s = (int64_t)(hk & (uint64_t)(nslots - 1));
  for (int64_t probe = 0; probe < nslots; ++probe) {
    const ulonglong2 q = *reinterpret_cast<const ulonglong2*>(&table[s]);
    if (q.x == key) {
      *off = (int)(uint32_t)q.y;
      *cnt = (int)(uint32_t)(q.y >> 32);
      return true;
    }
    if (q.x == kKeySentinel) return false;
    s = (s + 1) & (nslots - 1);
  }
  return false;
}

struct Grid {
  const float4* G;
  const int32_t* gi;
  const Slot* table;
  int64_t nslots;
  const uint32_t* filter;
  int fshift;
  double inv_h, h;
  const uint32_t* smax;
};

// Ring search, kGroup lanes per point: the lanes of a group share out the cells
// of each ring, then combine their minima with a butterfly of shuffles (the
// (value, index) order is total, so the result does not depend on who visited
// what). A group stops once its bound clears; the wavefront runs until every
// group has stopped, so every lane takes part in the shuffles.
constexpr int kGroup = 16;
static_assert(((2 * kRingMax + 1) * (2 * kRingMax + 1) * (2 * kRingMax + 1) + kGroup - 1) / kGroup <= 64,
              "a lane's cells of one ring must fit the 64-bit hit mask");

constexpr int kQueryThreads = 64;  // four points a workgroup: measured faster than 256-thread workgroups

__global__ void __launch_bounds__(kQueryThreads) query_kernel(const float* __restrict__ pts, int64_t n, Grid g, int has_cand,
                                                    float* __restrict__ val, int32_t* __restrict__ arg,
                                                    int32_t* __restrict__ fb, uint32_t* __restrict__ fb_n,
                                                    unsigned long long* __restrict__ bbest) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroup;
  const int gl = threadIdx.x & (kGroup - 1);
  float x = 0.f, y = 0.f, z = 0.f;
  bool live = false;
  if (i < n) {
    x = pts[3 * (size_t)i];
    y = pts[3 * (size_t)i + 1];
    z = pts[3 * (size_t)i + 2];
    const bool fin = isfinite(x) && isfinite(y) && isfinite(z);
    if (gl == 0 && !fin) {
      val[i] = __int_as_float(0x7fc00000);
      arg[i] = -1;
    } else if (gl == 0 && !has_cand) {
      val[i] = INFINITY;
      arg[i] = -1;
    }
    live = fin && has_cand;
  }
  const double smax = has_cand ? (double)float_unorder(*g.smax) : 0.0;
  const double kx = floor(__dmul_rn((double)x, g.inv_h));
  const double ky = floor(__dmul_rn((double)y, g.inv_h));
  const double kz = floor(__dmul_rn((double)z, g.inv_h));
  const double lim = (double)kKeyAxisLimit;
  float best = INFINITY;
  int bk = INT_MAX;
  bool done = !live;
  // the first pass takes the whole cube of radius 1 (rings 0 and 1 together: a point's own
  // cell alone almost never settles it), later passes one shell each
  for (int r = 1; r <= kRingMax; ++r) {
    if (!done) {
      // the shell of radius r: cells of the (2r+1)^3 cube with Chebyshev distance r (all 27
      // cells for r = 1). The
      // lane's cells t = gl + kGroup i go in two passes: first every filter load (independent,
      // so they overlap) into a mask of possibly occupied cells, then the table and the
      // Gaussians of those cells only.
      const int side = 2 * r + 1, nt = side * side * side;
      auto cell_key = [&](int t, bool* ok) {
        const int dz = t % side - r, dy = (t / side) % side - r, dx = t / (side * side) - r;
        const double cx = kx + dx, cy = ky + dy, cz = kz + dz;
        const int cheb = max(max(abs(dx), abs(dy)), abs(dz));
        *ok = (cheb == r || r == 1) && fabs(cx) <= lim && fabs(cy) <= lim && fabs(cz) <= lim;
        return *ok ? ((uint64_t)((int64_t)cx + kKeyBias) << (2 * kKeyFieldBits)) |
                         ((uint64_t)((int64_t)cy + kKeyBias) << kKeyFieldBits) | (uint64_t)((int64_t)cz + kKeyBias)
                   : 0ull;
      };
      uint64_t hits = 0;  // bit i: cell gl + kGroup i passed the filter (at most 43 cells a lane for r <= 3)
#pragma unroll 4
      for (int i = 0; gl + kGroup * i < nt; ++i) {
        bool ok;
        const uint64_t key = cell_key(gl + kGroup * i, &ok);
        const uint64_t fi = mix64(key) >> g.fshift;  // in range for any key
        const uint32_t word = g.filter[fi >> 5];
        if (ok && ((word >> (fi & 31)) & 1u)) hits |= 1ull << i;
      }
      while (hits) {
        const int i = __builtin_ctzll(hits);
        hits &= hits - 1;
        bool ok;
        const uint64_t key = cell_key(gl + kGroup * i, &ok);
        int off, cnt;
        if (!lookup(g.table, g.nslots, key, mix64(key), &off, &cnt)) continue;
        for (int j = off; j < off + cnt; ++j) take_min(gauss_value(x, y, z, g.G[j]), g.gi[j], &best, &bk);
      }
    }
#pragma unroll
    for (int o = 1; o < kGroup; o <<= 1) {
      const float ov = __shfl_xor(best, o, 64);
      const int ok = __shfl_xor(bk, o, 64);
      take_min(ov, ok, &best, &bk);
    }
    if (!done) {
      // distance from the point to the faces of the visited cube of cells
      const double lo = (double)r, hi = (double)(r + 1);
      double lb = (double)x - (kx - lo) * g.h;
      lb = fmin(lb, (kx + hi) * g.h - (double)x);
      lb = fmin(lb, (double)y - (ky - lo) * g.h);
      lb = fmin(lb, (ky + hi) * g.h - (double)y);
      lb = fmin(lb, (double)z - (kz - lo) * g.h);
      lb = fmin(lb, (kz + hi) * g.h - (double)z);
      // margin: float rounding of the values compared (a few ulps of the distances and scales involved)
      const double margin = 1e-5 * (fabs(lb) + fabs(smax) + fabs((double)best)) + 1e-7 * g.h;
      if (bk != INT_MAX && lb - smax > (double)best + margin) {
        done = true;
        if (gl == 0) {
          val[i] = best;
          arg[i] = bk;
        }
      }
    }
    if (__ballot(!done) == 0ull) break;
  }
  if (!done && gl == 0) {  // still open after kRingMax rings: the brute-force pass resolves it,
    // starting from the best value the rings found
    const uint32_t slot = atomicAdd(fb_n, 1u);
    fb[slot] = (int32_t)i;
    bbest[slot] = bk == INT_MAX ? ~0ull : pack_best(best, bk);
  }
}

// Bounding box and largest mean scale of each brute-force chunk (the Gaussians
// are in Morton cell order, so a chunk covers a compact region):
// (min x, y, z, max S), (max x, y, z, 0).
__global__ void __launch_bounds__(256) chunk_box_kernel(const float4* __restrict__ G, int64_t nvalid,
                                                        float4* __restrict__ box) {
  const int64_t g0 = (int64_t)blockIdx.x * kBruteChunk;
  const int cnt = (int)min((int64_t)kBruteChunk, nvalid - g0);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, sm = -INFINITY;
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const float4 q = G[g0 + t];
    lo[0] = fminf(lo[0], q.x);
    lo[1] = fminf(lo[1], q.y);
    lo[2] = fminf(lo[2], q.z);
    hi[0] = fmaxf(hi[0], q.x);
    hi[1] = fmaxf(hi[1], q.y);
    hi[2] = fmaxf(hi[2], q.z);
    sm = fmaxf(sm, q.w);
  }
  for (int o = 32; o > 0; o >>= 1) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
    }
    sm = fmaxf(sm, __shfl_xor(sm, o, 64));
  }
  __shared__ float red[4][7];
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[w][0] = lo[0], red[w][1] = lo[1], red[w][2] = lo[2];
    red[w][3] = hi[0], red[w][4] = hi[1], red[w][5] = hi[2], red[w][6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      for (int a = 0; a < 3; ++a) {
        red[0][a] = fminf(red[0][a], red[k][a]);
        red[0][3 + a] = fmaxf(red[0][3 + a], red[k][3 + a]);
      }
      red[0][6] = fmaxf(red[0][6], red[k][6]);
    }
    box[2 * blockIdx.x] = make_float4(red[0][0], red[0][1], red[0][2], red[0][6]);
    box[2 * blockIdx.x + 1] = make_float4(red[0][3], red[0][4], red[0][5], 0.0f);
  }
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, 64);
    const unsigned long long w = ((unsigned long long)hi << 32) | lo;
    v = w < v ? w : v;
  }
  return v;
}

// Nearest-first brute force for the points the rings left open, one wavefront
// per point, its lanes sharing out first the chunk boxes and then one chunk's
// Gaussians. Each round takes, among the chunks that the point cannot rule out
// (box distance minus the chunk's largest mean scale above its best so far by
// more than the rounding margin), the one with the nearest box that no earlier
// round took (ordered by that bound, then by chunk number), evaluates all of
// its Gaussians and tightens the best, kept as the minimum of (ordered value
// bits, index) over the rings' seed and every chunk taken. Rounds end when
// every chunk has been taken or ruled out. The best only falls, so a chunk
// ruled out once stays ruled out, and one is ruled out only when none of its
// values can reach the best: the result is that of evaluating every Gaussian.
// The nearest chunks usually hold the answer, so a point takes a few rounds.
__global__ void __launch_bounds__(256) nearest_kernel(const float* __restrict__ pts, const int32_t* __restrict__ fb,
                                                      uint32_t n_open, const float4* __restrict__ G,
                                                      const int32_t* __restrict__ gi, int64_t nvalid,
                                                      const float4* __restrict__ box, int nchunk,
                                                      const unsigned long long* __restrict__ seed,
                                                      float* __restrict__ val, int32_t* __restrict__ arg) {
  const uint32_t o = (uint32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (o >= n_open) return;  // whole wavefronts: o is uniform in a wavefront
  const int lane = lane_id();
  const int i = fb[o];
  const float x = pts[3 * (size_t)i], y = pts[3 * (size_t)i + 1], z = pts[3 * (size_t)i + 2];
  unsigned long long cur = seed[o];
  unsigned long long next = 0;  // smallest (bound, chunk) key a round may still take
  for (;;) {
    // box bounds in float: their rounding (a few ulps of the distance) is far inside the margin,
    // which exceeds 1e-5 (|lb| + |S|) >= 1e-5 x the distance
    const float cv = cur == ~0ull ? INFINITY : float_unorder((uint32_t)(cur >> 32));
    unsigned long long pick = ~0ull;
    for (int c = lane; c < nchunk; c += 64) {
      const float4 lo = box[2 * c], hi = box[2 * c + 1];
      const float ex = fmaxf(fmaxf(lo.x - x, x - hi.x), 0.0f);
      const float ey = fmaxf(fmaxf(lo.y - y, y - hi.y), 0.0f);
      const float ez = fmaxf(fmaxf(lo.z - z, z - hi.z), 0.0f);
      const float lb = __fsqrt_rn(ex * ex + ey * ey + ez * ez) - lo.w;
      if (lb > cv + 1e-5f * (fabsf(lb) + fabsf(cv) + fabsf(lo.w)) + 1e-7f) continue;
      const unsigned long long key = ((unsigned long long)float_order(lb) << 32) | (uint32_t)c;
      if (key >= next && key < pick) pick = key;
    }
    pick = wave_min_u64(pick);
    if (pick == ~0ull) break;
    next = pick + 1;
    const int64_t g0 = (int64_t)(uint32_t)pick * kBruteChunk;
    const int cnt = (int)min((int64_t)kBruteChunk, nvalid - g0);
    float b = INFINITY;
    int bk = INT_MAX;
#pragma unroll 4
    for (int t = lane; t < cnt; t += 64) take_min(gauss_value(x, y, z, G[g0 + t]), gi[g0 + t], &b, &bk);
    if (bk != INT_MAX) {
      const unsigned long long pb = pack_best(b, bk);
      cur = pb < cur ? pb : cur;
    }
    cur = wave_min_u64(cur);
  }
  if (lane == 0) {
    val[i] = cur == ~0ull ? INFINITY : float_unorder((uint32_t)(cur >> 32));
    arg[i] = cur == ~0ull ? -1 : (int32_t)(uint32_t)(cur & 0xffffffffull);
  }
}

// Deterministic sum of the finite points' values: fixed per-tile order, then
// the tiles in order.
__global__ void __launch_bounds__(256) sum_tiles(const float* __restrict__ val, const float* __restrict__ pts, int64_t n, double* __restrict__ tsum,
                                                 uint32_t* __restrict__ tcnt) {
  const int64_t base = (int64_t)blockIdx.x * kReduceTile + threadIdx.x * 4;
  double s = 0.0;
  uint32_t c = 0;
  for (int e = 0; e < 4; ++e) {
    const int64_t i = base + e;
    if (i < n) {
      const float x = pts[3 * (size_t)i], y = pts[3 * (size_t)i + 1], z = pts[3 * (size_t)i + 2];
      if (isfinite(x) && isfinite(y) && isfinite(z)) {
        s += (double)val[i];
        c += 1;
      }
    }
  }
  __shared__ double ss[256];
  __shared__ uint32_t sc[256];
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sc[threadIdx.x] += sc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tsum[blockIdx.x] = ss[0];
    tcnt[blockIdx.x] = sc[0];
  }
}

__global__ void __launch_bounds__(256) sum_final(const double* __restrict__ tsum, const uint32_t* __restrict__ tcnt,
                                                 int64_t nt, double* __restrict__ out) {
  __shared__ double ss[256];
  __shared__ unsigned long long sc[256];
  double s = 0.0;
  unsigned long long c = 0;
  for (int64_t t = threadIdx.x; t < nt; t += 256) {
    s += tsum[t];
    c += tcnt[t];
  }
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sc[threadIdx.x] += sc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ss[0];
    out[1] = (double)sc[0];
  }
}

}  // namespace
}  // namespace vgpr

using namespace vgpr;

extern "C" vgpr_status vgpr_structure_loss(vgpr_ctx* ctx, const float* d_pts, int64_t n_pts, const float* d_gauss,
                                           int64_t n_gauss, float cell_size, int scale_mode, float* d_value,
                                           int32_t* d_arg, double* h_loss, int64_t* h_n_valid) {
  if (!ctx || !h_loss) return VGPR_E_INVALID;
  *h_loss = NAN;
  if (h_n_valid) *h_n_valid = 0;
  if (n_pts < 0 || n_pts >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_INVALID, "n_pts out of range");
  if (n_gauss < 0 || n_gauss >= (int64_t(1) << 30)) return fail(ctx, VGPR_E_INVALID, "n_gauss out of range");
  if (!(cell_size > 0.0f) || !std::isfinite(cell_size)) return fail(ctx, VGPR_E_INVALID, "cell_size must be > 0");
  if (scale_mode != 0 && scale_mode != 1) return fail(ctx, VGPR_E_INVALID, "scale_mode must be 0 or 1");
  if (n_pts > 0 && !d_pts) return fail(ctx, VGPR_E_INVALID, "d_pts is NULL");
  if (n_gauss > 0 && !d_gauss) return fail(ctx, VGPR_E_INVALID, "d_gauss is NULL");
  if (n_gauss > 0 && (reinterpret_cast<uintptr_t>(d_gauss) & 15))
    return fail(ctx, VGPR_E_INVALID, "d_gauss must be 16-byte aligned");
  if (n_pts == 0) return VGPR_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  const int64_t n = n_pts, ng = n_gauss;
  int64_t ns = 2;
  while (ns < 2 * ng) ns <<= 1;
  const int64_t nt = (n + kReduceTile - 1) / kReduceTile;
  size_t head = 0;
  auto sub = [&](size_t bytes) {
    head = (head + 255) & ~size_t(255);
    size_t r = head;
    head += bytes;
    return r;
  };
  const size_t o_cen = sub(12 * (size_t)ng + 16), o_sb = sub(4 * (size_t)ng + 16), o_ck = sub(8 * (size_t)ng + 16),
               o_co = sub(4 * (size_t)ng + 16), o_cc = sub(4 * (size_t)ng + 16), o_pm = sub(4 * (size_t)ng + 16),
               o_G = sub(16 * (size_t)ng + 16), o_gi = sub(4 * (size_t)ng + 16), o_or = sub(4 * (size_t)ng + 16),
               o_tb = sub(sizeof(Slot) * (size_t)ns), o_fl = sub(16 * (size_t)ng + 64), o_fb = sub(4 * (size_t)n), o_bb = sub(8 * (size_t)n),
               o_box = sub(32 * (size_t)((ng + kBruteChunk - 1) / kBruteChunk) + 32),
               o_bmax = sub(4 * (size_t)((ng + 255) / 256) + 16), o_bc = sub(4 * (size_t)((ng + 255) / 256) + 16),
               o_bo = sub(4 * (size_t)((ng + 255) / 256) + 16),
               o_val = sub(d_value ? 0 : 4 * (size_t)n),
               o_arg = sub(d_arg ? 0 : 4 * (size_t)n), o_ts = sub(8 * (size_t)nt), o_tn = sub(4 * (size_t)nt),
               o_misc = sub(64);
  head = (head + 255) & ~size_t(255);
  vgpr_status st = reserve_work(ctx, head + 24 * (size_t)ng + 4096 * 16 + (1 << 20));
  if (st != VGPR_OK) return st;
  st = reserve_pinned(ctx, 64);
  if (st != VGPR_OK) return st;
  char* w = static_cast<char*>(ctx->work.ptr);
  float* cen = reinterpret_cast<float*>(w + o_cen);
  float* sb = reinterpret_cast<float*>(w + o_sb);
  uint64_t* ckeys = reinterpret_cast<uint64_t*>(w + o_ck);
  int32_t* coff = reinterpret_cast<int32_t*>(w + o_co);
  int32_t* ccnt = reinterpret_cast<int32_t*>(w + o_cc);
  int32_t* perm = reinterpret_cast<int32_t*>(w + o_pm);
  float4* G = reinterpret_cast<float4*>(w + o_G);
  int32_t* gi = reinterpret_cast<int32_t*>(w + o_gi);
  int32_t* orig = reinterpret_cast<int32_t*>(w + o_or);
  Slot* table = reinterpret_cast<Slot*>(w + o_tb);
  uint32_t* filter = reinterpret_cast<uint32_t*>(w + o_fl);
  int32_t* fb = reinterpret_cast<int32_t*>(w + o_fb);
  unsigned long long* bbest = reinterpret_cast<unsigned long long*>(w + o_bb);
  float4* cbox = reinterpret_cast<float4*>(w + o_box);
  uint32_t* bmax = reinterpret_cast<uint32_t*>(w + o_bmax);
  uint32_t* bcnt = reinterpret_cast<uint32_t*>(w + o_bc);
  uint32_t* boff = reinterpret_cast<uint32_t*>(w + o_bo);
  float* val = d_value ? d_value : reinterpret_cast<float*>(w + o_val);
  int32_t* arg = d_arg ? d_arg : reinterpret_cast<int32_t*>(w + o_arg);
  double* tsum = reinterpret_cast<double*>(w + o_ts);
  uint32_t* tcnt = reinterpret_cast<uint32_t*>(w + o_tn);
  // [0] largest mean scale (ordered bits), [1] open points, [2] candidates
  uint32_t* misc = reinterpret_cast<uint32_t*>(w + o_misc);
  double* dsum = reinterpret_cast<double*>(w + o_misc + 16);

  VGPR_HIP(ctx, hipMemsetAsync(misc, 0, 64, ctx->stream));
  int64_t nc = 0, n_bad = 0, n_cand = 0;
  if (ng > 0) {
    // candidates only (rows of unsolved voxels are NaN) go to the voxelizer
    const int64_t nb = (ng + 255) / 256;
    const float4* rows = reinterpret_cast<const float4*>(d_gauss);
    hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)nb), dim3(256), 0, ctx->stream, rows, ng, scale_mode, bcnt,
                       bmax);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, ctx->stream, bmax, bcnt, nb, boff, misc);
    hipLaunchKernelGGL(compact_kernel, dim3((unsigned)nb), dim3(256), 0, ctx->stream, rows, ng, scale_mode, boff,
                       cen, sb, orig);
    VGPR_HIP(ctx, hipGetLastError());
    void* hp0 = ctx->pinned;
    VGPR_HIP(ctx, hipMemcpyAsync(hp0, misc + 2, 4, hipMemcpyDeviceToHost, ctx->stream));
    VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    n_cand = static_cast<const uint32_t*>(hp0)[0];
    if (n_cand > 0) {
      st = voxelize_impl(ctx, cen, n_cand, nullptr, 1, cell_size, ckeys, coff, ccnt, perm, n_cand, &nc, nullptr,
                         &n_bad, head, true);
      if (st != VGPR_OK) return st;
      if (ctx->work.ptr != static_cast<void*>(w)) return fail(ctx, VGPR_E_DEVICE, "workspace moved during the loss");
    }
  }
  const int64_t nvalid = n_cand - n_bad;
  const bool has_cand = nvalid > 0;
  // table of at least twice the cell count (at most ns, since nc <= ng); filter
  // of at least 64 bits per cell (at most 16 ng bytes)
  int64_t nsl = 2;
  while (nsl < 2 * nc) nsl <<= 1;
  int lf = 6;
  while ((int64_t(1) << lf) < 64 * nc) ++lf;
  if (has_cand) {
    VGPR_HIP(ctx, hipMemsetAsync(table, 0xFF, sizeof(Slot) * (size_t)nsl, ctx->stream));
    VGPR_HIP(ctx, hipMemsetAsync(filter, 0, (size_t(1) << lf) / 8, ctx->stream));
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((nvalid + 255) / 256)), dim3(256), 0, ctx->stream, cen, sb,
                       orig, perm, nvalid, G, gi);
    hipLaunchKernelGGL(table_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, ctx->stream, ckeys, coff, ccnt,
                       nc, table, nsl, filter, 64 - lf);
    VGPR_HIP(ctx, hipGetLastError());
  }
  const double inv_h = 1.0 / (double)cell_size;
  Grid grid{G, gi, table, nsl, filter, 64 - lf, inv_h, (double)cell_size, misc};
  {
    ProfScope ps(ctx, "structure_loss");
    hipLaunchKernelGGL(query_kernel, dim3((unsigned)((n * kGroup + kQueryThreads - 1) / kQueryThreads)), dim3(kQueryThreads), 0, ctx->stream, d_pts, n, grid,
                       has_cand ? 1 : 0, val, arg, fb, misc + 1, bbest);
    VGPR_HIP(ctx, hipGetLastError());
  }
  // the voxelizer may have grown the pinned staging area: take its address only now
  void* hp = ctx->pinned;
  VGPR_HIP(ctx, hipMemcpyAsync(hp, misc, 8, hipMemcpyDeviceToHost, ctx->stream));
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const uint32_t n_open = static_cast<uint32_t*>(hp)[1];
  if (n_open > 0) {
    ProfScope ps(ctx, "structure_loss_brute");
    const unsigned gx = (unsigned)((nvalid + kBruteChunk - 1) / kBruteChunk);
    hipLaunchKernelGGL(chunk_box_kernel, dim3(gx), dim3(256), 0, ctx->stream, G, nvalid, cbox);
    hipLaunchKernelGGL(nearest_kernel, dim3((unsigned)(((int64_t)n_open * 64 + 255) / 256)), dim3(256), 0,
                       ctx->stream, d_pts, fb, n_open, G, gi, nvalid, cbox, (int)gx, bbest, val, arg);
    VGPR_HIP(ctx, hipGetLastError());
  }
  hipLaunchKernelGGL(sum_tiles, dim3((unsigned)nt), dim3(256), 0, ctx->stream, val, d_pts, n, tsum, tcnt);
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(256), 0, ctx->stream, tsum, tcnt, nt, dsum);
  VGPR_HIP(ctx, hipGetLastError());
  VGPR_HIP(ctx, hipMemcpyAsync(hp, dsum, 16, hipMemcpyDeviceToHost, ctx->stream));
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double res[2];
  std::memcpy(res, hp, 16);
  const int64_t n_valid = (int64_t)res[1];
  if (h_n_valid) *h_n_valid = n_valid;
  *h_loss = n_valid > 0 ? res[0] / (double)n_valid : NAN;
  return VGPR_OK;
}
