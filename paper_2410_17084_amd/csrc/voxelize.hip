// vgpr_voxelize: the STORE step of Alg. S1 (paper supplementary) on the GPU.
//
// 1. key kernel: one thread per point computes the packed 64-bit voxel key
//    (one IEEE double multiply by 1/s and a floor per axis) and seeds the
//    index array; non-finite points get the all-ones sentinel key.
// 2. stable LSD radix sort of (sort key, index), 8-bit digits, three kernels
//    per pass (tile histograms, per-digit scan across tiles, ranked scatter).
//    Ranks inside a tile come from 64-lane ballots, so equal digits keep
//    their input order and the sort is stable. The sort key is a compacted
//    form of the voxel key with the same order: each axis index minus the
//    batch minimum, packed into just the bits the batch's ranges need, then
//    an invalid-point bit, then the frame index (a batch is sorted by
//    (frame, key)). A spinning scan needs ~24 key bits, so three or four
//    passes instead of eight. If the packed form does not fit 64 bits the
//    frame index gets its own extra passes, read from the point's index.
// 3. segmentation: voxel heads (key change or frame start), a scan over the
//    heads, and scatter of keys / starts / counts; per-frame voxel ranges.
#include <algorithm>
#include <climits>

#include "scan.h"
#include "vgpr_internal.h"

namespace vgpr {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;                       // per lane (4 x 256: several tiles per CU at 1M points)
constexpr int kSortTile = kSortThreads * kSortItems;  // 1024 elements per block
constexpr int kSortWaves = kSortThreads / 64;

// Result words read back to the host after a voxelize call.
enum { R_NVOX = 0, R_INVALID = 1, R_RANGE = 2, R_NVALID = 3, R_MIN = 4, R_MAX = 7, R_FRAMES = 10 };

// Compacted sort key: fields (k - kmin) in bx / by / bz bits (x highest), the
// invalid flag at bit B = bx + by + bz, the frame index above it if embedded.
// In Morton form the B field bits are interleaved instead (see interleave3), so
// that runs of consecutive voxels cover compact 3-D regions.
struct KeyForm {
  int bx, by, bz, B;
  int embed;           // frame index in bits [B + 1, ...)
  int key_passes;      // radix passes over the packed key
  int morton;          // field bits interleaved (1) or concatenated (0)
  int64_t mn[3];       // per-axis minimum voxel index
};

// Morton interleave of fields of unequal widths: bit l of z, then of y, then
// of x, for l = 0, 1, ...; an axis drops out once l reaches its width, so the
// code takes exactly B bits and is a bijection of the three fields.
__device__ __forceinline__ uint64_t interleave3(uint64_t ux, uint64_t uy, uint64_t uz, const KeyForm& kf) {
  uint64_t tk = 0;
  int o = 0;
  const int top = max(kf.bx, max(kf.by, kf.bz));
  for (int l = 0; l < top; ++l) {
    if (l < kf.bz) tk |= ((uz >> l) & 1ull) << o++;
    if (l < kf.by) tk |= ((uy >> l) & 1ull) << o++;
    if (l < kf.bx) tk |= ((ux >> l) & 1ull) << o++;
  }
  return tk;
}

__device__ __forceinline__ void deinterleave3(uint64_t tk, const KeyForm& kf, uint64_t* ux, uint64_t* uy,
                                              uint64_t* uz) {
  uint64_t x = 0, y = 0, z = 0;
  int o = 0;
  const int top = max(kf.bx, max(kf.by, kf.bz));
  for (int l = 0; l < top; ++l) {
    if (l < kf.bz) z |= ((tk >> o++) & 1ull) << l;
    if (l < kf.by) y |= ((tk >> o++) & 1ull) << l;
    if (l < kf.bx) x |= ((tk >> o++) & 1ull) << l;
  }
  *ux = x;
  *uy = y;
  *uz = z;
}

__device__ __forceinline__ int frame_of(uint32_t idx, const int64_t* fo, int nf) {
  // largest f with fo[f] <= idx, for nf frames (fo has nf + 1 entries)
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (fo[mid] <= (int64_t)idx) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t digit_of(uint64_t key, uint32_t val, int pass, int key_passes, const int64_t* fo,
                                             int nf) {
  if (pass < key_passes) return (uint32_t)(key >> (8 * pass)) & 0xFFu;
  return ((uint32_t)frame_of(val, fo, nf) >> (8 * (pass - key_passes))) & 0xFFu;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
  return v;
}

// Voxel key of every point (packed, biased) and per-block min / max voxel index per axis.
__global__ void __launch_bounds__(256) key_kernel(const float* __restrict__ xyz, int n, double inv_s,
                                                  uint64_t* __restrict__ keys, int* __restrict__ part,
                                                  unsigned long long* __restrict__ res) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool invalid = false;
  bool range_err = false;
  int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
  if (i < n) {
    const float x = xyz[3 * (size_t)i + 0];
    const float y = xyz[3 * (size_t)i + 1];
    const float z = xyz[3 * (size_t)i + 2];
    uint64_t key = kKeySentinel;
    if (isfinite(x) && isfinite(y) && isfinite(z)) {
      const double kx = floor(__dmul_rn((double)x, inv_s));
      const double ky = floor(__dmul_rn((double)y, inv_s));
      const double kz = floor(__dmul_rn((double)z, inv_s));
      const double lim = (double)kKeyAxisLimit;
      if (fabs(kx) > lim || fabs(ky) > lim || fabs(kz) > lim) {
        range_err = true;
      } else {
        const int ix = (int)kx, iy = (int)ky, iz = (int)kz;
        mn[0] = mx[0] = ix;
        mn[1] = mx[1] = iy;
        mn[2] = mx[2] = iz;
        const uint64_t bx = (uint64_t)((int64_t)ix + kKeyBias);
        const uint64_t by = (uint64_t)((int64_t)iy + kKeyBias);
        const uint64_t bz = (uint64_t)((int64_t)iz + kKeyBias);
        key = (bx << (2 * kKeyFieldBits)) | (by << kKeyFieldBits) | bz;
      }
    } else {
      invalid = true;
    }
    keys[i] = key;
  }
  const unsigned long long inv_mask = __ballot(invalid);
  const unsigned long long rng_mask = __ballot(range_err);
  if (lane_id() == 0) {
    if (inv_mask) atomicAdd(&res[R_INVALID], (unsigned long long)__popcll(inv_mask));
    if (rng_mask) atomicOr(&res[R_RANGE], 1ull);
  }
  __shared__ int s[6][4];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int lo = wave_min_i(mn[a]), hi = wave_max_i(mx[a]);
    if (lane_id() == 0) {
      s[a][w] = lo;
      s[3 + a][w] = hi;
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    int r = s[a][0];
    for (int k = 1; k < 4; ++k) r = a < 3 ? min(r, s[a][k]) : max(r, s[a][k]);
    part[(size_t)blockIdx.x * 6 + a] = r;
  }
}

// Batch min / max per axis from the per-block partials.
__global__ void __launch_bounds__(1024) minmax_kernel(const int* __restrict__ part, int nparts,
                                                      unsigned long long* __restrict__ res) {
  __shared__ int s[6][16];
  int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
  for (int b = threadIdx.x; b < nparts; b += 1024) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mn[a] = min(mn[a], part[(size_t)b * 6 + a]);
      mx[a] = max(mx[a], part[(size_t)b * 6 + 3 + a]);
    }
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int lo = wave_min_i(mn[a]), hi = wave_max_i(mx[a]);
    if (lane_id() == 0) {
      s[a][w] = lo;
      s[3 + a][w] = hi;
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    int r = s[a][0];
    for (int k = 1; k < 16; ++k) r = a < 3 ? min(r, s[a][k]) : max(r, s[a][k]);
    res[(a < 3 ? R_MIN : R_MAX - 3) + a] = (unsigned long long)(long long)r;
  }
}

// Packed key -> compacted sort key (in place); seeds the index array the first pass reads.
__global__ void __launch_bounds__(256) compose_kernel(uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, int n,
                                                      KeyForm kf, const int64_t* __restrict__ fo, int nf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  vals[i] = (uint32_t)i;
  const uint64_t key = keys[i];
  uint64_t tk;
  if (key == kKeySentinel) {
    tk = 1ull << kf.B;
  } else {
    const int64_t mask = (int64_t(1) << kKeyFieldBits) - 1;
    const uint64_t ux = (uint64_t)((int64_t)((key >> (2 * kKeyFieldBits)) & mask) - kKeyBias - kf.mn[0]);
    const uint64_t uy = (uint64_t)((int64_t)((key >> kKeyFieldBits) & mask) - kKeyBias - kf.mn[1]);
    const uint64_t uz = (uint64_t)((int64_t)(key & mask) - kKeyBias - kf.mn[2]);
    tk = kf.morton ? interleave3(ux, uy, uz, kf) : (ux << (kf.by + kf.bz)) | (uy << kf.bz) | uz;
  }
  if (kf.embed && nf > 1) tk |= (uint64_t)frame_of((uint32_t)i, fo, nf) << (kf.B + 1);
  keys[i] = tk;
}

// Compacted sort key -> packed voxel key.
__device__ __forceinline__ uint64_t unpack_sort_key(uint64_t tk, const KeyForm& kf) {
  if (kf.morton) {
    uint64_t ux, uy, uz;
    deinterleave3(tk, kf, &ux, &uy, &uz);
    return ((uint64_t)((int64_t)ux + kf.mn[0] + kKeyBias) << (2 * kKeyFieldBits)) |
           ((uint64_t)((int64_t)uy + kf.mn[1] + kKeyBias) << kKeyFieldBits) | (uint64_t)((int64_t)uz + kf.mn[2] + kKeyBias);
  }
  const uint64_t mz = (kf.bz ? (1ull << kf.bz) : 1ull) - 1ull, my = (kf.by ? (1ull << kf.by) : 1ull) - 1ull,
                 mx = (kf.bx ? (1ull << kf.bx) : 1ull) - 1ull;
  const int64_t kz = (int64_t)(tk & mz) + kf.mn[2];
  const int64_t ky = (int64_t)((tk >> kf.bz) & my) + kf.mn[1];
  const int64_t kx = (int64_t)((tk >> (kf.by + kf.bz)) & mx) + kf.mn[0];
  return ((uint64_t)(kx + kKeyBias) << (2 * kKeyFieldBits)) | ((uint64_t)(ky + kKeyBias) << kKeyFieldBits) |
         (uint64_t)(kz + kKeyBias);
}

// Per-tile digit histogram, stored digit-major: hist[d * nblocks + b].
__global__ void __launch_bounds__(kSortThreads) radix_upsweep(const uint64_t* __restrict__ keys,
                                                              const uint32_t* __restrict__ vals, int n, int pass,
                                                              int key_passes, const int64_t* __restrict__ fo, int nf,
                                                              uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    const int i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(keys[i], vals[i], pass, key_passes, fo, nf)], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Block d: exclusive scan of digit d's row across tiles, in place; row total out.
__global__ void __launch_bounds__(1024) radix_rowscan(uint32_t* __restrict__ hist, int nblocks,
                                                      uint32_t* __restrict__ row_total) {
  __shared__ uint32_t smem[17];
  uint32_t* row = hist + (size_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (int s = 0; s < nblocks; s += 1024) {
    const int i = s + threadIdx.x;
    const uint32_t v = i < nblocks ? row[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_sum<1024>(v, smem, &tot);
    if (i < nblocks) row[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) row_total[blockIdx.x] = carry;
}

// Ranked scatter. Element order inside a tile is (wave, round, lane), which is
// the input order, so ranks from ballots preserve stability.
__global__ void __launch_bounds__(kSortThreads) radix_downsweep(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint64_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int n, int pass, int key_passes, const int64_t* __restrict__ fo, int nf,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ row_total, int nblocks) {
  __shared__ uint32_t cnt[kSortWaves][256];
  __shared__ uint32_t scan_smem[kSortWaves + 1];
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&cnt[0][0])[i] = 0;
  // global start of each digit: exclusive scan of the row totals
  uint32_t dtot;
  const uint32_t digit_start = block_exclusive_sum<kSortThreads>(row_total[threadIdx.x], scan_smem, &dtot);
  const uint32_t tile_base_for_digit = digit_start + hist[(size_t)threadIdx.x * nblocks + blockIdx.x];
  __syncthreads();

  const int base = blockIdx.x * kSortTile + wave * 64 * kSortItems;
  uint64_t k[kSortItems];
  uint32_t v[kSortItems];
  uint32_t d[kSortItems];
  uint32_t rank[kSortItems];
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = base + r * 64 + lane;
    const bool valid = i < n;
    k[r] = valid ? keys_in[i] : 0ull;
    v[r] = valid ? vals_in[i] : 0u;
    d[r] = valid ? digit_of(k[r], v[r], pass, key_passes, fo, nf) : 0u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d[r] >> b) & 1u;
      const unsigned long long bal = __ballot(valid && bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t before = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t total = (uint32_t)__popcll(peers);
    const bool leader = valid && before == 0;
    uint32_t old = 0;
    if (valid) old = cnt[wave][d[r]];
    rank[r] = old + before;
    __builtin_amdgcn_wave_barrier();
    if (leader) cnt[wave][d[r]] = old + total;
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: offset of each wave inside the tile, then the tile's global base
  {
    const int t = threadIdx.x;  // digit
    uint32_t run = tile_base_for_digit;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      const uint32_t c = cnt[w][t];
      cnt[w][t] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = base + r * 64 + lane;
    const uint32_t dst = cnt[wave][d[r]] + rank[r];
    if (i < n && dst < (uint32_t)n) {
      keys_out[dst] = k[r];
      vals_out[dst] = v[r];
    }
  }
}

__device__ __forceinline__ bool sort_key_valid(uint64_t k, const KeyForm& kf) { return ((k >> kf.B) & 1ull) == 0; }

__device__ __forceinline__ bool is_head(const uint64_t* keys, int i, const KeyForm& kf, const int64_t* fo, int nf) {
  const uint64_t k = keys[i];
  if (!sort_key_valid(k, kf)) return false;
  if (i == 0) return true;
  if (keys[i - 1] != k) return true;
  return !kf.embed && nf > 1 && frame_of((uint32_t)i, fo, nf) != frame_of((uint32_t)(i - 1), fo, nf);
}

__device__ __forceinline__ bool is_tail(const uint64_t* keys, int i, int n, const KeyForm& kf, const int64_t* fo,
                                        int nf) {
  const uint64_t k = keys[i];
  if (!sort_key_valid(k, kf)) return false;
  if (i == n - 1) return true;
  if (keys[i + 1] != k) return true;
  return !kf.embed && nf > 1 && frame_of((uint32_t)(i + 1), fo, nf) != frame_of((uint32_t)i, fo, nf);
}

__global__ void __launch_bounds__(kSortThreads) seg_reduce(const uint64_t* __restrict__ keys, int n, KeyForm kf,
                                                           const int64_t* __restrict__ fo, int nf,
                                                           uint32_t* __restrict__ block_sums) {
  uint32_t c = 0;
  const int base = blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    const int i = base + r * kSortThreads + threadIdx.x;
    if (i < n && is_head(keys, i, kf, fo, nf)) ++c;
  }
  c = wave_sum(c);
  __shared__ uint32_t s[kSortWaves];
  if (lane_id() == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kSortWaves; ++w) t += s[w];
    block_sums[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(1024) seg_scan_blocks(uint32_t* __restrict__ block_sums, int nblocks,
                                                        unsigned long long* __restrict__ res) {
  __shared__ uint32_t smem[17];
  uint32_t carry = 0;
  for (int s = 0; s < nblocks; s += 1024) {
    const int i = s + threadIdx.x;
    const uint32_t v = i < nblocks ? block_sums[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_sum<1024>(v, smem, &tot);
    if (i < nblocks) block_sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) res[R_NVOX] = carry;
}

// Heads write key and start; tails write end (turned into a count later).
__global__ void __launch_bounds__(kSortThreads) seg_scatter(const uint64_t* __restrict__ keys, int n, KeyForm kf,
                                                            const int64_t* __restrict__ fo, int nf,
                                                            const uint32_t* __restrict__ block_base,
                                                            int64_t cap, uint64_t* __restrict__ out_keys,
                                                            int32_t* __restrict__ out_off,
                                                            int32_t* __restrict__ out_cnt) {
  __shared__ uint32_t smem[kSortWaves + 1];
  const int base = blockIdx.x * kSortTile;
  uint32_t carry = block_base[blockIdx.x];
  for (int r = 0; r < kSortItems; ++r) {
    const int i = base + r * kSortThreads + threadIdx.x;
    const bool h = i < n && is_head(keys, i, kf, fo, nf);
    uint32_t tot;
    const uint32_t ex = block_exclusive_sum<kSortThreads>(h ? 1u : 0u, smem, &tot);
    const uint32_t vid_incl = carry + ex + (h ? 1u : 0u);  // heads up to and including i
    if (h && (int64_t)(vid_incl - 1) < cap) {
      out_keys[vid_incl - 1] = unpack_sort_key(keys[i], kf);
      out_off[vid_incl - 1] = i;
    }
    if (i < n && is_tail(keys, i, n, kf, fo, nf) && (int64_t)(vid_incl - 1) < cap) out_cnt[vid_incl - 1] = i + 1;
    carry += tot;
  }
}

__global__ void __launch_bounds__(256) seg_finish(const int32_t* __restrict__ out_off, int32_t* __restrict__ out_cnt,
                                                  int64_t cap, const int64_t* __restrict__ fo, int nf,
                                                  unsigned long long* __restrict__ res) {
  const int64_t nvox = (int64_t)res[R_NVOX];
  const int64_t lim = nvox < cap ? nvox : cap;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < lim) out_cnt[v] -= out_off[v];
  // frame f's first voxel = number of voxels starting before fo[f]
  if (v <= nf) {
    int64_t r;
    if (v == 0) r = 0;
    else if (v == nf || nvox > cap) r = (v == nf) ? nvox : 0;
    else {
      int64_t lo = 0, hi = lim;  // first voxel with start >= fo[v]
      const int64_t target = fo[v];
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)out_off[mid] < target) lo = mid + 1; else hi = mid;
      }
      r = lo;
    }
    res[R_FRAMES + v] = (unsigned long long)r;
  }
}

}  // namespace

vgpr_status voxelize_impl(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts, const int64_t* h_frame_offsets,
                          int32_t n_frames, float voxel_size, uint64_t* d_keys, int32_t* d_offsets,
                          int32_t* d_counts, int32_t* d_perm, int64_t cap_vox, int64_t* h_n_vox,
                          int64_t* h_frame_vox, int64_t* h_n_invalid, size_t work_offset, bool morton) {
  if (n_pts < 0 || n_pts >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_INVALID, "n_pts out of range");
  if (cap_vox < 0) return fail(ctx, VGPR_E_INVALID, "cap_vox < 0");
  if (!h_n_vox) return fail(ctx, VGPR_E_INVALID, "h_n_vox is NULL");
  if (n_pts > 0 && (!d_xyz || !d_perm)) return fail(ctx, VGPR_E_INVALID, "d_xyz / d_perm is NULL");
  if (cap_vox > 0 && (!d_keys || !d_offsets || !d_counts))
    return fail(ctx, VGPR_E_INVALID, "voxel output buffer is NULL");
  const int nf = n_frames < 1 ? 1 : n_frames;
  std::vector<int64_t> fo(nf + 1, 0);
  if (h_frame_offsets && n_frames >= 1) {
    for (int f = 0; f <= nf; ++f) fo[f] = h_frame_offsets[f];
    if (fo[0] != 0 || fo[nf] != n_pts) return fail(ctx, VGPR_E_INVALID, "frame offsets must span [0, n_pts]");
    for (int f = 0; f < nf; ++f)
      if (fo[f + 1] < fo[f]) return fail(ctx, VGPR_E_INVALID, "frame offsets must be ascending");
  } else {
    if (n_frames > 1) return fail(ctx, VGPR_E_INVALID, "h_frame_offsets is NULL with n_frames > 1");
    fo[1] = n_pts;
  }
  const int n = (int)n_pts;
  const int nblocks = n ? (n + kSortTile - 1) / kSortTile : 1;
  const size_t res_words = R_FRAMES + nf + 1;

  const int kblocks = n ? (n + 255) / 256 : 1;
  size_t need = work_offset + Carver::round(sizeof(uint64_t) * (size_t)n) * 2 +
                Carver::round(sizeof(uint32_t) * (size_t)n) + Carver::round(sizeof(uint32_t) * 256 * nblocks) +
                Carver::round(sizeof(uint32_t) * 256) + Carver::round(sizeof(uint32_t) * nblocks) +
                Carver::round(sizeof(int) * 6 * (size_t)kblocks) + Carver::round(sizeof(int64_t) * (nf + 1)) +
                Carver::round(sizeof(unsigned long long) * res_words) + 4096;
  vgpr_status st = reserve_work(ctx, need);
  if (st != VGPR_OK) return st;
  st = reserve_pinned(ctx, sizeof(int64_t) * (nf + 1) + sizeof(unsigned long long) * res_words + 64);
  if (st != VGPR_OK) return st;
  Carver cv(static_cast<char*>(ctx->work.ptr) + work_offset);
  uint64_t* keys_a = cv.take<uint64_t>(n);
  uint64_t* keys_b = cv.take<uint64_t>(n);
  uint32_t* vals_tmp = cv.take<uint32_t>(n);
  uint32_t* hist = cv.take<uint32_t>(256 * (size_t)nblocks);
  uint32_t* row_total = cv.take<uint32_t>(256);
  uint32_t* block_sums = cv.take<uint32_t>(nblocks);
  int* part = cv.take<int>(6 * (size_t)kblocks);
  int64_t* d_fo = cv.take<int64_t>(nf + 1);
  unsigned long long* d_res = cv.take<unsigned long long>(res_words);

  int64_t* h_fo = static_cast<int64_t*>(ctx->pinned);
  unsigned long long* h_res = reinterpret_cast<unsigned long long*>(h_fo + nf + 1);
  std::copy(fo.begin(), fo.end(), h_fo);
  VGPR_HIP(ctx, hipMemcpyAsync(d_fo, h_fo, sizeof(int64_t) * (nf + 1), hipMemcpyHostToDevice, ctx->stream));
  VGPR_HIP(ctx, hipMemsetAsync(d_res, 0, sizeof(unsigned long long) * res_words, ctx->stream));

  uint32_t* perm = reinterpret_cast<uint32_t*>(d_perm);
  KeyForm kf{};
  kf.B = 0;
  kf.morton = morton ? 1 : 0;
  if (n > 0) {
    const double inv_s = 1.0 / (double)voxel_size;
    // keys and the batch's index ranges; the ranges decide the sort key's width
    {
      ProfScope ps(ctx, "voxelize_key");
      hipLaunchKernelGGL(key_kernel, dim3(kblocks), dim3(256), 0, ctx->stream, d_xyz, n, inv_s, keys_a, part,
                         d_res);
      hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, ctx->stream, part, kblocks, d_res);
    }
    VGPR_HIP(ctx, hipGetLastError());
    VGPR_HIP(ctx, hipMemcpyAsync(h_res, d_res, sizeof(unsigned long long) * R_FRAMES, hipMemcpyDeviceToHost,
                                 ctx->stream));
    VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h_res[R_RANGE]) return fail(ctx, VGPR_E_RANGE, "a point's voxel index is outside +-(2^20 - 1)");
    auto bits = [](int64_t r) {
      int b = 0;
      while (r > 0) {
        ++b;
        r >>= 1;
      }
      return b;
    };
    const bool any_valid = (int64_t)h_res[R_INVALID] < n;
    for (int a = 0; a < 3; ++a) kf.mn[a] = any_valid ? (int64_t)(long long)h_res[R_MIN + a] : 0;
    const int b3[3] = {any_valid ? bits((int64_t)(long long)h_res[R_MAX + 0] - kf.mn[0]) : 0,
                       any_valid ? bits((int64_t)(long long)h_res[R_MAX + 1] - kf.mn[1]) : 0,
                       any_valid ? bits((int64_t)(long long)h_res[R_MAX + 2] - kf.mn[2]) : 0};
    kf.bx = b3[0];
    kf.by = b3[1];
    kf.bz = b3[2];
    kf.B = kf.bx + kf.by + kf.bz;
    const int bf = nf > 1 ? bits(nf - 1) : 0;
    kf.embed = (kf.B + 1 + bf) <= 64 ? 1 : 0;
    const int key_bits = kf.B + 1 + (kf.embed ? bf : 0);
    kf.key_passes = (key_bits + 7) / 8;
    int passes = kf.key_passes;
    if (!kf.embed && nf > 1) passes += (bf + 7) / 8;
    // choose index buffers so that the last pass writes them into d_perm:
    // pass p writes vbuf[(passes - 1 - p) & 1]; the input of pass 0 is the other one
    uint32_t* vbuf[2] = {perm, vals_tmp};
    const int first_in = (passes & 1) ? 1 : 0;
    hipLaunchKernelGGL(compose_kernel, dim3(kblocks), dim3(256), 0, ctx->stream, keys_a, vbuf[first_in], n, kf, d_fo,
                       nf);
    VGPR_HIP(ctx, hipGetLastError());
    int in = first_in;
    // keys ping-pong separately, starting in keys_a
    uint64_t* kcur = keys_a;
    uint64_t* kalt = keys_b;
    {
      ProfScope ps(ctx, "voxelize_sort");
      for (int p = 0; p < passes; ++p) {
        const int out = in ^ 1;
        hipLaunchKernelGGL(radix_upsweep, dim3(nblocks), dim3(kSortThreads), 0, ctx->stream, kcur, vbuf[in], n, p,
                           kf.key_passes, d_fo, nf, hist, nblocks);
        hipLaunchKernelGGL(radix_rowscan, dim3(256), dim3(1024), 0, ctx->stream, hist, nblocks, row_total);
        hipLaunchKernelGGL(radix_downsweep, dim3(nblocks), dim3(kSortThreads), 0, ctx->stream, kcur, vbuf[in], kalt,
                           vbuf[out], n, p, kf.key_passes, d_fo, nf, hist, row_total, nblocks);
        in = out;
        uint64_t* t = kcur;
        kcur = kalt;
        kalt = t;
      }
    }
    VGPR_HIP(ctx, hipGetLastError());
    const uint64_t* sorted = kcur;
    {
      ProfScope ps(ctx, "voxelize_segment");
      hipLaunchKernelGGL(seg_reduce, dim3(nblocks), dim3(kSortThreads), 0, ctx->stream, sorted, n, kf, d_fo, nf,
                         block_sums);
      hipLaunchKernelGGL(seg_scan_blocks, dim3(1), dim3(1024), 0, ctx->stream, block_sums, nblocks, d_res);
      hipLaunchKernelGGL(seg_scatter, dim3(nblocks), dim3(kSortThreads), 0, ctx->stream, sorted, n, kf, d_fo, nf,
                         block_sums, cap_vox, d_keys, d_offsets, d_counts);
      const int64_t fin = std::max<int64_t>(n, nf + 1);
      hipLaunchKernelGGL(seg_finish, dim3((unsigned)((fin + 255) / 256)), dim3(256), 0, ctx->stream, d_offsets,
                         d_counts, cap_vox, d_fo, nf, d_res);
    }
    VGPR_HIP(ctx, hipGetLastError());
  }
  VGPR_HIP(ctx, hipMemcpyAsync(h_res, d_res, sizeof(unsigned long long) * res_words, hipMemcpyDeviceToHost,
                               ctx->stream));
  VGPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h_res[R_RANGE]) return fail(ctx, VGPR_E_RANGE, "a point's voxel index is outside +-(2^20 - 1)");
  const int64_t nvox = (int64_t)h_res[R_NVOX];
  *h_n_vox = nvox;
  if (h_n_invalid) *h_n_invalid = (int64_t)h_res[R_INVALID];
  if (nvox > cap_vox)
    return fail(ctx, VGPR_E_CAPACITY, "voxel count " + std::to_string(nvox) + " exceeds cap_vox");
  if (h_frame_vox)
    for (int f = 0; f <= nf; ++f) h_frame_vox[f] = n > 0 ? (int64_t)h_res[R_FRAMES + f] : 0;
  return VGPR_OK;
}

}  // namespace vgpr

extern "C" vgpr_status vgpr_voxelize(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts, const int64_t* h_frame_offsets,
                                     int32_t n_frames, const vgpr_params* params, uint64_t* d_keys,
                                     int32_t* d_offsets, int32_t* d_counts, int32_t* d_perm, int64_t cap_vox,
                                     int64_t* h_n_vox, int64_t* h_frame_vox, int64_t* h_n_invalid) {
  if (!ctx) return VGPR_E_INVALID;
  vgpr_status st = vgpr::check_params(ctx, params);
  if (st != VGPR_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return vgpr::fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  return vgpr::voxelize_impl(ctx, d_xyz, n_pts, h_frame_offsets, n_frames, params->voxel_size, d_keys, d_offsets,
                             d_counts, d_perm, cap_vox, h_n_vox, h_frame_vox, h_n_invalid, 0);
}
