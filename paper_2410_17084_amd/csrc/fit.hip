// vgpr_fit_predict: Alg. 1 after STORE, Eq. (1)-(3) of the paper, per voxel.
//
// Three kernels per call (plus a re-solve pass in FP32 mode):
//
// 1. prep (one thread per voxel): kept count n, tau test, a slot in the
//    voxel's size bucket (one atomic per wavefront and bucket), the PCA frame
//    of Alg. 1 in double (centroid, covariance, cyclic Jacobi eigen-solve,
//    value axis = world axis closest to the smallest-eigenvalue eigenvector,
//    cyclic parameter axes, near-tie flag, optional per-voxel length scale)
//    written as a 64-byte slot record, and the kept points staged as float4
//    (x, y, z, noise variance) at their sorted positions, so that the solvers
//    read one record and one coalesced row of points per voxel. Voxels of more
//    than 64 points are staged and summed by a second kernel, one wavefront
//    per voxel, so that no thread walks up to 512 points alone.
// 2. solve: the posterior of Eq. (3) from an LDL^T elimination of the
//    augmented system whose rows are
//          [ K + S | f~ ]   n data rows      (S = noise variances on the diagonal)
//          [ K*^T       ]   m query rows
//    restricted to the n data columns. Eliminating the data columns turns
//    each query row into L^-1 k*_q and the right-hand side f~ (f minus its
//    mean, one extra value per data row) into y = L^-1 f~, so
//      var_q  = s_f^2 - sum_j a_qj^2 / d_j      (diagonal of Sigma*)
//      mean_q = mu    + sum_j a_qj * y_j / d_j   (K*^T (K+S)^-1 f~)
//    accumulate on the fly (d_j = pivots, a_qj = the query row's entry at
//    step j). K, K* and K** are never stored. Each row lives in registers;
//    after step j it shifts by one register so the active column is always
//    element 0 (no dynamic register indexing).
//    - wave solver (n <= 64, m <= 64): one voxel per wavefront, lane l holds
//      query row l and data row l; column j is broadcast with readlane, so
//      the elimination has no barriers at all.
//    - block solver (larger voxels or grids): one voxel per workgroup, one
//      row per lane, column j broadcast through LDS with one barrier a step.
// 3. NaN rows for voxels below tau.
//
// The elimination type T is float or double. In FP32 mode every voxel runs
// in float and voxels whose refinement score sum_j |y_j| / d_j exceeds the
// threshold (the amplification of FP32 rounding in K^-1 f~) are re-solved in
// double; in FP64 mode every voxel runs in double.
#include <algorithm>
#include <type_traits>
#include <utility>
#include <cfloat>

#include "scan.h"
#include "vgpr_internal.h"

namespace vgpr {
namespace {

constexpr int kBlockThreads = 256;  // upper bound of the block solver's workgroup
constexpr int kWaveThreads = 256;   // workgroup of the wave solver: 4 independent wavefronts
constexpr int kLists = kNumBuckets + 1;  // size buckets + the below-tau list
constexpr int kNanList = kNumBuckets;

struct FitParams {
  int cap;          // max_pts
  int tau;          // min_pts
  int nq;           // grid side
  int m;            // nq * nq
  int ls_mode;
  int frame_mode;   // 0 world value axis, 1 PCA-rotated frame
  int mode;         // 0 = FP32 first pass (flags), 1 = FP64 re-solve pass, 2 = FP64 only,
                    // 3 = FP32 pass with one FP64 refinement of alpha (flagged voxels)
  int bcap[kNumBuckets];  // bucket capacities
  float sf2;
  float noise;
  float eta;
  float refine_thr;
  float cond_thr;   // mixed mode: FP64 refinement of alpha above this n s_f^2 / min pivot
  double s;         // voxel size (float widened)
  double ell;       // fixed length scale
};

// Per-voxel frame of Alg. 1, written by prep and read by the solvers.
struct FrameRec {
  double mu;        // mean of the value coordinate
  double anc_u;     // voxel corner along u
  double anc_w;     // voxel corner along w
  double lam;       // 1 / (2 l^2)
  int ku, kw;       // voxel indices along u and w
  int axes;         // value axis | u << 2 | w << 4 | tie << 6
  int n;            // kept points
};

// One bucket slot: the voxel's frame and where its staged points are.
struct SlotRec {
  FrameRec fr;
  int v;            // voxel index (output row block)
  int off;          // first staged point (the voxel's sorted offset)
  int cnt;          // points before the cap
  int pad;
};

// Rotated local frame of one slot (frame_mode 1): centroid and the axes (e1, e2, v).
struct RotRec {
  double c[3];
  double e1[3], e2[3], v[3];
};

struct Lists {
  SlotRec* recs;         // kNumBuckets lists of `stride` slot records
  int32_t* nan_list;     // voxels below tau
  uint32_t* count;       // kLists counters
  int64_t stride;
  RotRec* rots;          // frame_mode 1: one rotated frame per slot record, else null
  int4* big;             // voxels of more than kPrepCoop points: (voxel, list, slot, 0)
  uint32_t* big_count;
};

// Voxels of more than this many kept points are staged and summed by a whole wavefront.
constexpr int kPrepCoop = 64;

__device__ __forceinline__ float k_exp(float x) { return __expf(x); }
__device__ __forceinline__ double k_exp(double x) { return exp(x); }

// Pivot reciprocal: the hardware estimate (1 ulp) in FP32, whose elimination error
// is far above it. In FP64 the hardware estimate refined by two Newton steps
// (each doubles the correct bits), within an ulp or two of 1/x for a normal
// positive pivot; a zero or non-finite pivot gives NaN and the voxel fails.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (double).
// On return w[] holds the eigenvalues and column k of V the k-th eigenvector.
__device__ void jacobi3(double A[3][3], double w[3], double V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-36 * dia || off == 0.0) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const int r = 3 - p - q;
      const double apq = A[p][q];
      if (apq != 0.0) {
        // rotation angle that annihilates A[p][q]: tan via the smaller root
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0);
        const double s = t * c;
        const double arp = A[r][p], arq = A[r][q];
        A[p][p] -= t * apq;
        A[q][q] += t * apq;
        A[p][q] = A[q][p] = 0.0;
        A[r][p] = A[p][r] = c * arp - s * arq;
        A[r][q] = A[q][r] = s * arp + c * arq;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
  w[0] = A[0][0];
  w[1] = A[1][1];
  w[2] = A[2][2];
}

__device__ __forceinline__ float pick(int axis, float x, float y, float z) { return axis == 0 ? x : (axis == 1 ? y : z); }

// The voxel's frame of Alg. 1 from the sums about its first point p0 (S1 = sum d,
// S2 = sum d d^T, d = p - p0, in the order s0, s1, s2, a00, a01, a02, a11, a12, a22),
// written as its slot record (and rotated frame).
__device__ __forceinline__ void prep_frame(const FitParams& P, const FitArgs& io, const Lists& L, int64_t v, int lst,
                                        int slot, int n, int c, int off, double p0x, double p0y, double p0z,
                                        const double (&sums)[9]) {
  const double s0 = sums[0], s1 = sums[1], s2 = sums[2], a00 = sums[3], a01 = sums[4], a02 = sums[5],
               a11 = sums[6], a12 = sums[7], a22 = sums[8];
  (void)off;
  const double inv_n = 1.0 / (double)n;
  const double m0 = s0 * inv_n, m1 = s1 * inv_n, m2 = s2 * inv_n;
  double A[3][3];
  A[0][0] = a00 * inv_n - m0 * m0;
  A[0][1] = A[1][0] = a01 * inv_n - m0 * m1;
  A[0][2] = A[2][0] = a02 * inv_n - m0 * m2;
  A[1][1] = a11 * inv_n - m1 * m1;
  A[1][2] = A[2][1] = a12 * inv_n - m1 * m2;
  A[2][2] = a22 * inv_n - m2 * m2;
  const double tr = A[0][0] + A[1][1] + A[2][2];
  double w[3], V[3][3];
  jacobi3(A, w, V);
  // eigenvector of the smallest eigenvalue (ties to the lower index)
  const int imin = (w[1] < w[0]) ? ((w[2] < w[1]) ? 2 : 1) : ((w[2] < w[0]) ? 2 : 0);
  const double v0 = imin == 0 ? V[0][0] : (imin == 1 ? V[0][1] : V[0][2]);
  const double v1 = imin == 0 ? V[1][0] : (imin == 1 ? V[1][1] : V[1][2]);
  const double v2 = imin == 0 ? V[2][0] : (imin == 1 ? V[2][1] : V[2][2]);
  const double wlo = fmin(fmin(w[0], w[1]), w[2]);
  const double whi = fmax(fmax(w[0], w[1]), w[2]);
  const double wmid = fmax(fmin(w[0], w[1]), fmin(fmax(w[0], w[1]), w[2]));
  const double b0 = fabs(v0), b1 = fabs(v1), b2 = fabs(v2);
  int ax = 0;
  double best = b0;
  if (b1 > best) { ax = 1; best = b1; }
  if (b2 > best) { ax = 2; best = b2; }
  const double second = (ax == 0) ? fmax(b1, b2) : (ax == 1 ? fmax(b0, b2) : fmax(b0, b1));
  const int tie = (best - second < 1e-6) || (wmid - wlo <= 1e-8 * tr);
  const int u = ax == 0 ? 1 : (ax == 1 ? 2 : 0);
  const int wv = ax == 0 ? 2 : (ax == 1 ? 0 : 1);
  double ell = P.ell;
  if (P.ls_mode == 1) {
    const double e = sqrt(3.0) * sqrt(fmax((wmid + whi) * 0.5, 0.0));
    ell = fmin(fmax(e, 0.05 * P.s), 2.0 * P.s);
  }
  const uint64_t key = io.keys[v];
  const int64_t mask = (int64_t(1) << kKeyFieldBits) - 1;
  const int kx = (int)((int64_t)((key >> (2 * kKeyFieldBits)) & mask) - kKeyBias);
  const int ky = (int)((int64_t)((key >> kKeyFieldBits) & mask) - kKeyBias);
  const int kz = (int)((int64_t)(key & mask) - kKeyBias);
  SlotRec r;
  r.fr.ku = u == 0 ? kx : (u == 1 ? ky : kz);
  r.fr.kw = wv == 0 ? kx : (wv == 1 ? ky : kz);
  const double pa = ax == 0 ? p0x : (ax == 1 ? p0y : p0z);
  const double ma = ax == 0 ? m0 : (ax == 1 ? m1 : m2);
  r.fr.mu = pa + ma;
  r.fr.anc_u = (double)r.fr.ku * P.s;
  r.fr.anc_w = (double)r.fr.kw * P.s;
  r.fr.lam = 1.0 / (2.0 * ell * ell);
  r.fr.axes = ax | (u << 2) | (wv << 4) | (tie << 6);
  r.fr.n = n;
  r.v = (int)v;
  r.off = off;
  r.cnt = c;
  r.pad = 0;
  if (P.frame_mode == 1) {
    // rotated frame: the normal with its largest component positive, e1 along e_k x v for the
    // world axis k least aligned with v (ties to the lower index), e2 = v x e1; local
    // coordinates are taken about the centroid, so the value's mean and the anchors are 0
    const double nv = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const double sg = (ax == 0 ? v0 : (ax == 1 ? v1 : v2)) < 0.0 ? -1.0 : 1.0;
    const double n0 = sg * v0 / nv, n1 = sg * v1 / nv, n2 = sg * v2 / nv;
    const double c0 = fabs(n0), c1 = fabs(n1), c2 = fabs(n2);
    const int k = (c1 < c0) ? ((c2 < c1) ? 2 : 1) : ((c2 < c0) ? 2 : 0);
    // e_k x n
    double a0 = k == 0 ? 0.0 : (k == 1 ? n2 : -n1);
    double a1 = k == 0 ? -n2 : (k == 1 ? 0.0 : n0);
    double a2 = k == 0 ? n1 : (k == 1 ? -n0 : 0.0);
    const double an = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
    a0 /= an;
    a1 /= an;
    a2 /= an;
    RotRec rr;
    rr.c[0] = p0x + m0;
    rr.c[1] = p0y + m1;
    rr.c[2] = p0z + m2;
    rr.e1[0] = a0;
    rr.e1[1] = a1;
    rr.e1[2] = a2;
    rr.e2[0] = n1 * a2 - n2 * a1;  // n x e1
    rr.e2[1] = n2 * a0 - n0 * a2;
    rr.e2[2] = n0 * a1 - n1 * a0;
    rr.v[0] = n0;
    rr.v[1] = n1;
    rr.v[2] = n2;
    L.rots[lst * L.stride + slot] = rr;
    r.fr.mu = 0.0;
    r.fr.anc_u = 0.0;
    r.fr.anc_w = 0.0;
  }
  L.recs[lst * L.stride + slot] = r;
}

// ---------------------------------------------------------------------------
// 1. prep: tau test, PCA frame, bucketing (one thread per voxel; one wavefront per
//    voxel of more than kPrepCoop points)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) prep_kernel(FitParams P, FitArgs io, float4* __restrict__ staged,
                                                   Lists L) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = v < io.n_vox;
  int lst = -1, n = 0, c = 0, off = 0;
  if (valid) {
    c = io.counts[v];
    off = io.offsets[v];
    n = c < P.cap ? c : P.cap;
    if (n < P.tau || off < 0 || (int64_t)off + n > io.n_pts) {
      // below tau (type (a)); a voxel whose points lie outside [0, n_pts) is not solved either
      const bool in_range = off >= 0 && (int64_t)off + n <= io.n_pts;
      io.status[v] = in_range ? (uint8_t)(VGPR_ST_BELOW_TAU | (c > P.cap ? VGPR_ST_CAPPED : 0)) : (uint8_t)0;
      io.axis[v] = -1;
      lst = kNanList;
    } else {
      lst = 0;
      while (lst < kNumBuckets - 1 && n > P.bcap[lst]) ++lst;
    }
  }
  // slot in the voxel's list: wavefront offsets within the workgroup through LDS,
  // then one global atomic per workgroup and list
  __shared__ uint32_t s_cnt[kLists], s_base[kLists];
  const int lane = lane_id();
  const unsigned long long lt = (1ull << lane) - 1ull;
  if (threadIdx.x < kLists) s_cnt[threadIdx.x] = 0u;
  __syncthreads();
  uint32_t woff = 0;
  unsigned long long mymask = 0;
#pragma unroll
  for (int l = 0; l < kLists; ++l) {
    const unsigned long long mk = __ballot(lst == l);
    if (mk) {
      const int leader = __ffsll((long long)mk) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&s_cnt[l], (uint32_t)__popcll(mk));
      base = __shfl(base, leader, 64);
      if (lst == l) {
        woff = base;
        mymask = mk;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kLists && s_cnt[threadIdx.x]) s_base[threadIdx.x] = atomicAdd(&L.count[threadIdx.x], s_cnt[threadIdx.x]);
  __syncthreads();
  int slot = 0;
  if (lst >= 0) slot = (int)(s_base[lst] + woff + __popcll(mymask & lt));
  if (lst == kNanList) L.nan_list[slot] = (int32_t)v;
  if (lst < 0 || lst == kNanList) return;
  if (n > kPrepCoop) {
    // staged, summed and framed by prep_big_kernel, one wavefront per voxel
    L.big[atomicAdd(L.big_count, 1u)] = make_int4((int)v, lst, slot, 0);
    return;
  }

  // stage the kept points and accumulate the covariance about the first point:
  // S1 = sum d, S2 = sum d d^T with d = p - p0. Loads of four points are issued
  // together so that a thread keeps several gathers in flight.
  const int* __restrict__ perm = io.perm;
  const float* __restrict__ xyz = io.xyz;
  const float* __restrict__ noise = io.noise;
  float4* __restrict__ st = staged;
  const int i0 = perm ? perm[off] : off;
  const float x0 = xyz[3 * (size_t)i0], y0 = xyz[3 * (size_t)i0 + 1], z0 = xyz[3 * (size_t)i0 + 2];
  st[off] = make_float4(x0, y0, z0, noise ? noise[i0] : P.noise);
  const double p0x = x0, p0y = y0, p0z = z0;
  double s0 = 0, s1 = 0, s2 = 0, a00 = 0, a01 = 0, a02 = 0, a11 = 0, a12 = 0, a22 = 0;
  for (int i = 1; i < n; i += 4) {
    float px[4], py[4], pz[4], pn[4];
#pragma unroll
    for (int u4 = 0; u4 < 4; ++u4) {
      const int ii = i + u4 < n ? i + u4 : i;
      const int idx = perm ? perm[off + ii] : off + ii;
      px[u4] = xyz[3 * (size_t)idx];
      py[u4] = xyz[3 * (size_t)idx + 1];
      pz[u4] = xyz[3 * (size_t)idx + 2];
      pn[u4] = noise ? noise[idx] : P.noise;
    }
#pragma unroll
    for (int u4 = 0; u4 < 4; ++u4) {
      if (i + u4 < n) {
        st[off + i + u4] = make_float4(px[u4], py[u4], pz[u4], pn[u4]);
        const double d0 = (double)px[u4] - p0x;
        const double d1 = (double)py[u4] - p0y;
        const double d2 = (double)pz[u4] - p0z;
        s0 += d0; s1 += d1; s2 += d2;
        a00 += d0 * d0; a01 += d0 * d1; a02 += d0 * d2;
        a11 += d1 * d1; a12 += d1 * d2; a22 += d2 * d2;
      }
    }
  }
  const double sums[9] = {s0, s1, s2, a00, a01, a02, a11, a12, a22};
  prep_frame(P, io, L, v, lst, slot, n, c, off, p0x, p0y, p0z, sums);
}

// prep for the voxels of more than kPrepCoop points: one wavefront per voxel stages its
// points (lane l takes points l, l + 64, ...) and sums its share of S1 and S2; the shares
// are added across the wavefront and lane 0 computes the frame. Grid-stride over the list.
__global__ void __launch_bounds__(256) prep_big_kernel(FitParams P, FitArgs io, float4* __restrict__ staged,
                                                       Lists L) {
  const int lane = lane_id();
  const int gw = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nw = (int)(((int64_t)gridDim.x * blockDim.x) >> 6);
  const int count = (int)*L.big_count;
  const int* __restrict__ perm = io.perm;
  const float* __restrict__ xyz = io.xyz;
  const float* __restrict__ noise = io.noise;
  for (int it = gw; it < count; it += nw) {
    const int4 e = L.big[it];
    const int v = e.x;
    const int c = io.counts[v];
    const int off = io.offsets[v];
    const int n = c < P.cap ? c : P.cap;
    const int i0 = perm ? perm[off] : off;
    const float x0 = xyz[3 * (size_t)i0], y0 = xyz[3 * (size_t)i0 + 1], z0 = xyz[3 * (size_t)i0 + 2];
    const double p0x = x0, p0y = y0, p0z = z0;
    double t[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = lane; i < n; i += 64) {
      const int idx = perm ? perm[off + i] : off + i;
      const float px = xyz[3 * (size_t)idx], py = xyz[3 * (size_t)idx + 1], pz = xyz[3 * (size_t)idx + 2];
      staged[off + i] = make_float4(px, py, pz, noise ? noise[idx] : P.noise);
      const double d0 = (double)px - p0x, d1 = (double)py - p0y, d2 = (double)pz - p0z;
      t[0] += d0; t[1] += d1; t[2] += d2;
      t[3] += d0 * d0; t[4] += d0 * d1; t[5] += d0 * d2;
      t[6] += d1 * d1; t[7] += d1 * d2; t[8] += d2 * d2;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) t[k] += __shfl_xor(t[k], d, 64);
    }
    if (lane == 0) prep_frame(P, io, L, v, e.y, e.z, n, c, off, p0x, p0y, p0z, t);
  }
}

// Zero the list counters with a kernel (no memset node when a caller captures the call in a graph).
__global__ void zero_kernel(uint32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Longest-first order of the tiled buckets' slots: a counting sort by kept point count,
// descending, one workgroup per bucket. The tiled solvers hand out voxels in this order, so
// the largest solves start first and the last ones to start are the shortest (list
// scheduling by longest processing time). Slots with equal counts may come in any order;
// every voxel is solved the same way whatever its position. One launch on the caller's
// stream before the buckets fork: a lone 1024-thread workgroup queued on a side stream
// could wait a millisecond for a CU while the solvers hold them.
// With count2, the slots of a second list at recs + stride2 join the sort (their order
// entries are stride2 + slot) and *total receives the combined count.
struct OrderJob {
  const SlotRec* recs;
  const uint32_t* count;
  int32_t* order;
  const uint32_t* count2;
  int32_t stride2;
  uint32_t* total;
};
struct OrderJobs {
  OrderJob job[kNumBuckets];
};
constexpr int kOrderThreads = 1024;
__global__ void __launch_bounds__(kOrderThreads) order_kernel(OrderJobs jobs) {
  static_assert(kMaxPtsLimit < kOrderThreads, "one count per thread in the scan");
  __shared__ uint32_t start[kMaxPtsLimit + 1];
  __shared__ uint32_t part[kOrderThreads / 64 + 1];
  const OrderJob& jb = jobs.job[blockIdx.x];
  const SlotRec* __restrict__ recs = jb.recs;
  const uint32_t* count2 = jb.count2;
  const int32_t stride2 = jb.stride2;
  int32_t* __restrict__ order = jb.order;
  const int items1 = (int)*jb.count;
  const int items = items1 + (count2 ? (int)*count2 : 0);
  auto slot_of = [&](int i) { return i < items1 ? i : stride2 + (i - items1); };
  for (int i = threadIdx.x; i <= kMaxPtsLimit; i += kOrderThreads) start[i] = 0u;
  __syncthreads();
  for (int i = threadIdx.x; i < items; i += kOrderThreads) atomicAdd(&start[recs[slot_of(i)].fr.n], 1u);
  __syncthreads();
  // first slot of each count, largest count first: thread t scans the count n = limit - t
  const int k = kMaxPtsLimit - (int)threadIdx.x;
  const uint32_t h = k >= 0 ? start[k] : 0u;
  uint32_t all;
  const uint32_t first = block_exclusive_sum<kOrderThreads>(h, part, &all);
  if (k >= 0) start[k] = first;
  __syncthreads();
  for (int i = threadIdx.x; i < items; i += kOrderThreads) {
    const int sl = slot_of(i);
    order[atomicAdd(&start[recs[sl].fr.n], 1u)] = sl;
  }
  if (jb.total && threadIdx.x == 0) *jb.total = (uint32_t)items;
}

// ---------------------------------------------------------------------------
// 3. NaN rows of voxels below tau (one wavefront per voxel, coalesced rows)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) nan_kernel(FitParams P, float* __restrict__ out, Lists L) {
  const int lane = lane_id();
  const int gw = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nw = (int)(((int64_t)gridDim.x * blockDim.x) >> 6);
  const int count = (int)L.count[kNanList];
  const float nan = __int_as_float(0x7fc00000);
  for (int it = gw; it < count; it += nw) {
    const int v = L.nan_list[it];
    float4* o = reinterpret_cast<float4*>(out) + (size_t)v * P.m;
    for (int q = lane; q < P.m; q += 64) o[q] = make_float4(nan, nan, nan, nan);
  }
}

// Status of a solved (or flagged) voxel; lane / thread 0 only.
__device__ __forceinline__ void finish_voxel(const FitParams& P, const FitArgs& io, int v, int slot, int cnt,
                                             int axes, bool failed, bool flag, float maxvar, int32_t* rlist,
                                             uint32_t* rcount, bool refined = false) {
  uint8_t st = VGPR_ST_SOLVED | (refined ? VGPR_ST_REFINED : 0);
  if (cnt > P.cap) st |= VGPR_ST_CAPPED;
  if ((axes >> 6) & 1) st |= VGPR_ST_AXIS_TIE;
  if (flag) {
    // FP32 pass: hand the voxel to the FP64 re-solve list
    const uint32_t k = atomicAdd(rcount, 1u);
    rlist[k] = slot;
    if (failed) st |= VGPR_ST_FACTOR_FAIL;
  } else {
    if (P.mode == 1) st |= VGPR_ST_REFINED | (io.status[v] & VGPR_ST_FACTOR_FAIL);
    if (failed) st = (uint8_t)((st & ~VGPR_ST_SOLVED) | VGPR_ST_FACTOR_FAIL);
    else if (maxvar <= P.eta) st |= VGPR_ST_CONVERGED;
  }
  io.status[v] = st;
  io.axis[v] = (int8_t)(axes & 3);
}

// Fraction (i + 0.5) / nq of grid index i, correctly rounded: voxel-independent,
// so the solvers compute it once per lane (or table) instead of once per voxel.
__device__ __forceinline__ double grid_frac(const FitParams& P, int i) {
  return __ddiv_rn((double)i + 0.5, (double)P.nq);
}

// Grid coordinates of the query with fractions (ti, tj) of its row and column.
__device__ __forceinline__ void coords_from_frac(const FitParams& P, const FrameRec& fr, double ti, double tj,
                                                 float* gu, float* gw) {
  if (P.frame_mode == 1) {
    // interval centres of an s x s square centred on the centroid, in the (e1, e2) plane
    *gu = (float)__dmul_rn(__dadd_rn(ti, -0.5), P.s);
    *gw = (float)__dmul_rn(__dadd_rn(tj, -0.5), P.s);
    return;
  }
  *gu = (float)__dmul_rn(__dadd_rn((double)fr.ku, ti), P.s);
  *gw = (float)__dmul_rn(__dadd_rn((double)fr.kw, tj), P.s);
}

__device__ __forceinline__ void query_coords(const FitParams& P, const FrameRec& fr, int q, float* gu, float* gw) {
  const int i = q / P.nq, j = q - (q / P.nq) * P.nq;
  coords_from_frac(P, fr, grid_frac(P, i), grid_frac(P, j), gu, gw);
}

__device__ __forceinline__ float4 out_row(int ax, int u, float mv, float gu, float gw, float vv) {
  float4 o;
  o.x = ax == 0 ? mv : (u == 0 ? gu : gw);
  o.y = ax == 1 ? mv : (u == 1 ? gu : gw);
  o.z = ax == 2 ? mv : (u == 2 ? gu : gw);
  o.w = vv;
  return o;
}

// Local coordinates of a staged point: (u, w) on the parameter plane and the centred value f.
__device__ __forceinline__ void local_point(const FitParams& P, const FrameRec& fr, const RotRec* __restrict__ rot,
                                            float4 pt, double* xu, double* xw, double* fv) {
  if (P.frame_mode == 1) {
    const double dx = (double)pt.x - rot->c[0], dy = (double)pt.y - rot->c[1], dz = (double)pt.z - rot->c[2];
    *xu = dx * rot->e1[0] + dy * rot->e1[1] + dz * rot->e1[2];
    *xw = dx * rot->e2[0] + dy * rot->e2[1] + dz * rot->e2[2];
    *fv = dx * rot->v[0] + dy * rot->v[1] + dz * rot->v[2] - fr.mu;
  } else {
    const int ax = fr.axes & 3, u = (fr.axes >> 2) & 3, wax = (fr.axes >> 4) & 3;
    *xu = (double)pick(u, pt.x, pt.y, pt.z) - fr.anc_u;
    *xw = (double)pick(wax, pt.x, pt.y, pt.z) - fr.anc_w;
    *fv = (double)pick(ax, pt.x, pt.y, pt.z) - fr.mu;
  }
}

// Output row of query (gu, gw) with predicted value fhat and variance vv, in world coordinates.
__device__ __forceinline__ float4 make_row(const FitParams& P, const FrameRec& fr, const RotRec* __restrict__ rot,
                                           double fhat, float gu, float gw, float vv) {
  if (P.frame_mode == 1) {
    const double a = gu, b = gw;
    return make_float4((float)(rot->c[0] + a * rot->e1[0] + b * rot->e2[0] + fhat * rot->v[0]),
                       (float)(rot->c[1] + a * rot->e1[1] + b * rot->e2[1] + fhat * rot->v[1]),
                       (float)(rot->c[2] + a * rot->e1[2] + b * rot->e2[2] + fhat * rot->v[2]), vv);
  }
  return out_row(fr.axes & 3, (fr.axes >> 2) & 3, (float)fhat, gu, gw, vv);
}

// One FP64 refinement step of alpha = (K + S)^-1 f~ with the FP32 factor K + S = L D L^T
// of the wave solver (lane i holds d_i and y_i = (L^-1 f~)_i, column j of the unit lower L
// is sL[j * NMAX + i], the data points in double are xd[0 | NMAX | 2 NMAX + i]):
//   alpha0 = L^-T D^-1 y,  r = f~ - (K + S) alpha0 (kernel entries in double),
//   alpha = alpha0 + L^-T D^-1 L^-1 r,
// then mean_q - mu = k*_q^T alpha in double for this lane's query rows (Eq. (3)).
template <int NMAX, int QR>
__device__ __forceinline__ void refine_mean(const FitParams& P, const FrameRec& fr, const double* __restrict__ xd,
                            const float* __restrict__ sL, int n, int lane, double dl, double yl, double nzl,
                            const float* gu, const float* gw, double* meanr) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const bool dl_ = lane < n;
  const double sf2 = (double)P.sf2, lam = fr.lam;
  // back substitution x = L^-T v for v held one value per lane
  auto back = [&](double v) {
    double acc = 0.0, x = 0.0;
    for (int k = n - 1; k >= 0; --k) {
      const double xk = bcast(v - acc, k);  // lane k's sum over rows below k is complete
      if (lane == k) x = xk;
      if (lane < k) acc += (double)sL[lane * NMAX + k] * xk;
    }
    return x;
  };
  double alpha = back(dl_ ? yl / dl : 0.0);
  // residual of (K + S) alpha = f~ in double
  double rr = 0.0;
  if (dl_) {
    const double ui = xd[lane], wi = xd[NMAX + lane];
    rr = xd[2 * NMAX + lane] - nzl * alpha;
    for (int c = 0; c < n; ++c) {
      const double ac = bcast(alpha, c);
      const double du = ui - xd[c], dw = wi - xd[NMAX + c];
      rr -= sf2 * exp(-(du * du + dw * dw) * lam) * ac;
    }
  } else {
    for (int c = 0; c < n; ++c) (void)bcast(alpha, c);  // every lane takes part in the broadcasts
  }
  // forward substitution w = L^-1 r, then D^-1 and the back substitution
  double w = 0.0;
  for (int j = 0; j < n; ++j) {
    const double wj = bcast(rr, j);  // lane j's value is final at step j
    if (lane == j) w = wj;
    if (lane > j && lane < n) rr -= (double)sL[j * NMAX + lane] * wj;
  }
  alpha += back(dl_ ? w / dl : 0.0);
  // mean of this lane's query rows from alpha (one row at a time: few registers on this rare path)
#pragma unroll
  for (int r = 0; r < QR; ++r) {
    const double qu = (double)gu[r] - fr.anc_u, qw = (double)gw[r] - fr.anc_w;
    double acc = 0.0;
    for (int c = 0; c < n; ++c) {
      const double ac = bcast(alpha, c);
      const double du = qu - xd[c], dw = qw - xd[NMAX + c];
      acc += sf2 * exp(-(du * du + dw * dw) * lam) * ac;
    }
    meanr[r] = acc;
  }
}

// ---------------------------------------------------------------------------
// 2a. wave solver: one voxel per wavefront, n <= min(NMAX, 64), m <= 64
// ---------------------------------------------------------------------------
template <typename T, int NMAX, int QR, bool REF = false>
__global__ void __launch_bounds__(kWaveThreads) fit_wave_kernel(FitParams P, FitArgs io,
                                                                const SlotRec* __restrict__ recs,
                                                                const RotRec* __restrict__ rots,
                                                                const float4* __restrict__ staged,
                                                                const int32_t* __restrict__ slots,
                                                                const uint32_t* __restrict__ count,
                                                                int32_t* __restrict__ rlist,
                                                                uint32_t* __restrict__ rcount,
                                                                int32_t* __restrict__ flist,
                                                                uint32_t* __restrict__ fcount) {
  constexpr bool kKInLds = NMAX <= 32;       // K from its upper triangle through LDS
  constexpr int kWaves = kWaveThreads / 64;
  constexpr int NQ = QR == 1 ? 8 : (QR == 2 ? 12 : 16);  // largest grid side for QR query rows per lane
  // REF: the FP32 pass over flagged voxels with one FP64 refinement step of alpha, which
  // keeps the float factor in the kernel-matrix region once K has been read. The first
  // FP32 pass of the 16-point shape hands those voxels to it and keeps its registers
  // (larger shapes re-solve them in FP64: their refinement would spill).
  static_assert(!REF || (sizeof(T) == 4 && NMAX == 16), "refinement pass: FP32, up to 16 points");
  constexpr bool kRefine = REF;
  constexpr bool kHandOff = sizeof(T) == 4 && NMAX == 16 && !REF;
  __shared__ T s_xu[kWaves][NMAX + NQ], s_xw[kWaves][NMAX + NQ];
  __shared__ T s_tab[kWaves][2 * NQ * NMAX];
  __shared__ T s_K[kWaves][kKInLds ? NMAX * NMAX : 1];
  __shared__ double s_xd[kWaves][kRefine ? 3 * NMAX : 1];  // data points (u, w, f~) in double
  const int wid = threadIdx.x >> 6;
  const int lane = lane_id();
  // wavefront-uniform indices (scalar registers): record loads become scalar loads
  const int gw = __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int nw = (int)(((int64_t)gridDim.x * blockDim.x) >> 6);
  const int cnt_items = (int)*count;
  const T sf2 = (T)P.sf2;
  // two-stage software pipeline: the record of item it + 2 nw and the points of
  // item it + nw are in flight while item it is solved
  int it = gw;
  SlotRec rn{};
  float4 pn = make_float4(0.f, 0.f, 0.f, 0.f);
  SlotRec rnn{};
  if (it < cnt_items) {
    rn = recs[slots ? slots[it] : it];
    if (lane < rn.fr.n) pn = staged[rn.off + lane];
  }
  if (it + nw < cnt_items) rnn = recs[slots ? slots[it + nw] : it + nw];
  // grid fractions of this lane's query rows and of grid index `lane` (voxel-independent)
  double fti[QR], ftj[QR];
  int qi[QR], qj[QR];
#pragma unroll
  for (int r = 0; r < QR; ++r) {
    const int q = lane + 64 * r < P.m ? lane + 64 * r : 0;
    qi[r] = q / P.nq;
    qj[r] = q - qi[r] * P.nq;
    fti[r] = grid_frac(P, qi[r]);
    ftj[r] = grid_frac(P, qj[r]);
  }
  const double flane = grid_frac(P, lane < P.nq ? lane : 0);
  for (; it < cnt_items; it += nw) {
    const SlotRec r = rn;
    const float4 pt = pn;
    if (it + nw < cnt_items) {
      rn = rnn;
      if (lane < rn.fr.n) pn = staged[rn.off + lane];
    }
    if (it + 2 * nw < cnt_items) rnn = recs[slots ? slots[it + 2 * nw] : it + 2 * nw];
    const FrameRec& fr = r.fr;
    const RotRec* rot = rots ? rots + (slots ? slots[it] : it) : nullptr;
    const int v = r.v;
    const int n = fr.n;
    const int ax = fr.axes & 3, u = (fr.axes >> 2) & 3, wax = (fr.axes >> 4) & 3;
    const int cnt = r.cnt;
    const T lam = (T)fr.lam;
    // this lane's data point (lanes < n)
    T xu = 0, xw = 0, fv = 0, nz = 0;
    if (lane < n) {
      double du, dw, df;
      local_point(P, fr, rot, pt, &du, &dw, &df);
      xu = (T)du;
      xw = (T)dw;
      fv = (T)df;
      nz = (T)pt.w;
      if constexpr (kRefine) {
        s_xd[wid][lane] = du;
        s_xd[wid][NMAX + lane] = dw;
        s_xd[wid][2 * NMAX + lane] = df;
      }
    }
    // this lane's query points q = lane + 64 r (r < QR, q < m): row i, column j of the grid
    float gu[QR], gwv[QR];
#pragma unroll
    for (int r = 0; r < QR; ++r) coords_from_frac(P, fr, fti[r], ftj[r], &gu[r], &gwv[r]);
    const bool dlane = lane < n;

    // Kernel entries with few exponentials. The query entries factor as
    // kappa(x*_q, x_c) = s_f^2 Eu[i][c] Ew[j][c], Eu[i][c] = exp(-lam (u*_i - u_c)^2),
    // so the wave builds the two nq x n tables; for n <= 32 the symmetric K
    // is built from its upper triangle. Both are spread over all 64 lanes and
    // exchanged through this wavefront's LDS region.
    T* __restrict__ su = s_xu[wid];
    T* __restrict__ sw = s_xw[wid];
    T* __restrict__ tu = s_tab[wid];
    T* __restrict__ tw = s_tab[wid] + NQ * NMAX;
    if (dlane) {
      su[lane] = xu;
      sw[lane] = xw;
    }
    if (lane < P.nq) {
      // grid coordinate i (and j) of the face: the same formula as query_coords
      float gi, gj;
      coords_from_frac(P, fr, flane, flane, &gi, &gj);
      su[NMAX + lane] = (T)((double)gi - fr.anc_u);
      sw[NMAX + lane] = (T)((double)gj - fr.anc_w);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nq = P.nq;
    for (int e = lane; e < nq * n; e += 64) {
      const int c = e / nq, i = e - c * nq;
      const T du = su[NMAX + i] - su[c], dw = sw[NMAX + i] - sw[c];
      tu[e] = k_exp(-(du * du) * lam);
      tw[e] = k_exp(-(dw * dw) * lam);
    }
    if constexpr (kKInLds) {
      // upper triangle (r <= c) folded into an (ne/2) x (ne+1) rectangle, ne = n rounded up to even
      T* __restrict__ Kt = s_K[wid];
      const int ne = (n + 1) & ~1;
      const int half = ne >> 1;
      for (int e = lane; e < half * (ne + 1); e += 64) {
        const int p = e / (ne + 1), k = e - p * (ne + 1);
        int r, c;
        if (k < ne - p) {
          r = p;
          c = p + k;
        } else {
          r = ne - 1 - p;
          c = r + (k - (ne - p));
        }
        if (c < n) {
          const T du = su[r] - su[c], dw = sw[r] - sw[c];
          const T kv = sf2 * k_exp(-(du * du + dw * dw) * lam);
          Kt[c * NMAX + r] = kv;
          Kt[r * NMAX + c] = kv;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // rows: A = query rows (q = lane + 64 r < m), B = data row (lanes < n) with its right-hand side fy
    T A[QR][NMAX], B[NMAX];
    T fy = fv;
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
      if (c < n) {
#pragma unroll
        for (int r = 0; r < QR; ++r) A[r][c] = sf2 * tu[c * nq + qi[r]] * tw[c * nq + qj[r]];
        T kb = 0;
        if constexpr (kKInLds) {
          // only data lanes (lane < n <= NMAX) read, so the index stays inside this wavefront's region
          if (dlane) kb = s_K[wid][c * NMAX + lane];
        } else {
          const T eu = xu - su[c], ew = xw - sw[c];
          kb = sf2 * k_exp(-(eu * eu + ew * ew) * lam);
        }
        B[c] = dlane ? kb + (c == lane ? nz : (T)0) : (T)0;
      } else {
#pragma unroll
        for (int r = 0; r < QR; ++r) A[r][c] = 0;
        B[c] = 0;
      }
      // keep the table loads of later columns from being hoisted (register pressure)
      if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    // the LDS region is rewritten for the next voxel only after every lane has read it
    __builtin_amdgcn_wave_barrier();
    T var[QR], mean[QR], tA[QR];
#pragma unroll
    for (int r = 0; r < QR; ++r) {
      var[r] = sf2;
      mean[r] = 0;
    }
    T minpiv = (T)FLT_MAX, score = 0;
    T dself = 1, yself = 0;  // this lane's pivot d_l and y_l
    T* __restrict__ sL = s_K[wid];  // FP32 pass: column j of the unit factor L at sL[j * NMAX + i]
    for (int j = 0; j < n; ++j) {
      const T cjB = B[0];
      const T d = bcast(cjB, j);
      const T y = bcast(fy, j);  // y_j = (L^-1 f~)_j, final once step j is reached
      const T inv = recip(d);
      const T tB = cjB * inv;
      if constexpr (kRefine) {
        if (lane == j) {
          dself = d;
          yself = y;
        }
        if (lane > j && lane < n) sL[j * NMAX + lane] = tB;  // K was read from this region before step 0
      }
#pragma unroll
      for (int r = 0; r < QR; ++r) {
        const T cjA = A[r][0];
        tA[r] = cjA * inv;
        var[r] -= tA[r] * cjA;
        mean[r] += tA[r] * y;
      }
      fy -= tB * y;
      minpiv = d < minpiv ? d : minpiv;
      score += (y < 0 ? -y : y) * inv;
      const int Lc = n - j - 1;
#pragma unroll
      for (int c0 = 0; c0 < NMAX - 1; c0 += 8) {
        if (c0 < Lc) {
#pragma unroll
          for (int k = c0; k < c0 + 8; ++k) {
            if (k < NMAX - 1) {
              // lane j+1+k holds data row j+1+k; past row n-1 the value is unused
              const T col = bcast(cjB, (j + 1 + k) & 63);
#pragma unroll
              for (int r = 0; r < QR; ++r) A[r][k] = A[r][k + 1] - tA[r] * col;
              B[k] = B[k + 1] - tB * col;
            }
          }
        }
      }
    }
    const bool failed = !(minpiv > (T)0) || !isfinite((double)score);
    // FP32 pass: a voxel whose smallest pivot is small against n s_f^2 (or whose rounding is
    // amplified, score sum_j |y_j| / d_j) refines alpha in FP64 here; a failed factor, or a
    // flagged voxel of a solver shape that keeps no factor, is re-solved in FP64 afterwards
    const bool want = (P.mode == 0 || P.mode == 3) && !failed &&
                      ((double)n * (double)P.sf2 > (double)P.cond_thr * (double)minpiv || score > (T)P.refine_thr);
    const bool refine = kRefine && want;
    const bool to_ref = P.mode == 0 && kHandOff && want;               // -> the refinement pass
    const bool to_fp64 = P.mode == 0 && (failed || (want && !kHandOff));  // -> the FP64 re-solve
    const bool flag = to_ref || to_fp64;
    double meanr[QR];
    if constexpr (kRefine) {
      if (refine) refine_mean<NMAX, QR>(P, fr, s_xd[wid], sL, n, lane, (double)dself, (double)yself, (double)nz,
                                        gu, gwv, meanr);
    }
    float mv_lane = 0.f;
#pragma unroll
    for (int r = 0; r < QR; ++r) {
      const int q = lane + 64 * r;
      if (!flag && q < P.m) {
        const float vv = failed ? __int_as_float(0x7fc00000) : (float)(var[r] > (T)0 ? var[r] : (T)0);
        const double fh = failed ? (double)__int_as_float(0x7fc00000) : fr.mu + (refine ? meanr[r] : (double)mean[r]);
        reinterpret_cast<float4*>(io.out)[(size_t)v * P.m + q] = make_row(P, fr, rot, fh, gu[r], gwv[r], vv);
        mv_lane = fmaxf(mv_lane, failed ? 0.f : vv);
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mv_lane = fmaxf(mv_lane, __shfl_xor(mv_lane, d, 64));
    if (lane == 0)
      finish_voxel(P, io, v, slots ? slots[it] : it, cnt, fr.axes, failed, flag, mv_lane, to_ref ? flist : rlist,
                   to_ref ? fcount : rcount, refine);
  }
}

// ---------------------------------------------------------------------------
// 2b. block solver: one voxel per workgroup, one row per lane
// ---------------------------------------------------------------------------
template <typename T, int NMAX>
__global__ void __launch_bounds__(kBlockThreads) fit_block_kernel(FitParams P, FitArgs io,
                                                                  const SlotRec* __restrict__ recs,
                                                                  const RotRec* __restrict__ rots,
                                                                  const float4* __restrict__ staged,
                                                                  const int32_t* __restrict__ slots,
                                                                  const uint32_t* __restrict__ count,
                                                                  uint32_t* __restrict__ next,
                                                                  int32_t* __restrict__ rlist,
                                                                  uint32_t* __restrict__ rcount) {
  __shared__ T su[NMAX + 4], sw[NMAX + 4], sf[NMAX + 4], sn[NMAX + 4];
  __shared__ __attribute__((aligned(16))) T col[2][NMAX + 8];
  __shared__ T piv[2][2];
  __shared__ double s_frac[kMaxGridSide];  // grid fractions (i + 0.5) / nq, written once
  __shared__ int s_item;
  __shared__ unsigned s_maxvar;
  __shared__ int s_flag;

  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int cnt_items = (int)*count;
  const T sf2 = (T)P.sf2;
  if (tid < P.nq) s_frac[tid] = grid_frac(P, tid);  // read after the first barrier of the loop

  for (;;) {
    if (tid == 0) {
      s_item = (int)atomicAdd(next, 1u);
      s_maxvar = 0u;
      s_flag = 0;
    }
    __syncthreads();
    const int item = s_item;
    if (item >= cnt_items) break;
    const int slot = slots ? slots[item] : item;
    const SlotRec r = recs[slot];
    const FrameRec& fr = r.fr;
    const RotRec* rot = rots ? rots + slot : nullptr;
    const int v = r.v;
    const int n = fr.n;
    const int ax = fr.axes & 3, u = (fr.axes >> 2) & 3, wax = (fr.axes >> 4) & 3;
    const int cnt = r.cnt;
    for (int i = tid; i < n; i += NT) {
      const float4 pt = staged[r.off + i];
      double du, dw, df;
      local_point(P, fr, rot, pt, &du, &dw, &df);
      su[i] = (T)du;
      sw[i] = (T)dw;
      sf[i] = (T)df;
      sn[i] = (T)pt.w;
    }
    __syncthreads();

    const T lam = (T)fr.lam;
    const int qchunk = NT - n;
    bool failed = false;
    for (int q0 = 0; q0 < P.m; q0 += qchunk) {
      // the previous chunk's last step may still be reading the pivot slots
      if (q0 > 0) __syncthreads();
      const bool is_data = tid < n;
      const int q = q0 + tid - n;
      const bool is_query = tid >= n && q < P.m;
      T a[NMAX];
      float gu = 0.f, gwv = 0.f;
      T xu = 0, xw = 0, nz = 0, fy = 0;
      if (is_data) {
        xu = su[tid];
        xw = sw[tid];
        fy = sf[tid];
        nz = sn[tid];
      } else if (is_query) {
        const int qi = q / P.nq;
        coords_from_frac(P, fr, s_frac[qi], s_frac[q - qi * P.nq], &gu, &gwv);
        xu = (T)((double)gu - fr.anc_u);
        xw = (T)((double)gwv - fr.anc_w);
      }
#pragma unroll
      for (int c = 0; c < NMAX; ++c) {
        if (c < n) {
          const T du = xu - su[c], dw = xw - sw[c];
          const T kv = sf2 * k_exp(-(du * du + dw * dw) * lam) + (c == tid ? nz : (T)0);
          a[c] = (is_data || is_query) ? kv : (T)0;
        } else {
          a[c] = 0;
        }
      }
      T var = sf2, mean = 0, minpiv = (T)FLT_MAX, score = 0;
      for (int j = 0; j < n; ++j) {
        const int b = j & 1;
        if (tid == j) {
          piv[b][0] = a[0];
          piv[b][1] = fy;  // y_j, final at its own step
        } else if (is_data && tid > j) {
          col[b][tid - j - 1] = a[0];
        }
        __syncthreads();
        const T d = piv[b][0];
        const T yj = piv[b][1];
        const T inv = recip(d);
        const T t = a[0] * inv;
        minpiv = d < minpiv ? d : minpiv;
        score += (yj < 0 ? -yj : yj) * inv;
        fy -= t * yj;
        if (is_query) {
          var -= t * a[0];
          mean += t * yj;
        }
        const int Lc = n - j - 1;
        const T* cb = col[b];
#pragma unroll
        for (int c0 = 0; c0 < NMAX - 1; c0 += 8) {
          if (c0 < Lc) {
#pragma unroll
            for (int k = c0; k < c0 + 8; ++k)
              if (k < NMAX - 1) a[k] = a[k + 1] - t * cb[k];
          }
        }
      }
      failed = !(minpiv > (T)0) || !isfinite((double)score);
      const bool flag = P.mode == 0 && (failed || score > (T)P.refine_thr);
      if (is_query && !flag) {
        const float vv = failed ? __int_as_float(0x7fc00000) : (float)(var > (T)0 ? var : (T)0);
        const double fh = failed ? (double)__int_as_float(0x7fc00000) : fr.mu + (double)mean;
        reinterpret_cast<float4*>(io.out)[(size_t)v * P.m + q] = make_row(P, fr, rot, fh, gu, gwv, vv);
        if (!failed) atomicMax(&s_maxvar, __float_as_uint(vv));
      }
      if (flag) {
        if (tid == 0) s_flag = 1 + (failed ? 1 : 0);
        break;
      }
    }
    __syncthreads();
    if (tid == 0)
      finish_voxel(P, io, v, slot, cnt, fr.axes, s_flag == 2 || (!s_flag && failed), s_flag != 0,
                   __uint_as_float(s_maxvar), rlist, rcount);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 2c. tiled solver (FP64, n up to 512): one voxel per workgroup of eight
//     wavefronts, 32 x 32 tiles, tile products on the FP64 matrix cores
// ---------------------------------------------------------------------------
// The augmented system is processed one block of 32 rows at a time, data rows
// first, then query rows: left-looking across row blocks and right-looking
// inside one,
//     L(I,J) = (A(I,J) - sum_{K<J} L(I,K) L(J,K)^T) L(J,J)^-T,
// the Cholesky factor of K + S tile by tile. The current row block lives in
// LDS. Finished data tiles L(I,J) and the inverses L(J,J)^-1 of the diagonal
// tiles go to the workgroup's scratch area, stored in matrix-core operand
// order so that a wavefront reads one operand fragment as 512 contiguous
// bytes. The right-hand side gives y = L^-1 f~ one block at a time, query rows
// become z_q = L^-1 k*_q, and
//     var_q = s_f^2 - |z_q|^2,   mean_q = mu + z_q . y      (Eq. (3)).
// Padding rows and columns of the last data block are identity rows, so they
// leave the factor of the real block unchanged.
// Order LDS writes of one wavefront before its later reads (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kTile = 32;
constexpr int kTileThreads = 512;
constexpr int kTileWaves = kTileThreads / 64;
constexpr int kTileDoubles = kTile * kTile;
constexpr int kXS = kTile + 1;  // row stride of the finished-tile buffer
constexpr int kQTiles = 8;             // 16-query column tiles per wavefront in the query product
constexpr int kQGroup = 16 * kQTiles;  // queries per group of the query product
constexpr int kQTabRows = 12;          // grid rows a group of 128 queries spans (at most 11 for n_q <= 16)

__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Accumulator layout of the 16 x 16 x 4 FP64 product: lane l, register k holds
// element (l / 16 + 4 k, l % 16) of the 16 x 16 result.
//
// Element (row, col) of a 32 x 32 tile in operand order: fragment (row half h,
// column quad s) is 64 consecutive doubles, lane l holding (16 h + l % 16, 4 s + l / 16).
__device__ __forceinline__ int frag_pos(int row, int col) {
  return (((row >> 4) * 8 + (col >> 2)) << 6) + (row & 15) + ((col & 3) << 4);
}

// Scratch doubles per workgroup: the lower data tiles and one inverse per diagonal tile.
constexpr size_t tile_scratch_doubles(int npad) {
  return (size_t)((npad / kTile) * (npad / kTile + 1) / 2 + npad / kTile) * kTileDoubles;
}

// Scratch doubles per workgroup of the mixed solver: FP32 lower tiles of L, inverses of the
// diagonal tiles, and the lower tiles of L^-1 twice (row-major, and in matrix-core operand order).
constexpr size_t tile_scratch_doubles_mixed(int npad) {
  return ((size_t)(3 * ((npad / kTile) * (npad / kTile + 1) / 2) + npad / kTile) * kTileDoubles + 1) / 2;
}

// f(std::integral_constant<int, 0>{}), ..., f(std::integral_constant<int, N - 1>{}): a loop whose
// index is a compile-time constant in every iteration.
template <typename F, int... T>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, T...>) {
  (f(std::integral_constant<int, T>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ double sum16(double v) {
#pragma unroll
  for (int d = 8; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <int NPAD>
__global__ void __launch_bounds__(kTileThreads) fit_tile_kernel(FitParams P, FitArgs io,
                                                                const SlotRec* __restrict__ recs,
                                                                const RotRec* __restrict__ rots,
                                                                const float4* __restrict__ staged,
                                                                const uint32_t* __restrict__ count,
                                                                uint32_t* __restrict__ next,
                                                                const int32_t* __restrict__ order,
                                                                double* __restrict__ scratch) {
  constexpr int NB = NPAD / kTile;
  constexpr int LD = NPAD + 2;  // row stride of the row block, in doubles
  // up to 128 points every finished tile and diagonal inverse stays in LDS (no scratch traffic)
  constexpr bool kLdsTiles = NPAD <= 128;
  __shared__ double s_tiles[kLdsTiles ? (NB * (NB + 1) / 2 + NB) * kTileDoubles : 1];
  __shared__ double rb[kTile * LD];
  __shared__ double xb[kTile * kXS];  // the tile finished in the current step
  __shared__ double pu[NPAD], pw[NPAD], pf[NPAD];
  __shared__ float pn[NPAD];
  __shared__ double sy[NPAD];
  __shared__ double srhs[kTile], squ[kTile], sqw[kTile];
  __shared__ double sdc[2 * kTile + 8];  // diagonal-tile column broadcast (lanes >= 32 hold zeros)
  __shared__ double srd[kTile];          // 1 / L_jj of the diagonal tile
  __shared__ double sdy;
  __shared__ int s_item, s_fail;
  __shared__ unsigned s_maxvar;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  double* __restrict__ Lt = kLdsTiles ? s_tiles : scratch + (size_t)blockIdx.x * tile_scratch_doubles(NPAD);
  double* __restrict__ Wt = Lt + (size_t)(NB * (NB + 1) / 2) * kTileDoubles;
  const int cnt_items = (int)*count;
  const double sf2 = (double)P.sf2;

  for (;;) {
    if (tid == 0) {
      s_item = (int)atomicAdd(next, 1u);
      s_fail = 0;
      s_maxvar = 0u;
    }
    __syncthreads();
    if (s_item >= cnt_items) break;
    const int item = order ? order[s_item] : s_item;  // slot of the voxel
    const SlotRec r = recs[item];
    const FrameRec& fr = r.fr;
    const RotRec* rot = rots ? rots + item : nullptr;
    const int n = fr.n;
    const int ax = fr.axes & 3, u = (fr.axes >> 2) & 3, wax = (fr.axes >> 4) & 3;
    const double lam = fr.lam;
    for (int i = tid; i < NPAD; i += kTileThreads) {
      double xu = 0, xw = 0, fv = 0;
      float nz = 0.f;
      if (i < n) {
        const float4 pt = staged[r.off + i];
        local_point(P, fr, rot, pt, &xu, &xw, &fv);
        nz = pt.w;
      }
      pu[i] = xu;
      pw[i] = xw;
      pf[i] = fv;
      pn[i] = nz;
    }
    const int nbd = (n + kTile - 1) / kTile;
    const int nbe = (P.m + kTile - 1) / kTile;
    // entry (rr, c) of row block Ib of the augmented system: K + S for data blocks (identity
    // rows and columns past n), K*^T for query blocks (zero past the grid and past n)
    auto entry = [&](int Ib, int rr, int c) -> double {
      if (Ib < nbd) {
        const int i = Ib * kTile + rr;
        if (i < n && c < n) {
          const double du = pu[i] - pu[c], dw = pw[i] - pw[c];
          return sf2 * exp(-(du * du + dw * dw) * lam) + (i == c ? (double)pn[i] : 0.0);
        }
        return i == c ? 1.0 : 0.0;
      }
      const int q = (Ib - nbd) * kTile + rr;
      if (q < P.m && c < n) {
        const double du = squ[rr] - pu[c], dw = sqw[rr] - pw[c];
        return sf2 * exp(-(du * du + dw * dw) * lam);
      }
      return 0.0;
    };
    // query coordinates of the first query block now: its rows are built in part during the
    // last data block's diagonal phase
    if (tid < kTile) {
      float gu = 0.f, gw = 0.f;
      if (tid < P.m) query_coords(P, fr, tid, &gu, &gw);
      squ[tid] = (double)gu - fr.anc_u;
      sqw[tid] = (double)gw - fr.anc_w;
    }
    int c_pre = 0;  // columns [0, c_pre) of block I were built during the previous diagonal phase
    for (int I = 0; I < nbd + nbe; ++I) {
      const bool data = I < nbd;
      const int ncols = data ? (I + 1) * kTile : nbd * kTile;
      if (I > nbd && tid < kTile) {
        const int q = (I - nbd) * kTile + tid;
        float gu = 0.f, gw = 0.f;
        if (q < P.m) query_coords(P, fr, q, &gu, &gw);
        squ[tid] = (double)gu - fr.anc_u;
        sqw[tid] = (double)gw - fr.anc_w;
      }
      __syncthreads();
      // the block's rows of the augmented system (the columns not built ahead)
      {
        // thread t fills row t % 32, every 16th column from c_pre + t / 32
        const int rr = tid & (kTile - 1);
        for (int c = c_pre + tid / kTile; c < ncols; c += kTileThreads / kTile) rb[rr * LD + c] = entry(I, rr, c);
      }
      c_pre = 0;
      __syncthreads();
      const int jend = data ? I : nbd;
      // operand fragment of L(J,J)^-1 for this wavefront's quarter of X, fetched one step ahead
      // (the fetch of step J + 1 is in flight during step J's updates and barriers)
      double wfn[8];
      if (wid < 4 && jend > 0) {
#pragma unroll
        for (int s = 0; s < 8; ++s) wfn[s] = Wt[(((wid & 1) * 8 + s) << 6) + lane];
      }
      for (int J = 0; J < jend; ++J) {
        // finish tile J: X = A(I,J) L(J,J)^-T, one 16 x 16 quarter on each of
        // wavefronts 0-3, into the tile buffer (the row block is still being read)
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        const int a = (wid >> 1) & 1, b = wid & 1;
        if (wid < 4) {
#pragma unroll
          for (int s = 0; s < 8; ++s) acc = mfma_f64(rb[(a * 16 + l16) * LD + J * kTile + 4 * s + l4], wfn[s], acc);
          if (J + 1 < jend) {
            const double* __restrict__ W = Wt + (size_t)(J + 1) * kTileDoubles;
#pragma unroll
            for (int s = 0; s < 8; ++s) wfn[s] = W[((b * 8 + s) << 6) + lane];
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) xb[(a * 16 + l4 + 4 * k) * kXS + b * 16 + l16] = acc[k];
        }
        __syncthreads();
        if (wid < 4) {
          double* __restrict__ Lij = Lt + (size_t)(I * (I + 1) / 2 + J) * kTileDoubles;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int row = a * 16 + l4 + 4 * k, col = b * 16 + l16;
            rb[row * LD + J * kTile + col] = acc[k];
            if (data) Lij[frag_pos(row, col)] = acc[k];
          }
        }
        // right-looking update of the block's later tiles: A(I,J') -= X L(J',J)^T. With the
        // tiles in scratch a unit is a 32 x 16 column half (both row halves share the operand
        // fragment of L(J',J), fetched once); with the tiles in LDS, a 16 x 16 quarter (twice
        // the units to spread over the wavefronts). The next unit's operand is fetched while
        // the current one runs.
        constexpr int kHalves = kLdsTiles ? 1 : 2;  // row halves per unit
        constexpr int kUnitsPerTile = 4 / kHalves;
        const int jlast = data ? I : nbd - 1;
        const int units = (jlast - J) * kUnitsPerTile;
        int un = wid;
        double bf[8], bn[8];
        auto fetch = [&](int uu, double* dst) {
          const int Jp = J + 1 + uu / kUnitsPerTile, b2 = uu & 1;
          if (data && Jp == I) {  // L(I,J) itself: the tile buffer
#pragma unroll
            for (int s = 0; s < 8; ++s) dst[s] = xb[(b2 * 16 + l16) * kXS + 4 * s + l4];
          } else {
            const double* __restrict__ Lpj = Lt + (size_t)(Jp * (Jp + 1) / 2 + J) * kTileDoubles;
#pragma unroll
            for (int s = 0; s < 8; ++s) dst[s] = Lpj[((b2 * 8 + s) << 6) + lane];
          }
        };
        if (un < units) fetch(un, bf);
        for (; un < units; un += kTileWaves) {
          if (un + kTileWaves < units) fetch(un + kTileWaves, bn);
          const int Jp = J + 1 + un / kUnitsPerTile, b2 = un & 1;
          const int a0 = kHalves == 2 ? 0 : (un >> 1) & 1;  // first row half of the unit
          double* __restrict__ cp = rb + Jp * kTile + b2 * 16 + l16;
          dbl4 c[kHalves];
#pragma unroll
          for (int h = 0; h < kHalves; ++h) {
#pragma unroll
            for (int k = 0; k < 4; ++k) c[h][k] = cp[((a0 + h) * 16 + l4 + 4 * k) * LD];
          }
#pragma unroll
          for (int s = 0; s < 8; ++s) {
#pragma unroll
            for (int h = 0; h < kHalves; ++h) c[h] = mfma_f64(-xb[((a0 + h) * 16 + l16) * kXS + 4 * s + l4], bf[s], c[h]);
          }
#pragma unroll
          for (int h = 0; h < kHalves; ++h) {
#pragma unroll
            for (int k = 0; k < 4; ++k) cp[((a0 + h) * 16 + l4 + 4 * k) * LD] = c[h][k];
          }
#pragma unroll
          for (int s = 0; s < 8; ++s) bf[s] = bn[s];
        }
        __syncthreads();
      }
      if (data) {
        // right-hand side of the block: f~_I - sum_{J<I} L(I,J) y_J, sixteen lanes per row
        {
          const int rr = tid >> 4, sub = tid & 15;
          double t = 0.0;
          for (int c = sub; c < I * kTile; c += 16) t += rb[rr * LD + c] * sy[c];
          t = sum16(t);
          if (sub == 0) srhs[rr] = pf[I * kTile + rr] - t;
        }
        __syncthreads();
        if (wid == 0) {
          // diagonal tile by wavefront 0: LDL^T with lane r holding row r (shifted so
          // that element 0 is the active column), y_I on the fly, L(I,I) = U sqrt(D)
          double B[kTile];
          double fy = lane < kTile ? srhs[lane] : 0.0;
#pragma unroll
          for (int c = 0; c < kTile; ++c) B[c] = lane < kTile ? rb[lane * LD + I * kTile + c] : 0.0;
          bool bad = false;
          // four groups of eight pivot steps: group g reads and updates the 31 - 8 g entries
          // that can still be live in its steps (B[1 .. 31 - j] at step j), not all 31
          static_for<kTile / 8>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            constexpr int R = kTile - 1 - 8 * g;  // entries right of the group's first pivot
            constexpr int H = R / 2;              // read before the reciprocal, so the reads overlap it
#pragma unroll 1
            for (int j = 8 * g; j < 8 * g + 8; ++j) {
              // column j of the remaining rows through LDS (one wavefront: no workgroup barrier)
              const double cj = B[0];
              sdc[lane] = cj;
              if (lane == j) sdy = fy;
              wave_sync();
              double col[R];
#pragma unroll
              for (int k = 0; k < H; ++k) col[k] = sdc[j + 1 + k];
              const double d = sdc[j];
              const double yj = sdy;
              // 1/sqrt(d) from the hardware estimate and two Newton steps (each doubles the
              // correct bits), then 1/d = rs^2 and sqrt(d) = d rs
              double rs = __builtin_amdgcn_rsq(d);
              rs = rs * (1.5 - 0.5 * d * rs * rs);
              rs = rs * (1.5 - 0.5 * d * rs * rs);
              const double inv = rs * rs;
              const double t = cj * inv;
              bad |= !(d > 0.0);
              if (lane == j) {
                rb[lane * LD + I * kTile + j] = d * rs;  // sqrt(d)
                srd[j] = rs;
                sy[I * kTile + j] = yj * rs;
              } else if (lane > j && lane < kTile) {
                rb[lane * LD + I * kTile + j] = cj * rs;
              }
              fy -= t * yj;
#pragma unroll
              for (int k = H; k < R; ++k) col[k] = sdc[j + 1 + k];
#pragma unroll
              for (int k = 0; k < R; ++k) B[k] = B[k + 1] - t * col[k];
              wave_sync();  // every lane has read column j before it is overwritten
            }
          });
          if (bad && lane == 0) s_fail = 1;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          // L(I,I)^-1 by forward substitution, lane k computing column k; the sums
          // run as four independent chains and the division is by the stored 1/L_ii.
          // Entries above the diagonal of a column are exactly zero, so the sums
          // start at zero and the unit right-hand side enters as + 1/L_ii on the
          // diagonal (an identity constant per row would be hoisted out of the
          // voxel loop and spilled).
          if (lane < kTile) {
            double x[kTile];
            const double* __restrict__ Ld = rb + I * kTile;
#pragma unroll
            for (int i = 0; i < kTile; ++i) {
              double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
              for (int j0 = 0; j0 < i; j0 += 8) {
                // eight entries of row i read together, then four independent chains
                double lr[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) lr[e] = j0 + e < i ? Ld[i * LD + j0 + e] : 0.0;
#pragma unroll
                for (int e = 0; e < 8; e += 4) {
                  if (j0 + e < i) s0 -= lr[e] * x[j0 + e];
                  if (j0 + e + 1 < i) s1 -= lr[e + 1] * x[j0 + e + 1];
                  if (j0 + e + 2 < i) s2 -= lr[e + 2] * x[j0 + e + 2];
                  if (j0 + e + 3 < i) s3 -= lr[e + 3] * x[j0 + e + 3];
                }
              }
              const double ri = srd[i];
              x[i] = ((s0 + s1) + (s2 + s3)) * ri + (i == lane ? ri : 0.0);
            }
            double* __restrict__ Wi = Wt + (size_t)I * kTileDoubles;
#pragma unroll
            for (int i = 0; i < kTile; ++i) Wi[frag_pos(i, lane)] = x[i];
          }
        } else if (wid != kTileWaves / 2) {
          // meanwhile six wavefronts (not the one sharing wavefront 0's SIMD) build columns
          // [0, 32 I) of the next block, which no one reads any more in this block (the
          // diagonal phase works on columns [32 I, 32 I + 32))
          const int pc = I * kTile;
          const int w6 = wid < kTileWaves / 2 ? wid - 1 : wid - 2;
          const int rr = lane & (kTile - 1);
          for (int c = 2 * w6 + lane / kTile; c < pc; c += 2 * (kTileWaves - 2)) rb[rr * LD + c] = entry(I + 1, rr, c);
        }
        c_pre = I * kTile;
        __syncthreads();
      } else {
        // query rows of the block: variance and mean, sixteen lanes per row
        const int rr = tid >> 4, sub = tid & 15;
        double zz = 0.0, zy = 0.0;
        for (int c = sub; c < nbd * kTile; c += 16) {
          const double z = rb[rr * LD + c];
          zz += z * z;
          zy += z * sy[c];
        }
        zz = sum16(zz);
        zy = sum16(zy);
        const int q = (I - nbd) * kTile + rr;
        if (sub == 0 && q < P.m) {
          float gu, gw;
          query_coords(P, fr, q, &gu, &gw);
          const bool failed = s_fail != 0;
          const double var = sf2 - zz;
          const float vv = failed ? __int_as_float(0x7fc00000) : (float)(var > 0.0 ? var : 0.0);
          const double fh = failed ? (double)__int_as_float(0x7fc00000) : fr.mu + zy;
          reinterpret_cast<float4*>(io.out)[(size_t)r.v * P.m + q] = make_row(P, fr, rot, fh, gu, gw, vv);
          if (!failed) atomicMax(&s_maxvar, __float_as_uint(vv));
        }
        __syncthreads();
      }
    }
    if (tid == 0)
      finish_voxel(P, io, r.v, item, r.cnt, fr.axes, s_fail != 0, false, __uint_as_float(s_maxvar), nullptr, nullptr);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 2d. mixed-precision tiled solver (n up to 512): the tiled solver's block
//     structure in FP32, the query rows as one product with the formed inverse
// ---------------------------------------------------------------------------
// - K and its Cholesky factor in FP32: tile products on the FP32 matrix cores
//   (16 x 16 x 4), diagonal tiles by LDL^T on one wavefront.
// - L^-1 formed row block by row block as the factor is finished (FP32 matrix
//   cores): L^-1(I,K) = -L(I,I)^-1 sum_{K <= J < I} L(I,J) L^-1(J,K).
// - alpha = L^-T L^-1 f~ by block substitution from the FP32 factor,
//   accumulated in double; when n s_f^2 / min pivot exceeds cond_threshold
//   (small pivots) or the amplification score sum_j |y_j| / d_j exceeds
//   refine_threshold, two refinement steps alpha += (K + S)^-1 (f~ - (K + S) alpha)
//   with the residual in FP64 (kernel entries recomputed in double).
// - mean_q = mu + sum_c kappa(x*_q, x_c) alpha_c in FP64, so the mean does not
//   depend on the reduced-precision products below.
// - z_q = L^-1 k*_q for every query as one product (FP32 matrix cores, no
//   barrier inside a group of 128 queries), var_q = s_f^2 - |z_q|^2. Forming
//   z through the triangular recurrence instead lets rounding compound from
//   block to block; with split-BF16 tile products (hi x hi + hi x lo + lo x hi)
//   that reached 1.3e-3 s_f^2 of variance error on 200-point voxels.
// Data tiles, diagonal inverses and L^-1 go to the workgroup's scratch area.
typedef float flt4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ flt4 mfma_f32(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Operand and accumulator layout of the 16 x 16 x 4 FP32 product: lane l holds A(l % 16, l / 16)
// and B(l / 16, l % 16); register k of the result holds element (4 (l / 16) + k, l % 16).

template <int NPAD>
__global__ void __launch_bounds__(kTileThreads) fit_tile_mixed_kernel(FitParams P, FitArgs io,
                                                                      const SlotRec* __restrict__ recs,
                                                                      const RotRec* __restrict__ rots,
                                                                      const float4* __restrict__ staged,
                                                                      const uint32_t* __restrict__ count,
                                                                      uint32_t* __restrict__ next,
                                                                      const int32_t* __restrict__ order,
                                                                      double* __restrict__ scratch) {
  constexpr int NB = NPAD / kTile;
  constexpr int NT = NB * (NB + 1) / 2;  // lower data tiles
  constexpr int LD = NPAD + 4;           // row stride of the row block, in floats
  constexpr int XS = kTile + 4;
  // the row block and finished tile of the factorisation share LDS with the query product's
  // kernel tables (rows of the group, columns) and its per-wavefront partial sums
  constexpr int kTabRows = kQTabRows + 1;  // the group's grid rows and one zero row
  constexpr int kRowBlock = kTile * LD + kTile * XS;
  constexpr int kTables = NPAD * kTabRows + NPAD * kMaxGridSide + kTileWaves * kQGroup;
  __shared__ __attribute__((aligned(16))) float s_bigf[kRowBlock > kTables ? kRowBlock : kTables];
  float* const rb = s_bigf;
  float* const xb = s_bigf + kTile * LD;
  __shared__ double pu[NPAD], pw[NPAD], pf[NPAD];
  __shared__ float pn[NPAD];
  __shared__ float sy[NPAD];
  __shared__ double sal[NPAD], sz[NPAD];
  __shared__ double sred[16][kTile];
  __shared__ double smq[kMaxGridSide * kMaxGridSide];  // mean of each query
  __shared__ float sT[kTileWaves][kTile * 16];         // per wavefront: a 32 x 16 strip while L^-1 is formed
  __shared__ int s_qoff[kQGroup];                      // table offsets of the group's queries
  __shared__ float srhs[kTile];
  __shared__ float sdcf[2 * kTile + 8];
  __shared__ float srdf[kTile];
  __shared__ float sdyf;
  __shared__ int s_item;
  __shared__ int s_fail;
  __shared__ float s_minpiv;
  __shared__ float s_score;
  __shared__ unsigned s_maxvar;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  // scratch of this workgroup (FP32, 32 x 32 tiles): L row-major, the diagonal inverses, and L^-1
  // row-major (right operand while L^-1 is formed) and in operand order (left operand of the
  // query product); L^-1 tile (I, K) at tile I (I + 1) / 2 + K
  float* __restrict__ Lf = reinterpret_cast<float*>(scratch + (size_t)blockIdx.x * tile_scratch_doubles_mixed(NPAD));
  float* __restrict__ Wf = Lf + (size_t)NT * kTileDoubles;
  float* __restrict__ Vr = Wf + (size_t)NB * kTileDoubles;
  float* __restrict__ Va = Vr + (size_t)NT * kTileDoubles;
  const int cnt_items = (int)*count;
  const double sf2 = (double)P.sf2;
  const float sf2f = P.sf2;

  for (;;) {
    if (tid == 0) {
      s_item = (int)atomicAdd(next, 1u);
      s_fail = 0;
      s_minpiv = FLT_MAX;
      s_score = 0.f;
      s_maxvar = 0u;
    }
    __syncthreads();
    if (s_item >= cnt_items) break;
    const int item = order ? order[s_item] : s_item;  // slot of the voxel
    const SlotRec r = recs[item];
    const FrameRec& fr = r.fr;
    const RotRec* rot = rots ? rots + item : nullptr;
    const int n = fr.n;
    const int ax = fr.axes & 3, u = (fr.axes >> 2) & 3, wax = (fr.axes >> 4) & 3;
    const double lam = fr.lam;
    const float lamf = (float)fr.lam;
    for (int i = tid; i < NPAD; i += kTileThreads) {
      double xu = 0, xw = 0, fv = 0;
      float nz = 0.f;
      if (i < n) {
        const float4 pt = staged[r.off + i];
        local_point(P, fr, rot, pt, &xu, &xw, &fv);
        nz = pt.w;
      }
      pu[i] = xu;
      pw[i] = xw;
      pf[i] = fv;
      pn[i] = nz;
    }
    const int nbd = (n + kTile - 1) / kTile;
    const int nbe = (P.m + kTile - 1) / kTile;
    __syncthreads();

    // ---- data row blocks: FP32 Cholesky tile by tile ----
    for (int I = 0; I < nbd; ++I) {
      const int ncols = (I + 1) * kTile;
      for (int e = tid; e < kTile * ncols; e += kTileThreads) {
        const int rr = e / ncols, c = e - rr * ncols;
        const int i = I * kTile + rr;
        float val;
        if (i < n && c < n) {
          const float du = (float)(pu[i] - pu[c]), dw = (float)(pw[i] - pw[c]);
          val = sf2f * __expf(-(du * du + dw * dw) * lamf) + (i == c ? pn[i] : 0.f);
        } else {
          val = i == c ? 1.f : 0.f;
        }
        rb[rr * LD + c] = val;
      }
      __syncthreads();
      for (int J = 0; J < I; ++J) {
        flt4 acc = {0.f, 0.f, 0.f, 0.f};
        const int a = (wid >> 1) & 1, b = wid & 1;
        if (wid < 4) {
          const float* __restrict__ W = Wf + (size_t)J * kTileDoubles;
#pragma unroll
          for (int s = 0; s < 8; ++s)
            acc = mfma_f32(rb[(a * 16 + l16) * LD + J * kTile + 4 * s + l4], W[(b * 16 + l16) * kTile + 4 * s + l4], acc);
#pragma unroll
          for (int k = 0; k < 4; ++k) xb[(a * 16 + 4 * l4 + k) * XS + b * 16 + l16] = acc[k];
        }
        __syncthreads();
        if (wid < 4) {
          const size_t t = (size_t)(I * (I + 1) / 2 + J) * kTileDoubles;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int row = a * 16 + 4 * l4 + k, col = b * 16 + l16;
            const float v = acc[k];
            rb[row * LD + J * kTile + col] = v;
            Lf[t + row * kTile + col] = v;
          }
        }
        const int units = (I - J) * 4;
        for (int un = wid; un < units; un += kTileWaves) {
          const int Jp = J + 1 + (un >> 2), a2 = (un >> 1) & 1, b2 = un & 1;
          float* __restrict__ cp = rb + Jp * kTile + b2 * 16 + l16;
          flt4 c4;
#pragma unroll
          for (int k = 0; k < 4; ++k) c4[k] = cp[(a2 * 16 + 4 * l4 + k) * LD];
          const float* __restrict__ Bt = Lf + (size_t)(Jp * (Jp + 1) / 2 + J) * kTileDoubles;
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const float bv = Jp == I ? xb[(b2 * 16 + l16) * XS + 4 * s + l4] : Bt[(b2 * 16 + l16) * kTile + 4 * s + l4];
            c4 = mfma_f32(-xb[(a2 * 16 + l16) * XS + 4 * s + l4], bv, c4);
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) cp[(a2 * 16 + 4 * l4 + k) * LD] = c4[k];
        }
        __syncthreads();
      }
      {
        const int rr = tid >> 4, sub = tid & 15;
        float t = 0.f;
        for (int c = sub; c < I * kTile; c += 16) t += rb[rr * LD + c] * sy[c];
#pragma unroll
        for (int d = 8; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
        if (sub == 0) srhs[rr] = (float)pf[I * kTile + rr] - t;
      }
      __syncthreads();
      if (wid == 0) {
        float B[kTile];
        float fy = lane < kTile ? srhs[lane] : 0.f;
#pragma unroll
        for (int c = 0; c < kTile; ++c) B[c] = lane < kTile ? rb[lane * LD + I * kTile + c] : 0.f;
        bool bad = false;
        float mp = FLT_MAX;
        float sc = 0.f;  // sum_j |y_j| / d_j of the unit-diagonal factor (the FP32 amplification score)
        for (int j = 0; j < kTile; ++j) {
          const float cj = B[0];
          sdcf[lane] = cj;
          if (lane == j) sdyf = fy;
          wave_sync();
          float colv[kTile - 1];  // the column up front: the LDS reads overlap the reciprocal
#pragma unroll
          for (int k = 0; k < kTile - 1; ++k) colv[k] = sdcf[j + 1 + k];
          const float d = sdcf[j];
          const float yj = sdyf;
          const float inv = 1.f / d;
          const float rs = sqrtf(inv);
          const float t = cj * inv;
          bad |= !(d > 0.f);
          if (I * kTile + j < n) {
            mp = fminf(mp, d);
            sc += fabsf(yj) * inv;
          }
          if (lane == j) {
            rb[lane * LD + I * kTile + j] = d * rs;
            srdf[j] = rs;
            sy[I * kTile + j] = yj * rs;
          } else if (lane > j && lane < kTile) {
            rb[lane * LD + I * kTile + j] = cj * rs;
          }
          fy -= t * yj;
#pragma unroll
          for (int k = 0; k < kTile - 1; ++k) B[k] = B[k + 1] - t * colv[k];
          B[kTile - 1] = 0.f;
          wave_sync();
        }
        if (lane == 0) {
          if (bad) s_fail = 1;
          s_minpiv = fminf(s_minpiv, mp);
          s_score += sc;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < kTile) {
          float x[kTile];
          const float* __restrict__ Ld = rb + I * kTile;
#pragma unroll
          for (int i = 0; i < kTile; ++i) {
            float s0 = 0.f, s1 = 0.f;  // as in the FP64 solver: the unit enters on the diagonal
#pragma unroll
            for (int j = 0; j + 1 < i; j += 2) {
              s0 -= Ld[i * LD + j] * x[j];
              s1 -= Ld[i * LD + j + 1] * x[j + 1];
            }
            if (i & 1) s0 -= Ld[i * LD + i - 1] * x[i - 1];
            const float ri = srdf[i];
            x[i] = (s0 + s1) * ri + (i == lane ? ri : 0.f);
          }
          const size_t t = (size_t)I * kTileDoubles;
#pragma unroll
          for (int i = 0; i < kTile; ++i) Wf[t + i * kTile + lane] = x[i];
        }
      }
      __syncthreads();
      // row block I of L^-1: the diagonal tile is L(I,I)^-1; for K < I,
      //   L^-1(I,K) = -L(I,I)^-1 sum_{K <= J < I} L(I,J) L^-1(J,K),
      // one 32 x 16 strip (K, column half b2) per unit on the FP32 matrix cores
      {
        const float* __restrict__ Wi = Wf + (size_t)I * kTileDoubles;
        float* __restrict__ Vi = Vr + (size_t)(I * (I + 1) / 2 + I) * kTileDoubles;
        float* __restrict__ Ai = Va + (size_t)(I * (I + 1) / 2 + I) * kTileDoubles;
        for (int e = tid; e < kTileDoubles; e += kTileThreads) {
          const int row = e >> 5, col = e & 31;
          Vi[e] = Wi[e];
          Ai[frag_pos(row, col)] = Wi[e];
        }
      }
      for (int un = wid; un < 2 * I; un += kTileWaves) {
        const int K = un >> 1, b2 = un & 1;
        flt4 t0 = {0.f, 0.f, 0.f, 0.f}, t1 = {0.f, 0.f, 0.f, 0.f};
        for (int J = K; J < I; ++J) {
          const float* __restrict__ Vj = Vr + (size_t)(J * (J + 1) / 2 + K) * kTileDoubles + b2 * 16 + l16;
#pragma unroll
          for (int s8 = 0; s8 < 8; ++s8) {
            const float bv = Vj[(4 * s8 + l4) * kTile];
            t0 = mfma_f32(rb[l16 * LD + J * kTile + 4 * s8 + l4], bv, t0);
            t1 = mfma_f32(rb[(16 + l16) * LD + J * kTile + 4 * s8 + l4], bv, t1);
          }
        }
        // the sum through this wavefront's LDS strip, then the product with L(I,I)^-1
        float* __restrict__ st = sT[wid];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          st[(4 * l4 + k) * 16 + l16] = t0[k];
          st[(16 + 4 * l4 + k) * 16 + l16] = t1[k];
        }
        wave_sync();
        const float* __restrict__ Wi = Wf + (size_t)I * kTileDoubles;
        flt4 o0 = {0.f, 0.f, 0.f, 0.f}, o1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
          const float tb = st[(4 * s8 + l4) * 16 + l16];
          if (s8 < 4) o0 = mfma_f32(Wi[l16 * kTile + 4 * s8 + l4], tb, o0);  // rows 0-15: zero right of 16
          o1 = mfma_f32(Wi[(16 + l16) * kTile + 4 * s8 + l4], tb, o1);
        }
        wave_sync();  // the strip is rewritten by this wavefront's next unit
        float* __restrict__ Vi = Vr + (size_t)(I * (I + 1) / 2 + K) * kTileDoubles;
        float* __restrict__ Ai = Va + (size_t)(I * (I + 1) / 2 + K) * kTileDoubles;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int col = b2 * 16 + l16, r0 = 4 * l4 + k, r1 = 16 + 4 * l4 + k;
          Vi[r0 * kTile + col] = -o0[k];
          Vi[r1 * kTile + col] = -o1[k];
          Ai[frag_pos(r0, col)] = -o0[k];
          Ai[frag_pos(r1, col)] = -o1[k];
        }
      }
      __syncthreads();
    }

    // ---- alpha: block back substitution L^T alpha = y, then the optional FP64 refinement ----
    // back(src, dst): dst = L^-T src (double accumulation, FP32 factor); rows >= n of src are 0
    auto back = [&](const float* ysrc, const double* dsrc, double* dst) {
      for (int I = nbd - 1; I >= 0; --I) {
        const int c = tid & 31, g = tid >> 5;
        double t = 0.0;
        for (int J = I + 1; J < nbd; ++J) {
          const float* __restrict__ T = Lf + (size_t)(J * (J + 1) / 2 + I) * kTileDoubles;
          for (int rr = g; rr < kTile; rr += 16) t += (double)T[rr * kTile + c] * dst[J * kTile + rr];
        }
        sred[g][c] = t;
        __syncthreads();
        if (tid < kTile) {
          double s = ysrc ? (double)ysrc[I * kTile + tid] : dsrc[I * kTile + tid];
#pragma unroll
          for (int k = 0; k < 16; ++k) s -= sred[k][tid];
          sred[0][tid] = s;  // t_I
        }
        __syncthreads();
        if (tid < kTile) {
          const float* __restrict__ W = Wf + (size_t)I * kTileDoubles;
          double s = 0.0;
          for (int cc = tid; cc < kTile; ++cc) s += (double)W[cc * kTile + tid] * sred[0][cc];
          dst[I * kTile + tid] = s;
        }
        __syncthreads();
      }
    };
    back(sy, nullptr, sal);
    const bool refine = !s_fail && ((double)n * sf2 / (double)s_minpiv > (double)P.cond_thr ||
                                    !(s_score <= P.refine_thr));
    // Two steps: one step with an FP32 factor leaves about (kappa eps_32)^2 of alpha's relative
    // error, and kappa = n s_f^2 / sigma^2 reaches 2.6e5 at 256 points (one step left 1.5e-4 m of
    // mean error on such voxels); the second takes it to (kappa eps_32)^3.
    for (int step = 0; refine && step < 2; ++step) {
      // residual f~ - (K + S) alpha in FP64, one row per thread
      for (int i = tid; i < nbd * kTile; i += kTileThreads) {
        double rsd = 0.0;
        if (i < n) {
          rsd = pf[i] - (double)pn[i] * sal[i];
          for (int c = 0; c < n; ++c) {
            const double du = pu[i] - pu[c], dw = pw[i] - pw[c];
            rsd -= sf2 * exp(-(du * du + dw * dw) * lam) * sal[c];
          }
        }
        sz[i] = rsd;
      }
      __syncthreads();
      // forward substitution L w = residual, in place in sz
      for (int I = 0; I < nbd; ++I) {
        const int rr = tid & 31, g = tid >> 5;
        double t = 0.0;
        for (int J = 0; J < I; ++J) {
          const float* __restrict__ T = Lf + (size_t)(I * (I + 1) / 2 + J) * kTileDoubles;
          for (int c = g; c < kTile; c += 16) t += (double)T[rr * kTile + c] * sz[J * kTile + c];
        }
        sred[g][rr] = t;
        __syncthreads();
        if (tid < kTile) {
          double s = sz[I * kTile + tid];
#pragma unroll
          for (int k = 0; k < 16; ++k) s -= sred[k][tid];
          sred[0][tid] = s;
        }
        __syncthreads();
        if (tid < kTile) {
          const float* __restrict__ W = Wf + (size_t)I * kTileDoubles;
          double s = 0.0;
          for (int cc = 0; cc <= tid; ++cc) s += (double)W[tid * kTile + cc] * sred[0][cc];
          sz[I * kTile + tid] = s;
        }
        __syncthreads();
      }
      // back substitution, in place: delta = L^-T w
      back(nullptr, sz, sz);
      for (int i = tid; i < nbd * kTile; i += kTileThreads) sal[i] += sz[i];
      __syncthreads();
    }

    // ---- queries: the mean from alpha in FP64, the variance from z = L^-1 K* ----
    // mean_q = mu + k*_q^T alpha with kernel entries in double, four threads per query
    for (int q0 = 0; q0 < P.m; q0 += kTileThreads / 4) {
      const int q = q0 + (tid >> 2), sub = tid & 3;
      double macc = 0.0;
      if (q < P.m) {
        float gu, gw;
        query_coords(P, fr, q, &gu, &gw);
        const double qu = (double)gu - fr.anc_u, qw = (double)gw - fr.anc_w;
        for (int c = sub; c < n; c += 4) {
          const double du = qu - pu[c], dw = qw - pw[c];
          macc += sf2 * exp(-(du * du + dw * dw) * lam) * sal[c];
        }
      }
      macc += __shfl_xor(macc, 1, 64);
      macc += __shfl_xor(macc, 2, 64);
      if (q < P.m && sub == 0) smq[q] = macc;
    }
    // var_q = s_f^2 - |z_q|^2 with z_q = L^-1 k*_q as one product with the formed inverse on the
    // FP32 matrix cores, 128 queries at a time: each wavefront takes whole 16-row strips of
    // L^-1 (zig-zag order, pairing long and short strips) against all eight 16-query column
    // tiles of the group, so one operand fragment of L^-1 feeds eight products; no barrier
    // inside a group. The cross-covariance entries come from two tables (the grid is
    // separable): k*(c, q) = [s_f^2 exp(-lam du_i^2)] [exp(-lam dw_j^2)], each rounded to
    // float from double. Each product's error stays that of one FP32 matrix product (no
    // recurrence through earlier blocks); partial sums combine across lanes by shuffles and
    // across wavefronts in a fixed order.
    {
      float* const tu = s_bigf;                           // [c][kTabRows]: row factors of the group
      float* const tw = s_bigf + NPAD * kTabRows;         // [c][16]: column factors
      float* const part = tw + NPAD * kMaxGridSide;       // [wavefront][query of the group]
      const int nq = P.nq;
      const int ns = (n + 15) >> 4;  // strips holding data rows; the rest of z is zero
      const int n4 = (n + 3) & ~3;   // table columns from n on are zero
      for (int e = tid; e < NPAD * kMaxGridSide; e += kTileThreads) {
        const int c = e >> 4, j = e & 15;
        float v = 0.f;
        if (c < n && j < nq) {
          float gu, gw;
          coords_from_frac(P, fr, grid_frac(P, 0), grid_frac(P, j), &gu, &gw);
          const double dw = ((double)gw - fr.anc_w) - pw[c];
          v = (float)exp(-(dw * dw) * lam);
        }
        tw[e] = v;
      }
      for (int q0 = 0; q0 < P.m; q0 += kQGroup) {
        const int i0 = q0 / nq;
        const int irows = ((q0 + kQGroup < P.m ? q0 + kQGroup : P.m) - 1) / nq - i0 + 1;
        for (int e = tid; e < NPAD * kTabRows; e += kTileThreads) {
          const int c = e / kTabRows, i = e - c * kTabRows;
          float v = 0.f;
          if (c < n && i < irows) {
            float gu, gw;
            coords_from_frac(P, fr, grid_frac(P, i0 + i), grid_frac(P, 0), &gu, &gw);
            const double du = ((double)gu - fr.anc_u) - pu[c];
            v = (float)(sf2 * exp(-(du * du) * lam));
          }
          tu[e] = v;
        }
        // with n_q = 16 a group is eight whole grid rows: row factor t, column factor l % 16
        const bool full16 = nq == kMaxGridSide;
        if (!full16 && tid < kQGroup) {
          const int q = q0 + tid;
          s_qoff[tid] = q < P.m ? ((q / nq - i0) << 8) | (q % nq) : (kQTabRows << 8);  // past the grid: zero row
        }
        __syncthreads();
        float zz[kQTiles];
#pragma unroll
        for (int t = 0; t < kQTiles; ++t) zz[t] = 0.f;
        auto strips = [&](auto full16_tag) {
          constexpr bool FULL16 = decltype(full16_tag)::value;
          for (int rr = 0; kTileWaves * rr < ns; ++rr) {
            const int sx = kTileWaves * rr + ((rr & 1) ? kTileWaves - 1 - wid : wid);
            if (sx >= ns) continue;
            const int I = sx >> 1;
            const int kend = (16 * sx + 16 < n4 ? 16 * sx + 16 : n4) >> 2;  // steps of 4 columns
            const float* __restrict__ A0 =
                Va + (size_t)(I * (I + 1) / 2) * kTileDoubles + (((sx & 1) * 8) << 6) + lane;
            auto afrag = [&](int ks) { return A0[(size_t)(ks >> 3) * kTileDoubles + ((ks & 7) << 6)]; };
            flt4 acc[kQTiles];
#pragma unroll
            for (int t = 0; t < kQTiles; ++t) acc[t] = flt4{0.f, 0.f, 0.f, 0.f};
            float an1 = afrag(0);
            float an2 = kend > 1 ? afrag(1) : 0.f;
            for (int ks = 0; ks < kend; ++ks) {
              const float a = an1;
              an1 = an2;
              an2 = ks + 2 < kend ? afrag(ks + 2) : 0.f;
              const int c = 4 * ks + l4;
              const float* __restrict__ tuc = tu + c * kTabRows;
              const float* __restrict__ twc = tw + c * kMaxGridSide;
              if constexpr (FULL16) {
                const float wv = twc[l16];
#pragma unroll
                for (int t = 0; t < kQTiles; ++t) acc[t] = mfma_f32(a, tuc[t] * wv, acc[t]);
              } else {
#pragma unroll
                for (int t = 0; t < kQTiles; ++t) {
                  const int o = s_qoff[16 * t + l16];
                  acc[t] = mfma_f32(a, tuc[o >> 8] * twc[o & 255], acc[t]);
                }
              }
            }
            // lane l, register k holds z of row 16 sx + 4 (l / 16) + k for query column l % 16 of tile t
#pragma unroll
            for (int t = 0; t < kQTiles; ++t)
#pragma unroll
              for (int k = 0; k < 4; ++k) zz[t] += acc[t][k] * acc[t][k];
          }
        };
        if (full16)
          strips(std::integral_constant<bool, true>{});
        else
          strips(std::integral_constant<bool, false>{});
#pragma unroll
        for (int t = 0; t < kQTiles; ++t) {
          zz[t] += __shfl_xor(zz[t], 16, 64);
          zz[t] += __shfl_xor(zz[t], 32, 64);
          if (l4 == 0) part[wid * kQGroup + 16 * t + l16] = zz[t];
        }
        __syncthreads();
        if (tid < kQGroup && q0 + tid < P.m) {
          const int q = q0 + tid;
          double zzs = 0.0;
#pragma unroll
          for (int w = 0; w < kTileWaves; ++w) zzs += (double)part[w * kQGroup + tid];
          float gu, gw;
          query_coords(P, fr, q, &gu, &gw);
          const bool failed = s_fail != 0;
          const double var = sf2 - zzs;
          const float vv = failed ? __int_as_float(0x7fc00000) : (float)(var > 0.0 ? var : 0.0);
          const double fh = failed ? (double)__int_as_float(0x7fc00000) : fr.mu + smq[q];
          reinterpret_cast<float4*>(io.out)[(size_t)r.v * P.m + q] = make_row(P, fr, rot, fh, gu, gw, vv);
          if (!failed) atomicMax(&s_maxvar, __float_as_uint(vv));
        }
        __syncthreads();  // the tables and partial sums are rewritten for the next group
      }
    }
    if (tid == 0) {
      finish_voxel(P, io, r.v, item, r.cnt, fr.axes, s_fail != 0, false, __uint_as_float(s_maxvar), nullptr,
                   nullptr);
      if (refine) io.status[r.v] |= (uint8_t)VGPR_ST_REFINED;
    }
    __syncthreads();
  }
}

template <typename K>
int occupancy(K kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

// Timing family of each launch: pass (FP32, FP64 re-solve, FP64 only) and bucket capacity.
const char* const kFam[3][kNumBuckets] = {
    {"fit_f32_n16", "fit_f32_n32", "fit_f32_n64", "fit_f32_n96", "fit_f32_n128", "fit_f32_n256", "fit_f32_n512"},
    {"refine_f64_n16", "refine_f64_n32", "refine_f64_n64", "refine_f64_n96", "refine_f64_n128", "refine_f64_n256",
     "refine_f64_n512"},
    {"fit_f64_n16", "fit_f64_n32", "fit_f64_n64", "fit_f64_n96", "fit_f64_n128", "fit_f64_n256", "fit_f64_n512"}};
const char* const kFamRefine = "refine_f32_n16";
const char* const kFamMixed[kNumBuckets] = {"fit_mix_n16", "fit_mix_n32", "fit_mix_n64", "fit_mix_n96",
                                            "fit_mix_n128", "fit_mix_n256", "fit_mix_n512"};


struct Launch {
  hipStream_t stream;
  int grid_scale;            // x 1/4 of the resident workgroups
  const SlotRec* recs;
  const RotRec* rots;        // frame_mode 1: rotated frames parallel to recs, else null
  const int32_t* slots;      // nullable: item -> slot indirection (re-solve lists)
  const uint32_t* count;
  uint32_t* next;
  int32_t* rlist;
  uint32_t* rcount;
  int64_t max_items;
  const char* fam;
  int32_t* flist = nullptr;   // FP32 pass: voxels for the refinement pass
  uint32_t* fcount = nullptr;
};

template <typename T, int NMAX, int QR, bool REF = false>
vgpr_status launch_wave(vgpr_ctx* ctx, const FitParams& P, const FitArgs& io, const float4* staged,
                        const Launch& l) {
  static int per_cu = -1;
  if (per_cu < 0) per_cu = occupancy(fit_wave_kernel<T, NMAX, QR, REF>, kWaveThreads);
  int64_t grid = (int64_t)per_cu * ctx->cu_count * l.grid_scale / 4;
  const int64_t need = (l.max_items + kWaveThreads / 64 - 1) / (kWaveThreads / 64);
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  ProfScope ps(ctx, l.fam, l.stream);
  hipLaunchKernelGGL((fit_wave_kernel<T, NMAX, QR, REF>), dim3((unsigned)grid), dim3(kWaveThreads), 0, l.stream, P,
                     io, l.recs, l.rots, staged, l.slots, l.count, l.rlist, l.rcount, l.flist, l.fcount);
  VGPR_HIP(ctx, hipGetLastError());
  return VGPR_OK;
}

template <typename T, int NMAX>
vgpr_status launch_block(vgpr_ctx* ctx, const FitParams& P, const FitArgs& io, const float4* staged,
                         const Launch& l) {
  int threads = NMAX + P.m;
  if (threads > kBlockThreads) threads = kBlockThreads;
  threads = (threads + 63) & ~63;
  static int per_cu = -1;
  if (per_cu < 0) per_cu = occupancy(fit_block_kernel<T, NMAX>, kBlockThreads);
  int64_t grid = (int64_t)per_cu * (kBlockThreads / threads) * ctx->cu_count * l.grid_scale / 4;
  if (grid > l.max_items) grid = l.max_items;
  if (grid < 1) grid = 1;
  ProfScope ps(ctx, l.fam, l.stream);
  hipLaunchKernelGGL((fit_block_kernel<T, NMAX>), dim3((unsigned)grid), dim3(threads), 0, l.stream, P, io,
                     l.recs, l.rots, staged, l.slots, l.count, l.next, l.rlist, l.rcount);
  VGPR_HIP(ctx, hipGetLastError());
  return VGPR_OK;
}

template <int NPAD, bool MIXED>
int tile_per_cu() {
  static int per_cu = -1;
  if (per_cu < 0)
    per_cu = MIXED ? occupancy(fit_tile_mixed_kernel<NPAD>, kTileThreads) : occupancy(fit_tile_kernel<NPAD>, kTileThreads);
  return per_cu;
}

int tile_per_cu_of(int b, bool mixed) {
  switch (kBucketCap[b]) {
    case 64: return mixed ? tile_per_cu<64, true>() : tile_per_cu<64, false>();
    case 96: return mixed ? tile_per_cu<96, true>() : tile_per_cu<96, false>();
    case 128: return mixed ? tile_per_cu<128, true>() : tile_per_cu<128, false>();
    case 256: return mixed ? tile_per_cu<256, true>() : tile_per_cu<256, false>();
    default: return mixed ? tile_per_cu<512, true>() : tile_per_cu<512, false>();
  }
}

// Buckets from this one on run the tiled solvers.
int first_tile_bucket(const vgpr_ctx* ctx) { return ctx->tune.tile_first_bucket; }

// Workgroups of a tiled solver for bucket b: at most one resident wave of them,
// since each holds a scratch area.
int tile_grid(const vgpr_ctx* ctx, int b, bool mixed, int grid_scale) {
  const int gs = grid_scale < 4 ? grid_scale : 4;
  const int64_t g = (int64_t)tile_per_cu_of(b, mixed) * ctx->cu_count * gs / 4;
  return g < 1 ? 1 : (int)g;
}

size_t tile_bucket_bytes(const vgpr_ctx* ctx, int b, bool mixed) {
  if (!mixed && kBucketCap[b] <= 128) return 0;  // the FP64 tiled solver keeps these tiles in LDS
  const size_t per = mixed ? tile_scratch_doubles_mixed(kBucketCap[b]) : tile_scratch_doubles(kBucketCap[b]);
  return (size_t)tile_per_cu_of(b, mixed) * ctx->cu_count * per * sizeof(double);
}

template <bool MIXED>
void launch_tile_kernel(int npad, dim3 g, dim3 t, hipStream_t s, const FitParams& P, const FitArgs& io,
                        const Launch& l, const float4* staged, double* scratch) {
#define VGPR_TILE_CASE(NP)                                                                                   \
  case NP:                                                                                                   \
    if (MIXED)                                                                                               \
      hipLaunchKernelGGL(fit_tile_mixed_kernel<NP>, g, t, 0, s, P, io, l.recs, l.rots, staged, l.count, l.next,     \
                         l.slots, scratch);                                                                   \
    else                                                                                                     \
      hipLaunchKernelGGL(fit_tile_kernel<NP>, g, t, 0, s, P, io, l.recs, l.rots, staged, l.count, l.next, l.slots,  \
                         scratch);                                                                            \
    break;
  switch (npad) {
    VGPR_TILE_CASE(64)
    VGPR_TILE_CASE(96)
    VGPR_TILE_CASE(128)
    VGPR_TILE_CASE(256)
    default:
    VGPR_TILE_CASE(512)
  }
#undef VGPR_TILE_CASE
}

vgpr_status launch_tile(vgpr_ctx* ctx, int b, bool mixed, const FitParams& P, const FitArgs& io,
                        const float4* staged, const Launch& l, double* scratch) {
  int64_t grid = tile_grid(ctx, b, mixed, l.grid_scale);
  if (grid > l.max_items) grid = l.max_items;
  ProfScope ps(ctx, l.fam, l.stream);
  if (mixed)
    launch_tile_kernel<true>(kBucketCap[b], dim3((unsigned)grid), dim3(kTileThreads), l.stream, P, io, l, staged, scratch);
  else
    launch_tile_kernel<false>(kBucketCap[b], dim3((unsigned)grid), dim3(kTileThreads), l.stream, P, io, l, staged, scratch);
  VGPR_HIP(ctx, hipGetLastError());
  return VGPR_OK;
}

// One solver launch for bucket b, in precision T.
template <typename T>
vgpr_status launch_bucket(vgpr_ctx* ctx, int b, bool wave, const FitParams& P, const FitArgs& io,
                          const float4* staged, const Launch& l) {
  if (wave) {
    // query rows per lane; combinations that do not fit the register file fall back to the block solver
    const int qr = P.m <= 64 ? 1 : (P.m <= 128 ? 2 : 4);
    if (b == 0) {
      if (qr == 1) return launch_wave<T, 16, 1>(ctx, P, io, staged, l);
      if (qr == 2) return launch_wave<T, 16, 2>(ctx, P, io, staged, l);
      return launch_wave<T, 16, 4>(ctx, P, io, staged, l);
    }
    if (b == 1) {
      if (qr == 1) return launch_wave<T, 32, 1>(ctx, P, io, staged, l);
      if (qr == 2) return launch_wave<T, 32, 2>(ctx, P, io, staged, l);
      if constexpr (sizeof(T) == 4) return launch_wave<T, 32, 4>(ctx, P, io, staged, l);
    }
    if (b == 2 && qr == 1) return launch_wave<T, 64, 1>(ctx, P, io, staged, l);
  }
  switch (b) {
    case 0: return launch_block<T, 16>(ctx, P, io, staged, l);
    case 1: return launch_block<T, 32>(ctx, P, io, staged, l);
    case 2: return launch_block<T, 64>(ctx, P, io, staged, l);
    case 3: return launch_block<T, 96>(ctx, P, io, staged, l);
    default: return launch_block<T, 128>(ctx, P, io, staged, l);
  }
}

// The refinement pass of the FP32 16-point wave bucket over the voxels its first pass flagged.
vgpr_status launch_refine(vgpr_ctx* ctx, const FitParams& P, const FitArgs& io, const float4* staged,
                          const Launch& l) {
  const int qr = P.m <= 64 ? 1 : (P.m <= 128 ? 2 : 4);
  if (qr == 1) return launch_wave<float, 16, 1, true>(ctx, P, io, staged, l);
  if (qr == 2) return launch_wave<float, 16, 2, true>(ctx, P, io, staged, l);
  return launch_wave<float, 16, 4, true>(ctx, P, io, staged, l);
}

}  // namespace

size_t fit_work_bytes(const vgpr_ctx* ctx, int64_t n_vox, int64_t n_pts, const vgpr_params* p) {
  size_t tiles = 0;
  const bool mixed = p->precision == VGPR_PREC_MIXED;
  for (int b = first_tile_bucket(ctx); b < kNumBuckets; ++b)
    if (p->max_pts > kBucketCap[b - 1]) tiles += Carver::round(tile_bucket_bytes(ctx, b, mixed));
  const size_t rot_bytes = p->frame_mode == 1 ? Carver::round(sizeof(RotRec) * (size_t)n_vox * kNumBuckets) : 0;
  return rot_bytes + Carver::round(sizeof(SlotRec) * (size_t)n_vox * kNumBuckets) + Carver::round(sizeof(float4) * (size_t)n_pts) +
         Carver::round(sizeof(int32_t) * (size_t)n_vox) + Carver::round(sizeof(int4) * (size_t)n_vox) +
         2 * Carver::round(sizeof(int32_t) * (size_t)n_vox * kNumBuckets) +
         Carver::round(sizeof(uint32_t) * 64) + tiles + 4096;
}

vgpr_status fit_predict_impl(vgpr_ctx* ctx, const FitArgs& a, const vgpr_params* p, size_t work_offset,
                             char* fixed_work) {
  if (a.n_vox < 0 || a.n_vox >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_INVALID, "n_vox out of range");
  if (a.n_pts < 0 || a.n_pts >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_INVALID, "n_pts out of range");
  if (a.n_vox == 0) return VGPR_OK;
  if (!a.xyz || !a.keys || !a.offsets || !a.counts || !a.out || !a.axis || !a.status)
    return fail(ctx, VGPR_E_INVALID, "null device pointer");
  if (reinterpret_cast<uintptr_t>(a.out) & 15) return fail(ctx, VGPR_E_INVALID, "d_out must be 16-byte aligned");
  const int m = p->grid_side * p->grid_side;
  vgpr_status st = VGPR_OK;
  if (!fixed_work) {
    st = reserve_work(ctx, work_offset + fit_work_bytes(ctx, a.n_vox, a.n_pts, p));
    if (st != VGPR_OK) return st;
  }
  Carver cv(fixed_work ? fixed_work : static_cast<char*>(ctx->work.ptr) + work_offset);
  RotRec* rots = p->frame_mode == 1 ? cv.take<RotRec>((size_t)a.n_vox * kNumBuckets) : nullptr;
  SlotRec* recs = cv.take<SlotRec>((size_t)a.n_vox * kNumBuckets);
  float4* staged = cv.take<float4>((size_t)a.n_pts);
  int32_t* nan_list = cv.take<int32_t>((size_t)a.n_vox);
  int4* big_list = cv.take<int4>((size_t)a.n_vox);
  int32_t* rlists = cv.take<int32_t>((size_t)a.n_vox * kNumBuckets);
  int32_t* flists = cv.take<int32_t>((size_t)a.n_vox * kNumBuckets);
  // [0,8) list counts, [8,15) fetch, [16,23) re-solve counts, [24,31) fetch, [32,39) refinement counts, [40,47) fetch,
  // 48 voxels of more than kPrepCoop points, 49 the merged 256/512-point list
  uint32_t* ctr = cv.take<uint32_t>(64);
  double* tile_scratch[kNumBuckets] = {};
  const bool mixed = p->precision == VGPR_PREC_MIXED;
  for (int b = first_tile_bucket(ctx); b < kNumBuckets; ++b)
    if (p->max_pts > kBucketCap[b - 1])
      tile_scratch[b] = cv.take<double>(tile_bucket_bytes(ctx, b, mixed) / sizeof(double));
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, ctx->stream, ctr, 64);

  // the wave solver holds up to four query rows per lane (grids up to 256 points) for voxels of up
  // to 32 points, one row per lane (grids up to 64 points) for voxels of up to 64 points
  auto wave_ok = [&](int b) { return b <= 1 ? m <= 256 : m <= 64; };
  FitParams P;
  P.cap = p->max_pts;
  P.tau = p->min_pts;
  P.nq = p->grid_side;
  P.m = m;
  P.ls_mode = p->ls_mode;
  P.frame_mode = p->frame_mode;
  for (int b = 0; b < kNumBuckets; ++b) P.bcap[b] = kBucketCap[b];
  P.sf2 = p->signal_var;
  P.noise = p->noise_var;
  P.eta = p->converge_var;
  P.refine_thr = p->refine_threshold;
  P.cond_thr = p->cond_threshold;
  P.s = (double)p->voxel_size;
  P.ell = (double)p->length_scale;
  const bool fp32 = p->precision == VGPR_PREC_FP32 || p->precision == VGPR_PREC_MIXED;
  P.mode = 2;

  Lists L{recs, nan_list, ctr, a.n_vox, rots, big_list, ctr + 48};
  {
    ProfScope ps(ctx, "classify");
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)((a.n_vox + 255) / 256)), dim3(256), 0, ctx->stream, P, a,
                       staged, L);
    VGPR_HIP(ctx, hipGetLastError());
    if (p->max_pts > kPrepCoop) {
      hipLaunchKernelGGL(prep_big_kernel, dim3((unsigned)std::min<int64_t>((a.n_vox + 3) / 4, 2048)), dim3(256), 0,
                         ctx->stream, P, a, staged, L);
      VGPR_HIP(ctx, hipGetLastError());
    }
  }
  // Buckets run concurrently on the caller's stream and the three side streams
  // (bucket_stream of the launch choices; by default the 96/128-point buckets on
  // side stream 1, the 32/64-point buckets on side stream 2, the 256/512-point
  // buckets on side stream 3, the 16-point bucket and its passes on the caller's
  // stream), joined back before the call returns (with tiled_first, the tiled
  // buckets run before the fork instead). Many small voxels fill the CUs that
  // the few long large-voxel solves leave idle.
  st = ensure_aux(ctx);
  if (st != VGPR_OK) return st;
  const vgpr_tuning& tu = ctx->tune;
  // tiled_first: the tiled buckets run alone on the caller's stream before the
  // fork (their workgroups need whole CUs, which concurrent buckets would hold)
  const bool tiles_first = tu.streams != 1 && tu.tiled_first != 0;
  auto stream_of = [&](int b) {
    if (tu.streams == 1 || (tiles_first && b >= first_tile_bucket(ctx))) return ctx->stream;
    const int s = tu.bucket_stream[b];
    return s == 0 ? ctx->stream : ctx->aux[s - 1];
  };
  bool merge_top = false;  // set below, once the launched buckets are known
  auto launch_b = [&](int b) -> vgpr_status {
    const bool tiled = b >= first_tile_bucket(ctx);
    const bool wave = wave_ok(b) && b <= tu.wave_last_bucket;
    const bool in_fp32 = fp32 && b <= tu.fp32_last_bucket && !tiled;
    FitParams Pb = P;
    Pb.mode = in_fp32 ? 0 : 2;
    const RotRec* rb_ = rots ? rots + (size_t)b * a.n_vox : nullptr;
    Launch l{stream_of(b), tu.grid_scale[b], recs + (size_t)b * a.n_vox, rb_, nullptr, ctr + b, ctr + 8 + b,
             rlists + (size_t)b * a.n_vox, ctr + 16 + b, a.n_vox, kFam[in_fp32 ? 0 : 2][b]};
    if (tiled) {
      if (mixed) l.fam = kFamMixed[b];
      // largest voxels first: the bucket's (otherwise unused) re-solve list holds the order,
      // sorted before the fork
      if (b == kNumBuckets - 1 && merge_top) {
        // the 256- and 512-point buckets as one launch: slots of both lists relative to the
        // 256-point bucket's records (the 512-point list follows it at a.n_vox)
        l.recs = recs + (size_t)(b - 1) * a.n_vox;
        l.rots = rots ? rots + (size_t)(b - 1) * a.n_vox : nullptr;
        l.count = ctr + 49;
      }
      l.slots = rlists + (size_t)b * a.n_vox;
      return launch_tile(ctx, b, mixed, Pb, a, staged, l, tile_scratch[b]);
    }
    const bool refine_pass = in_fp32 && wave && b == 0;  // the wave shape that hands voxels to the refinement pass
    if (refine_pass) {
      l.flist = flists + (size_t)b * a.n_vox;
      l.fcount = ctr + 32 + b;
    }
    vgpr_status s2 = in_fp32 ? launch_bucket<float>(ctx, b, wave, Pb, a, staged, l)
                             : launch_bucket<double>(ctx, b, wave, Pb, a, staged, l);
    if (s2 != VGPR_OK || !in_fp32) return s2;
    if (refine_pass) {
      // FP32 again over the voxels with small pivots, each with one FP64 refinement step of alpha
      FitParams F = P;
      F.mode = 3;
      Launch lf{stream_of(b), tu.grid_scale[b], recs + (size_t)b * a.n_vox, rb_, flists + (size_t)b * a.n_vox,
                ctr + 32 + b, ctr + 40 + b, nullptr, nullptr, a.n_vox, kFamRefine};
      if ((s2 = launch_refine(ctx, F, a, staged, lf)) != VGPR_OK) return s2;
    }
    // FP64 re-solve of this bucket's flagged voxels, on the same stream right after it
    FitParams R = P;
    R.mode = 1;
    Launch lr{stream_of(b), tu.grid_scale[b], recs + (size_t)b * a.n_vox, rb_, rlists + (size_t)b * a.n_vox,
              ctr + 16 + b, ctr + 24 + b, nullptr, nullptr, a.n_vox, kFam[1][b]};
    return launch_bucket<double>(ctx, b, wave, R, a, staged, lr);
  };
  auto launched = [&](int b) { return p->max_pts > (b ? P.bcap[b - 1] : 0); };
  // 256- and 512-point buckets merged into the 512-point launch (the combined slots must fit int32)
  merge_top = tu.tiled_merge != 0 && launched(kNumBuckets - 1) && first_tile_bucket(ctx) <= kNumBuckets - 2 &&
              a.n_vox < (int64_t(1) << 30);
  auto skipped = [&](int b) { return merge_top && b == kNumBuckets - 2; };
  {
    // longest-first orders of the tiled buckets, one workgroup each
    OrderJobs oj{};
    int nj = 0;
    for (int b = first_tile_bucket(ctx); b < kNumBuckets; ++b) {
      if (!launched(b) || skipped(b)) continue;
      const bool merged = b == kNumBuckets - 1 && merge_top;
      OrderJob& j = oj.job[nj++];
      j.recs = recs + (size_t)(merged ? b - 1 : b) * a.n_vox;
      j.count = ctr + (merged ? b - 1 : b);
      j.order = rlists + (size_t)b * a.n_vox;
      j.count2 = merged ? ctr + b : nullptr;
      j.stride2 = merged ? (int32_t)a.n_vox : 0;
      j.total = merged ? ctr + 49 : nullptr;
    }
    if (nj > 0) {
      hipLaunchKernelGGL(order_kernel, dim3((unsigned)nj), dim3(kOrderThreads), 0, ctx->stream, oj);
      VGPR_HIP(ctx, hipGetLastError());
    }
  }
  if (tiles_first)
    for (int b = kNumBuckets - 1; b >= first_tile_bucket(ctx); --b)
      if (launched(b) && !skipped(b) && (st = launch_b(b)) != VGPR_OK) return st;
  VGPR_HIP(ctx, hipEventRecord(ctx->fork_ev, ctx->stream));
  for (int i = 0; i < vgpr_ctx::kAux; ++i) VGPR_HIP(ctx, hipStreamWaitEvent(ctx->aux[i], ctx->fork_ev, 0));
  for (int b = kNumBuckets - 1; b >= 0; --b) {
    if (!launched(b) || skipped(b) || (tiles_first && b >= first_tile_bucket(ctx))) continue;
    if ((st = launch_b(b)) != VGPR_OK) return st;
  }
  {
    // NaN rows of the voxels below tau: HBM writes only, queued behind the caller's stream's
    // buckets so that they overlap the long solves instead of delaying the fork
    ProfScope ps(ctx, "nan_rows");
    hipLaunchKernelGGL(nan_kernel, dim3((unsigned)std::min<int64_t>((a.n_vox + 3) / 4, 4096)), dim3(256), 0,
                       ctx->stream, P, a.out, L);
    VGPR_HIP(ctx, hipGetLastError());
  }
  for (int i = 0; i < vgpr_ctx::kAux; ++i) {
    VGPR_HIP(ctx, hipEventRecord(ctx->join_ev[i], ctx->aux[i]));
    VGPR_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->join_ev[i], 0));
  }
  return VGPR_OK;
}

}  // namespace vgpr

extern "C" vgpr_status vgpr_fit_predict(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts, const uint64_t* d_keys,
                                        const int32_t* d_offsets, const int32_t* d_counts, const int32_t* d_perm,
                                        int64_t n_vox, const float* d_noise_var, const vgpr_params* params,
                                        float* d_out, int8_t* d_axis, uint8_t* d_status) {
  if (!ctx) return VGPR_E_INVALID;
  vgpr_status st = vgpr::check_params(ctx, params);
  if (st != VGPR_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return vgpr::fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  vgpr::FitArgs a{d_xyz, n_pts, d_keys, d_offsets, d_counts, d_perm, d_noise_var, n_vox, d_out, d_axis, d_status};
  return vgpr::fit_predict_impl(ctx, a, params, 0);
}

// No-allocation variant: the same launches, with the scratch carved from the
// context device's fixed scratch array (its address looked up at vgpr_create).
extern "C" vgpr_status vgpr_fit_predict_noalloc(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts,
                                                const uint64_t* d_keys, const int32_t* d_offsets,
                                                const int32_t* d_counts, const int32_t* d_perm, int64_t n_vox,
                                                const float* d_noise_var, const vgpr_params* params, float* d_out,
                                                int8_t* d_axis, uint8_t* d_status) {
  using namespace vgpr;
  if (!ctx) return VGPR_E_INVALID;
  vgpr_status st = check_params(ctx, params);
  if (st != VGPR_OK) return st;
  if (!ctx->fixed_scratch || !ctx->aux[0]) return fail(ctx, VGPR_E_DEVICE, "context has no fixed scratch");
  if (n_vox < 0 || n_vox >= (int64_t(1) << 31) || n_pts < 0 || n_pts >= (int64_t(1) << 31))
    return fail(ctx, VGPR_E_INVALID, "n_vox and n_pts must be in [0, 2^31)");
  const size_t need = fit_work_bytes(ctx, n_vox, n_pts, params);
  if (need > kFixedScratchBytes)
    return fail(ctx, VGPR_E_CAPACITY,
                "scratch of " + std::to_string(need) + " bytes exceeds the fixed scratch of " +
                    std::to_string(kFixedScratchBytes) + " bytes (fewer voxels or points, or max_pts <= 128 "
                    "outside MIXED mode, keep it within)");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  FitArgs a{d_xyz, n_pts, d_keys, d_offsets, d_counts, d_perm, d_noise_var, n_vox, d_out, d_axis, d_status};
  const bool prof = ctx->profiling;
  ctx->profiling = false;  // timing events would be created on demand
  st = fit_predict_impl(ctx, a, params, 0, static_cast<char*>(ctx->fixed_scratch));
  ctx->profiling = prof;
  return st;
}

// ---------------------------------------------------------------------------
// Captured fit_predict: the same launches recorded once as a HIP graph and
// replayed. The graph owns its scratch, so later calls that grow the context
// workspace cannot invalidate it.
// ---------------------------------------------------------------------------
struct vgpr_graph {
  vgpr_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* work = nullptr;
  size_t bytes = 0;
};

extern "C" vgpr_status vgpr_fit_graph_create(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts,
                                             const uint64_t* d_keys, const int32_t* d_offsets,
                                             const int32_t* d_counts, const int32_t* d_perm, int64_t n_vox,
                                             const float* d_noise_var, const vgpr_params* params, float* d_out,
                                             int8_t* d_axis, uint8_t* d_status, vgpr_graph** out) {
  using namespace vgpr;
  if (!ctx || !out) return VGPR_E_INVALID;
  *out = nullptr;
  vgpr_status st = check_params(ctx, params);
  if (st != VGPR_OK) return st;
  if (ctx->stream == nullptr) return fail(ctx, VGPR_E_INVALID, "graph capture needs a context on a non-default stream");
  if (n_vox <= 0 || n_vox >= (int64_t(1) << 31) || n_pts <= 0 || n_pts >= (int64_t(1) << 31))
    return fail(ctx, VGPR_E_INVALID, "graph capture needs 0 < n_vox, n_pts < 2^31");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  st = ensure_aux(ctx);
  if (st != VGPR_OK) return st;
  auto* g = new vgpr_graph();
  g->ctx = ctx;
  g->bytes = fit_work_bytes(ctx, n_vox, n_pts, params);
  st = alloc_owned(ctx, &g->work, g->bytes);
  if (st != VGPR_OK) {
    delete g;
    return st;
  }
  FitArgs a{d_xyz, n_pts, d_keys, d_offsets, d_counts, d_perm, d_noise_var, n_vox, d_out, d_axis, d_status};
  const bool prof = ctx->profiling;
  ctx->profiling = false;  // no timing events inside the graph
  hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = fit_predict_impl(ctx, a, params, 0, static_cast<char*>(g->work));
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(ctx->stream, &graph);
    g->graph = graph;
    if (st == VGPR_OK && e2 != hipSuccess) st = hip_fail(ctx, e2, "hipStreamEndCapture");
  } else {
    st = hip_fail(ctx, e, "hipStreamBeginCapture");
  }
  ctx->profiling = prof;
  if (st == VGPR_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) st = hip_fail(ctx, e, "hipGraphInstantiate");
  }
  if (st != VGPR_OK) {
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    free_owned(ctx, g->work, g->bytes);
    delete g;
    return st;
  }
  ctx->live_graphs += 1;
  *out = g;
  return VGPR_OK;
}

extern "C" vgpr_status vgpr_graph_launch(vgpr_graph* g) {
  using namespace vgpr;
  if (!g) return VGPR_E_INVALID;
  vgpr_ctx* ctx = g->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  VGPR_HIP(ctx, hipGraphLaunch(g->exec, ctx->stream));
  return VGPR_OK;
}

extern "C" vgpr_status vgpr_graph_destroy(vgpr_graph* g) {
  using namespace vgpr;
  if (!g) return VGPR_E_INVALID;
  vgpr_ctx* ctx = g->ctx;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);  // no replay may still use the scratch
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  free_owned(ctx, g->work, g->bytes);
  ctx->live_graphs -= 1;
  delete g;
  return VGPR_OK;
}
