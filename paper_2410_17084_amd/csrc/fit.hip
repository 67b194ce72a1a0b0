// vgpr_fit_predict: Alg. 1 after STORE, Eq. (1)-(3) of the paper, per voxel.
//
// Design (MI355X): one workgroup solves one voxel at a time, pulling voxel
// indices from a size bucket's list with an atomic counter (persistent grid).
// The workgroup's lanes own the rows of the augmented system
//
//          [ K + S ]   n data rows      (S = noise variances on the diagonal)
//          [ f~^T  ]   1 right-hand-side row (f minus its mean)
//          [ K*^T  ]   m query rows
//
// restricted to the n columns of the data points. A right-looking LDL^T
// elimination over those n columns (no square roots) turns the data rows into
// the factor, the f row into y = L^-1 f~ and every query row into L^-1 k*_q, so
// the posterior of Eq. (3) accumulates on the fly:
//   var_q  = s_f^2 - sum_j a_qj^2 / d_j          (diagonal of Sigma*)
//   mean_q = mu    + sum_j a_qj * y_j / d_j       (K*^T (K+S)^-1 f~)
// where d_j is the j-th pivot and a_qj the query row's entry at step j. Each
// lane keeps its row in registers; after step j the row is shifted by one
// register so the active column is always element 0 (no dynamic register
// indexing). Column j of the data rows is broadcast through LDS, double
// buffered, with one barrier per step. K, K* and K** are never stored.
//
// The elimination type T is float or double. In FP32 mode every voxel runs
// in float and those whose refinement score sum_j |y_j| / d_j exceeds the
// threshold (the FP32 rounding amplification of K^-1 f~) are re-solved in
// double; in FP64 mode every voxel runs in double. The PCA frame is double in
// both.
#include <cfloat>

#include "scan.cuh"
#include "vgpr_internal.h"

namespace vgpr {
namespace {

constexpr int kFitThreads = 256;  // upper bound of the workgroup size

struct FitParams {
  int cap;          // max_pts
  int tau;          // min_pts
  int nq;           // grid side
  int m;            // nq * nq
  int ls_mode;
  int mode;         // 0 = FP32 first pass (flags), 1 = FP64 re-solve pass, 2 = FP64 only
  float sf2;
  float noise;
  float eta;
  float refine_thr;
  double s;         // voxel size (float widened)
  double ell;       // fixed length scale
};

struct WorkList {
  const int32_t* list;        // voxel indices
  const uint32_t* count;      // number of entries (device)
  uint32_t* next;             // fetch counter (device)
  int32_t* refine_list;       // FP32 pass: voxels to re-solve (nullable)
  uint32_t* refine_count;
};

__device__ __forceinline__ float k_exp(float x) { return __expf(x); }
__device__ __forceinline__ double k_exp(double x) { return exp(x); }

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
      if (apq == 0.0) continue;
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
  w[0] = A[0][0];
  w[1] = A[1][1];
  w[2] = A[2][2];
}

struct FrameInfo {
  double mu;        // mean of the value coordinate
  double anc_u;     // voxel corner along u
  double anc_w;     // voxel corner along w
  double lam;       // 1 / (2 l^2)
  int axis, u, w;
  int ku, kw;
  int tie;
};

template <typename T, int NMAX>
__global__ void __launch_bounds__(kFitThreads) fit_kernel(FitParams P, FitArgs io, WorkList wl) {
  __shared__ float sp[3][NMAX];
  __shared__ T su[NMAX + 4], sw[NMAX + 4], sf[NMAX + 4];
  __shared__ __attribute__((aligned(16))) T col[2][NMAX + 8];
  __shared__ T piv[2][2];
  __shared__ FrameInfo fr;
  __shared__ int s_item;
  __shared__ unsigned s_maxvar;
  __shared__ int s_flag;

  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int lane = tid & 63;

  for (;;) {
    if (tid == 0) {
      s_item = (int)atomicAdd(wl.next, 1u);
      s_maxvar = 0u;
      s_flag = 0;
    }
    __syncthreads();
    const int item = s_item;
    if (item >= (int)*wl.count) break;
    const int v = wl.list[item];
    const int off = io.offsets[v];
    const int cnt = io.counts[v];
    const int n = cnt < P.cap ? cnt : P.cap;
    const int* perm = io.perm;

    // ---- gather the voxel's points (coalesced over consecutive sorted slots)
    for (int i = tid; i < n; i += NT) {
      const int idx = perm ? perm[off + i] : off + i;
      sp[0][i] = io.xyz[3 * (size_t)idx + 0];
      sp[1][i] = io.xyz[3 * (size_t)idx + 1];
      sp[2][i] = io.xyz[3 * (size_t)idx + 2];
    }
    __syncthreads();

    // ---- PCA frame and value-axis switch (wave 0, double)
    if (tid < 64) {
      double c0 = 0, c1 = 0, c2 = 0;
      for (int i = 0; i < n; ++i) {
        c0 += (double)sp[0][i];
        c1 += (double)sp[1][i];
        c2 += (double)sp[2][i];
      }
      const double inv_n = 1.0 / (double)n;
      c0 *= inv_n;
      c1 *= inv_n;
      c2 *= inv_n;
      double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int i = 0; i < n; ++i) {
        const double d0 = (double)sp[0][i] - c0, d1 = (double)sp[1][i] - c1, d2 = (double)sp[2][i] - c2;
        A[0][0] += d0 * d0;
        A[0][1] += d0 * d1;
        A[0][2] += d0 * d2;
        A[1][1] += d1 * d1;
        A[1][2] += d1 * d2;
        A[2][2] += d2 * d2;
      }
      A[0][0] *= inv_n; A[0][1] *= inv_n; A[0][2] *= inv_n;
      A[1][1] *= inv_n; A[1][2] *= inv_n; A[2][2] *= inv_n;
      A[1][0] = A[0][1]; A[2][0] = A[0][2]; A[2][1] = A[1][2];
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
      const double a0 = fabs(v0), a1 = fabs(v1), a2 = fabs(v2);
      int ax = 0;
      double best = a0;
      if (a1 > best) { ax = 1; best = a1; }
      if (a2 > best) { ax = 2; best = a2; }
      // second largest |v_k|
      const double second = (ax == 0) ? fmax(a1, a2) : (ax == 1 ? fmax(a0, a2) : fmax(a0, a1));
      const int tie = (best - second < 1e-6) || (wmid - wlo <= 1e-8 * tr);
      const int u = ax == 0 ? 1 : (ax == 1 ? 2 : 0);
      const int wv = ax == 0 ? 2 : (ax == 1 ? 0 : 1);
      double ell = P.ell;
      if (P.ls_mode == 1) {
        const double e = sqrt(3.0) * sqrt(fmax((wmid + whi) * 0.5, 0.0));
        ell = fmin(fmax(e, 0.05 * P.s), 2.0 * P.s);
      }
      if (tid == 0) {
        const uint64_t key = io.keys[v];
        const int64_t mask = (int64_t(1) << kKeyFieldBits) - 1;
        const int kx = (int)((int64_t)((key >> (2 * kKeyFieldBits)) & mask) - kKeyBias);
        const int ky = (int)((int64_t)((key >> kKeyFieldBits) & mask) - kKeyBias);
        const int kz = (int)((int64_t)(key & mask) - kKeyBias);
        const int ku = u == 0 ? kx : (u == 1 ? ky : kz);
        const int kw = wv == 0 ? kx : (wv == 1 ? ky : kz);
        fr.axis = ax;
        fr.u = u;
        fr.w = wv;
        fr.ku = ku;
        fr.kw = kw;
        fr.mu = ax == 0 ? c0 : (ax == 1 ? c1 : c2);
        fr.anc_u = (double)ku * P.s;
        fr.anc_w = (double)kw * P.s;
        fr.lam = 1.0 / (2.0 * ell * ell);
        fr.tie = tie;
      }
    }
    __syncthreads();
    const int ax = fr.axis, u = fr.u, wax = fr.w;
    const double mu = fr.mu;
    for (int i = tid; i < n; i += NT) {
      su[i] = (T)((double)sp[u][i] - fr.anc_u);
      sw[i] = (T)((double)sp[wax][i] - fr.anc_w);
      sf[i] = (T)((double)sp[ax][i] - mu);
    }
    __syncthreads();

    const T lam = (T)fr.lam;
    const T sf2 = (T)P.sf2;
    const int qchunk = NT - n - 1;
    bool failed = false;
    T minpiv = (T)FLT_MAX;
    T score = 0;
    for (int q0 = 0; q0 < P.m; q0 += qchunk) {
      // ---- row roles for this chunk
      const bool is_data = tid < n;
      const bool is_f = tid == n;
      const int q = q0 + tid - n - 1;
      const bool is_query = tid > n && q < P.m;
      T a[NMAX];
      float gu = 0.f, gw = 0.f;
      T xu = 0, xw = 0, nz = 0;
      if (is_data) {
        xu = su[tid];
        xw = sw[tid];
        nz = (T)P.noise;
        if (io.noise) nz = (T)io.noise[perm ? perm[off + tid] : off + tid];
      } else if (is_query) {
        const int i = q / P.nq, j = q - (q / P.nq) * P.nq;
        const double ti = __ddiv_rn((double)i + 0.5, (double)P.nq);
        const double tj = __ddiv_rn((double)j + 0.5, (double)P.nq);
        gu = (float)__dmul_rn(__dadd_rn((double)fr.ku, ti), P.s);
        gw = (float)__dmul_rn(__dadd_rn((double)fr.kw, tj), P.s);
        xu = (T)((double)gu - fr.anc_u);
        xw = (T)((double)gw - fr.anc_w);
      }
      if (is_data || is_query) {
        // kernel row: kappa(x_row, x_c) for the n data points, noise on the diagonal
#pragma unroll
        for (int c = 0; c < NMAX; ++c) {
          if (c < n) {
            const T du = xu - su[c], dw = xw - sw[c];
            a[c] = sf2 * k_exp(-(du * du + dw * dw) * lam) + (c == tid ? nz : (T)0);
          } else {
            a[c] = 0;
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < NMAX; ++c) a[c] = (is_f && c < n) ? sf[c] : (T)0;
      }
      T var = sf2;
      T mean = 0;
      minpiv = (T)FLT_MAX;
      score = 0;

      // ---- right-looking LDL^T over the n data columns
      for (int j = 0; j < n; ++j) {
        const int b = j & 1;
        if (is_data && tid >= j) {
          if (tid == j) piv[b][0] = a[0];
          else col[b][tid - j - 1] = a[0];
        }
        if (is_f) piv[b][1] = a[0];
        __syncthreads();
        const T d = piv[b][0];
        const T yj = piv[b][1];
        const T inv = (T)1 / d;
        const T t = a[0] * inv;
        minpiv = d < minpiv ? d : minpiv;
        score += (yj < 0 ? -yj : yj) * inv;
        if (is_query) {
          var -= t * a[0];
          mean += t * yj;
        }
        const int L = n - j - 1;
        const T* cb = col[b];
#pragma unroll
        for (int c0 = 0; c0 < NMAX - 1; c0 += 8) {
          if (c0 < L) {
#pragma unroll
            for (int k = c0; k < c0 + 8; ++k)
              if (k < NMAX - 1) a[k] = a[k + 1] - t * cb[k];
          }
        }
      }
      failed = !(minpiv > (T)0) || !isfinite((double)score);
      const bool flag = P.mode == 0 && (failed || score > (T)P.refine_thr);

      // ---- outputs
      if (is_query && !flag) {
        const float vv = failed ? __int_as_float(0x7fc00000) : (float)(var > (T)0 ? var : (T)0);
        const float mv = failed ? __int_as_float(0x7fc00000) : (float)(mu + (double)mean);
        float4 o;
        o.x = ax == 0 ? mv : (u == 0 ? gu : gw);
        o.y = ax == 1 ? mv : (u == 1 ? gu : gw);
        o.z = ax == 2 ? mv : (u == 2 ? gu : gw);
        o.w = vv;
        reinterpret_cast<float4*>(io.out)[(size_t)v * P.m + q] = o;
        if (!failed) atomicMax(&s_maxvar, __float_as_uint(vv));
      }
      if (flag) {
        if (tid == 0) s_flag = 1 + (failed ? 1 : 0);
        break;
      }
    }
    __syncthreads();
    if (tid == 0) {
      uint8_t st = VGPR_ST_SOLVED;
      if (cnt > P.cap) st |= VGPR_ST_CAPPED;
      if (fr.tie) st |= VGPR_ST_AXIS_TIE;
      if (s_flag) {
        // FP32 pass: hand the voxel to the FP64 re-solve list
        const uint32_t slot = atomicAdd(wl.refine_count, 1u);
        wl.refine_list[slot] = v;
        if (s_flag == 2) st |= VGPR_ST_FACTOR_FAIL;
        io.status[v] = st;
      } else {
        if (P.mode == 1) st |= VGPR_ST_REFINED | (io.status[v] & VGPR_ST_FACTOR_FAIL);
        if (failed) {
          st = (uint8_t)((st & ~VGPR_ST_SOLVED) | VGPR_ST_FACTOR_FAIL);
        } else if (__uint_as_float(s_maxvar) <= P.eta) {
          st |= VGPR_ST_CONVERGED;
        }
        io.status[v] = st;
      }
      io.axis[v] = (int8_t)ax;
    }
    __syncthreads();
  }
}

// Sort voxels into size buckets; voxels below tau get NaN rows.
__global__ void __launch_bounds__(256) classify_kernel(const int32_t* __restrict__ counts, int64_t n_vox, int cap,
                                                       int tau, int m, int32_t* __restrict__ lists,
                                                       uint32_t* __restrict__ list_counts, int64_t list_stride,
                                                       float* __restrict__ out, int8_t* __restrict__ axis,
                                                       uint8_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_vox) return;
  const int c = counts[v];
  const int n = c < cap ? c : cap;
  if (n < tau) {
    status[v] = (uint8_t)(VGPR_ST_BELOW_TAU | (c > cap ? VGPR_ST_CAPPED : 0));
    axis[v] = -1;
    const float nan = __int_as_float(0x7fc00000);
    float4* o = reinterpret_cast<float4*>(out) + (size_t)v * m;
    for (int q = 0; q < m; ++q) o[q] = make_float4(nan, nan, nan, nan);
    return;
  }
  int b = 0;
  while (b < kNumBuckets - 1 && n > kBucketCap[b]) ++b;
  const uint32_t slot = atomicAdd(&list_counts[b], 1u);
  lists[b * list_stride + slot] = (int32_t)v;
}

template <typename T, int NMAX>
int blocks_per_cu() {
  static int cached = -1;
  if (cached < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_kernel<T, NMAX>, kFitThreads, 0) != hipSuccess ||
        nb < 1)
      nb = 1;
    cached = nb;
  }
  return cached;
}

// Timing family of each launch: precision, pass and bucket capacity.
const char* const kFamFit32[kNumBuckets] = {"fit_f32_n16", "fit_f32_n32", "fit_f32_n64", "fit_f32_n128"};
const char* const kFamFit64[kNumBuckets] = {"fit_f64_n16", "fit_f64_n32", "fit_f64_n64", "fit_f64_n128"};
const char* const kFamRefine[kNumBuckets] = {"refine_f64_n16", "refine_f64_n32", "refine_f64_n64",
                                             "refine_f64_n128"};

template <typename T>
vgpr_status launch_bucket(vgpr_ctx* ctx, int b, const FitParams& P, const FitArgs& io, const WorkList& wl,
                          int64_t max_items, const char* fam) {
  const int nmax = kBucketCap[b];
  int threads = nmax + 1 + P.m;
  if (threads > kFitThreads) threads = kFitThreads;
  threads = (threads + 63) & ~63;
  int per_cu = 1;
  switch (b) {
    case 0: per_cu = blocks_per_cu<T, 16>(); break;
    case 1: per_cu = blocks_per_cu<T, 32>(); break;
    case 2: per_cu = blocks_per_cu<T, 64>(); break;
    default: per_cu = blocks_per_cu<T, 128>(); break;
  }
  // occupancy was computed for the largest workgroup; smaller groups fit more
  per_cu = per_cu * (kFitThreads / threads);
  int64_t grid = (int64_t)per_cu * ctx->cu_count;
  if (grid > max_items) grid = max_items;
  if (grid < 1) grid = 1;
  ProfScope ps(ctx, fam);
  switch (b) {
    case 0: hipLaunchKernelGGL((fit_kernel<T, 16>), dim3(grid), dim3(threads), 0, ctx->stream, P, io, wl); break;
    case 1: hipLaunchKernelGGL((fit_kernel<T, 32>), dim3(grid), dim3(threads), 0, ctx->stream, P, io, wl); break;
    case 2: hipLaunchKernelGGL((fit_kernel<T, 64>), dim3(grid), dim3(threads), 0, ctx->stream, P, io, wl); break;
    default: hipLaunchKernelGGL((fit_kernel<T, 128>), dim3(grid), dim3(threads), 0, ctx->stream, P, io, wl); break;
  }
  VGPR_HIP(ctx, hipGetLastError());
  return VGPR_OK;
}

}  // namespace

size_t fit_work_bytes(int64_t n_vox) {
  return Carver::round(sizeof(int32_t) * (size_t)n_vox * kNumBuckets) * 2 + Carver::round(sizeof(uint32_t) * 64) +
         1024;
}

vgpr_status fit_predict_impl(vgpr_ctx* ctx, const FitArgs& a, const vgpr_params* p, size_t work_offset) {
  if (a.n_vox < 0 || a.n_vox >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_INVALID, "n_vox out of range");
  if (a.n_vox == 0) return VGPR_OK;
  if (!a.xyz || !a.keys || !a.offsets || !a.counts || !a.out || !a.axis || !a.status)
    return fail(ctx, VGPR_E_INVALID, "null device pointer");
  if (reinterpret_cast<uintptr_t>(a.out) & 15) return fail(ctx, VGPR_E_INVALID, "d_out must be 16-byte aligned");
  const int m = p->grid_side * p->grid_side;
  if (kBucketCap[kNumBuckets - 1] + 2 > kFitThreads - 1)
    return fail(ctx, VGPR_E_UNSUPPORTED, "workgroup too small");
  vgpr_status st = reserve_work(ctx, work_offset + fit_work_bytes(a.n_vox));
  if (st != VGPR_OK) return st;
  Carver cv(static_cast<char*>(ctx->work.ptr) + work_offset);
  int32_t* lists = cv.take<int32_t>((size_t)a.n_vox * kNumBuckets);
  int32_t* rlists = cv.take<int32_t>((size_t)a.n_vox * kNumBuckets);
  uint32_t* ctr = cv.take<uint32_t>(64);  // [0,4) counts, [4,8) next, [8,12) refine counts, [12,16) refine next
  VGPR_HIP(ctx, hipMemsetAsync(ctr, 0, sizeof(uint32_t) * 64, ctx->stream));

  {
    ProfScope ps(ctx, "classify");
    hipLaunchKernelGGL(classify_kernel, dim3((unsigned)((a.n_vox + 255) / 256)), dim3(256), 0, ctx->stream, a.counts,
                       a.n_vox, p->max_pts, p->min_pts, m, lists, ctr, a.n_vox, a.out, a.axis, a.status);
  }
  VGPR_HIP(ctx, hipGetLastError());

  FitParams P;
  P.cap = p->max_pts;
  P.tau = p->min_pts;
  P.nq = p->grid_side;
  P.m = m;
  P.ls_mode = p->ls_mode;
  P.sf2 = p->signal_var;
  P.noise = p->noise_var;
  P.eta = p->converge_var;
  P.refine_thr = p->refine_threshold;
  P.s = (double)p->voxel_size;
  P.ell = (double)p->length_scale;

  const bool fp32 = p->precision == VGPR_PREC_FP32;
  P.mode = fp32 ? 0 : 2;
  for (int b = 0; b < kNumBuckets; ++b) {
    if (p->max_pts <= (b ? kBucketCap[b - 1] : 0)) break;
    WorkList wl;
    wl.list = lists + (size_t)b * a.n_vox;
    wl.count = ctr + b;
    wl.next = ctr + 4 + b;
    wl.refine_list = rlists + (size_t)b * a.n_vox;
    wl.refine_count = ctr + 8 + b;
    st = fp32 ? launch_bucket<float>(ctx, b, P, a, wl, a.n_vox, kFamFit32[b])
              : launch_bucket<double>(ctx, b, P, a, wl, a.n_vox, kFamFit64[b]);
    if (st != VGPR_OK) return st;
  }
  if (fp32) {
    FitParams R = P;
    R.mode = 1;
    for (int b = 0; b < kNumBuckets; ++b) {
      if (p->max_pts <= (b ? kBucketCap[b - 1] : 0)) break;
      WorkList wl;
      wl.list = rlists + (size_t)b * a.n_vox;
      wl.count = ctr + 8 + b;
      wl.next = ctr + 12 + b;
      wl.refine_list = nullptr;
      wl.refine_count = nullptr;
      st = launch_bucket<double>(ctx, b, R, a, wl, a.n_vox, kFamRefine[b]);
      if (st != VGPR_OK) return st;
    }
  }
  return VGPR_OK;
}

}  // namespace vgpr

extern "C" vgpr_status vgpr_fit_predict(vgpr_ctx* ctx, const float* d_xyz, const uint64_t* d_keys,
                                        const int32_t* d_offsets, const int32_t* d_counts, const int32_t* d_perm,
                                        int64_t n_vox, const float* d_noise_var, const vgpr_params* params,
                                        float* d_out, int8_t* d_axis, uint8_t* d_status) {
  if (!ctx) return VGPR_E_INVALID;
  vgpr_status st = vgpr::check_params(ctx, params);
  if (st != VGPR_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return vgpr::fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  vgpr::FitArgs a{d_xyz, d_keys, d_offsets, d_counts, d_perm, d_noise_var, n_vox, d_out, d_axis, d_status};
  return vgpr::fit_predict_impl(ctx, a, params, 0);
}
