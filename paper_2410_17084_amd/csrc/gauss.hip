// vgpr_gauss_init: initial 3D Gaussians from the predicted grids (Sec. 3.2).
//
// The n_q x n_q grid of a solved voxel splits into n_s x n_s subgrids of
// n_r x n_r predicted points (n_q = n_s n_r). For each subgrid the Gaussian's
// position is the inverse-variance weighted mean of its points, its
// covariance the weighted scatter about that mean normalised by the weight
// sum, its scale the covariance diagonal, its rotation the identity (not
// stored). One thread per Gaussian: two passes over the subgrid's rows
// (mean, then scatter) with double accumulation, so the result does not
// depend on cancellation in a one-pass formula. The kernel reads the rows of
// solved voxels once and the status byte of every voxel, and writes 32 bytes
// per Gaussian (NaN for voxels that were not solved): it is bound by HBM.
#include "vgpr_internal.h"

namespace vgpr {
namespace {

// One thread per Gaussian. NR > 0: subgrids of NR x NR rows, all loaded before
// any arithmetic and kept in registers (with their weights) for both passes;
// NR = 0: any n_r, rows loaded as the passes go. The sums run in the same order
// either way, so both give the same bits.
constexpr int kGaussThreads = 64;  // one wavefront a workgroup: measured faster than 128 or 256

template <int NR>
__global__ void __launch_bounds__(kGaussThreads) gauss_kernel(const float4* __restrict__ rows, const uint8_t* __restrict__ status,
                                                    int64_t n_gauss, int gs, int nr, int ns, float var_floor,
                                                    float4* __restrict__ gauss) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_gauss) return;
  const int per = ns * ns;
  const int64_t v = t / per;
  const int beta = (int)(t - v * per);
  const int bi = beta / ns, bj = beta - (beta / ns) * ns;
  float4* o = gauss + 2 * t;
  if (!(status[v] & VGPR_ST_SOLVED)) {
    const float nan = __int_as_float(0x7fc00000);
    o[0] = make_float4(nan, nan, nan, nan);
    o[1] = make_float4(nan, nan, nan, nan);
    return;
  }
  const float4* __restrict__ g = rows + v * gs * gs + (int64_t)(bi * nr) * gs + bj * nr;
  const double fl = (double)var_floor;
  double sw = 0, sx = 0, sy = 0, sz = 0, cx = 0, cy = 0, cz = 0, px, py, pz;
  if constexpr (NR > 0) {
    float4 r[NR * NR];
    double w[NR * NR];
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int j = 0; j < NR; ++j) r[i * NR + j] = g[i * gs + j];
#pragma unroll
    for (int k = 0; k < NR * NR; ++k) {
      w[k] = 1.0 / fmax((double)r[k].w, fl);
      sw += w[k];
      sx += w[k] * (double)r[k].x;
      sy += w[k] * (double)r[k].y;
      sz += w[k] * (double)r[k].z;
    }
    px = sx / sw, py = sy / sw, pz = sz / sw;
#pragma unroll
    for (int k = 0; k < NR * NR; ++k) {
      const double dx = (double)r[k].x - px, dy = (double)r[k].y - py, dz = (double)r[k].z - pz;
      cx += w[k] * dx * dx;
      cy += w[k] * dy * dy;
      cz += w[k] * dz * dz;
    }
  } else {
    for (int i = 0; i < nr; ++i) {
      for (int j = 0; j < nr; ++j) {
        const float4 r = g[i * gs + j];
        const double w = 1.0 / fmax((double)r.w, fl);
        sw += w;
        sx += w * (double)r.x;
        sy += w * (double)r.y;
        sz += w * (double)r.z;
      }
    }
    px = sx / sw, py = sy / sw, pz = sz / sw;
    for (int i = 0; i < nr; ++i) {
      for (int j = 0; j < nr; ++j) {
        const float4 r = g[i * gs + j];
        const double w = 1.0 / fmax((double)r.w, fl);
        const double dx = (double)r.x - px, dy = (double)r.y - py, dz = (double)r.z - pz;
        cx += w * dx * dx;
        cy += w * dy * dy;
        cz += w * dz * dz;
      }
    }
  }
  o[0] = make_float4((float)px, (float)py, (float)pz, (float)sw);
  o[1] = make_float4((float)(cx / sw), (float)(cy / sw), (float)(cz / sw), 0.f);
}

}  // namespace
}  // namespace vgpr

extern "C" vgpr_status vgpr_gauss_init(vgpr_ctx* ctx, const float* d_out, const uint8_t* d_status, int64_t n_vox,
                                       int32_t grid_side, int32_t n_r, float var_floor, float* d_gauss) {
  using namespace vgpr;
  if (!ctx) return VGPR_E_INVALID;
  if (n_vox < 0 || n_vox >= (int64_t(1) << 31)) return fail(ctx, VGPR_E_INVALID, "n_vox out of range");
  if (grid_side < 1 || grid_side > kMaxGridSide) return fail(ctx, VGPR_E_INVALID, "grid_side must be in [1, 16]");
  if (n_r < 1 || grid_side % n_r != 0) return fail(ctx, VGPR_E_INVALID, "n_r must divide grid_side");
  if (!(var_floor > 0.f)) return fail(ctx, VGPR_E_INVALID, "var_floor must be > 0");
  if (n_vox == 0) return VGPR_OK;
  if (!d_out || !d_status || !d_gauss) return fail(ctx, VGPR_E_INVALID, "null device pointer");
  if ((reinterpret_cast<uintptr_t>(d_out) | reinterpret_cast<uintptr_t>(d_gauss)) & 15)
    return fail(ctx, VGPR_E_INVALID, "d_out and d_gauss must be 16-byte aligned");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VGPR_E_DEVICE, "hipSetDevice");
  const int ns = grid_side / n_r;
  const int64_t n_gauss = n_vox * ns * ns;
  const int64_t blocks = (n_gauss + kGaussThreads - 1) / kGaussThreads;
  if (blocks > INT32_MAX) return fail(ctx, VGPR_E_INVALID, "n_vox * (grid_side / n_r)^2 too large for one launch");
  ProfScope ps(ctx, "gauss_init");
  auto kernel = n_r == 1 ? gauss_kernel<1>
              : n_r == 2 ? gauss_kernel<2>
              : n_r == 3 ? gauss_kernel<3>
              : n_r == 4 ? gauss_kernel<4>
                         : gauss_kernel<0>;
  hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kGaussThreads), 0, ctx->stream,
                     reinterpret_cast<const float4*>(d_out), d_status, n_gauss, grid_side, n_r, ns, var_floor,
                     reinterpret_cast<float4*>(d_gauss));
  VGPR_HIP(ctx, hipGetLastError());
  return VGPR_OK;
}
