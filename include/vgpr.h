/*
 * vgpr.h - C ABI of the batched Voxel-GPR hot path (GS-LIVM, arXiv 2410.17084)
 * on one MI355X (gfx950).
 *
 * The library densifies sparse LiDAR points voxel by voxel with Gaussian
 * Process Regression (paper Sec. 3.1, Alg. 1):
 *
 *   vgpr_voxelize    - Alg. S1 (STORE): voxel key per point, the visited-voxel
 *                      list S_updated, each voxel's points in arrival order.
 *   vgpr_fit_predict - the rest of Alg. 1 after STORE: per-voxel PCA and
 *                      value-axis switch, kernel matrices K, K*, K**, and the
 *                      posterior mean and variance of Eq. (3) on a query grid
 *                      (also captured as a HIP graph: vgpr_fit_graph_*).
 *   vgpr_map_update  - the voxel-map update of Sec. 3.3: points stacked into
 *                      a persistent map, voxels of types (b)/(c) re-solved,
 *                      types (a)/(d) skipped; with update mode 1 the
 *                      covariance-centred update of type (c) voxels
 *                      (vgpr_map_create_ex); vgpr_map_export / _import
 *                      checkpoint and resume a map.
 *   vgpr_gauss_init  - the initial 3D Gaussians of Sec. 3.2 from the grids.
 *   vgpr_structure_loss - the structure similarity loss L_p of Eq. (9).
 *
 * Conventions shared by every call
 * - Pointers named d_* are device pointers (HIP global memory on the
 *   context's device) owned by the caller; pointers named h_* are host
 *   pointers. The library never frees caller memory.
 * - Work is enqueued on the context's HIP stream. Device outputs are valid
 *   once that stream has completed. A host out-parameter that depends on a
 *   device count (n_vox, n_upd) is written before the call returns, which
 *   synchronises the stream.
 * - No exception crosses the ABI. A call that fails returns a status other
 *   than VGPR_OK and leaves its outputs unspecified; vgpr_last_error gives a
 *   message. Per-voxel numerical events are not call errors: they are reported
 *   in the per-voxel status bits below.
 * - Points are float32 x, y, z interleaved (12 bytes per point), world frame,
 *   metres. Non-finite points are dropped and counted.
 * - Calls on one context are not thread-safe; use one context per host thread.
 */
#ifndef VGPR_H
#define VGPR_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define VGPR_API __attribute__((visibility("default")))
#else
#define VGPR_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vgpr_ctx vgpr_ctx;
typedef struct vgpr_map vgpr_map;

typedef enum {
  VGPR_OK = 0,
  VGPR_E_INVALID = 1,     /* bad argument (null pointer, negative size, bad params) */
  VGPR_E_NOMEM = 2,       /* device allocation failed */
  VGPR_E_CAPACITY = 3,    /* caller buffer too small: the required size is written back */
  VGPR_E_RANGE = 4,       /* a finite point's voxel index is outside +-(2^20 - 1) */
  VGPR_E_BUDGET = 5,      /* the work does not fit the context's HBM budget */
  VGPR_E_DEVICE = 6,      /* a HIP runtime call failed */
  VGPR_E_UNSUPPORTED = 7  /* parameter combination the library does not implement */
} vgpr_status;

/* Per-voxel status bits (uint8 per voxel). */
enum {
  VGPR_ST_SOLVED = 1,       /* fitted and predicted */
  VGPR_ST_BELOW_TAU = 2,    /* fewer than min_pts kept points: not solved (Sec. 3.3 type (a)) */
  VGPR_ST_CAPPED = 4,       /* more than max_pts points; the first max_pts in order were kept */
  VGPR_ST_REFINED = 8,      /* an FP32 solve whose alpha took one FP64 refinement step (small
                               pivots or amplified rounding), or which was re-solved in FP64 */
  VGPR_ST_FACTOR_FAIL = 16, /* a non-positive pivot in the FP32 factorisation (then re-solved in
                               FP64); in FP64 mode, the FP64 factorisation failed (rows are NaN) */
  VGPR_ST_CONVERGED = 32,   /* max predicted variance <= converge_var (Sec. 3.3 type (d)) */
  VGPR_ST_AXIS_TIE = 64     /* value-axis decision within rounding of a tie (either axis valid) */
};

/* Arithmetic of the posterior (kernel entries and factorisation). */
enum {
  VGPR_PREC_FP32 = 0,  /* buckets up to the tuning's fp32_last_bucket (by default voxels of up
                          to 16 points): FP32 build and LDL^T; a voxel whose n s_f^2 / min
                          pivot exceeds cond_threshold, or whose refinement score
                          sum_j |y_j| / d_j exceeds refine_threshold, takes one FP64 residual
                          refinement step of alpha = (K + S)^-1 f~ with the FP32 factor and
                          its mean from K*^T alpha in FP64 (16-point shape; larger FP32
                          shapes re-solve such voxels in FP64), a failed FP32 factor is
                          re-solved in FP64 (status REFINED); larger voxels run in FP64 */
  VGPR_PREC_MIXED = 1, /* buckets below tile_first_bucket as in FP32 mode; larger voxels: FP32
                          kernel build and tiled Cholesky on the FP32 matrix cores, L^-1 formed
                          from the FP32 factor, var = s_f^2 - |L^-1 k*_q|^2 as one FP32 matrix
                          product, the mean from K*^T alpha in FP64 with alpha = (K + S)^-1 f~
                          from the FP32 factor and, when n s_f^2 / min pivot exceeds
                          cond_threshold or the refinement score sum_j |y_j| / d_j exceeds
                          refine_threshold, two FP64 residual refinement steps of alpha
                          (status REFINED) */
  VGPR_PREC_FP64 = 2   /* FP64 build and LDL^T for every voxel */
};

/*
 * Hyper-parameters (plain data, copied at call time).
 * Paper defaults (Table S6, Sec. 3.1): voxel_size 0.2 m, min_pts (tau) 10,
 * grid_side = n_s * n_r = 9, converge_var (eta) 0.3, and the kernel
 * exp(-lambda d^2) with lambda = 1, i.e. signal_var 1, length_scale 1/sqrt(2).
 */
typedef struct {
  float voxel_size;       /* s, metres, > 0 */
  int32_t max_pts;        /* cap of points per voxel, 1..512 */
  int32_t min_pts;        /* tau: solve a voxel only with at least this many kept points (>= 1) */
  int32_t grid_side;      /* n_q: queries per side of the voxel face; m = n_q^2, 1..16 */
  float signal_var;       /* s_f^2 of the squared-exponential kernel, > 0 */
  float length_scale;     /* l of exp(-d^2 / (2 l^2)), metres, > 0 (ls_mode 0) */
  float noise_var;        /* sigma_n^2, the sensor noise variance added to K's diagonal, >= 0 */
  int32_t ls_mode;        /* 0: fixed length_scale; 1: per voxel from PCA eigenvalues,
                             l = sqrt(3 (lambda_mid + lambda_max) / 2) clamped to [0.05 s, 2 s] */
  int32_t frame_mode;     /* 0: world value axis of Alg. 1 (value = world coordinate a, grid on
                             the voxel face); 1: PCA-rotated frame: value along the normal v
                             (largest component positive), parameters along e1 = unit(e_k x v),
                             e_k the world axis least aligned with v, and e2 = v x e1, about the
                             centroid; grid = interval centres of an s x s square centred on the
                             centroid in the (e1, e2) plane; output rows are world points
                             centroid + u e1 + w e2 + mean v (noiseless planes are reproduced
                             exactly in any orientation) */
  int32_t precision;      /* VGPR_PREC_* */
  float refine_threshold; /* FP32 / MIXED: refine in FP64 when sum_j |y_j| / d_j exceeds this */
  float converge_var;     /* eta: converged when the max predicted variance <= eta */
  float cond_threshold;   /* FP32 / MIXED: refine alpha in FP64 when n s_f^2 / min pivot exceeds this */
} vgpr_params;

/* Fill *p with the paper's defaults (see above), FP32 precision. */
VGPR_API void vgpr_params_default(vgpr_params* p);

/* Human-readable name of a status code (static string). */
VGPR_API const char* vgpr_status_str(vgpr_status s);

/*
 * Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream). Scratch memory for
 * sorting, bucketing and refinement lists is allocated on demand and never
 * exceeds `hbm_budget_bytes` (0 = no limit); exceeding it returns
 * VGPR_E_BUDGET. The context owns that scratch memory.
 */
VGPR_API vgpr_status vgpr_create(int device, void* hip_stream, size_t hbm_budget_bytes, vgpr_ctx** out);
/* Fails with VGPR_E_INVALID (and frees nothing) while maps created on ctx are alive. */
VGPR_API vgpr_status vgpr_destroy(vgpr_ctx* ctx);
VGPR_API vgpr_status vgpr_set_stream(vgpr_ctx* ctx, void* hip_stream);
/* Message of the last failed call on this context (static until the next call);
 * with ctx = NULL, why the calling thread's last vgpr_create failed. */
VGPR_API const char* vgpr_last_error(const vgpr_ctx* ctx);
/* Device bytes the context currently holds: its scratch, the staging area of
 * its maps' updates, and the maps created on it. */
VGPR_API size_t vgpr_workspace_bytes(const vgpr_ctx* ctx);

/*
 * vgpr_voxelize - Alg. S1 (STORE) for one frame or a batch of frames.
 *
 * Key of a point p (float32) with s = voxel_size: k = floor(double(p) * (1/s))
 * per axis, 1/s computed once in double from the float32 s, one IEEE double
 * multiply; voxels are half-open [k s, (k+1) s). The 64-bit key packs the
 * biased fields k + 2^20 in 21 bits each, x highest:
 *   key = (kx + 2^20) << 42 | (ky + 2^20) << 21 | (kz + 2^20).
 * Non-finite points get key UINT64_MAX and belong to no voxel.
 *
 * Frames: h_frame_offsets (host, n_frames + 1 entries, ascending, first 0,
 * last n_pts) splits d_xyz into frames voxelized independently; NULL with
 * n_frames <= 1 means one frame. The voxel list is ordered by frame, then by
 * ascending key; within a voxel, points keep their input order (stable).
 *
 * Outputs (caller-allocated, device):
 *   d_keys[cap_vox]    voxel keys
 *   d_offsets[cap_vox] start of each voxel in the sorted point order
 *   d_counts[cap_vox]  points per voxel (before the max_pts cap)
 *   d_perm[n_pts]      sorted position -> input point index; frame f's
 *                      positions stay inside frame f's input range, and its
 *                      non-finite points come after its voxels
 * Host outputs: *h_n_vox = voxel count; h_frame_vox (nullable, n_frames + 1)
 * = cumulative voxel count per frame; h_n_invalid (nullable) = non-finite
 * points. If the voxel count exceeds cap_vox the call returns
 * VGPR_E_CAPACITY with *h_n_vox set to the required size. n_pts < 2^31.
 */
VGPR_API vgpr_status vgpr_voxelize(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts,
                          const int64_t* h_frame_offsets, int32_t n_frames,
                          const vgpr_params* params, uint64_t* d_keys, int32_t* d_offsets,
                          int32_t* d_counts, int32_t* d_perm, int64_t cap_vox,
                          int64_t* h_n_vox, int64_t* h_frame_vox, int64_t* h_n_invalid);

/*
 * vgpr_fit_predict - Alg. 1 per voxel after STORE (Sec. 3.1, Eq. (1)-(3)).
 *
 * For voxel v, its kept points are d_xyz[d_perm[d_offsets[v] + i]],
 * i < min(d_counts[v], max_pts) (d_perm may be NULL: then the points are
 * d_xyz[d_offsets[v] + i]). n_pts is the number of points d_xyz holds (the
 * length of d_perm); it sizes a staging scratch of 16 * n_pts bytes. Voxels
 * must satisfy 0 <= d_offsets[v] and d_offsets[v] + min(d_counts[v], max_pts)
 * <= n_pts; a voxel that does not is skipped (status 0, NaN rows).
 * With n kept points and n >= min_pts:
 *  - PCA (double): centroid c, covariance (1/n) sum (p - c)(p - c)^T, eigenvector
 *    of its smallest eigenvalue v; value axis a = argmax_k |v_k| (ties to the
 *    lower index); parameter axes (u, w) = (Y,Z), (Z,X), (X,Y) for a = X, Y, Z.
 *  - f_i = p_i[a] with the constant prior mean mu = mean(f); x_i = (p_i[u], p_i[w]).
 *  - queries x*_q on the voxel face: coordinate (k + (i + 1/2)/n_q) s evaluated
 *    in double and rounded to float, q = i n_q + j, i along u.
 *  - kappa(x, x') = s_f^2 exp(-|x - x'|^2 / (2 l^2)); K + diag(sigma^2) with
 *    sigma^2 = noise_var, or d_noise_var[input index] when d_noise_var != NULL.
 *  - mean_q = mu + k*_q^T (K + S)^-1 (f - mu), var_q = s_f^2 - k*_q^T (K + S)^-1 k*_q
 *    (the diagonal of Sigma* of Eq. (3)), var clamped at 0.
 * Outputs (caller-allocated, device):
 *   d_out[n_vox * m * 4]  float x, y, z, var of query q of voxel v at row v*m + q:
 *                         coordinate a = mean_q, (u, w) = x*_q; NaN rows for
 *                         unsolved voxels
 *   d_axis[n_vox]         value axis 0/1/2, -1 when not solved
 *   d_status[n_vox]       VGPR_ST_* bits
 * Asynchronous: returns after enqueueing.
 */
VGPR_API vgpr_status vgpr_fit_predict(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts, const uint64_t* d_keys,
                             const int32_t* d_offsets, const int32_t* d_counts,
                             const int32_t* d_perm, int64_t n_vox, const float* d_noise_var,
                             const vgpr_params* params, float* d_out, int8_t* d_axis,
                             uint8_t* d_status);

/*
 * vgpr_fit_predict_noalloc - vgpr_fit_predict for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, outputs and results as
 * vgpr_fit_predict (the same kernels run), but its scratch comes from a fixed
 * device array of 64 MiB, one per GPU, held until the process ends; the call
 * itself allocates nothing (no hipMalloc / hipFree, no stream or event
 * creation: the context made its side streams at vgpr_create). The caller
 * still owns every input and output buffer.
 * Limit: the call's scratch (about 525 bytes per voxel + 16 bytes per point,
 * plus the tiled solvers' areas when max_pts > 128 or in MIXED mode) must fit
 * in the 64 MiB; otherwise it returns VGPR_E_CAPACITY and enqueues nothing.
 * Concurrency: every call on one GPU (from any context) shares that GPU's
 * array, which keeps the last call's contents; calls whose work overlaps on
 * one GPU race, so callers serialise them (one stream, or events).
 * Asynchronous like vgpr_fit_predict.
 */
VGPR_API vgpr_status vgpr_fit_predict_noalloc(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts,
                                              const uint64_t* d_keys, const int32_t* d_offsets,
                                              const int32_t* d_counts, const int32_t* d_perm, int64_t n_vox,
                                              const float* d_noise_var, const vgpr_params* params,
                                              float* d_out, int8_t* d_axis, uint8_t* d_status);

/*
 * Device-resident voxel map (the global map C of Alg. S1 with the voxel
 * states of Sec. 3.3). Holds up to max_voxels voxels, each with up to
 * params.max_pts points stored in arrival order; later points of a full voxel
 * are dropped. The map owns its device memory (about
 * max_voxels * (32 + 12 * max_pts) bytes plus a hash table of
 * 2 * max_voxels 8-byte slots), counted against the context's budget. Its
 * updates' solves run from a staging area that the context holds and its
 * maps share, grown to the largest update so far: the re-solved voxels'
 * stored points back to back (28 bytes per point with the solver's copy),
 * about 530 bytes per re-solved voxel, and the tiled solvers' fixed scratch
 * when max_pts > 64. An update's scratch therefore scales with the voxels it
 * re-solves, not with max_voxels.
 */
VGPR_API vgpr_status vgpr_map_create(vgpr_ctx* ctx, const vgpr_params* params, int64_t max_voxels,
                            vgpr_map** out);

/*
 * vgpr_map_create_ex - as vgpr_map_create with an update mode.
 * update_mode 0: the map above (type (c) voxels re-solved on their stored
 * points). update_mode 1: the covariance-centred update of Sec. 3.3 (Fig. 4).
 * A voxel's first solve (type (b), on its pooled points) puts it in the map
 * with its m = grid_side^2 predicted rows (x, y, z, var), kept as float32;
 * its pool then stops growing. A later frame that touches it (type (c))
 * re-solves Alg. 1 on the m carried rows, each with its posterior variance
 * (raised to 1e-6 signal_var) as its noise variance, stacked with the
 * frame's first max_pts points in that voxel (sensor noise_var); the new
 * rows replace the carried ones, and the voxel is converged (type (d)) once
 * their max variance <= converge_var. CAPPED then reports that the frame
 * brought more than max_pts points to the voxel. Needs grid_side^2 + max_pts
 * <= 512 and max_voxels * grid_side^2 < 2^31; the map owns an extra
 * max_voxels * (16 m + 1) bytes, and its updates take about
 * 48 (m + max_pts) bytes per re-solved voxel of the context's staging area.
 * Errors: E_INVALID for another update_mode or those limits.
 */
VGPR_API vgpr_status vgpr_map_create_ex(vgpr_ctx* ctx, const vgpr_params* params, int64_t max_voxels,
                               int update_mode, vgpr_map** out);
VGPR_API vgpr_status vgpr_map_destroy(vgpr_map* map);

/*
 * vgpr_map_update - one frame through the map (Sec. 3.3).
 * The frame's points (world frame) are voxelized (Alg. S1) and appended to
 * their voxels. Every voxel the frame touched that now holds >= min_pts
 * points and is not converged (types (b) and (c)) is re-solved on all its
 * stored points; it becomes converged (type (d)) once its max predicted
 * variance <= converge_var and is skipped afterwards, as are voxels with
 * too few points (type (a)).
 * Outputs: the re-solved voxels in ascending key order, *h_n_upd of them:
 * d_upd_keys[cap_upd], d_out[cap_upd * m * 4], d_axis[cap_upd],
 * d_status[cap_upd] as in vgpr_fit_predict. VGPR_E_CAPACITY when the map
 * would exceed max_voxels (the frame is then not applied) or when more than
 * cap_upd voxels were re-solved (*h_n_upd = required; the map state is
 * updated but outputs are incomplete).
 */
VGPR_API vgpr_status vgpr_map_update(vgpr_map* map, const float* d_xyz, int64_t n_pts, uint64_t* d_upd_keys,
                            float* d_out, int8_t* d_axis, uint8_t* d_status, int64_t cap_upd,
                            int64_t* h_n_upd);

/* Map counters: voxels held, points stored, converged voxels (host outputs, nullable). */
VGPR_API vgpr_status vgpr_map_stats(vgpr_map* map, int64_t* h_n_voxels, int64_t* h_n_points,
                           int64_t* h_n_converged);

/*
 * vgpr_map_export / vgpr_map_import - checkpoint and resume of a map (the
 * state of Sec. 3.3 that the paper keeps across frames), through host memory.
 *
 * Export writes the map's whole state into the caller's host buffer h_buf of
 * buf_bytes bytes: an 80-byte header (magic "VGPRMAP1" at byte 0, version 1
 * as u32 at 8, update mode as i32 at 12, voxel count V as i64 at 16, the
 * vgpr_params the map was created with at 24), then in native
 * (little-endian) byte order: V voxel keys (u64, in insertion order), V
 * stored point counts (i32), V arrived point counts (i32), V converged flags
 * (u8), for update mode 1 V in-map flags (u8), the point pool (V * max_pts *
 * 3 float32), and for update mode 1 the predicted rows (V * grid_side^2 *
 * 4 float32). *h_needed receives the size; with h_buf = NULL only the size is
 * returned. Synchronises the map's stream. Errors: E_CAPACITY when buf_bytes <
 * *h_needed.
 *
 * Import creates a new map on ctx (as vgpr_map_create_ex, with the serialised
 * parameters and update mode, and max_voxels >= V) holding that state: later
 * updates of it give the same results as updates of the exported map would.
 * Errors: E_INVALID (not a serialised map, wrong version, truncated buffer,
 * max_voxels < V, a stored count outside [0, max_pts], parameters the library
 * rejects), E_BUDGET, E_DEVICE.
 */
VGPR_API vgpr_status vgpr_map_export(vgpr_map* map, void* h_buf, size_t buf_bytes, size_t* h_needed);
VGPR_API vgpr_status vgpr_map_import(vgpr_ctx* ctx, const void* h_buf, size_t buf_bytes, int64_t max_voxels,
                                     vgpr_map** out);

/*
 * vgpr_gauss_init - initial 3D Gaussians from the predicted grids (Sec. 3.2).
 *
 * d_out / d_status: n_vox voxels as written by vgpr_fit_predict (or
 * vgpr_map_update) with grid side grid_side (m = grid_side^2 float4 rows per
 * voxel, row q = i grid_side + j). The grid splits into n_s x n_s subgrids of
 * n_r x n_r points, n_s = grid_side / n_r (the paper's n_s intervals with n_r
 * neighbours each); subgrid beta = bi n_s + bj holds rows i in [bi n_r,
 * (bi + 1) n_r) and columns j in [bj n_r, (bj + 1) n_r). Each point's weight
 * is 1 / max(var, var_floor). Per subgrid, d_gauss receives 8 floats:
 * (p_x, p_y, p_z, sum of weights, S_x, S_y, S_z, 0) with p the weighted mean
 * position and S the diagonal of the weighted scatter sum w (P - p)(P - p)^T
 * / sum w; the rotation is the identity. d_gauss: n_vox * n_s^2 * 8 floats,
 * caller-owned, 16-byte aligned. Voxels without the SOLVED bit get NaN.
 * Enqueued on the context's stream. Errors: E_INVALID (n_r does not divide
 * grid_side, grid_side outside 1..16, var_floor <= 0, null or misaligned
 * pointers).
 */
VGPR_API vgpr_status vgpr_gauss_init(vgpr_ctx* ctx, const float* d_out, const uint8_t* d_status, int64_t n_vox,
                                     int32_t grid_side, int32_t n_r, float var_floor, float* d_gauss);

/*
 * vgpr_structure_loss - structure similarity loss L_p of Eq. (9) (Sec. 3.3).
 *
 * d_pts: n_pts scan points (float32 x, y, z). d_gauss: n_gauss Gaussians of 8
 * floats in the vgpr_gauss_init layout (p_x, p_y, p_z, *, S_x, S_y, S_z, *),
 * 16-byte aligned. S-bar_k = mean of S_x, S_y, S_z (scale_mode 0) or of their
 * square roots (scale_mode 1: S holds variances, as vgpr_gauss_init writes).
 * A Gaussian whose centre or S-bar is not finite (an unsolved voxel's NaN row)
 * is not a candidate. For every point: value = min over candidates of
 * (|P - p_k|_2 - S-bar_k) in float32, index = the k attaining it (the lowest k
 * among equal values); *h_loss = the mean of the values over the finite
 * points (accumulated in double, in a fixed order), *h_n_valid their number.
 * Non-finite points get value NaN and index -1 and are left out; with no
 * candidate every finite point gets +inf and -1 and the loss is +inf; with no
 * finite point the loss is NaN. The search is exact on a uniform grid of
 * cell_size (> 0; a spacing near that of the Gaussians is fastest); the
 * result does not depend on cell_size. d_value (n_pts floats) and d_arg
 * (n_pts int32) are caller-owned and nullable. Synchronises the context's
 * stream. Errors: E_INVALID (sizes, null or misaligned pointers, cell_size,
 * scale_mode), E_RANGE (a Gaussian's cell index beyond +-(2^20 - 1)),
 * E_BUDGET.
 */
VGPR_API vgpr_status vgpr_structure_loss(vgpr_ctx* ctx, const float* d_pts, int64_t n_pts, const float* d_gauss,
                                         int64_t n_gauss, float cell_size, int scale_mode, float* d_value,
                                         int32_t* d_arg, double* h_loss, int64_t* h_n_valid);

/*
 * Captured form of vgpr_fit_predict (the batching form: every size bucket's
 * persistent launch, the side-stream fork and join, recorded once as a HIP
 * graph and replayed with one launch).
 *
 * vgpr_fit_graph_create takes exactly the arguments of vgpr_fit_predict and
 * records that call on the context's stream, which must not be the default
 * (NULL) stream. Nothing runs at capture time. Every buffer pointer, n_pts,
 * n_vox, the parameters and the context's launch choices are fixed in the
 * graph; the buffers' contents are read when the graph runs, so a replay
 * after the inputs were rewritten (for example a new batch voxelized into the
 * same buffers with the same n_vox) computes that batch. The caller keeps the
 * buffers alive and unchanged in size until vgpr_graph_destroy. The graph owns
 * its scratch (allocated at creation inside the context's HBM budget).
 * Errors: E_INVALID (default stream, n_vox or n_pts <= 0), E_BUDGET / E_NOMEM
 * for the scratch, E_DEVICE if capture or instantiation fails.
 *
 * vgpr_graph_launch enqueues one replay on the context's stream (asynchronous,
 * like vgpr_fit_predict). vgpr_graph_destroy waits for the context's stream
 * and frees the graph; a context cannot be destroyed while graphs are alive.
 */
typedef struct vgpr_graph vgpr_graph;

VGPR_API vgpr_status vgpr_fit_graph_create(vgpr_ctx* ctx, const float* d_xyz, int64_t n_pts,
                                           const uint64_t* d_keys, const int32_t* d_offsets,
                                           const int32_t* d_counts, const int32_t* d_perm, int64_t n_vox,
                                           const float* d_noise_var, const vgpr_params* params, float* d_out,
                                           int8_t* d_axis, uint8_t* d_status, vgpr_graph** out);
VGPR_API vgpr_status vgpr_graph_launch(vgpr_graph* graph);
VGPR_API vgpr_status vgpr_graph_destroy(vgpr_graph* graph);

/*
 * Launch choices of vgpr_fit_predict. streams, grid_scale and tiled_first
 * change only timing (results are bit-identical); fp32_last_bucket and wave_last_bucket
 * change the rounding (which arithmetic and which solver a voxel gets), and
 * every choice stays within the stated tolerances. Buckets hold voxels of up to
 * 16, 32, 64, 96, 128, 256 and 512 kept points (index 0..6); buckets from
 * tile_first_bucket on run the tiled FP64 solver. Defaults come from the project's
 * autotuner on the spinning-scan workload.
 */
typedef struct {
  int32_t fp32_last_bucket;   /* FP32 mode: buckets 0..this run in float first (-1: none) */
  int32_t wave_last_bucket;   /* grids of up to 64 points: buckets 0..this use the one-voxel-per-
                                 wavefront solver (max 2), the others one voxel per workgroup */
  int32_t streams;            /* 1: every bucket on the context's stream; 3: buckets fork onto
                                 the three side streams as bucket_stream says and join back */
  int32_t grid_scale[7];      /* persistent grid of bucket b = grid_scale[b] / 4 x the resident
                                 workgroups the device holds (1..64; buckets 5 and 6 use at
                                 most 4, one resident wave of workgroups) */
  int32_t tile_first_bucket;  /* buckets from this one on (2..5) run a tiled solver on the
                                 matrix cores (FP64, or the mixed form in MIXED mode); buckets
                                 5 and 6 always do */
  int32_t tiled_first;        /* with streams = 3: 1 runs the tiled buckets first, alone on the
                                 context's stream (their workgroups need whole CUs, which other
                                 buckets' workgroups would hold), and forks the others after
                                 them; 0 forks every bucket at once */
  int32_t bucket_stream[7];   /* with streams = 3: stream of bucket b, 0 the context's stream,
                                 1..3 the side streams; buckets on one stream run one after
                                 another, largest first (default {0, 2, 2, 1, 1, 3, 3}: 16
                                 points on the context's stream, 96/128, 32/64 and 256/512
                                 points each on one side stream) */
  int32_t tiled_merge;        /* 1: the 256- and 512-point buckets run as one longest-first
                                 launch of the 512-point tiled solver (the smaller voxels fill
                                 the CUs the larger ones leave idle); 0: one launch each */
} vgpr_tuning;

VGPR_API vgpr_status vgpr_set_tuning(vgpr_ctx* ctx, const vgpr_tuning* t);
VGPR_API vgpr_status vgpr_get_tuning(const vgpr_ctx* ctx, vgpr_tuning* t);

/*
 * Kernel timing for measurement. When enabled, the library records HIP
 * events on the context's stream around each launch of its kernels.
 * vgpr_profile_read synchronises the stream and returns, for the kernel
 * family `name`, the summed duration in milliseconds and the number of
 * launches since the last read of that family, then resets it. Families:
 * "voxelize_key", "voxelize_sort" (all radix passes of a call),
 * "voxelize_segment", "classify" (tau test, frames and bucket slots), "nan_rows"
 * (the rows of voxels below tau), "gauss_init", "structure_loss" (the ring-search
 * kernel of vgpr_structure_loss), "structure_loss_brute" (its brute-force pass
 * over points far from every Gaussian), "fit_mix_n<C>" (MIXED mode tiled
 * solver), "fit_f32_n<C>" / "fit_f64_n<C>" (the
 * per-voxel solver over the size bucket of capacity C = 16, 32, 64, 96, 128, 256, 512) and
 * "refine_f64_n<C>" (the FP64 re-solve of flagged voxels of that bucket).
 */
VGPR_API vgpr_status vgpr_profile_enable(vgpr_ctx* ctx, int on);
VGPR_API vgpr_status vgpr_profile_read(vgpr_ctx* ctx, const char* name, double* h_total_ms,
                              int64_t* h_launches);

#ifdef __cplusplus
}
#endif

#endif /* VGPR_H */
