"""FP64 CPU oracle for the Voxel-GPR hot path (GS-LIVM, arXiv 2410.17084).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link
or execute this module: only the tests, the smoke check and the bench's CPU
baseline leg use it. It shares no code, header, table or constant generator
with the HIP library; the only thing both sides consume in common are the
seeded point clouds from the synthetic generators.

What it computes, in the paper's order (Sec. 3.1, Alg. 1; supplementary Alg. S1):

1. ``voxelize`` - the STORE step of Alg. S1: every point gets a voxel key
   (the paper's HASH, unspecified there; read here as a packed floor key, see
   ``voxel_coords`` / ``pack_keys``) and is pushed into its voxel's point list.
   The voxel list is S_updated.
2. ``local_frame`` - Alg. 1's PCA and axis switch: the value axis is the world
   axis making the smallest angle with the voxel's PCA eigenvector, the two
   parameter axes follow in the cyclic order the algorithm lists.
3. ``query_grid`` - Alg. 1's MeshGrid: an evenly spaced grid of interval
   centres on the voxel face spanned by the parameter axes (Sec. 3.1, and
   Sec. 3.2 for n_q = n_s * n_r points per side).
4. ``gp_posterior`` - Eq. (2)-(3): the squared-exponential kernel of Sec. 3.1
   and the GP posterior mean and covariance of the predictions.
5. ``fit_predict_voxel`` / ``fit_predict`` - Alg. 1 end to end for one voxel /
   for every voxel of a frame: predicted points (f*, x*) plus their variances.
6. ``map_update`` - the voxel state machine of Sec. 3.3 (types (a)-(d)).
7. ``gauss_init`` - Sec. 3.2: one 3D Gaussian per n_r x n_r subgrid of a
   voxel's predicted points, position = inverse-variance weighted mean,
   covariance = weighted scatter about it, scale = its diagonal, rotation =
   identity.

Precision: all arithmetic is float64 on the float32 inputs converted exactly.
Library primitives used as single steps: ``numpy.argsort`` (stable sort),
``numpy.linalg.eigh`` (symmetric eigensolver), ``scipy.linalg.cho_factor`` /
``cho_solve`` / ``solve_triangular`` (the SPD solve of Eq. (3)).

Readings of points the paper leaves open: the key packing, half-open voxels,
stable point order, the cap policy, smallest-eigenvalue eigenvector, |v| for
the angle, cyclic parameter axes, a constant prior mean equal to the sample
mean of f, the kernel scale s_f^2 and length scale l in place of lambda, the
grid of interval centres, output of the diagonal of Sigma*, convergence as
max var <= eta, the axis convention of the rotated frame (frame_mode 1), the
carried rows and noise of the covariance-centred type (c) update, and for
Eq. (9) the mean over the n points with S-bar the mean of the three scales.

Parity status: every function here is pinned by closed forms, invariants,
brute force or an independent library routine in tests/test_oracle_pins.py.
The per-voxel length-scale rule ``pca_length_scale`` (ls_mode 1, for the large
aggregated-map workload) is not defined by the paper: the rule is a reading of
this implementation, and what is pinned is that the oracle computes that rule
(closed forms on lattice rectangles with distinct in-plane variances, the
uniform square, both clamp edges).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np
import scipy.linalg

# ----------------------------------------------------------------------------
# Interface constants (status bits and key layout). They are restated here on
# purpose rather than shared with the C header: the two sides must agree by
# specification, not by a common file.
# ----------------------------------------------------------------------------
KEY_FIELD_BITS = 21
KEY_BIAS = 1 << 20                 # per-axis bias: field = k + 2^20
KEY_AXIS_LIMIT = (1 << 20) - 1     # |k| above this is out of range
KEY_SENTINEL = np.uint64(0xFFFFFFFFFFFFFFFF)  # key of a non-finite point

ST_SOLVED = 1       # the GP was fitted and the grid predicted
ST_BELOW_TAU = 2    # kept point count below tau: not solved (type (a))
ST_CAPPED = 4       # more points than the cap arrived; extras dropped in order
ST_REFINED = 8      # (GPU only) FP64 refinement step applied
ST_FACTOR_FAIL = 16  # (GPU only) FP32 factor broke down, FP64 fallback used
ST_CONVERGED = 32   # max predicted variance <= eta (type (d))
ST_AXIS_TIE = 64    # value-axis decision is numerically ambiguous

# Cyclic parameter axes for each value axis (Alg. 1: X -> (Y, Z), Y -> (Z, X),
# Z -> (X, Y)).
PARAM_AXES = {0: (1, 2), 1: (2, 0), 2: (0, 1)}

# Ambiguity margins for the value-axis decision (see ``local_frame``).
AXIS_MARGIN = 1e-6
EIGEN_GAP_REL = 1e-8


class OracleRangeError(ValueError):
    """A finite point's voxel index lies outside the 21-bit key range."""


@dataclass(frozen=True)
class Params:
    """Hyper-parameters of one Voxel-GPR run.

    Defaults follow the paper where it fixes a value: tau = 10, n_s = n_r = 3
    (n_q = 9), eta = 0.3, voxel 0.2 m (Table S6); lambda = 1 (Sec. 3.1) is
    s_f^2 = 1 and l = 1/sqrt(2) m.
    """
    voxel_size: float = 0.2
    max_pts: int = 128
    min_pts: int = 10
    grid_side: int = 9
    signal_var: float = 1.0
    length_scale: float = 1.0 / math.sqrt(2.0)
    noise_var: float = 1e-3
    ls_mode: int = 0          # 0 fixed l, 1 per-voxel l from PCA eigenvalues
    converge_var: float = 0.3
    frame_mode: int = 0       # 0 world value axis (Alg. 1), 1 PCA-rotated local frame


# ----------------------------------------------------------------------------
# 1. STORE / HASH (Alg. S1)
# ----------------------------------------------------------------------------
def voxel_coords(xyz: np.ndarray, voxel_size: float):
    """Integer voxel index of every point and a finiteness mask.

    k = floor(p * (1/s)) per axis, where 1/s is computed once in float64 from
    the float32 voxel size, and the product is one IEEE float64 multiply of
    the exactly converted float32 coordinate. Voxels are half-open
    [k s, (k+1) s).
    """
    p = np.asarray(xyz, dtype=np.float32).astype(np.float64)
    inv_s = 1.0 / np.float64(np.float32(voxel_size))
    valid = np.all(np.isfinite(p), axis=1)
    with np.errstate(invalid="ignore", over="ignore"):
        k = np.floor(p * inv_s)
    k[~valid] = 0
    if valid.any() and np.abs(k[valid]).max() > KEY_AXIS_LIMIT:
        raise OracleRangeError("voxel index outside +-(2^20 - 1)")
    return k.astype(np.int64), valid


def pack_keys(k: np.ndarray, valid: np.ndarray | None = None) -> np.ndarray:
    """Pack (kx, ky, kz) into one 64-bit key: biased 21-bit fields, x highest."""
    k = np.asarray(k, dtype=np.int64)
    b = (k + KEY_BIAS).astype(np.uint64)
    key = (b[:, 0] << np.uint64(2 * KEY_FIELD_BITS)) | (b[:, 1] << np.uint64(KEY_FIELD_BITS)) | b[:, 2]
    if valid is not None:
        key = np.where(valid, key, KEY_SENTINEL)
    return key.astype(np.uint64)


def unpack_key(key) -> tuple[int, int, int]:
    key = int(key)
    m = (1 << KEY_FIELD_BITS) - 1
    return ((key >> (2 * KEY_FIELD_BITS)) & m) - KEY_BIAS, ((key >> KEY_FIELD_BITS) & m) - KEY_BIAS, \
        (key & m) - KEY_BIAS


def voxelize(xyz: np.ndarray, voxel_size: float, frame_offsets=None) -> dict:
    """Alg. S1 for one or several frames.

    Each frame's points are grouped by voxel key; S_updated is the frame's
    list of distinct keys in ascending order, and each voxel's points keep
    their arrival order (a stable sort). Several frames are voxelized
    independently and their lists concatenated in frame order. Non-finite
    points get the sentinel key, sort after the frame's voxels and belong to
    no voxel.

    Returns keys (V,) uint64; offsets (V,) start of each voxel in the sorted
    order; counts (V,); perm (N,) sorted position -> input index (frame f's
    points stay in frame f's index range); frame_vox (F+1,) voxel ranges per
    frame; n_invalid.
    """
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    n = len(xyz)
    if frame_offsets is None:
        frame_offsets = np.array([0, n], dtype=np.int64)
    frame_offsets = np.asarray(frame_offsets, dtype=np.int64)
    if n:
        k, valid = voxel_coords(xyz, voxel_size)
        allkeys = pack_keys(k, valid)
    else:
        valid = np.zeros(0, dtype=bool)
        allkeys = np.zeros(0, dtype=np.uint64)
    perm = np.empty(n, dtype=np.int64)
    keys, offsets, counts, frame_vox = [], [], [], [0]
    for f in range(len(frame_offsets) - 1):
        a, b = int(frame_offsets[f]), int(frame_offsets[f + 1])
        order = np.argsort(allkeys[a:b], kind="stable")
        perm[a:b] = a + order
        sk = allkeys[a:b][order]
        nv = int(np.count_nonzero(sk != KEY_SENTINEL))
        sk = sk[:nv]
        if nv:
            head = np.ones(nv, dtype=bool)
            head[1:] = sk[1:] != sk[:-1]
            starts = np.flatnonzero(head)
            ends = np.append(starts[1:], nv)
            keys.extend(sk[starts].tolist())
            offsets.extend((a + starts).tolist())
            counts.extend((ends - starts).tolist())
        frame_vox.append(len(keys))
    return {
        "keys": np.asarray(keys, dtype=np.uint64),
        "offsets": np.asarray(offsets, dtype=np.int64),
        "counts": np.asarray(counts, dtype=np.int64),
        "perm": perm,
        "frame_vox": np.asarray(frame_vox, dtype=np.int64),
        "n_invalid": int(np.count_nonzero(~valid)),
    }


# ----------------------------------------------------------------------------
# 2. PCA frame and value-axis switch (Alg. 1)
# ----------------------------------------------------------------------------
@dataclass
class Frame:
    axis: int                  # value axis (0 = X, 1 = Y, 2 = Z)
    params: tuple[int, int]    # parameter axes (u, w), cyclic
    centroid: np.ndarray       # (3,)
    eigvals: np.ndarray        # ascending
    normal: np.ndarray         # eigenvector of the smallest eigenvalue
    ambiguous: bool = False


def local_frame(P: np.ndarray) -> Frame:
    """PCA of the voxel's points and the value-axis decision.

    Covariance C = (1/n) sum (p - c)(p - c)^T about the centroid c. The
    eigenvector taken is the one of the smallest eigenvalue (the local surface
    normal), so the parameter axes span the surface and the grid on them is a
    graph of the value coordinate. The angle between that eigenvector (a line:
    its sign is arbitrary) and world axis k is arccos |v_k|, so the smallest
    angle is the largest |v_k|; exact ties go to the lower axis index.

    The decision is flagged ambiguous when the two largest |v_k| are within
    AXIS_MARGIN or the two smallest eigenvalues are within EIGEN_GAP_REL of
    the trace: there a rounding-level difference can flip the axis.
    """
    P = np.asarray(P, dtype=np.float64)
    c = P.mean(axis=0)
    D = P - c
    C = (D.T @ D) / len(P)
    w, V = np.linalg.eigh(C)
    v = V[:, 0]
    av = np.abs(v)
    a = int(np.argmax(av))
    s = np.sort(av)
    tr = float(np.trace(C))
    amb = bool((s[2] - s[1]) < AXIS_MARGIN or (w[1] - w[0]) <= EIGEN_GAP_REL * tr)
    return Frame(axis=a, params=PARAM_AXES[a], centroid=c, eigvals=w, normal=v, ambiguous=amb)


def rotated_frame(fr: Frame) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Orthonormal local frame (e1, e2, v) of the PCA-rotated variant (frame_mode 1).

    v is the surface normal of `local_frame` with its largest component made
    positive (the sign of an eigenvector is arbitrary). The in-plane axes are
    not the other two eigenvectors, whose directions are undefined when their
    eigenvalues coincide (a roughly isotropic patch); instead e1 is the unit
    vector along e_k x v, e_k the world axis least aligned with v (smallest
    |v_k|, ties to the lower index), and e2 = v x e1, a right-handed frame
    that depends continuously on v.
    """
    v = np.asarray(fr.normal, dtype=np.float64)
    v = v / np.linalg.norm(v)
    if v[fr.axis] < 0:
        v = -v
    k = int(np.argmin(np.abs(v)))
    ek = np.zeros(3)
    ek[k] = 1.0
    e1 = np.cross(ek, v)
    e1 = e1 / np.linalg.norm(e1)
    e2 = np.cross(v, e1)
    return e1, e2, v


def rotated_grid(voxel_size: float, n_q: int) -> np.ndarray:
    """Query grid of frame_mode 1: interval centres of an s x s square centred
    on the voxel's centroid in its (e1, e2) plane; row q = i n_q + j, i along e1."""
    s = float(np.float32(voxel_size))
    t = np.array([((i + 0.5) / n_q - 0.5) * s for i in range(n_q)])
    return np.stack([np.repeat(t, n_q), np.tile(t, n_q)], axis=1)


def pca_length_scale(eigvals: np.ndarray, voxel_size: float) -> float:
    """Per-voxel length scale for the aggregated-map workload (ls_mode 1).

    l = sqrt(3) * sqrt((lambda_mid + lambda_max) / 2), clamped to
    [0.05 s, 2 s]. For points uniform on an a x b rectangle the in-plane
    variances are a^2/12 and b^2/12, so l = sqrt((a^2 + b^2) / 8); for a face of
    side s that is s/2. Not defined by the paper (a reading of this
    implementation); the pins check the oracle against that rule.
    """
    s = float(np.float32(voxel_size))
    ell = math.sqrt(3.0) * math.sqrt(max((eigvals[1] + eigvals[2]) / 2.0, 0.0))
    return min(max(ell, 0.05 * s), 2.0 * s)


# ----------------------------------------------------------------------------
# 3. MeshGrid (Alg. 1, Sec. 3.1-3.2)
# ----------------------------------------------------------------------------
def query_grid(k_u: int, k_w: int, voxel_size: float, n_q: int) -> np.ndarray:
    """Query points x* on the voxel face spanned by the parameter axes.

    Each side of the voxel [k s, (k+1) s) is split into n_q equal intervals
    and one query sits at every interval centre: coordinate
    (k + (i + 1/2)/n_q) * s, evaluated in float64 as written ((i + 0.5) / n_q,
    then + k, then * s) and rounded once to float32, so that both
    implementations query the very same points. Row q = i * n_q + j with i
    along u and j along w.
    """
    s = np.float64(np.float32(voxel_size))
    t = (np.arange(n_q, dtype=np.float64) + 0.5) / np.float64(n_q)
    gu = ((np.float64(k_u) + t) * s).astype(np.float32).astype(np.float64)
    gw = ((np.float64(k_w) + t) * s).astype(np.float32).astype(np.float64)
    U, W = np.meshgrid(gu, gw, indexing="ij")
    return np.stack([U.ravel(), W.ravel()], axis=1)


# ----------------------------------------------------------------------------
# 4. GP posterior (Eq. (2)-(3))
# ----------------------------------------------------------------------------
def se_kernel(A: np.ndarray, B: np.ndarray, signal_var: float, length_scale: float) -> np.ndarray:
    """kappa(a, b) = s_f^2 exp(-||a - b||^2 / (2 l^2)).

    The paper writes exp(-lambda ||a - b||^2) with lambda = 1, i.e.
    s_f^2 = 1 and l = 1/sqrt(2).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    d2 = ((A[:, None, :] - B[None, :, :]) ** 2).sum(axis=-1)
    return signal_var * np.exp(-d2 / (2.0 * length_scale * length_scale))


def gp_posterior(x, f, xq, signal_var, length_scale, noise_var, full=False):
    """Posterior mean and variance of Eq. (3) with a constant prior mean.

    mu* = mu_f + K*^T (K + S)^-1 (f - mu_f),  Sigma* = K** - K*^T (K + S)^-1 K*,
    where mu_f is the sample mean of f (the constant mean of Eq. (1)),
    K = kappa(x, x), K* = kappa(x, x*), K** = kappa(x*, x*) and S = sigma^2 I
    (or diag of per-point noise variances). The SPD solve goes through a
    Cholesky factor K + S = L L^T; the variance is s_f^2 - ||L^-1 k*_q||^2,
    the diagonal of Sigma*.
    """
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    xq = np.asarray(xq, dtype=np.float64)
    n = len(x)
    mu_f = f.mean()
    ft = f - mu_f
    K = se_kernel(x, x, signal_var, length_scale)
    K[np.diag_indices(n)] += np.broadcast_to(np.asarray(noise_var, dtype=np.float64), (n,))
    Ks = se_kernel(x, xq, signal_var, length_scale)
    L = scipy.linalg.cholesky(K, lower=True)
    alpha = scipy.linalg.cho_solve((L, True), ft)
    mean = mu_f + Ks.T @ alpha
    V = scipy.linalg.solve_triangular(L, Ks, lower=True)
    var = signal_var - (V * V).sum(axis=0)
    if not full:
        return mean, var
    Kss = se_kernel(xq, xq, signal_var, length_scale)
    return mean, var, Kss - V.T @ V


# ----------------------------------------------------------------------------
# 5. Alg. 1 per voxel and per frame
# ----------------------------------------------------------------------------
def fit_predict_voxel(P: np.ndarray, key, params: Params, axis: int | None = None,
                      noise_var=None, n_total: int | None = None) -> dict:
    """Alg. 1 for one voxel.

    P holds the voxel's points in their stored order; only the first
    params.max_pts are used (the cap). Below tau nothing is solved. Otherwise
    the frame picks the value axis a and parameter axes (u, w); f = p[a],
    x = (p[u], p[w]); the query grid sits on the voxel face of (u, w); each
    output row is the world point with coordinate a = mu*_q, (u, w) = x*_q,
    followed by var_q.

    `axis` forces the value axis (used where the decision is ambiguous and
    the implementation under test reports another valid choice).
    """
    P = np.asarray(P, dtype=np.float32).astype(np.float64)
    n_total = len(P) if n_total is None else n_total
    n = min(len(P), params.max_pts)
    P = P[:n]
    m = params.grid_side * params.grid_side
    out = np.full((m, 4), np.nan)
    status = ST_CAPPED if n_total > params.max_pts else 0
    res = {"out": out, "axis": -1, "status": status, "ambiguous": False, "n": n}
    if n < params.min_pts:
        res["status"] |= ST_BELOW_TAU
        return res
    fr = local_frame(P)
    if params.frame_mode == 1:
        return _fit_predict_rotated(P, fr, params, noise_var, n, res)
    a = fr.axis if axis is None else int(axis)
    u, w = PARAM_AXES[a]
    k = unpack_key(key)
    xq = query_grid(k[u], k[w], params.voxel_size, params.grid_side)
    ell = params.length_scale if params.ls_mode == 0 else pca_length_scale(fr.eigvals, params.voxel_size)
    nv = params.noise_var if noise_var is None else np.asarray(noise_var, dtype=np.float64)[:n]
    mean, var = gp_posterior(P[:, [u, w]], P[:, a], xq, params.signal_var, ell, nv)
    out[:, a] = mean
    out[:, u] = xq[:, 0]
    out[:, w] = xq[:, 1]
    out[:, 3] = var
    res["status"] |= ST_SOLVED
    if var.max() <= params.converge_var:
        res["status"] |= ST_CONVERGED
    if fr.ambiguous:
        res["status"] |= ST_AXIS_TIE
    res.update(axis=a, ambiguous=fr.ambiguous, length_scale=ell, frame=fr)
    return res


def _fit_predict_rotated(P, fr, params, noise_var, n, res):
    """frame_mode 1: Alg. 1 in the PCA-rotated frame. With c the centroid,
    x = ((p - c).e1, (p - c).e2) and f = (p - c).v; the predicted world point
    of query x*_q is c + x*_q,1 e1 + x*_q,2 e2 + mu*_q v. Points of a noiseless
    plane have f = 0, so every prediction lies on that plane exactly."""
    e1, e2, v = rotated_frame(fr)
    c = fr.centroid
    D = P - c
    x = np.stack([D @ e1, D @ e2], axis=1)
    f = D @ v
    xq = rotated_grid(params.voxel_size, params.grid_side)
    ell = params.length_scale if params.ls_mode == 0 else pca_length_scale(fr.eigvals, params.voxel_size)
    nv = params.noise_var if noise_var is None else np.asarray(noise_var, dtype=np.float64)[:n]
    mean, var = gp_posterior(x, f, xq, params.signal_var, ell, nv)
    out = res["out"]
    out[:, :3] = c + xq[:, :1] * e1 + xq[:, 1:] * e2 + mean[:, None] * v
    out[:, 3] = var
    res["status"] |= ST_SOLVED
    if var.max() <= params.converge_var:
        res["status"] |= ST_CONVERGED
    if fr.ambiguous:
        res["status"] |= ST_AXIS_TIE
    res.update(axis=fr.axis, ambiguous=fr.ambiguous, length_scale=ell, frame=fr, rotation=(e1, e2, v))
    return res


def voxel_points(xyz, vox, v):
    o = int(vox["offsets"][v])
    c = int(vox["counts"][v])
    return np.asarray(xyz, dtype=np.float32)[vox["perm"][o:o + c]]


def fit_predict(xyz: np.ndarray, vox: dict, params: Params, voxels=None, axes=None) -> dict:
    """Alg. 1 for every voxel of `vox` (or the listed subset).

    Returns out (V, m, 4), axis (V,), status (V,), ambiguous (V,) in voxel
    list order; voxels not listed keep NaN rows and status 0.
    """
    V = len(vox["keys"])
    m = params.grid_side * params.grid_side
    out = np.full((V, m, 4), np.nan)
    axis = np.full(V, -1, dtype=np.int64)
    status = np.zeros(V, dtype=np.int64)
    amb = np.zeros(V, dtype=bool)
    idx = range(V) if voxels is None else voxels
    for v in idx:
        P = voxel_points(xyz, vox, v)
        r = fit_predict_voxel(P, vox["keys"][v], params, axis=None if axes is None else axes[v])
        out[v] = r["out"]
        axis[v] = r["axis"]
        status[v] = r["status"]
        amb[v] = r["ambiguous"]
    return {"out": out, "axis": axis, "status": status, "ambiguous": amb}


# ----------------------------------------------------------------------------
# 6. Voxel state machine across frames (Sec. 3.3, Fig. 4)
# ----------------------------------------------------------------------------
@dataclass
class VoxelMap:
    """Global voxel map C of Alg. S1 with the per-voxel state of Sec. 3.3.

    Each voxel stores up to max_pts points in arrival order (later points are
    dropped once full) and a converged flag. A frame's update solves the
    voxels it touched that hold at least tau points and are not converged
    (types (b) and (c)); types (a) (too few points) and (d) (converged) are
    skipped. A solved voxel becomes converged when its max variance <= eta.

    feedback=True takes the covariance-centred update of type (c) voxels
    (Sec. 3.3, Fig. 4): once a voxel has been solved (it is in the map) it
    keeps its predicted grid rows, stored as float32 like the output rows, and
    the pool is no longer extended. A later frame that touches it re-solves
    Alg. 1 on those rows, each carrying its posterior variance as its noise
    variance, stacked with the frame's new points (the first max_pts of them in
    arrival order, sensor noise), and the new prediction replaces the old one;
    this repeats until the max variance reaches eta (type (d)). Voxels not yet
    in the map accumulate points and take their first solve as without feedback.
    """
    params: Params
    feedback: bool = False
    points: dict = field(default_factory=dict)
    converged: dict = field(default_factory=dict)
    total: dict = field(default_factory=dict)
    pred: dict = field(default_factory=dict)

    def update(self, xyz: np.ndarray) -> dict:
        vox = voxelize(xyz, self.params.voxel_size)
        keys_upd, outs, axes, stats = [], [], [], []
        for v, key in enumerate(vox["keys"].tolist()):
            P = voxel_points(xyz, vox, v)
            self.total[key] = self.total.get(key, 0) + len(P)
            if self.feedback and key in self.pred:
                if self.converged.get(key, False):
                    continue
                r = self._feedback_solve(key, P)
            else:
                have = self.points.get(key)
                stored = P if have is None else np.concatenate([have, P])
                self.points[key] = stored[: self.params.max_pts]
                if self.converged.get(key, False) or len(self.points[key]) < self.params.min_pts:
                    continue
                r = fit_predict_voxel(self.points[key], key, self.params, n_total=self.total[key])
                if self.feedback and r["status"] & ST_SOLVED:
                    self.pred[key] = r["out"].astype(np.float32)
            if r["status"] & ST_CONVERGED:
                self.converged[key] = True
            keys_upd.append(key)
            outs.append(r["out"])
            axes.append(r["axis"])
            stats.append(r["status"])
        m = self.params.grid_side ** 2
        return {
            "keys": np.asarray(keys_upd, dtype=np.uint64),
            "out": np.asarray(outs).reshape(-1, m, 4) if outs else np.zeros((0, m, 4)),
            "axis": np.asarray(axes, dtype=np.int64),
            "status": np.asarray(stats, dtype=np.int64),
        }

    def _feedback_solve(self, key, P: np.ndarray) -> dict:
        """Type (c) re-solve: Alg. 1 on the carried rows stacked with the new
        points; the cap applies to the new points, so the stacked set holds up
        to m + max_pts points. CAPPED reports that the frame brought more than
        max_pts new points; the prediction is kept only when SOLVED."""
        prm = self.params
        X, nz = feedback_inputs(self.pred[key], P, prm)
        m = prm.grid_side ** 2
        r = fit_predict_voxel(X, key, with_params(prm, max_pts=m + prm.max_pts), noise_var=nz)
        r["status"] = (r["status"] & ~ST_CAPPED) | (ST_CAPPED if len(P) > prm.max_pts else 0)
        if r["status"] & ST_SOLVED:
            self.pred[key] = r["out"].astype(np.float32)
        return r


# Smallest noise variance, relative to s_f^2, that a carried prediction takes
# into a type (c) re-solve (a posterior variance can round to 0).
PRED_NOISE_FLOOR = 1e-6


def feedback_inputs(prev: np.ndarray, P: np.ndarray, params: Params):
    """Stacked training set of a type (c) re-solve (Sec. 3.3, Fig. 4): the
    previous prediction's m rows (x, y, z) first, with their posterior
    variances (raised to PRED_NOISE_FLOOR s_f^2) as noise variances, then the
    first max_pts new points in arrival order with the sensor noise variance."""
    prev = np.asarray(prev, dtype=np.float32)
    new = np.asarray(P, dtype=np.float32)[: params.max_pts]
    X = np.concatenate([prev[:, :3], new])
    carried = np.maximum(prev[:, 3].astype(np.float64), PRED_NOISE_FLOOR * params.signal_var)
    nz = np.concatenate([carried, np.full(len(new), params.noise_var)])
    return X, nz


def with_params(p: Params, **kw) -> Params:
    return replace(p, **kw)


def gauss_init(out: np.ndarray, status: np.ndarray, grid_side: int, n_r: int, var_floor: float) -> np.ndarray:
    """Initial 3D Gaussians of Sec. 3.2 from predicted grids.

    out: (V, m, 4) predicted points (x, y, z) and variances, m = grid_side^2,
    row q = i * grid_side + j. The grid splits into n_s x n_s subgrids of
    n_r x n_r points (n_s = grid_side / n_r); subgrid beta = bi * n_s + bj
    holds rows i in [bi n_r, (bi + 1) n_r), columns j in [bj n_r, (bj + 1) n_r).
    Each point gets the weight w = 1 / var (var raised to var_floor first, so a
    zero variance gives a finite weight); the Gaussian's position is the
    weighted mean p = sum w P / sum w, its covariance Phi = Q^T diag(w) Q / sum w
    with Q = P - p, its scale S = diag(Phi) and its rotation the identity.

    Returns (V, n_s^2, 8): (p_x, p_y, p_z, sum w, S_x, S_y, S_z, 0); voxels
    whose status lacks SOLVED get NaN rows.
    """
    out = np.asarray(out, dtype=np.float64)
    V, m = out.shape[0], out.shape[1]
    assert m == grid_side * grid_side and grid_side % n_r == 0
    n_s = grid_side // n_r
    res = np.full((V, n_s * n_s, 8), np.nan)
    for v in range(V):
        if not int(status[v]) & ST_SOLVED:
            continue
        g = out[v].reshape(grid_side, grid_side, 4)
        for bi in range(n_s):
            for bj in range(n_s):
                blk = g[bi * n_r:(bi + 1) * n_r, bj * n_r:(bj + 1) * n_r].reshape(-1, 4)
                P = blk[:, :3]
                w = 1.0 / np.maximum(blk[:, 3], var_floor)
                sw = w.sum()
                p = (P * w[:, None]).sum(axis=0) / sw
                Q = P - p
                phi = Q.T @ np.diag(w) @ Q / sw
                res[v, bi * n_s + bj] = [p[0], p[1], p[2], sw, phi[0, 0], phi[1, 1], phi[2, 2], 0.0]
    return res


def gaussian_mean_scale(gauss: np.ndarray, scale_mode: int) -> np.ndarray:
    """S-bar_k of Eq. (9): the mean of Gaussian k's three scale values. Rows are
    in the layout gauss_init returns (p_x, p_y, p_z, sum w, S_x, S_y, S_z, 0).
    scale_mode 0 averages S as stored; scale_mode 1 averages their square roots
    (S holding variances, as the initial Gaussians of Sec. 3.2 do)."""
    G = np.asarray(gauss, dtype=np.float32).astype(np.float64).reshape(-1, 8)
    S = G[:, 4:7]
    if scale_mode == 1:
        with np.errstate(invalid="ignore"):
            S = np.sqrt(S)
    elif scale_mode != 0:
        raise ValueError("scale_mode must be 0 or 1")
    return S.mean(axis=1)


def structure_loss(pts: np.ndarray, gauss: np.ndarray, scale_mode: int = 0, chunk: int = 2048) -> dict:
    """Structure similarity loss L_p of Eq. (9) (Sec. 3.3).

    For every scan point P_j: value_j = min over Gaussians k of
    (|P_j - p_k|_2 - S-bar_k), and the k attaining it (the lowest k among equal
    values); L_p is the mean of value_j over the frame's points. Readings: the
    sum runs over the n points (Eq. (9) writes j = 0..n against 1/n);
    non-finite points are left out of the mean (value NaN, index -1); a Gaussian
    whose centre or S-bar is not finite (an unsolved voxel's NaN row) is not a
    candidate. With no candidate at all every finite point gets +inf and index
    -1, and L_p is +inf; with no finite point L_p is NaN.

    Returns {"value": (n,), "arg": (n,), "loss": float, "n_valid": int}.
    """
    P = np.asarray(pts, dtype=np.float32).astype(np.float64).reshape(-1, 3)
    G = np.asarray(gauss, dtype=np.float32).astype(np.float64).reshape(-1, 8)
    sbar = gaussian_mean_scale(G, scale_mode)
    cand = np.flatnonzero(np.isfinite(G[:, :3]).all(axis=1) & np.isfinite(sbar))
    n = len(P)
    value = np.full(n, np.nan)
    arg = np.full(n, -1, dtype=np.int64)
    fin = np.isfinite(P).all(axis=1)
    idx = np.flatnonzero(fin)
    if len(cand) == 0:
        value[idx] = np.inf
    else:
        C = G[cand, :3]
        s = sbar[cand]
        for a in range(0, len(idx), chunk):
            rows = idx[a:a + chunk]
            D = np.sqrt(((P[rows, None, :] - C[None, :, :]) ** 2).sum(axis=2)) - s[None, :]
            j = np.argmin(D, axis=1)  # first minimum: candidates are in ascending k
            value[rows] = D[np.arange(len(rows)), j]
            arg[rows] = cand[j]
    n_valid = int(fin.sum())
    loss = float(value[idx].mean()) if n_valid else float("nan")
    return {"value": value, "arg": arg, "loss": loss, "n_valid": n_valid}
