"""Plant plausible mistakes in the oracle (on the CPU) and check a pin catches each.

Each mutant patches one oracle function with a small, realistic slip (a dropped
term, a wrong sign, a wrong index, a transposed operand, an unstable sort, a
wrong eigenvector, a non-cyclic axis order, grid points on interval edges) and
runs the pins of tests/test_oracle_pins.py against it: at least one must fail.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import vgpr_oracle as O
from tests import test_oracle_pins as pins

_orig_posterior = O.gp_posterior
_orig_kernel = O.se_kernel
_orig_frame = O.local_frame
_orig_grid = O.query_grid


def _posterior_no_noise(x, f, xq, sf2, ell, sn, full=False):
    return _orig_posterior(x, f, xq, sf2, ell, 0.0 * np.asarray(sn) + 1e-14, full)


def _posterior_no_centering(x, f, xq, sf2, ell, sn, full=False):
    x = np.asarray(x, float)
    f = np.asarray(f, float)
    K = O.se_kernel(x, x, sf2, ell) + np.eye(len(x)) * sn
    Ks = O.se_kernel(x, xq, sf2, ell)
    L = scipy.linalg.cholesky(K, lower=True)
    mean = Ks.T @ scipy.linalg.cho_solve((L, True), f)  # zero prior mean in world coordinates
    V = scipy.linalg.solve_triangular(L, Ks, lower=True)
    var = sf2 - (V * V).sum(0)
    if full:
        return mean, var, O.se_kernel(xq, xq, sf2, ell) - V.T @ V
    return mean, var


def _posterior_sign_slip(x, f, xq, sf2, ell, sn, full=False):
    r = _orig_posterior(x, f, xq, sf2, ell, sn, full)
    mu = np.mean(f)
    return (2 * mu - r[0],) + tuple(r[1:])


def _posterior_var_plus(x, f, xq, sf2, ell, sn, full=False):
    r = list(_orig_posterior(x, f, xq, sf2, ell, sn, full))
    r[1] = 2 * sf2 - r[1]  # K** + K*^T K^-1 K*
    return tuple(r)


def _kernel_missing_half(A, B, sf2, ell):
    return _orig_kernel(A, B, sf2, ell / np.sqrt(2.0))  # exp(-d^2 / l^2)


def _kernel_transposed(A, B, sf2, ell):
    K = _orig_kernel(A, B, sf2, ell)
    if K.shape[0] == K.shape[1]:
        return K
    # a transposed operand reaching the cross-covariance: rows and columns swap roles
    return _orig_kernel(B[: len(A)] if len(B) >= len(A) else np.resize(B, A.shape), A, sf2, ell).T


def _frame_largest_eigvec(P):
    fr = _orig_frame(P)
    P = np.asarray(P, float)
    D = P - P.mean(0)
    w, V = np.linalg.eigh(D.T @ D / len(P))
    v = V[:, 2]
    a = int(np.argmax(np.abs(v)))
    fr.axis, fr.params, fr.normal = a, O.PARAM_AXES[a], v
    return fr


def _frame_signed_angle(P):
    fr = _orig_frame(P)
    a = int(np.argmax(fr.normal))  # forgets |v|: a negative normal component never wins
    fr.axis, fr.params = a, O.PARAM_AXES[a]
    return fr


def _grid_edges(ku, kw, s, nq):
    g = _orig_grid(ku, kw, s, nq)
    S = float(np.float32(s))
    return g - 0.5 * S / nq


def _unstable_voxelize(xyz, s, frame_offsets=None):
    vox = _orig_voxelize(xyz, s, frame_offsets)
    perm = vox["perm"].copy()
    for o, c in zip(vox["offsets"], vox["counts"]):
        perm[o:o + c] = perm[o:o + c][::-1]
    vox["perm"] = perm
    return vox


_orig_voxelize = O.voxelize
_non_cyclic = {0: (1, 2), 1: (0, 2), 2: (0, 1)}

PIN_TESTS = [
    lambda: pins.test_posterior_n1_closed_form(),
    lambda: pins.test_posterior_n2_closed_form(),
    lambda: pins.test_posterior_vs_mpmath_50_digits(),
    lambda: pins.test_posterior_vs_explicit_inverse(),
    lambda: pins.test_interpolation_as_noise_vanishes(),
    lambda: pins.test_variance_bounds_and_monotone_in_data(),
    lambda: pins.test_far_field_returns_prior(),
    lambda: pins.test_plane_normal_to_value_axis_is_exact(),
    lambda: pins.test_voxel_outputs_layout_and_status(),
    lambda: pins.test_cyclic_relabelling_equivariance(),
    lambda: pins.test_grid_exact_small_case(),
    lambda: pins.test_grid_interval_centres(-3, 7, 0.2, 9),
    lambda: pins.test_keys_match_bruteforce_grouping(),
    lambda: pins.test_multi_frame_equals_concatenation(),
    lambda: [pins.test_frame_axis_of_known_planes(n, a) for n, a in
             [([0, 0, 1], 2), ([1, 0, 0], 0), ([0, 1, 0], 1), ([0.2, -0.3, 1.0], 2), ([1.0, 0.5, -0.4], 0),
              ([-0.1, 0.9, 0.6], 1)]],
]


def _caught():
    for t in PIN_TESTS:
        try:
            t()
        except (AssertionError, np.linalg.LinAlgError, ValueError, IndexError):
            return True
    return False


def test_pins_green_on_unmodified_oracle():
    assert not _caught()


@pytest.mark.parametrize("name,target,mutant", [
    ("noise term dropped", "gp_posterior", _posterior_no_noise),
    ("prior mean not subtracted", "gp_posterior", _posterior_no_centering),
    ("sign slip in the mean", "gp_posterior", _posterior_sign_slip),
    ("variance term added", "gp_posterior", _posterior_var_plus),
    ("factor 2 missing in 2 l^2", "se_kernel", _kernel_missing_half),
    ("transposed cross-covariance", "se_kernel", _kernel_transposed),
    ("largest eigenvector", "local_frame", _frame_largest_eigvec),
    ("signed angle", "local_frame", _frame_signed_angle),
    ("grid on interval edges", "query_grid", _grid_edges),
    ("unstable point order", "voxelize", _unstable_voxelize),
    ("non-cyclic parameter axes", "PARAM_AXES", _non_cyclic),
])
def test_pins_catch_mutant(monkeypatch, name, target, mutant):
    monkeypatch.setattr(O, target, mutant)
    assert _caught(), f"no pin caught the mutant: {name}"


# ---------------------------------------------------------------------------
# Sec. 3.2 Gaussian initialisation: mutants of gauss_init
# ---------------------------------------------------------------------------
def _gauss_variant(weight="inv", transpose=False, std=False, norm="sum"):
    def f(out, status, grid_side, n_r, var_floor):
        out = np.asarray(out, dtype=np.float64)
        V = out.shape[0]
        ns = grid_side // n_r
        res = np.full((V, ns * ns, 8), np.nan)
        for v in range(V):
            if not int(status[v]) & O.ST_SOLVED:
                continue
            g = out[v].reshape(grid_side, grid_side, 4)
            for bi in range(ns):
                for bj in range(ns):
                    a, b = (bj, bi) if transpose else (bi, bj)
                    blk = g[a * n_r:(a + 1) * n_r, b * n_r:(b + 1) * n_r].reshape(-1, 4)
                    var = np.maximum(blk[:, 3], var_floor)
                    w = var if weight == "var" else (np.ones_like(var) if weight == "one" else 1.0 / var)
                    p = (blk[:, :3] * w[:, None]).sum(0) / w.sum()
                    Q = blk[:, :3] - p
                    den = w.sum() if norm == "sum" else len(w)
                    phi = np.diag(Q.T @ np.diag(w) @ Q) / den
                    if std:
                        phi = np.sqrt(phi)
                    res[v, bi * ns + bj] = [*p, w.sum(), *phi, 0.0]
        return res
    return f


GAUSS_PINS = [
    lambda: pins.test_gauss_uniform_weights_regular_grid_closed_form(),
    lambda: pins.test_gauss_matches_numpy_weighted_covariance(),
    lambda: pins.test_gauss_dominant_weight_and_invariances(),
    lambda: pins.test_gauss_floor_unsolved_and_single_point_subgrids(),
]


def _gauss_caught():
    for t in GAUSS_PINS:
        try:
            t()
        except (AssertionError, ValueError, IndexError, FloatingPointError):
            return True
    return False


def test_gauss_pins_green_on_unmodified_oracle():
    assert not _gauss_caught()


@pytest.mark.parametrize("name,mutant", [
    ("weight = variance", _gauss_variant(weight="var")),
    ("unweighted", _gauss_variant(weight="one")),
    ("subgrids transposed", _gauss_variant(transpose=True)),
    ("scale as standard deviation", _gauss_variant(std=True)),
    ("scatter divided by the point count", _gauss_variant(norm="count")),
])
def test_gauss_pins_catch_mutant(monkeypatch, name, mutant):
    monkeypatch.setattr(O, "gauss_init", mutant)
    assert _gauss_caught(), f"no pin caught the mutant: {name}"


# ---------------------------------------------------------------------------
# PCA-rotated frame (frame_mode 1): mutants
# ---------------------------------------------------------------------------
_orig_rot_frame = O.rotated_frame
_orig_rot_grid = O.rotated_grid


def _rot_frame_swapped(fr):
    e1, e2, v = _orig_rot_frame(fr)
    return e2, -e1, v  # still right-handed, but the grid's i axis runs along e2


def _rot_frame_fixed_axis(fr):
    # e1 from a fixed world axis (x) instead of the one least aligned with the normal
    v = _orig_rot_frame(fr)[2]
    e1 = np.cross([1.0, 0.0, 0.0], v)
    e1 = e1 / np.linalg.norm(e1)
    return e1, np.cross(v, e1), v


def _rot_frame_world_axis(fr):
    # value along the world axis of Alg. 1 instead of the normal
    a = fr.axis
    v = np.zeros(3)
    v[a] = 1.0
    u, w = O.PARAM_AXES[a]
    e1 = np.zeros(3)
    e1[u] = 1.0
    return e1, np.cross(v, e1), v


def _rot_grid_uncentred(s, nq):
    return _orig_rot_grid(s, nq) + 0.5 * float(np.float32(s))


ROT_PINS = [
    lambda: [pins.test_rotated_frame_recovers_noiseless_tilted_planes_exactly(c) for c in
             [(0.5, 0.25, 0.125, [0, 1, 2]), (1.5, -0.25, 0.0, [1, 2, 0])]],
    lambda: pins.test_rotated_frame_closed_form_and_grid_geometry(),
    lambda: pins.test_rotated_frame_orthonormal_and_continuous(),
]


def _rot_caught():
    for t in ROT_PINS:
        try:
            t()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            return True
    return False


def test_rotated_pins_green_on_unmodified_oracle():
    assert not _rot_caught()


@pytest.mark.parametrize("name,target,mutant", [
    ("in-plane axes swapped", "rotated_frame", _rot_frame_swapped),
    ("in-plane axis from a fixed world axis", "rotated_frame", _rot_frame_fixed_axis),
    ("value along the world axis", "rotated_frame", _rot_frame_world_axis),
    ("grid not centred on the centroid", "rotated_grid", _rot_grid_uncentred),
])
def test_rotated_pins_catch_mutant(monkeypatch, name, target, mutant):
    monkeypatch.setattr(O, target, mutant)
    assert _rot_caught(), f"no pin caught the mutant: {name}"


# ---------------------------------------------------------------------------
# Sec. 3.3 covariance-centred update (VoxelMap(feedback=True))
# ---------------------------------------------------------------------------
_orig_fb_inputs = O.feedback_inputs


def _fb_sensor_noise(prev, P, params):
    X, nz = _orig_fb_inputs(prev, P, params)
    return X, np.full(len(X), params.noise_var)  # carried rows keep the sensor variance


def _fb_dropped(prev, P, params):
    X, nz = _orig_fb_inputs(prev, P, params)
    m = len(prev)
    return X[m:], nz[m:]  # re-solve on the new points only


def _fb_uncapped(prev, P, params):
    prev = np.asarray(prev, np.float32)
    new = np.asarray(P, np.float32)  # every new point, past max_pts
    X = np.concatenate([prev[:, :3], new])
    nz = np.concatenate([np.maximum(prev[:, 3].astype(np.float64), 1e-6), np.full(len(new), params.noise_var)])
    return X, nz


def _fb_std_dev(prev, P, params):
    X, nz = _orig_fb_inputs(prev, P, params)
    m = len(prev)
    nz = nz.copy()
    nz[:m] = np.sqrt(nz[:m])  # standard deviation where a variance belongs
    return X, nz


def _fb_pool_grows(self, xyz):
    # the pool keeps growing after the voxel entered the map
    vox = O.voxelize(xyz, self.params.voxel_size)
    for v, key in enumerate(vox["keys"].tolist()):
        if key in self.pred:
            P = O.voxel_points(xyz, vox, v)
            self.points[key] = np.concatenate([self.points[key], P])[: self.params.max_pts]
    return _orig_map_update(self, xyz)


_orig_map_update = O.VoxelMap.update

FB_PINS = [
    lambda: pins.test_feedback_update_closed_form_sequence(),
    lambda: pins.test_feedback_variance_never_exceeds_single_pseudo_observation(),
    lambda: pins.test_feedback_state_machine(),
]


def _fb_caught():
    for t in FB_PINS:
        try:
            t()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            return True
    return False


def test_feedback_pins_green_on_unmodified_oracle():
    assert not _fb_caught()


@pytest.mark.parametrize("name,mutant", [
    ("carried rows keep the sensor variance", _fb_sensor_noise),
    ("carried rows dropped", _fb_dropped),
    ("new points not capped", _fb_uncapped),
    ("standard deviation as the carried noise", _fb_std_dev),
])
def test_feedback_pins_catch_input_mutant(monkeypatch, name, mutant):
    monkeypatch.setattr(O, "feedback_inputs", mutant)
    assert _fb_caught(), f"no pin caught the mutant: {name}"


def test_feedback_pins_catch_growing_pool(monkeypatch):
    monkeypatch.setattr(O.VoxelMap, "update", _fb_pool_grows)
    assert _fb_caught()


# ---------------------------------------------------------------------------
# Eq. (9) structure similarity loss
# ---------------------------------------------------------------------------
_orig_sloss = O.structure_loss
_orig_mean_scale = O.gaussian_mean_scale


def _sloss_variant(P, G, scale_mode=0, squared=False, plus=False, nearest_first=False):
    P = np.asarray(P, np.float32).astype(np.float64).reshape(-1, 3)
    G = np.asarray(G, np.float32).astype(np.float64).reshape(-1, 8)
    s = O.gaussian_mean_scale(G, scale_mode)
    cand = np.flatnonzero(np.isfinite(G[:, :3]).all(1) & np.isfinite(s))
    n = len(P)
    value, arg = np.full(n, np.nan), np.full(n, -1)
    fin = np.isfinite(P).all(1)
    for j in np.flatnonzero(fin):
        if len(cand) == 0:
            value[j] = np.inf
            continue
        d2 = ((P[j] - G[cand, :3]) ** 2).sum(1)
        d = d2 if squared else np.sqrt(d2)
        if nearest_first:
            k = int(np.argmin(d))
            v = d[k] - s[cand][k]
        else:
            vals = d + s[cand] if plus else d - s[cand]
            k = int(np.argmin(vals))
            v = vals[k]
        value[j], arg[j] = v, cand[k]
    nv = int(fin.sum())
    return {"value": value, "arg": arg, "loss": float(value[fin].mean()) if nv else float("nan"), "n_valid": nv}


def _sloss_squared(P, G, scale_mode=0, chunk=2048):
    return _sloss_variant(P, G, scale_mode, squared=True)


def _sloss_plus(P, G, scale_mode=0, chunk=2048):
    return _sloss_variant(P, G, scale_mode, plus=True)


def _sloss_nearest_first(P, G, scale_mode=0, chunk=2048):
    return _sloss_variant(P, G, scale_mode, nearest_first=True)


def _sloss_sum(P, G, scale_mode=0, chunk=2048):
    r = _orig_sloss(P, G, scale_mode, chunk)
    r["loss"] = r["loss"] * max(r["n_valid"], 1)  # sum where the mean belongs
    return r


def _mean_scale_max(G, scale_mode):
    G = np.asarray(G, np.float32).astype(np.float64).reshape(-1, 8)
    S = np.sqrt(G[:, 4:7]) if scale_mode == 1 else G[:, 4:7]
    return S.max(axis=1)  # largest scale instead of the mean


def _mean_scale_no_sqrt(G, scale_mode):
    return _orig_mean_scale(G, 0)  # variances averaged as if they were scales


SLOSS_PINS = [
    lambda: pins.test_structure_loss_worked_example_exact(),
    lambda: pins.test_structure_loss_zero_scale_is_nearest_neighbour(),
    lambda: pins.test_structure_loss_minimises_the_difference_not_the_distance(),
    lambda: pins.test_structure_loss_scale_modes_and_invariances(),
    lambda: pins.test_structure_loss_invalid_rows_points_and_empty_map(),
]


def _sloss_caught():
    for t in SLOSS_PINS:
        try:
            t()
        except (AssertionError, ValueError, IndexError):
            return True
    return False


def test_structure_loss_pins_green_on_unmodified_oracle():
    assert not _sloss_caught()


@pytest.mark.parametrize("name,target,mutant", [
    ("squared distance", "structure_loss", _sloss_squared),
    ("scale added", "structure_loss", _sloss_plus),
    ("nearest centre first, then its scale", "structure_loss", _sloss_nearest_first),
    ("sum over points", "structure_loss", _sloss_sum),
    ("largest scale instead of the mean", "gaussian_mean_scale", _mean_scale_max),
    ("variances averaged without the square root", "gaussian_mean_scale", _mean_scale_no_sqrt),
])
def test_structure_loss_pins_catch_mutant(monkeypatch, name, target, mutant):
    monkeypatch.setattr(O, target, mutant)
    assert _sloss_caught(), f"no pin caught the mutant: {name}"


# ---------------------------------------------------------------------------
# Per-voxel length scale (ls_mode 1): mutants of pca_length_scale
# ---------------------------------------------------------------------------
def _ls_variant(mix="midmax", root3=True, lo=0.05, hi=2.0):
    def f(eigvals, voxel_size):
        s = float(np.float32(voxel_size))
        w = np.asarray(eigvals, dtype=np.float64)
        v = {"midmax": (w[1] + w[2]) / 2.0, "max": w[2], "minmid": (w[0] + w[1]) / 2.0,
             "sum": w[1] + w[2]}[mix]
        ell = (np.sqrt(3.0) if root3 else 1.0) * np.sqrt(max(v, 0.0))
        return min(max(ell, lo * s), hi * s)
    return f


LS_PINS = [
    lambda: pins.test_pca_length_scale_uniform_square(),
    lambda: [pins.test_pca_length_scale_rectangle_closed_form(*c) for c in
             [(0.06, 0.1, 12, 20), (0.1, 0.02, 25, 5), (0.03, 0.09, 7, 40)]],
    lambda: [pins.test_pca_length_scale_clamp_edges(s) for s in (0.1, 0.2, 1.0)],
]


def _ls_caught():
    for t in LS_PINS:
        try:
            t()
        except AssertionError:
            return True
    return False


def test_length_scale_pins_green_on_unmodified_oracle():
    assert not _ls_caught()


@pytest.mark.parametrize("name,mutant", [
    ("largest eigenvalue alone", _ls_variant(mix="max")),
    ("smallest and middle eigenvalues", _ls_variant(mix="minmid")),
    ("sum instead of the mean", _ls_variant(mix="sum")),
    ("sqrt(3) missing", _ls_variant(root3=False)),
    ("lower clamp edge 0.1 s", _ls_variant(lo=0.1)),
    ("lower clamp edge 0.01 s", _ls_variant(lo=0.01)),
    ("upper clamp edge s", _ls_variant(hi=1.0)),
    ("upper clamp edge 4 s", _ls_variant(hi=4.0)),
])
def test_length_scale_pins_catch_mutant(monkeypatch, name, mutant):
    monkeypatch.setattr(O, "pca_length_scale", mutant)
    assert _ls_caught(), f"no pin caught the mutant: {name}"
