"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-derive the oracle's own formulas: each checks a property that
holds independently of how the oracle is written (brute force over tiny
inputs, exact rational arithmetic, closed forms of the GP posterior for n = 1
and n = 2, an mpmath 50-digit evaluation of Eq. (3), invariants of GP
regression, and symmetries of Alg. 1). tests/test_oracle_mutants.py plants
plausible mistakes in the oracle and checks that these pins catch them.
"""
import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import vgpr_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Table S6 / Sec. 3.1 defaults
# ---------------------------------------------------------------------------
def test_defaults_match_table_s6():
    with open(os.path.join(GOLDEN, "table_s6_hyperparameters.json")) as fh:
        g = json.load(fh)
    p = O.Params()
    assert p.voxel_size == pytest.approx(g["size"])
    assert p.min_pts == g["tau"]
    assert p.grid_side == g["n_s"] * g["n_r"]
    assert p.converge_var == pytest.approx(g["eta"])
    # exp(-lambda d^2) with lambda = 1  <=>  s_f^2 = 1, l = 1/sqrt(2)
    lam = 1.0 / (2.0 * p.length_scale ** 2)
    assert lam == pytest.approx(g["lambda"], rel=1e-15)
    assert p.signal_var == 1.0


# ---------------------------------------------------------------------------
# Keys and grouping (Alg. S1)
# ---------------------------------------------------------------------------
def _brute_group(xyz, s):
    """Python-dict grouping with exact rational voxel membership checks."""
    s32 = Fraction(float(np.float32(s)))
    groups = {}
    for i, p in enumerate(np.asarray(xyz, dtype=np.float32).tolist()):
        if not all(math.isfinite(c) for c in p):
            continue
        k = []
        for c in p:
            fc = Fraction(c)
            q = math.floor(fc / s32)  # exact floor of the exact quotient
            k.append(q)
        groups.setdefault(tuple(k), []).append(i)
    return groups


def test_keys_match_bruteforce_grouping():
    r = rng(1)
    s = 0.25
    xyz = r.uniform(-3, 3, size=(3000, 3)).astype(np.float32)
    # points exactly on voxel boundaries and negative zero
    xyz[:50] = (r.integers(-12, 12, size=(50, 3)) * s).astype(np.float32)
    xyz[50] = [-0.0, 0.0, -0.0]
    vox = O.voxelize(xyz, s)
    g = _brute_group(xyz, s)
    # voxel order = ascending (kx, ky, kz): the packed key orders like the tuple
    exp_keys = sorted(g)
    got = [O.unpack_key(k) for k in vox["keys"]]
    assert got == exp_keys
    for v, k in enumerate(exp_keys):
        o, c = int(vox["offsets"][v]), int(vox["counts"][v])
        assert vox["perm"][o:o + c].tolist() == g[k]  # arrival order kept


def test_keys_rounded_product_vs_exact_quotient():
    """Away from boundaries the float64 product floor equals the exact floor."""
    r = rng(2)
    s = np.float32(0.2)  # not a binary fraction
    xyz = r.uniform(-50, 50, size=(20000, 3)).astype(np.float32)
    k, valid = O.voxel_coords(xyz, s)
    assert valid.all()
    S = Fraction(float(s))
    for p, kk in zip(xyz[:2000].tolist(), k[:2000].tolist()):
        for c, q in zip(p, kk):
            exact = Fraction(c) / S
            fl = math.floor(exact)
            if abs(exact - round(exact)) > Fraction(1, 10 ** 9):
                assert q == fl
            else:
                assert q in (fl, fl - 1, fl + 1)


@pytest.mark.parametrize("p,s,k", [
    (0.5, 0.5, 1), (0.0, 0.5, 0), (-0.0, 0.5, 0), (-0.25, 0.5, -1), (-0.5, 0.5, -1),
    (0.49999997, 0.5, 0), (1.0, 1.0, 1), (-1e-30, 1.0, -1), (3.0, 0.75, 4),
])
def test_key_half_open_special_values(p, s, k):
    kk, valid = O.voxel_coords(np.array([[p, p, p]], np.float32), s)
    assert valid.all() and kk.tolist() == [[k, k, k]]


def test_key_packing_roundtrip_and_order():
    r = rng(3)
    k = r.integers(-O.KEY_AXIS_LIMIT, O.KEY_AXIS_LIMIT + 1, size=(500, 3))
    k[:6] = [[O.KEY_AXIS_LIMIT] * 3, [-O.KEY_AXIS_LIMIT] * 3, [0, 0, 0], [-1, 0, 1], [1, -1, 0], [0, 1, -1]]
    keys = O.pack_keys(k)
    assert [O.unpack_key(x) for x in keys] == [tuple(x) for x in k.tolist()]
    order_keys = np.argsort(keys, kind="stable")
    order_tuple = sorted(range(len(k)), key=lambda i: tuple(k[i]))
    assert order_keys.tolist() == order_tuple
    assert int(keys.max()) < 2 ** 63  # the sentinel sorts after every valid key


def test_nonfinite_points_dropped_and_counted():
    xyz = np.array([[0.1, 0.1, 0.1], [np.nan, 0, 0], [0.2, 0.1, 0.1], [np.inf, 1, 1], [0, -np.inf, 0]],
                   np.float32)
    vox = O.voxelize(xyz, 1.0)
    assert vox["n_invalid"] == 3
    assert len(vox["keys"]) == 1 and vox["counts"].tolist() == [2]
    assert vox["perm"][:2].tolist() == [0, 2]


def test_key_range_limit():
    s = 1.0
    ok = np.array([[O.KEY_AXIS_LIMIT + 0.5, -O.KEY_AXIS_LIMIT, 0]], np.float32)
    O.voxel_coords(ok, s)
    bad = np.array([[O.KEY_AXIS_LIMIT + 1.0, 0, 0]], np.float32)
    with pytest.raises(O.OracleRangeError):
        O.voxel_coords(bad, s)


def test_empty_and_single_point():
    v0 = O.voxelize(np.zeros((0, 3), np.float32), 0.5)
    assert len(v0["keys"]) == 0 and v0["n_invalid"] == 0 and len(v0["perm"]) == 0
    v1 = O.voxelize(np.array([[0.3, -0.3, 7.1]], np.float32), 0.5)
    assert [O.unpack_key(k) for k in v1["keys"]] == [(0, -1, 14)]


def test_multi_frame_equals_concatenation():
    r = rng(4)
    frames = [r.uniform(-2, 2, size=(n, 3)).astype(np.float32) for n in (100, 0, 57, 300)]
    xyz = np.concatenate(frames)
    offs = np.cumsum([0] + [len(f) for f in frames])
    vb = O.voxelize(xyz, 0.5, offs)
    keys, counts, starts = [], [], []
    for f, fr in enumerate(frames):
        v = O.voxelize(fr, 0.5)
        keys += v["keys"].tolist()
        counts += v["counts"].tolist()
        starts += (v["offsets"] + offs[f]).tolist()
        assert (vb["perm"][offs[f]:offs[f + 1]] - offs[f]).tolist() == v["perm"].tolist()
    assert vb["keys"].tolist() == keys and vb["counts"].tolist() == counts
    assert vb["offsets"].tolist() == starts
    assert np.diff(vb["frame_vox"]).tolist() == [len(O.voxelize(f, 0.5)["keys"]) for f in frames]


# ---------------------------------------------------------------------------
# PCA frame and value axis (Alg. 1)
# ---------------------------------------------------------------------------
def _plane_points(normal, n=200, seed=0, noise=0.0):
    r = rng(seed)
    normal = np.asarray(normal, float)
    normal /= np.linalg.norm(normal)
    a = np.cross(normal, [1, 0, 0] if abs(normal[0]) < 0.9 else [0, 1, 0])
    a /= np.linalg.norm(a)
    b = np.cross(normal, a)
    uv = r.uniform(-0.4, 0.4, size=(n, 2))
    return uv[:, :1] * a + uv[:, 1:] * b + r.normal(0, noise, size=(n, 1)) * normal


@pytest.mark.parametrize("normal,axis", [
    ([0, 0, 1], 2), ([1, 0, 0], 0), ([0, 1, 0], 1), ([0.2, -0.3, 1.0], 2), ([1.0, 0.5, -0.4], 0),
    ([-0.1, 0.9, 0.6], 1),
])
def test_frame_axis_of_known_planes(normal, axis):
    fr = O.local_frame(_plane_points(normal, noise=0.005))
    assert fr.axis == axis
    assert fr.params == {0: (1, 2), 1: (2, 0), 2: (0, 1)}[axis]
    nrm = np.asarray(normal, float) / np.linalg.norm(normal)
    assert abs(abs(fr.normal @ nrm) - 1) < 1e-3


def test_frame_eigen_vs_mpmath():
    for seed in range(5):
        P = rng(10 + seed).normal(size=(5, 3)) * [1.0, 0.5, 0.1]
        fr = O.local_frame(P)
        mpmath.mp.dps = 50
        Pm = mpmath.matrix(P.tolist())
        n = P.shape[0]
        c = [sum(Pm[i, j] for i in range(n)) / n for j in range(3)]
        C = mpmath.matrix(3, 3)
        for i in range(3):
            for j in range(3):
                C[i, j] = sum((Pm[k, i] - c[i]) * (Pm[k, j] - c[j]) for k in range(n)) / n
        E, Q = mpmath.eigsy(C)
        order = sorted(range(3), key=lambda i: E[i])
        assert np.allclose([float(E[i]) for i in order], fr.eigvals, rtol=1e-12, atol=1e-15)
        v = np.array([float(Q[i, order[0]]) for i in range(3)])
        assert abs(abs(v @ fr.normal) - 1) < 1e-12


def test_frame_axis_ties_go_low_and_are_flagged():
    # normal exactly at 45 deg between X and Y: |v_x| == |v_y|
    P = np.array([[0, 0, 0], [1, -1, 0], [0, 0, 1], [1, -1, 1], [0.5, -0.5, 0.5]], float)
    fr = O.local_frame(P)
    assert fr.ambiguous
    assert fr.axis in (0, 1)


# ---------------------------------------------------------------------------
# MeshGrid (Alg. 1, Sec. 3.1-3.2)
# ---------------------------------------------------------------------------
def test_grid_exact_small_case():
    g = O.query_grid(0, 0, 1.0, 4)
    assert sorted(set(g[:, 0].tolist())) == [0.125, 0.375, 0.625, 0.875]
    assert g[:4, 0].tolist() == [0.125] * 4 and g[:4, 1].tolist() == [0.125, 0.375, 0.625, 0.875]


@pytest.mark.parametrize("ku,kw,s,nq", [(-3, 7, 0.2, 9), (12, -1, 0.5, 8), (1000, -2000, 0.1, 16)])
def test_grid_interval_centres(ku, kw, s, nq):
    g = O.query_grid(ku, kw, s, nq)
    S = float(np.float32(s))
    assert g.shape == (nq * nq, 2)
    for col, k in ((0, ku), (1, kw)):
        vals = np.unique(g[:, col])
        assert len(vals) == nq
        exact = [(k + (i + 0.5) / nq) * S for i in range(nq)]
        # within float32 rounding of the exact interval centre
        assert np.allclose(vals, exact, rtol=0, atol=4 * np.spacing(np.float32(abs(k * S) + S)))
        assert vals.min() > k * S and vals.max() < (k + 1) * S
    assert np.mean(g, axis=0) == pytest.approx([(ku + 0.5) * S, (kw + 0.5) * S], abs=1e-5 * (1 + abs(ku) * S))


# ---------------------------------------------------------------------------
# GP posterior (Eq. (2)-(3))
# ---------------------------------------------------------------------------
def _se(a, b, sf2, ell):
    d2 = sum((x - y) ** 2 for x, y in zip(a, b))
    return sf2 * math.exp(-d2 / (2 * ell * ell))


def test_posterior_n1_closed_form():
    x = np.array([[0.3, -0.2]])
    f = np.array([1.7])
    xq = rng(5).uniform(-1, 1, size=(7, 2))
    sf2, ell, sn = 1.3, 0.4, 2e-3
    mean, var = O.gp_posterior(x, f, xq, sf2, ell, sn)
    for q in range(len(xq)):
        k = _se(xq[q], x[0], sf2, ell)
        assert mean[q] == pytest.approx(1.7, abs=1e-14)  # f - mean(f) = 0
        assert var[q] == pytest.approx(sf2 - k * k / (sf2 + sn), rel=1e-13, abs=1e-15)


def test_posterior_n2_closed_form():
    x = np.array([[0.0, 0.0], [0.3, 0.1]])
    f = np.array([0.5, -0.25])
    xq = np.array([[0.1, 0.05], [0.7, -0.2], [0.0, 0.0]])
    sf2, ell, sn = 1.0, 0.5, 1e-3
    mean, var = O.gp_posterior(x, f, xq, sf2, ell, sn)
    a = sf2 + sn
    b = _se(x[0], x[1], sf2, ell)
    det = a * a - b * b
    inv = [[a / det, -b / det], [-b / det, a / det]]
    mu = (f[0] + f[1]) / 2
    ft = [f[0] - mu, f[1] - mu]
    for q in range(len(xq)):
        k = [_se(x[0], xq[q], sf2, ell), _se(x[1], xq[q], sf2, ell)]
        ik = [inv[0][0] * k[0] + inv[0][1] * k[1], inv[1][0] * k[0] + inv[1][1] * k[1]]
        assert mean[q] == pytest.approx(mu + ik[0] * ft[0] + ik[1] * ft[1], rel=1e-12, abs=1e-13)
        assert var[q] == pytest.approx(sf2 - (ik[0] * k[0] + ik[1] * k[1]), rel=1e-11, abs=1e-13)


def test_posterior_vs_mpmath_50_digits():
    mpmath.mp.dps = 50
    for seed, n in ((20, 3), (21, 5), (22, 6)):
        r = rng(seed)
        x = r.uniform(0, 0.5, size=(n, 2))
        f = r.normal(0, 0.1, size=n)
        xq = r.uniform(0, 0.5, size=(4, 2))
        sf2, ell, sn = 1.0, 0.25, 1e-3
        mean, var = O.gp_posterior(x, f, xq, sf2, ell, sn)

        def k(a, b):
            return sf2 * mpmath.exp(-((mpmath.mpf(a[0]) - b[0]) ** 2 + (mpmath.mpf(a[1]) - b[1]) ** 2)
                                    / (2 * mpmath.mpf(ell) ** 2))
        K = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                K[i, j] = k(x[i], x[j]) + (mpmath.mpf(sn) if i == j else 0)
        Ki = mpmath.inverse(K)
        mu = mpmath.fsum([mpmath.mpf(v) for v in f]) / n
        ft = mpmath.matrix([mpmath.mpf(v) - mu for v in f])
        for q in range(len(xq)):
            ks = mpmath.matrix([k(x[i], xq[q]) for i in range(n)])
            m = mu + (ks.T * Ki * ft)[0]
            v = sf2 - (ks.T * Ki * ks)[0]
            assert abs(float(m) - mean[q]) <= 1e-9
            assert abs(float(v) - var[q]) <= 1e-9


def test_posterior_vs_explicit_inverse():
    for seed in range(6):
        r = rng(30 + seed)
        n = int(r.integers(3, 17))
        x = r.uniform(0, 1, size=(n, 2))
        f = r.normal(size=n)
        xq = r.uniform(0, 1, size=(9, 2))
        sf2, ell, sn = 0.8, 0.3, 1e-2
        mean, var, S = O.gp_posterior(x, f, xq, sf2, ell, sn, full=True)
        d = lambda A, B: ((A[:, None] - B[None]) ** 2).sum(-1)
        K = sf2 * np.exp(-d(x, x) / (2 * ell ** 2)) + sn * np.eye(n)
        Ks = sf2 * np.exp(-d(x, xq) / (2 * ell ** 2))
        Kss = sf2 * np.exp(-d(xq, xq) / (2 * ell ** 2))
        Ki = np.linalg.inv(K)
        mu = f.mean()
        assert np.allclose(mean, mu + Ks.T @ Ki @ (f - mu), rtol=1e-10, atol=1e-12)
        assert np.allclose(S, Kss - Ks.T @ Ki @ Ks, rtol=1e-10, atol=1e-12)
        assert np.allclose(np.diag(S), var, rtol=1e-12, atol=1e-14)
        assert np.allclose(S, S.T, atol=1e-14)
        assert np.linalg.eigvalsh(S).min() > -1e-10


def test_interpolation_as_noise_vanishes():
    r = rng(40)
    x = r.uniform(0, 0.5, size=(8, 2))
    f = r.normal(0, 0.1, size=8)
    mean, var = O.gp_posterior(x, f, x, 1.0, 0.25, 1e-10)
    assert np.allclose(mean, f, atol=1e-6)
    assert np.all(np.abs(var) < 1e-6)


def test_variance_bounds_and_monotone_in_data():
    r = rng(41)
    x = r.uniform(0, 0.5, size=(20, 2))
    f = r.normal(0, 0.1, size=20)
    xq = r.uniform(-0.2, 0.7, size=(50, 2))
    prev = None
    for n in range(1, 21):
        _, var = O.gp_posterior(x[:n], f[:n], xq, 1.0, 0.25, 1e-3)
        assert np.all(var >= -1e-12) and np.all(var <= 1.0 + 1e-12)
        if prev is not None:
            assert np.all(var <= prev + 1e-12)  # adding a point never raises a variance
        prev = var


def test_far_field_returns_prior():
    r = rng(42)
    x = r.uniform(0, 0.5, size=(10, 2))
    f = r.normal(3.0, 0.1, size=10)
    xq = np.array([[50.0, 50.0], [-80.0, 10.0]])
    mean, var = O.gp_posterior(x, f, xq, 2.0, 0.25, 1e-3)
    assert np.allclose(mean, f.mean(), atol=1e-12)
    assert np.allclose(var, 2.0, atol=1e-12)


def test_permutation_invariance_and_scaling():
    r = rng(43)
    x = r.uniform(0, 0.5, size=(15, 2))
    f = r.normal(0, 0.1, size=15)
    xq = r.uniform(0, 0.5, size=(16, 2))
    m0, v0 = O.gp_posterior(x, f, xq, 1.0, 0.25, 1e-3)
    p = r.permutation(15)
    m1, v1 = O.gp_posterior(x[p], f[p], xq, 1.0, 0.25, 1e-3)
    assert np.abs(m0 - m1).max() <= 1e-12 and np.abs(v0 - v1).max() <= 1e-12
    c = 3.0
    m2, v2 = O.gp_posterior(c * x, c * f, c * xq, 1.0, c * 0.25, 1e-3 * c * c)
    # scaling every coordinate (and l) by c scales mu* - mu_f by c when the noise scales by c^2 too
    # only when s_f^2 scales as well; with fixed s_f^2 check the kernel-invariant part instead
    m3, v3 = O.gp_posterior(c * x, f, c * xq, 1.0, c * 0.25, 1e-3)
    assert np.allclose(m3, m0, atol=1e-12) and np.allclose(v3, v0, atol=1e-12)
    m4, _ = O.gp_posterior(x, c * f, xq, 1.0, 0.25, 1e-3)
    assert np.allclose(m4 - c * f.mean(), c * (m0 - f.mean()), atol=1e-12)
    del m2, v2


def test_condition_bound():
    r = rng(44)
    for n in (4, 32, 128):
        x = r.uniform(0, 0.5, size=(n, 2))
        x[n // 2:] = x[: n - n // 2] + 1e-6  # near duplicates
        d2 = ((x[:, None] - x[None]) ** 2).sum(-1)
        K = np.exp(-d2 / (2 * 0.25 ** 2)) + 1e-3 * np.eye(n)
        assert np.linalg.cond(K) <= 1 + n * 1.0 / 1e-3 + 1e-6


# ---------------------------------------------------------------------------
# Alg. 1 end to end per voxel
# ---------------------------------------------------------------------------
def _params(**kw):
    base = dict(voxel_size=0.5, max_pts=64, min_pts=3, grid_side=4, signal_var=1.0, length_scale=0.25,
                noise_var=1e-3, converge_var=0.3)
    base.update(kw)
    return O.Params(**base)


def test_plane_normal_to_value_axis_is_exact():
    r = rng(50)
    n = 40
    P = np.zeros((n, 3), np.float32)
    P[:, 0] = r.uniform(2.0, 2.5, n)
    P[:, 1] = r.uniform(-1.0, -0.5, n)
    P[:, 2] = np.float32(0.3125)  # plane z = const inside voxel kz = 0
    key = O.pack_keys(np.array([[4, -2, 0]]))[0]
    res = O.fit_predict_voxel(P, key, _params())
    assert res["axis"] == 2
    assert np.abs(res["out"][:, 2] - 0.3125).max() <= 1e-12


def test_tilted_noiseless_plane_error_shrinks_with_density():
    errs = []
    for n in (12, 48, 160):
        r = rng(51)
        uv = r.uniform(0.0, 0.5, size=(n, 2))
        z = 0.2 + 0.1 * uv[:, 0] - 0.05 * uv[:, 1]
        P = np.stack([uv[:, 0], uv[:, 1], z], 1).astype(np.float32)
        key = O.pack_keys(np.array([[0, 0, 0]]))[0]
        res = O.fit_predict_voxel(P, key, _params(max_pts=256, noise_var=1e-6))
        g = res["out"]
        truth = 0.2 + 0.1 * g[:, 0] - 0.05 * g[:, 1]
        errs.append(np.abs(g[:, 2] - truth).max())
    assert errs[2] < errs[0] and errs[2] < 5e-3


def test_voxel_outputs_layout_and_status():
    r = rng(52)
    P = np.stack([r.uniform(0, 0.5, 30), r.uniform(0, 0.5, 30), 0.25 + r.normal(0, 0.01, 30)], 1)
    key = O.pack_keys(np.array([[0, 0, 0]]))[0]
    prm = _params(max_pts=20)
    res = O.fit_predict_voxel(P.astype(np.float32), key, prm)
    assert res["n"] == 20 and res["status"] & O.ST_CAPPED and res["status"] & O.ST_SOLVED
    g = O.query_grid(0, 0, 0.5, 4)
    assert np.array_equal(res["out"][:, 0], g[:, 0]) and np.array_equal(res["out"][:, 1], g[:, 1])
    conv = res["out"][:, 3].max() <= prm.converge_var
    assert bool(res["status"] & O.ST_CONVERGED) == conv
    small = O.fit_predict_voxel(P[:2].astype(np.float32), key, prm)
    assert small["status"] & O.ST_BELOW_TAU and not small["status"] & O.ST_SOLVED
    assert np.isnan(small["out"]).all()


def test_cyclic_relabelling_equivariance():
    """Mapping (x, y, z) -> (z, x, y) permutes axes cyclically and leaves every value identical."""
    r = rng(53)
    P = np.stack([r.uniform(1.0, 1.5, 25), r.uniform(-0.5, 0.0, 25), 0.7 + 0.2 * r.uniform(0, 0.5, 25)
                  + r.normal(0, 0.01, 25)], 1).astype(np.float32)
    k = np.floor(P.astype(np.float64)[0] / 0.5).astype(np.int64)
    key = O.pack_keys(k[None])[0]
    Q = P[:, [2, 0, 1]]
    keyq = O.pack_keys(k[[2, 0, 1]][None])[0]
    a = O.fit_predict_voxel(P, key, _params())
    b = O.fit_predict_voxel(Q, keyq, _params())
    assert b["axis"] == (a["axis"] + 1) % 3
    assert np.array_equal(b["out"][:, [1, 2, 0, 3]], a["out"])


def test_pca_length_scale_uniform_square():
    r = rng(54)
    s = 0.4
    P = np.stack([r.uniform(0, s, 200000), r.uniform(0, s, 200000), np.zeros(200000)], 1)
    fr = O.local_frame(P)
    assert O.pca_length_scale(fr.eigvals, s) == pytest.approx(s / 2, rel=5e-3)


def _lattice_rectangle(a, b, ka, kb, tilt):
    """ka x kb points at the interval centres of an a x b rectangle, rotated by the
    orthonormal matrix `tilt` (columns: the two in-plane axes and the normal)."""
    ia = (np.arange(ka) + 0.5) / ka * a
    ib = (np.arange(kb) + 0.5) / kb * b
    U, W = np.meshgrid(ia, ib, indexing="ij")
    local = np.stack([U.ravel(), W.ravel(), np.zeros(U.size)], 1)
    return local @ tilt.T + np.array([0.3, -0.2, 0.05])


def _rotation(seed):
    q, _ = np.linalg.qr(rng(seed).normal(size=(3, 3)))
    return q


@pytest.mark.parametrize("a,b,ka,kb", [(0.06, 0.1, 12, 20), (0.1, 0.02, 25, 5), (0.03, 0.09, 7, 40)])
def test_pca_length_scale_rectangle_closed_form(a, b, ka, kb):
    """Points on a ka x kb lattice of interval centres of an a x b rectangle (any
    orientation): the discrete uniform law gives in-plane variances
    a^2 (1 - 1/ka^2) / 12 and b^2 (1 - 1/kb^2) / 12 and a zero normal variance, so the
    rule's l = sqrt(3) sqrt((lambda_mid + lambda_max) / 2) is
    sqrt((a^2 (1 - 1/ka^2) + b^2 (1 - 1/kb^2)) / 8), which tends to sqrt((a^2 + b^2) / 8)
    for a dense rectangle. a != b separates lambda_mid from lambda_max; the same value
    reaches the posterior through Alg. 1 with ls_mode 1."""
    s = 0.1
    va = a * a * (1.0 - 1.0 / ka ** 2) / 12.0
    vb = b * b * (1.0 - 1.0 / kb ** 2) / 12.0
    expect = math.sqrt((a * a * (1.0 - 1.0 / ka ** 2) + b * b * (1.0 - 1.0 / kb ** 2)) / 8.0)
    assert expect == pytest.approx(math.sqrt(3.0) * math.sqrt((va + vb) / 2.0), rel=1e-14)
    P = _lattice_rectangle(a, b, ka, kb, _rotation(int(1000 * a + kb)))
    fr = O.local_frame(P)
    assert np.sort(fr.eigvals) == pytest.approx(sorted([0.0, va, vb]), abs=1e-15)
    assert O.pca_length_scale(fr.eigvals, s) == pytest.approx(expect, rel=1e-10)
    # dense limit of the same rectangle
    Pd = _lattice_rectangle(a, b, 400, 400, _rotation(5))
    assert O.pca_length_scale(O.local_frame(Pd).eigvals, s) == pytest.approx(math.sqrt((a * a + b * b) / 8.0),
                                                                           rel=2e-5)
    # end to end: the length scale Alg. 1 uses under ls_mode 1
    prm = O.Params(voxel_size=s, max_pts=10 ** 6, min_pts=3, grid_side=3, ls_mode=1)
    k = np.floor(P[0] / s).astype(np.int64)
    res = O.fit_predict_voxel(P[:64].astype(np.float32), O.pack_keys(k[None])[0], prm)
    ev = O.local_frame(P[:64].astype(np.float32).astype(np.float64)).eigvals
    assert res["length_scale"] == pytest.approx(math.sqrt(1.5 * (ev[1] + ev[2])), rel=1e-12)


@pytest.mark.parametrize("s", [0.1, 0.2, 1.0])
def test_pca_length_scale_clamp_edges(s):
    """The clamp [0.05 s, 2 s], s the float32 voxel size: values inside pass unchanged,
    values outside take the nearer edge, and the edges themselves are reached exactly.
    The eigenvalues are chosen so that (lambda_mid + lambda_max) / 2 = l^2 / 3 exactly
    in the rule's formula; lambda_min must not enter."""
    sf = float(np.float32(s))

    def ell_for(target, lam_min=0.0):
        half = target * target / 3.0
        return O.pca_length_scale(np.array([lam_min, 0.5 * half, 1.5 * half]), s)

    for frac in (0.051, 0.3, 0.5, 1.0, 1.99):
        assert ell_for(frac * sf) == pytest.approx(frac * sf, rel=1e-12)
        assert ell_for(frac * sf, lam_min=0.25 * (frac * sf) ** 2 / 3.0) == pytest.approx(frac * sf, rel=1e-12)
    for frac in (1e-4, 0.01, 0.049):
        assert ell_for(frac * sf) == 0.05 * sf
    for frac in (2.01, 3.0, 50.0):
        assert ell_for(frac * sf) == 2.0 * sf
    assert O.pca_length_scale(np.zeros(3), s) == 0.05 * sf          # a single repeated point
    # a line segment: lambda_mid = 0
    assert O.pca_length_scale(np.array([0.0, 0.0, 1.5 * sf * sf]), s) == pytest.approx(1.5 * sf, rel=1e-12)


# ---------------------------------------------------------------------------
# Voxel state machine (Sec. 3.3)
# ---------------------------------------------------------------------------
def test_map_state_machine_types():
    prm = _params(min_pts=10, max_pts=40, converge_var=0.05)
    m = O.VoxelMap(prm)
    r = rng(60)

    def pts(n, base):
        return np.stack([base[0] + r.uniform(0.01, 0.49, n), base[1] + r.uniform(0.01, 0.49, n),
                         base[2] + 0.25 + r.normal(0, 0.005, n)], 1).astype(np.float32)
    A = (0.0, 0.0, 0.0)
    B = (1.0, 0.0, 0.0)
    u1 = m.update(np.concatenate([pts(6, A), pts(12, B)]))          # A: type (a); B: type (b)
    kB = O.pack_keys(np.array([[2, 0, 0]]))[0]
    kA = O.pack_keys(np.array([[0, 0, 0]]))[0]
    assert u1["keys"].tolist() == [kB]
    u2 = m.update(pts(6, A))                                          # A reaches tau with stacked points
    assert u2["keys"].tolist() == [kA]
    assert len(m.points[kA]) == 12
    if not m.converged.get(kB, False):
        u3 = m.update(pts(30, B))                                     # B type (c): re-solved on stacked points
        assert kB in u3["keys"].tolist()
        assert len(m.points[kB]) == 40                                # cap keeps the first 40 in arrival order
    m.converged[kB] = True
    u4 = m.update(pts(5, B))                                          # type (d): skipped
    assert kB not in u4["keys"].tolist()


# ---------------------------------------------------------------------------
# Sec. 3.3 / Fig. 4: covariance-centred update of type (c) voxels
# ---------------------------------------------------------------------------
# Lattice sites at >= 0.1 from the interval centres 0.25 / 0.75 of a 2x2 grid on
# the unit voxel's face; with l = 1e-3 every kernel entry between distinct sites
# or between a site and a grid point underflows to 0, so the posterior at a grid
# point sees only the carried prediction at that point: with prior s_f^2 and a
# pseudo-observation c of noise variance v at the point itself,
#   var = s_f^2 v / (s_f^2 + v),  mean = mu + s_f^2 / (s_f^2 + v) (c - mu),
# mu being the mean value of the stacked set (Eq. (3) for one observation).
_FB_SITES = [0.05, 0.15, 0.35, 0.45, 0.55, 0.65, 0.85, 0.95]


def _fb_frame(r, n, z):
    idx = r.choice(64, n, replace=False)
    x = np.array([_FB_SITES[i // 8] for i in idx])
    y = np.array([_FB_SITES[i % 8] for i in idx])
    return np.stack([x, y, np.asarray(z, float)], 1).astype(np.float32)


def test_feedback_update_closed_form_sequence():
    prm = _params(voxel_size=1.0, grid_side=2, min_pts=3, max_pts=8, length_scale=1e-3, converge_var=0.3)
    m = O.VoxelMap(prm, feedback=True)
    r = rng(90)
    key = int(O.pack_keys(np.array([[0, 0, 0]]))[0])
    frames = [_fb_frame(r, 5, 0.5 + r.uniform(-0.01, 0.01, 5)),
              _fb_frame(r, 4, 0.5 + r.uniform(-0.01, 0.01, 4)),
              _fb_frame(r, 3, 0.5 + r.uniform(-0.01, 0.01, 3)),
              _fb_frame(r, 11, np.concatenate([0.5 + r.uniform(-0.01, 0.01, 8), [0.56] * 3])),
              _fb_frame(r, 2, [0.5, 0.5])]
    sf2 = prm.signal_var
    grid = np.array([[0.25, 0.25], [0.25, 0.75], [0.75, 0.25], [0.75, 0.75]])
    c = v = None
    for k, F in enumerate(frames):
        u = m.update(F)
        if k == 4:  # converged at the fourth solve: type (d), skipped
            assert u["keys"].tolist() == []
            break
        assert u["keys"].tolist() == [key] and u["axis"].tolist() == [2]
        z = F[:, 2].astype(np.float64)
        if k == 0:  # type (b): no grid point sees a data point
            mean = np.full(4, z.mean())
            var = np.full(4, sf2)
        else:
            zn = z[: prm.max_pts]
            mu = (4 * c + zn.sum()) / (4 + len(zn))
            mean = np.full(4, mu + sf2 / (sf2 + v) * (c - mu))
            var = np.full(4, sf2 * v / (sf2 + v))
        out = u["out"][0]
        assert np.allclose(out[:, :2], grid, atol=0)
        assert np.allclose(out[:, 2], mean, rtol=0, atol=1e-12), (k, out[:, 2], mean)
        assert np.allclose(out[:, 3], var, rtol=0, atol=1e-12), (k, out[:, 3], var)
        st = int(u["status"][0])
        assert bool(st & O.ST_CAPPED) == (len(F) > prm.max_pts)
        assert bool(st & O.ST_CONVERGED) == (k == 3), (k, var)
        c = float(np.float32(mean[0]))
        v = float(np.float32(var[0]))


def test_feedback_variance_never_exceeds_single_pseudo_observation():
    """Posterior variance with more observations is no larger than with a subset:
    at a grid point that carries a prediction of variance v, a type (c) re-solve
    (same value axis, hence the same grid) gives var <= s_f^2 v / (s_f^2 + v) < v."""
    prm = _params(voxel_size=0.5, grid_side=4, min_pts=3, max_pts=24, length_scale=0.25, converge_var=1e-4)
    m = O.VoxelMap(prm, feedback=True)
    r = rng(91)
    n_checked = 0
    axes = {}
    for f in range(5):
        pts = []
        for b in range(6):
            o = np.array([0.5 * (b % 3), 0.5 * (b // 3), 0.0])
            n = int(r.integers(2, 30))
            xy = r.uniform(0.02, 0.48, (n, 2))
            z = 0.2 + 0.3 * xy[:, 0] - 0.2 * xy[:, 1] + r.normal(0, 0.01, n)
            pts.append(o + np.stack([xy[:, 0], xy[:, 1], z], 1))
        F = np.concatenate(pts).astype(np.float32)
        prev = {k: v.copy() for k, v in m.pred.items()}
        pool = {k: len(v) for k, v in m.points.items()}
        u = m.update(F)
        for i, key in enumerate(u["keys"].tolist()):
            st = int(u["status"][i])
            if key in prev:
                assert len(m.points[key]) == pool[key]  # the pool stops growing once in the map
                if st & O.ST_SOLVED and axes.get(key) == int(u["axis"][i]):
                    vq = np.maximum(prev[key][:, 3].astype(np.float64), O.PRED_NOISE_FLOOR * prm.signal_var)
                    bound = prm.signal_var * vq / (prm.signal_var + vq)
                    assert (u["out"][i][:, 3] <= bound * (1 + 1e-9) + 1e-12).all(), (f, key)
                    n_checked += 1
            if st & O.ST_SOLVED:
                axes[key] = int(u["axis"][i])
    assert n_checked >= 10


def test_feedback_state_machine():
    """Types (a)-(d) with feedback: points pool until tau, the first solve puts the
    voxel in the map, a later frame re-solves on the m carried rows plus the new
    points (capped), converged voxels are skipped."""
    prm = _params(min_pts=10, max_pts=12, grid_side=3, converge_var=1e-6)
    m = O.VoxelMap(prm, feedback=True)
    r = rng(92)

    def pts(n, base):
        return np.stack([base[0] + r.uniform(0.01, 0.49, n), base[1] + r.uniform(0.01, 0.49, n),
                         base[2] + 0.25 + r.normal(0, 0.005, n)], 1).astype(np.float32)
    A, B = (0.0, 0.0, 0.0), (1.0, 0.0, 0.0)
    kA = int(O.pack_keys(np.array([[0, 0, 0]]))[0])
    kB = int(O.pack_keys(np.array([[2, 0, 0]]))[0])
    u1 = m.update(np.concatenate([pts(6, A), pts(12, B)]))   # A: (a); B: (b) -> in the map
    assert u1["keys"].tolist() == [kB] and kB in m.pred and kA not in m.pred
    u2 = m.update(np.concatenate([pts(5, A), pts(3, B)]))    # A: (b) on 11 pooled points; B: (c) on 9 + 3
    assert u2["keys"].tolist() == [kA, kB]
    assert len(m.points[kA]) == 11 and len(m.points[kB]) == 12
    assert not u2["status"][1] & O.ST_CAPPED
    u3 = m.update(pts(20, B))                                 # (c) with 20 new points: 12 taken, CAPPED
    assert u3["keys"].tolist() == [kB] and u3["status"][0] & O.ST_CAPPED
    assert len(m.points[kB]) == 12
    m.converged[kB] = True
    assert m.update(pts(4, B))["keys"].tolist() == []         # (d): skipped
    # the re-solve sees exactly the carried rows and the capped new points
    X, nz = O.feedback_inputs(m.pred[kA], pts(15, A), prm)
    assert X.shape == (9 + 12, 3) and np.all(nz[9:] == prm.noise_var)


# ---------------------------------------------------------------------------
# Sec. 3.2: initial 3D Gaussians from the predicted grid
# ---------------------------------------------------------------------------
def _grid_rows(gs, h, z, var):
    rows = np.zeros((1, gs * gs, 4))
    for i in range(gs):
        for j in range(gs):
            rows[0, i * gs + j] = [i * h, j * h, z(i, j), var(i, j)]
    return rows


def test_gauss_uniform_weights_regular_grid_closed_form():
    """Equal variances: position = centroid of the block, parameter-axis scales =
    h^2 (n_r^2 - 1) / 12 (population variance of n_r equally spaced values),
    value-axis scale = exact rational variance of the block's values."""
    gs, nr = 6, 3
    h = Fraction(1, 10)
    zf = lambda i, j: Fraction(1, 2) + Fraction(1, 100) * i * i + Fraction(1, 1000) * j  # noqa: E731
    rows = _grid_rows(gs, float(h), lambda i, j: float(zf(i, j)), lambda i, j: 0.04)
    g = O.gauss_init(rows, np.array([O.ST_SOLVED]), gs, nr, 1e-12)
    ns = gs // nr
    assert g.shape == (1, ns * ns, 8)
    for bi in range(ns):
        for bj in range(ns):
            pts = [(i, j) for i in range(bi * nr, bi * nr + nr) for j in range(bj * nr, bj * nr + nr)]
            zs = [zf(i, j) for i, j in pts]
            zm = sum(zs) / len(zs)
            zv = sum((z - zm) ** 2 for z in zs) / len(zs)
            e = g[0, bi * ns + bj]
            assert e[0] == pytest.approx(float(h * (bi * nr + Fraction(nr - 1, 2))), abs=1e-15)
            assert e[1] == pytest.approx(float(h * (bj * nr + Fraction(nr - 1, 2))), abs=1e-15)
            assert e[2] == pytest.approx(float(zm), abs=1e-15)
            assert e[3] == pytest.approx(nr * nr / 0.04, rel=1e-15)
            assert e[4] == pytest.approx(float(h * h * (nr * nr - 1) / 12), rel=1e-12)
            assert e[5] == pytest.approx(float(h * h * (nr * nr - 1) / 12), rel=1e-12)
            assert e[6] == pytest.approx(float(zv), rel=1e-10, abs=1e-18)


def test_gauss_matches_numpy_weighted_covariance():
    """Brute force: numpy.average and numpy.cov(aweights=1/var, bias=True) per subgrid."""
    r = rng(40)
    gs, nr = 8, 4
    rows = np.concatenate([r.normal(size=(3, gs * gs, 3)), r.uniform(1e-3, 0.5, size=(3, gs * gs, 1))], axis=2)
    g = O.gauss_init(rows, np.array([O.ST_SOLVED] * 3), gs, nr, 1e-12)
    ns = gs // nr
    for v in range(3):
        grid = rows[v].reshape(gs, gs, 4)
        for bi in range(ns):
            for bj in range(ns):
                blk = grid[bi * nr:(bi + 1) * nr, bj * nr:(bj + 1) * nr].reshape(-1, 4)
                w = 1.0 / blk[:, 3]
                p = np.average(blk[:, :3], axis=0, weights=w)
                C = np.cov(blk[:, :3].T, aweights=w, bias=True)
                e = g[v, bi * ns + bj]
                assert np.allclose(e[:3], p, rtol=0, atol=1e-13)
                assert np.allclose(e[4:7], np.diag(C), rtol=1e-11, atol=1e-15)
                assert e[7] == 0.0


def test_gauss_dominant_weight_and_invariances():
    r = rng(41)
    gs, nr = 6, 3
    rows = np.concatenate([r.normal(size=(1, gs * gs, 3)), np.ones((1, gs * gs, 1))], axis=2)
    st = np.array([O.ST_SOLVED])
    base = O.gauss_init(rows, st, gs, nr, 1e-30)
    # one point with a tiny variance pulls its Gaussian onto itself and shrinks the scales
    q = 1 * gs + 4  # (i, j) = (1, 4): subgrid (0, 1)
    r2 = rows.copy()
    r2[0, q, 3] = 1e-14
    g = O.gauss_init(r2, st, gs, nr, 1e-30)
    assert np.allclose(g[0, 1, :3], rows[0, q, :3], atol=1e-12)
    assert np.all(g[0, 1, 4:7] < 1e-12)
    assert np.array_equal(g[0, [0, 2, 3]], base[0, [0, 2, 3]])
    # scaling every variance leaves position and scale unchanged and divides sum w
    r3 = rows.copy()
    r3[..., 3] *= 7.5
    g3 = O.gauss_init(r3, st, gs, nr, 1e-30)
    assert np.allclose(g3[..., [0, 1, 2, 4, 5, 6]], base[..., [0, 1, 2, 4, 5, 6]], rtol=1e-12, atol=1e-14)
    assert np.allclose(g3[..., 3] * 7.5, base[..., 3], rtol=1e-12)
    # translation moves positions only
    r4 = rows.copy()
    r4[..., :3] += np.array([3.0, -2.0, 0.5])
    g4 = O.gauss_init(r4, st, gs, nr, 1e-30)
    assert np.allclose(g4[..., :3] - base[..., :3], [3.0, -2.0, 0.5], atol=1e-12)
    assert np.allclose(g4[..., 4:7], base[..., 4:7], rtol=1e-9, atol=1e-14)


def test_gauss_floor_unsolved_and_single_point_subgrids():
    r = rng(42)
    gs = 4
    rows = np.concatenate([r.normal(size=(2, gs * gs, 3)), r.uniform(0.1, 1, size=(2, gs * gs, 1))], axis=2)
    rows[0, 5, 3] = 0.0  # a zero variance takes the floor: finite weight 1 / floor
    g = O.gauss_init(rows, np.array([O.ST_SOLVED, O.ST_BELOW_TAU]), gs, 2, 1e-6)
    assert np.isfinite(g[0]).all() and np.isnan(g[1]).all()
    q = 5  # (1, 1): subgrid (0, 0)
    assert g[0, 0, 3] == pytest.approx(1e6 + sum(1.0 / rows[0, k, 3] for k in (0, 1, 4)), rel=1e-12)
    # n_r = 1: every point is its own Gaussian with zero scale
    g1 = O.gauss_init(rows, np.array([O.ST_SOLVED, O.ST_SOLVED]), gs, 1, 1e-6)
    assert np.allclose(g1[:, :, :3], rows[:, :, :3], rtol=1e-15, atol=1e-15)
    assert np.all(np.abs(g1[:, :, 4:7]) <= 1e-28)  # zero up to the rounding of w P / w
    assert q == 5


# ---------------------------------------------------------------------------
# PCA-rotated local frame (frame_mode 1)
# ---------------------------------------------------------------------------
def _dyadic_plane_points(coef, n=40, seed=0):
    """Points with dyadic coordinates on z = a x + b y + c (exact in float32),
    or on the same plane with the axes cyclically relabelled."""
    r = rng(seed)
    a, b, c, perm = coef
    xy = r.integers(0, 32, size=(n, 2)) / 64.0
    z = a * xy[:, 0] + b * xy[:, 1] + c
    P = np.stack([xy[:, 0], xy[:, 1], z], axis=1)[:, perm]
    assert np.array_equal(P.astype(np.float32).astype(np.float64), P)
    return P


@pytest.mark.parametrize("coef", [(0.5, 0.25, 0.125, [0, 1, 2]), (-0.75, 0.5, 0.25, [0, 1, 2]),
                                  (1.5, -0.25, 0.0, [1, 2, 0]), (0.25, 2.0, 0.5, [2, 0, 1]),
                                  (-3.0, 0.5, 0.75, [0, 2, 1])])
def test_rotated_frame_recovers_noiseless_tilted_planes_exactly(coef):
    """Every prediction lies on the plane of the data, for any tilt (the value
    coordinate of coplanar points is zero in the rotated frame)."""
    P = _dyadic_plane_points(coef)
    a, b, c, perm = coef
    nrm = np.array([-a, -b, 1.0])[perm]  # normal in the relabelled axes: column j is axis perm[j]
    key = O.pack_keys(O.voxel_coords(P[:1], 1.0)[0])[0]
    for nq in (3, 8):
        prm = O.Params(voxel_size=1.0, min_pts=3, grid_side=nq, frame_mode=1, length_scale=0.3)
        r = O.fit_predict_voxel(P, key, prm)
        assert r["status"] & O.ST_SOLVED
        out = r["out"][:, :3]
        # distance of every predicted point to the plane through the data
        off = (out - P[0]) @ nrm / np.linalg.norm(nrm)
        assert np.abs(off).max() <= 1e-12, np.abs(off).max()


def test_rotated_frame_closed_form_and_grid_geometry():
    """Plane z = x / 2: normal (-1, 0, 2)/sqrt(5) with its z component positive,
    e1 = e_y x v = (2, 0, 1)/sqrt(5), e2 = v x e1 = (0, 1, 0); the predicted points
    project onto (e1, e2) about the centroid as the interval centres of an s x s square."""
    P = _dyadic_plane_points((0.5, 0.0, 0.25, [0, 1, 2]), n=30, seed=3)
    prm = O.Params(voxel_size=0.5, min_pts=3, grid_side=4, frame_mode=1, length_scale=0.2)
    key = O.pack_keys(O.voxel_coords(P[:1], 0.5)[0])[0]
    r = O.fit_predict_voxel(P, key, prm)
    e1, e2, v = r["rotation"]
    s5 = math.sqrt(5.0)
    assert np.allclose(v, [-1 / s5, 0, 2 / s5], atol=1e-14)
    assert np.allclose(e1, [2 / s5, 0, 1 / s5], atol=1e-14)
    assert np.allclose(e2, [0, 1, 0], atol=1e-14)
    assert np.allclose(np.cross(e1, e2), v, atol=1e-14)
    c = P.mean(axis=0)
    d = r["out"][:, :3] - c
    t = [((i + 0.5) / 4 - 0.5) * 0.5 for i in range(4)]
    assert np.allclose(d @ e1, np.repeat(t, 4), atol=1e-12)
    assert np.allclose(d @ e2, np.tile(t, 4), atol=1e-12)


def test_rotated_frame_orthonormal_and_continuous():
    r0 = rng(50)
    for _ in range(20):
        P = r0.normal(size=(30, 3)) * [1.0, 0.7, 0.05]
        Q, _ = np.linalg.qr(r0.normal(size=(3, 3)))
        P = P @ Q.T
        fr = O.local_frame(P)
        e1, e2, v = O.rotated_frame(fr)
        M = np.stack([e1, e2, v])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-13)
        assert np.linalg.det(M) > 0 and v[fr.axis] > 0
        # a tiny perturbation of the points moves the frame only a little
        e1b, e2b, vb = O.rotated_frame(O.local_frame(P + 1e-9 * r0.normal(size=P.shape)))
        if np.argmin(np.abs(v)) == np.argmin(np.abs(vb)):
            assert np.abs(np.stack([e1b, e2b, vb]) - M).max() < 1e-6


# ---------------------------------------------------------------------------
# Eq. (9): structure similarity loss L_p
# ---------------------------------------------------------------------------
def _gauss_rows(centres, scales):
    G = np.zeros((len(centres), 8), np.float32)
    G[:, :3] = centres
    G[:, 4:7] = scales
    return G


def test_structure_loss_worked_example_exact():
    """Hand-computed: 3-4-5 and 5-12-13 distances with rational scale means."""
    G = _gauss_rows([[0, 0, 0], [6, 8, 0], [0, 0, 13]],
                    [[0.5, 0.5, 0.5], [1.0, 2.0, 3.0], [0.25, 0.25, 0.25]])
    P = np.array([[3, 4, 0], [0, 5, 1], [6, 8, 0.5]], np.float32)
    # point 0: |.|=5 -> 4.5; |(3,4,0)-(6,8,0)|=5 -> 3; to (0,0,13): sqrt(9+16+169) -> larger
    # point 1: to (0,0,0): sqrt(26) - 0.5; to (6,8,0): sqrt(36+9+1) - 2; to (0,0,13): 13 - 0.25
    # point 2: to (6,8,0): 0.5 - 2 = -1.5
    r = O.structure_loss(P, G)
    v1 = [math.sqrt(26) - 0.5, math.sqrt(46) - 2, 13 - 0.25]
    assert r["arg"].tolist() == [1, int(np.argmin(v1)), 1]
    assert r["value"][0] == pytest.approx(3.0, abs=1e-12)
    assert r["value"][1] == pytest.approx(min(v1), abs=1e-12)
    assert r["value"][2] == pytest.approx(-1.5, abs=1e-12)
    assert r["loss"] == pytest.approx((3.0 + min(v1) - 1.5) / 3, abs=1e-12)
    assert r["n_valid"] == 3


def test_structure_loss_zero_scale_is_nearest_neighbour():
    """S-bar = 0 reduces Eq. (9) to the nearest-neighbour distance (scipy's k-d tree);
    a common S-bar = c shifts every value by -c with the same nearest index."""
    import scipy.spatial
    r = rng(70)
    C = r.uniform(-5, 5, (400, 3)).astype(np.float32)
    P = r.uniform(-6, 6, (300, 3)).astype(np.float32)
    d, k = scipy.spatial.cKDTree(C.astype(np.float64)).query(P.astype(np.float64))
    r0 = O.structure_loss(P, _gauss_rows(C, np.zeros((400, 3))))
    assert np.allclose(r0["value"], d, rtol=0, atol=1e-12)
    assert np.array_equal(r0["arg"], k)
    rc = O.structure_loss(P, _gauss_rows(C, np.full((400, 3), 0.75)))
    assert np.allclose(rc["value"], d - 0.75, rtol=0, atol=1e-12)
    assert np.array_equal(rc["arg"], k)
    assert rc["loss"] == pytest.approx(d.mean() - 0.75, abs=1e-12)


def test_structure_loss_minimises_the_difference_not_the_distance():
    """A farther Gaussian with a larger scale wins: the minimum is over
    |P - p_k| - S-bar_k, not S-bar of the nearest centre."""
    G = _gauss_rows([[1, 0, 0], [3, 0, 0]], [[0, 0, 0], [2.5, 2.5, 2.5]])
    r = O.structure_loss(np.array([[0, 0, 0]], np.float32), G)
    assert r["arg"].tolist() == [1] and r["value"][0] == pytest.approx(0.5, abs=1e-12)


def test_structure_loss_scale_modes_and_invariances():
    G = _gauss_rows([[0, 0, 0]], [[1.0, 4.0, 9.0]])
    P = np.array([[0, 0, 10]], np.float32)
    assert O.structure_loss(P, G, scale_mode=0)["value"][0] == pytest.approx(10 - 14 / 3, abs=1e-12)
    assert O.structure_loss(P, G, scale_mode=1)["value"][0] == pytest.approx(10 - 2.0, abs=1e-12)
    r = rng(71)
    C = r.uniform(-2, 2, (60, 3)).astype(np.float32)
    S = r.uniform(0, 0.3, (60, 3)).astype(np.float32)
    Q = r.uniform(-3, 3, (50, 3)).astype(np.float32)
    base = O.structure_loss(Q, _gauss_rows(C, S))
    # translation by a dyadic offset (exact in float32 at these magnitudes)
    t = np.array([8.0, -4.0, 2.0], np.float32)
    moved = O.structure_loss(Q + t, _gauss_rows(C + t, S))
    assert np.allclose(moved["value"], base["value"], rtol=0, atol=1e-6)
    # permuting the Gaussians permutes the indices only
    perm = r.permutation(60)
    pr = O.structure_loss(Q, _gauss_rows(C[perm], S[perm]))
    assert np.allclose(pr["value"], base["value"], rtol=0, atol=1e-12)
    assert np.array_equal(perm[pr["arg"]], base["arg"])


def test_structure_loss_invalid_rows_points_and_empty_map():
    G = _gauss_rows([[0, 0, 0], [1, 0, 0]], [[0.1] * 3, [0.1] * 3])
    G[0, :] = np.nan                                           # an unsolved voxel's row
    P = np.array([[0, 0, 0], [np.nan, 0, 0], [2, 0, 0]], np.float32)
    r = O.structure_loss(P, G)
    assert r["arg"].tolist() == [1, -1, 1] and np.isnan(r["value"][1])
    assert r["n_valid"] == 2
    assert r["loss"] == pytest.approx(((1 - 0.1) + (1 - 0.1)) / 2, abs=1e-7)
    e = O.structure_loss(P, G[:1])
    assert np.isinf(e["value"][0]) and e["arg"][0] == -1 and np.isinf(e["loss"])
    assert np.isnan(O.structure_loss(np.zeros((0, 3), np.float32), G)["loss"])
