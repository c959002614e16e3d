"""Pins for the FP64 oracle: closed forms, invariants and special cases that
fix what the lift computes independently of the oracle's own code.

Paper references are to the Method section ("Semantic Embedding"): the
rasterizer call that yields per-pixel weights of the contributing Gaussians,
the parameter-masking step and the aggregation equation.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import make_custom_scene

F32 = np.float32


def _cam(w, h, f, cx=None, cy=None, R=None, t=None):
    return dict(fx=f, fy=f, cx=w / 2 if cx is None else cx, cy=h / 2 if cy is None else cy,
                R=np.eye(3) if R is None else R, t=np.zeros(3) if t is None else t,
                width=w, height=h)


def _pixel_ids(w, h):
    return np.arange(w * h, dtype=np.int32).reshape(h, w)


def _unit_feats(n, d, seed=0):
    f = np.random.default_rng(seed).standard_normal((n, d))
    return (f / np.linalg.norm(f, axis=1, keepdims=True)).astype(np.float32)


def _alpha(o, dx, dy, sxx, syy, sxy=0.0):
    det = sxx * syy - sxy * sxy
    q = (syy * dx * dx - 2 * sxy * dx * dy + sxx * dy * dy) / det
    return np.minimum(0.99, o * np.exp(-0.5 * q))


# --------------------------------------------------------------------------
# projection

def test_projection_on_axis_closed_form():
    """On the optical axis an axis-aligned Gaussian projects with a diagonal
    Jacobian: Sigma2 = diag(fx^2 sx^2 / z^2, fy^2 sy^2 / z^2) + 0.3 I, mean at
    the principal point."""
    f, z = 40.0, 3.0
    s = np.array([0.11, 0.07, 0.05])
    sc = make_custom_scene([0, 0, z], s, [1, 0, 0, 0], [0.5], [_cam(64, 48, f)],
                           [np.zeros((48, 64), np.int32)], _unit_feats(1, 4))
    mu, cov, con, zc = oracle.project64_view(sc, 0)
    s32 = s.astype(F32).astype(np.float64)
    exp_cov = [f * f * s32[0] ** 2 / z ** 2 + 0.3, 0.0, f * f * s32[1] ** 2 / z ** 2 + 0.3]
    np.testing.assert_allclose(cov[0], exp_cov, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(mu[0], [32.0, 24.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(con[0], [1 / exp_cov[0], 0.0, 1 / exp_cov[2]], rtol=1e-12, atol=1e-15)
    assert zc[0] == z


@pytest.mark.parametrize("angle_deg", [45.0, -30.0])
def test_projection_rotated_closed_form(angle_deg):
    """A rotation theta about the optical axis (quaternion (cos t/2, 0, 0,
    sin t/2), Hamilton convention, active) turns the screen covariance by
    theta: Sigma_xy = (f/z)^2 (sx^2 - sy^2) cos sin.  The sign fixes the
    quaternion convention and the order of the covariance products."""
    f, z = 40.0, 3.0
    sx, sy, sz = 0.2, 0.05, 0.05
    th = math.radians(angle_deg)
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    sc = make_custom_scene([0, 0, z], [sx, sy, sz], q, [0.5], [_cam(64, 64, f)],
                           [np.zeros((64, 64), np.int32)], _unit_feats(1, 4))
    _, cov, _, _ = oracle.project64_view(sc, 0)
    # the quaternion is rounded to float32 in the scene; use its exact value
    qq = sc.quats[0].astype(np.float64)
    qq /= np.linalg.norm(qq)
    th32 = 2 * math.atan2(qq[3], qq[0])
    c, s = math.cos(th32), math.sin(th32)
    sx, sy = [float(v) for v in sc.scales[0, :2].astype(np.float64)]
    k = f * f / (z * z)
    exp = [k * (c * c * sx * sx + s * s * sy * sy) + 0.3, k * c * s * (sx * sx - sy * sy),
           k * (s * s * sx * sx + c * c * sy * sy) + 0.3]
    np.testing.assert_allclose(cov[0], exp, rtol=1e-9, atol=1e-12)


def test_projection_matches_sampled_perspective():
    """EWA projection is the first-order (Jacobian) image of the 3D Gaussian
    under the pinhole map x = fx X/Z + cx: for a small Gaussian it equals the
    covariance of projected samples.  Catches transposed rotations, wrong
    Jacobian terms or a wrong world-to-camera product."""
    rng = np.random.default_rng(5)
    # camera looking at the origin from an oblique pose
    pos = np.array([2.0, -1.5, 1.2])
    fwd = -pos / np.linalg.norm(pos)
    right = np.cross(fwd, [0, 0, 1.0]); right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ pos
    mean = np.array([0.3, -0.2, 0.25])
    scale = np.array([0.004, 0.0015, 0.0025])
    q = rng.standard_normal(4); q /= np.linalg.norm(q)
    sc = make_custom_scene(mean, scale, q, [0.5],
                           [_cam(320, 240, 256.0, R=R.astype(F32), t=t.astype(F32))],
                           [np.zeros((240, 320), np.int32)], _unit_feats(1, 4))
    mu, cov, _, _ = oracle.project64_view(sc, 0)
    # sample in float64 from the float32 parameters the oracle sees
    m = sc.means[0].astype(np.float64)
    s = sc.scales[0].astype(np.float64)
    w, x, y, z = (sc.quats[0].astype(np.float64) / np.linalg.norm(sc.quats[0].astype(np.float64)))
    Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                   [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                   [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    n = 400_000
    pts = m + (rng.standard_normal((n, 3)) * s) @ Rq.T
    Rc = sc.cams[0]["R"].astype(np.float64).reshape(3, 3)
    tc = sc.cams[0]["t"].astype(np.float64)
    pc = pts @ Rc.T + tc
    u = 256.0 * pc[:, 0] / pc[:, 2] + 160.0
    v = 256.0 * pc[:, 1] / pc[:, 2] + 120.0
    C = np.cov(np.stack([u, v]))
    got = np.array([[cov[0, 0] - 0.3, cov[0, 1]], [cov[0, 1], cov[0, 2] - 0.3]])
    assert np.linalg.norm(got - C) / np.linalg.norm(C) < 1.5e-2
    np.testing.assert_allclose(mu[0], [u.mean(), v.mean()], atol=2e-3 * math.sqrt(C[0, 0]) + 1e-3)


def test_mirror_depth_and_box_agree_with_fp64(scene_2k):
    """The FP32 decision path agrees with FP64 to rounding, and its pixel box
    contains every pixel where the FP64 weight reaches 1/255."""
    for v in range(scene_2k.n_views):
        mv = oracle.mirror_view(scene_2k, v)
        mu, cov, con, zc = oracle.project64_view(scene_2k, v)
        vis = mv.vis == 1
        assert vis.sum() > 100
        np.testing.assert_allclose(mv.z32[vis], zc[vis], rtol=3e-7)
        np.testing.assert_allclose(mv.mu[vis], mu[vis], rtol=0, atol=2e-4)
        np.testing.assert_allclose(mv.cov[vis], cov[vis], rtol=1e-4, atol=1e-4)
        # conservative box: a ring of pixels just outside has alpha < 1/255
        W, H = int(scene_2k.cams[v]["width"]), int(scene_2k.cams[v]["height"])
        for g in np.flatnonzero(vis)[:300]:
            x0, x1, y0, y1 = mv.box[g]
            xs = np.arange(max(x0 - 3, 0), min(x1 + 4, W))
            ys = np.arange(max(y0 - 3, 0), min(y1 + 4, H))
            X, Y = np.meshgrid(xs + 0.5, ys + 0.5)
            inside = (X >= x0) & (X <= x1 + 1) & (Y >= y0) & (Y <= y1 + 1)
            a = _alpha(float(scene_2k.opacity[g]), X - mu[g, 0], Y - mu[g, 1],
                       cov[g, 0], cov[g, 2], cov[g, 1])
            assert not np.any((a >= 1 / 255) & ~inside)


# --------------------------------------------------------------------------
# blending weights

def _axis_scene(gs, w=32, h=32, f=25.6, cx=None, cy=None, ids=None, feats=None):
    means = [[0, 0, z] for z, _, _ in gs]
    scales = [s for _, s, _ in gs]
    ops = [o for _, _, o in gs]
    ids = _pixel_ids(w, h) if ids is None else ids
    nseg = int(ids.max()) + 1
    feats = _unit_feats(nseg, 4) if feats is None else feats
    return make_custom_scene(means, scales, [[1, 0, 0, 0]] * len(gs), ops,
                             [_cam(w, h, f, cx, cy)], [ids], feats)


def _screen_diag(sc, g):
    f = float(sc.cams[0]["fx"])          # the float32 focal length the oracle sees
    z = float(sc.means[g, 2])
    s = sc.scales[g].astype(np.float64)
    return f * f * s[0] ** 2 / z ** 2 + 0.3, f * f * s[1] ** 2 / z ** 2 + 0.3


def _dense_w(res, g, npix):
    out = np.zeros(npix)
    m = res.g == g
    out[res.s[m]] = res.w[m]
    return out


def test_single_gaussian_closed_form():
    """One Gaussian, T = 1: w(p) = min(0.99, o exp(-q/2)) wherever it reaches
    1/255, else 0 (per-pixel segments expose every pixel's weight)."""
    sc = _axis_scene([(3.0, [0.3, 0.15, 0.1], 0.8)])
    r = oracle.lift_view(sc, 0, pixels=True)
    sxx, syy = _screen_diag(sc, 0)
    u, v = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    a = _alpha(float(sc.opacity[0]), u - 16.0, v - 16.0, sxx, syy)
    exp = np.where(a >= 1 / 255, a, 0.0).ravel()
    got = _dense_w(r, 0, 32 * 32)
    np.testing.assert_allclose(got, exp, rtol=1e-12, atol=0)
    assert (got > 0).sum() == (exp > 0).sum() > 50


def test_two_gaussian_occlusion_closed_form():
    """Front-to-back blending: behind a front Gaussian the back one gets
    w_b = alpha_b (1 - alpha_f) where the front one is blended."""
    sc = _axis_scene([(4.0, [0.5, 0.4, 0.1], 0.8), (2.0, [0.15, 0.25, 0.1], 0.9)])
    r = oracle.lift_view(sc, 0)
    u, v = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    ab = _alpha(float(sc.opacity[0]), u - 16.0, v - 16.0, *_screen_diag(sc, 0)).ravel()
    af = _alpha(float(sc.opacity[1]), u - 16.0, v - 16.0, *_screen_diag(sc, 1)).ravel()
    af = np.where(af >= 1 / 255, af, 0.0)
    exp_b = np.where(ab >= 1 / 255, ab * (1 - af), 0.0)
    np.testing.assert_allclose(_dense_w(r, 1, 1024), af, rtol=1e-12)
    np.testing.assert_allclose(_dense_w(r, 0, 1024), exp_b, rtol=1e-12)
    assert (af > 0.5).any() and (exp_b > 0).sum() > 100


def test_termination_is_exclusive():
    """The walk stops before the Gaussian that would take T below 1e-4: with
    alpha = 0.95 at a pixel centre, three Gaussians blend (T = 0.05^3 =
    1.25e-4) and the fourth does not; a Gaussian whose alpha stays below
    1/255 never blends and leaves T untouched."""
    gs = [(2.0 + 0.1 * k, [0.05, 0.05, 0.05], 0.95) for k in range(5)]
    gs.insert(1, (2.05, [0.3, 0.3, 0.05], 0.0035))   # alpha < 1/255 everywhere
    sc = _axis_scene(gs, cx=16.5, cy=16.5)
    r = oracle.lift_view(sc, 0, pixels=True)
    p = 16 * 32 + 16                         # pixel whose centre is (16.5, 16.5)
    a = float(np.float32(0.95))
    order = [0, 2, 3, 4, 5]                  # depth order without the faint one
    exp = [a * (1 - a) ** k for k in range(3)]
    for k, g in enumerate(order):
        got = _dense_w(r, g, 1024)[p]
        assert got == pytest.approx(exp[k], rel=1e-13) if k < 3 else got == 0.0
    assert not np.any(r.g == 1)
    assert r.T.ravel()[p] == pytest.approx((1 - a) ** 3, rel=1e-12)
    assert r.T.ravel()[p] >= 1e-4


def test_pixel_invariant_and_bounds(oracle_2k):
    """Telescoping: sum_k w_kp = 1 - T_final(p), and T_final >= 1e-4."""
    for r in oracle_2k.views:
        np.testing.assert_allclose(r.wsum, 1.0 - r.T, rtol=0, atol=1e-12)
        assert r.T.min() >= 1e-4
        assert r.T.max() <= 1.0


# --------------------------------------------------------------------------
# masking and aggregation

def test_identical_features_reproduce_feature(scene_2k):
    """If every segment carries the same vector f, the normalised weighted
    average is f for every Gaussian with non-zero weight."""
    import dataclasses
    f = _unit_feats(1, scene_2k.dim, seed=9)[0]
    sc = dataclasses.replace(scene_2k, feats=np.tile(f, (scene_2k.feats.shape[0], 1)))
    r = oracle.lift(sc)
    nz = r.den > 0
    assert nz.sum() > 1000
    np.testing.assert_allclose(r.E[nz], np.broadcast_to(f.astype(np.float64), r.E[nz].shape),
                               rtol=0, atol=1e-12)
    assert np.all(r.E[~nz] == 0)


def test_symmetric_split_averages_features():
    """A centred, axis-aligned Gaussian over an image split at the principal
    point gets equal weight from both halves: E = (f_left + f_right) / 2."""
    ids = np.zeros((32, 32), np.int32)
    ids[:, 16:] = 1
    feats = _unit_feats(2, 8, seed=3)
    sc = _axis_scene([(3.0, [0.4, 0.2, 0.1], 0.7)], ids=ids, feats=feats)
    r = oracle.lift(sc)
    wl, wr = r.views[0].w
    assert wl == pytest.approx(wr, rel=1e-13)
    np.testing.assert_allclose(r.E[0], (feats[0].astype(np.float64) + feats[1]) / 2, atol=1e-13)


def test_background_pixels_occlude_but_do_not_count():
    """Pixels with id -1 are blended (they still occlude) but add nothing to
    the aggregation sums: with the left half as background only the right
    half's weight remains, and the back Gaussian is still attenuated there."""
    ids = np.full((32, 32), -1, np.int32)
    ids[:, 16:] = 0
    sc = _axis_scene([(4.0, [0.5, 0.4, 0.1], 0.8), (2.0, [0.15, 0.25, 0.1], 0.9)],
                     ids=ids, feats=_unit_feats(1, 4))
    full = _axis_scene([(4.0, [0.5, 0.4, 0.1], 0.8), (2.0, [0.15, 0.25, 0.1], 0.9)])
    rf = oracle.lift_view(full, 0)
    r = oracle.lift_view(sc, 0)
    right = (np.arange(1024) % 32) >= 16
    for g in (0, 1):
        assert r.w[r.g == g][0] == pytest.approx(_dense_w(rf, g, 1024)[right].sum(), rel=1e-12)


def test_embeddings_are_convex_combinations(oracle_2k):
    """E_k is a convex combination of unit vectors: |E_k| <= 1."""
    nz = oracle_2k.den > 0
    assert np.linalg.norm(oracle_2k.E[nz], axis=1).max() <= 1.0 + 1e-12


def test_gaussian_permutation_equivariance(scene_2k, oracle_2k):
    """Relabelling the Gaussians relabels the result and changes nothing else
    (given no depth ties among Gaussians, asserted here)."""
    import dataclasses
    for v in range(scene_2k.n_views):
        mv = oracle.mirror_view(scene_2k, v)
        z = mv.z32[mv.vis == 1]
        assert np.unique(z).size == z.size
    perm = np.random.default_rng(1).permutation(scene_2k.n)
    sc = dataclasses.replace(scene_2k, means=scene_2k.means[perm], scales=scene_2k.scales[perm],
                             quats=scene_2k.quats[perm], opacity=scene_2k.opacity[perm])
    r = oracle.lift(sc)
    inv = np.argsort(perm)
    assert np.array_equal(r.num[inv], oracle_2k.num)
    assert np.array_equal(r.den[inv], oracle_2k.den)


def test_brute_and_box_agree_bitwise(scene_2k, oracle_2k):
    """Boxes only prune Gaussians that cannot reach 1/255: the brute-force
    walk over every Gaussian gives the identical result."""
    rb = oracle.lift(scene_2k, mode="brute", pixels=True)
    assert np.array_equal(rb.num, oracle_2k.num)
    assert np.array_equal(rb.den, oracle_2k.den)
    for a, b in zip(rb.views, oracle_2k.views):
        assert np.array_equal(a.T, b.T)
        assert a.n_tests == b.n_tests and a.n_contrib == b.n_contrib


def test_depth_ties_break_by_gaussian_index():
    """Identical Gaussians have identical depth keys; the reference order
    visits the lower index first, so only it sees T = 1."""
    sc = _axis_scene([(3.0, [0.2, 0.2, 0.1], 0.6)] * 3)
    t, zb, g = oracle.sorted_keys(sc, 0, 16, 16)
    for tile in np.unique(t):
        assert list(g[t == tile]) == [0, 1, 2]
    r = oracle.lift_view(sc, 0)
    w = [_dense_w(r, k, 1024).sum() for k in range(3)]
    assert w[0] > w[1] > w[2] > 0


def test_sorted_keys_cover_boxes(scene_2k):
    """Every visible Gaussian appears in exactly the tiles its box touches,
    ordered by (tile, depth, index)."""
    for tw, th in [(16, 16), (8, 8), (16, 8)]:
        t, zb, g = oracle.sorted_keys(scene_2k, 1, tw, th)
        key = t.astype(np.int64) * 2 ** 32 + zb.astype(np.int64)
        assert np.all(np.diff(key) >= 0)
        ties = np.diff(key) == 0
        assert np.all(np.diff(g.astype(np.int64))[ties] > 0)
        mv = oracle.mirror_view(scene_2k, 1)
        b = mv.box[mv.vis == 1]
        exp = ((b[:, 1] // tw - b[:, 0] // tw + 1) * (b[:, 3] // th - b[:, 2] // th + 1)).sum()
        assert t.size == exp


# --------------------------------------------------------------------------
# rasterizer constants as options (the reading of the constants the paper
# leaves to the rasterizer: they are the library's options, and the oracle
# takes the same values)

def test_custom_alpha_bounds_and_dilation_closed_form():
    """With alpha_max = 0.6, alpha_min = 0.05 and 1.0 px^2 of dilation one
    Gaussian weighs w(p) = min(0.6, o exp(-q/2)) where that reaches 0.05,
    Sigma2 = diag(f^2 s^2 / z^2) + 1.0 I."""
    amax, amin, dil = F32(0.6), F32(0.05), F32(1.0)
    sc = _axis_scene([(3.0, [0.3, 0.15, 0.1], 0.8)])
    with oracle.constants(alpha_max=amax, alpha_min=amin, dilation=dil):
        r = oracle.lift_view(sc, 0, pixels=True)
        mu, cov, _, _ = oracle.project64_view(sc, 0)
    f, z = float(sc.cams[0]["fx"]), 3.0
    s = sc.scales[0].astype(np.float64)
    sxx, syy = f * f * s[0] ** 2 / z ** 2 + float(dil), f * f * s[1] ** 2 / z ** 2 + float(dil)
    np.testing.assert_allclose(cov[0], [sxx, 0.0, syy], rtol=1e-12, atol=1e-15)
    u, v = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    o = float(sc.opacity[0])
    a = np.minimum(float(amax), o * np.exp(-0.5 * ((u - 16.0) ** 2 / sxx + (v - 16.0) ** 2 / syy)))
    exp = np.where(a >= float(amin), a, 0.0).ravel()
    got = _dense_w(r, 0, 32 * 32)
    np.testing.assert_allclose(got, exp, rtol=1e-12, atol=0)
    assert (got == float(amax)).sum() > 4 and 20 < (got > 0).sum() < (exp.size - 50)
    # the defaults are restored afterwards (alpha above 0.6 is kept again)
    r0 = oracle.lift_view(sc, 0)
    assert _dense_w(r0, 0, 1024).max() > float(amax)


def test_custom_stop_is_exclusive():
    """t_min = 0.01 and alpha = 0.95: after one blend T = 0.05; the second
    would take T to 0.0025 < 0.01, so exactly one Gaussian blends."""
    gs = [(2.0 + 0.1 * k, [0.05, 0.05, 0.05], 0.95) for k in range(4)]
    sc = _axis_scene(gs, cx=16.5, cy=16.5)
    p = 16 * 32 + 16
    a = float(np.float32(0.95))
    with oracle.constants(t_min=F32(0.01)):
        r = oracle.lift_view(sc, 0, pixels=True)
    assert _dense_w(r, 0, 1024)[p] == pytest.approx(a, rel=1e-13)
    assert all(_dense_w(r, g, 1024)[p] == 0.0 for g in (1, 2, 3))
    assert r.T.ravel()[p] == pytest.approx(1 - a, rel=1e-12)


def test_custom_near_plane_and_guard():
    """near_z = 0.5 culls a Gaussian at depth 0.3 and keeps one at 0.8; with
    guard g a Gaussian beyond the clamp projects with the Jacobian at
    x/z = g tan(half FOV): Sigma2_xx = (f / z)^2 (sx^2 + t^2 sz^2) + 0.3."""
    cam = _cam(64, 48, 40.0)
    sc = make_custom_scene([[0, 0, 0.3], [0, 0, 0.8]], [[0.01] * 3] * 2, [[1, 0, 0, 0]] * 2,
                           [0.5, 0.5], [cam], [np.zeros((48, 64), np.int32)], _unit_feats(1, 4))
    with oracle.constants(near_z=F32(0.5)):
        mv = oracle.mirror_view(sc, 0)
    assert mv.vis[0] == 0 and mv.vis[1] == 1
    assert np.all(oracle.mirror_view(sc, 0).vis == 1)
    z, x = 2.0, 3.0                     # x/z = 1.5, beyond 1.3 * 32/40 and 1.1 * 32/40
    s = np.array([0.05, 0.04, 0.2], np.float32)
    sc2 = make_custom_scene([[x, 0, z]], [s], [[1, 0, 0, 0]], [0.5], [cam],
                            [np.zeros((48, 64), np.int32)], _unit_feats(1, 4))
    for g in (1.1, 1.3):
        with oracle.constants(guard=F32(g)):
            _, cov, _, _ = oracle.project64_view(sc2, 0)
        t = float(F32(g)) * 0.5 * 64 / 40.0
        sd = s.astype(np.float64)
        exp = (40.0 / z) ** 2 * (sd[0] ** 2 + t * t * sd[2] ** 2) + 0.3
        assert cov[0, 0] == pytest.approx(exp, rel=1e-12)


# --------------------------------------------------------------------------
# overlapping masks (a pixel may lie in several masks M_j: parameter masking
# gives its weight to each of them, and the aggregation sums over every mask
# and its pixels)

def test_disjoint_masks_reproduce_single_labels(scene_2k, oracle_2k):
    """A second label layer of -1 everywhere changes nothing, bit for bit."""
    import dataclasses
    ids2 = [np.stack([i, np.full_like(i, -1)], axis=-1) for i in scene_2k.ids]
    sc2 = dataclasses.replace(scene_2k, ids=ids2)
    for v in range(scene_2k.n_views):
        r2 = oracle.lift_view(sc2, v)
        r1 = oracle_2k.views[v]
        assert np.array_equal(r1.g, r2.g) and np.array_equal(r1.s, r2.s)
        assert np.array_equal(r1.w, r2.w) and np.array_equal(r1.u, r2.u)


def test_pixel_in_two_masks_adds_weight_to_both():
    """Per-pixel masks plus one large mask over the left half: every pixel's
    own mask keeps its single-label weight, and the large mask receives the
    sum of the weights of its pixels."""
    sc = _axis_scene([(3.0, [0.3, 0.15, 0.1], 0.8)])
    r1 = oracle.lift_view(sc, 0)
    big = np.full((32, 32), -1, np.int32)
    big[:, :16] = 32 * 32
    ids2 = np.stack([sc.ids[0], big], axis=-1)
    sc2 = make_custom_scene(sc.means, sc.scales, sc.quats, sc.opacity,
                            [dict(fx=float(sc.cams[0]["fx"]), fy=float(sc.cams[0]["fy"]),
                                  cx=float(sc.cams[0]["cx"]), cy=float(sc.cams[0]["cy"]),
                                  width=32, height=32)],
                            [ids2], _unit_feats(32 * 32 + 1, 4), nseg=[32 * 32 + 1])
    r2 = oracle.lift_view(sc2, 0)
    per_pixel = _dense_w(r1, 0, 32 * 32)
    got = np.zeros(32 * 32 + 1)
    got[r2.s[r2.g == 0]] = r2.w[r2.g == 0]
    np.testing.assert_array_equal(got[:32 * 32], per_pixel)
    left = (np.arange(32 * 32) % 32) < 16
    assert got[32 * 32] == pytest.approx(per_pixel[left].sum(), rel=1e-13)
    assert got[32 * 32] > 0


def test_two_full_masks_average_their_features():
    """Two masks that both cover the whole image: every Gaussian's weight goes
    to both in equal amounts, so E = (f1 + f2) / 2 exactly."""
    sc = _axis_scene([(3.0, [0.3, 0.15, 0.1], 0.8), (2.5, [0.1, 0.2, 0.1], 0.6)])
    ids2 = np.stack([np.zeros((32, 32), np.int32), np.ones((32, 32), np.int32)], axis=-1)
    f = _unit_feats(2, 8, seed=3)
    c = sc.cams[0]
    sc2 = make_custom_scene(sc.means, sc.scales, sc.quats, sc.opacity,
                            [dict(fx=float(c["fx"]), fy=float(c["fy"]), cx=float(c["cx"]),
                                  cy=float(c["cy"]), width=32, height=32)], [ids2], f, nseg=[2])
    ref = oracle.lift(sc2)
    want = (f[0].astype(np.float64) + f[1].astype(np.float64)) / 2
    for g in range(2):
        np.testing.assert_allclose(ref.E[g], want, rtol=0, atol=1e-15)


def test_kernel_weights_closed_form():
    """weight_mode = 1 (the paper's weight equation): every Gaussian the walk
    blends gets w = exp(-q/2), its kernel value, independent of opacity and of
    the Gaussians in front; the contributing set is the walk's (alpha >= 1/255,
    before the stop)."""
    sc = _axis_scene([(4.0, [0.5, 0.4, 0.1], 0.8), (2.0, [0.15, 0.25, 0.1], 0.9)])
    with oracle.constants(weight_mode=1.0):
        r = oracle.lift_view(sc, 0)
    u, v = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    for g in (0, 1):
        sxx, syy = _screen_diag(sc, g)
        kv = np.exp(-0.5 * ((u - 16.0) ** 2 / sxx + (v - 16.0) ** 2 / syy)).ravel()
        a = float(sc.opacity[g]) * kv
        exp = np.where(np.minimum(0.99, a) >= 1 / 255, kv, 0.0)
        np.testing.assert_allclose(_dense_w(r, g, 1024), exp, rtol=1e-12, atol=0)
    # the back Gaussian's kernel weight is not reduced by the front one
    assert _dense_w(r, 0, 1024).max() > 0.9


def test_kernel_weights_fp32_rewalk_within_bound():
    """The FP32 re-walk with kernel weights stays within the oracle's
    rounding and decision masses."""
    sc = make_scene_small()
    with oracle.constants(weight_mode=1.0):
        r64 = oracle.lift_view(sc, 0)
        r32 = oracle.lift_view(sc, 0, fp32=True)
    k64 = r64.g.astype(np.int64) << 32 | r64.s.astype(np.int64)
    k32 = r32.g.astype(np.int64) << 32 | r32.s.astype(np.int64)
    allk = np.union1d(k64, k32)
    W64, W32, B = np.zeros(allk.size), np.zeros(allk.size), np.full(allk.size, oracle.SUM_ABS)
    i64 = np.searchsorted(allk, k64)
    W64[i64] = r64.w
    B[i64] = oracle.weight_bound(r64.w, r64.u, r64.r)
    W32[np.searchsorted(allk, k32)] = r32.w
    assert np.all(np.abs(W32 - W64) <= B), (np.abs(W32 - W64) / B).max()


# --------------------------------------------------------------------------
# render-back (Method, the rendering equation with the lift's weights)

def test_render_two_gaussian_closed_form():
    """Two Gaussians on the optical axis: out = (w_f a_f + w_b a_b) /
    (w_f + w_b) with w_f = alpha_f, w_b = alpha_b (1 - alpha_f) (each where it
    reaches 1/255), 0 where neither blends."""
    sc = _axis_scene([(4.0, [0.5, 0.4, 0.1], 0.8), (2.0, [0.15, 0.25, 0.1], 0.9)])
    attr = np.array([[1.0, -2.0, 0.5], [3.0, 0.25, -1.0]], np.float32)
    rr = oracle.render_view(sc, 0, attr)
    u, v = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    ab = _alpha(float(sc.opacity[0]), u - 16.0, v - 16.0, *_screen_diag(sc, 0))
    af = _alpha(float(sc.opacity[1]), u - 16.0, v - 16.0, *_screen_diag(sc, 1))
    af = np.where(af >= 1 / 255, af, 0.0)
    wb = np.where(ab >= 1 / 255, ab * (1 - af), 0.0)
    ws = af + wb
    a = attr.astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        want = np.where(ws[..., None] > 0,
                        (af[..., None] * a[1] + wb[..., None] * a[0]) / ws[..., None], 0.0)
    np.testing.assert_allclose(rr.wsum, ws, rtol=1e-12, atol=0)
    np.testing.assert_allclose(rr.out, want, rtol=1e-12, atol=1e-15)
    assert (ws == 0).any() and (af > 0.5).any() and (wb > 0).sum() > 100


def _random_small_scene(seed, n=300, w=48, h=40):
    rng = np.random.default_rng(seed)
    means = np.c_[rng.uniform(-1.2, 1.2, n), rng.uniform(-1.0, 1.0, n), rng.uniform(2.0, 5.0, n)]
    scales = rng.uniform(0.03, 0.25, (n, 3))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    ops = rng.uniform(0.05, 0.99, n)
    ids = _pixel_ids(w, h)
    return make_custom_scene(means, scales, q, ops, [_cam(w, h, 40.0)], [ids],
                             _unit_feats(w * h, 4, seed))


@pytest.mark.parametrize("kernel", [False, True])
def test_render_is_the_lift_weights_per_pixel(kernel):
    """With one segment per pixel the lift's W_v[g, p] is the weight of
    Gaussian g at pixel p, so the render must equal sum_g W[g, p] a_g /
    sum_g W[g, p] at every pixel, with wsum = sum_g W[g, p] (alpha T weights
    and kernel weights); constant attributes render as that constant wherever
    something blends."""
    sc = _random_small_scene(11)
    n, npix = sc.n, 48 * 40
    attr = np.random.default_rng(5).standard_normal((n, 5)).astype(np.float32)
    attr[:, 4] = 0.625
    with oracle.constants(weight_mode=1.0 if kernel else 0.0):
        r = oracle.lift_view(sc, 0)
        rr = oracle.render_view(sc, 0, attr)
    Wd = np.zeros((npix, n))
    Wd[r.s, r.g] = r.w
    ws = Wd.sum(axis=1)
    num = Wd @ attr.astype(np.float64)
    want = np.where(ws[:, None] > 0, num / np.where(ws > 0, ws, 1.0)[:, None], 0.0)
    np.testing.assert_allclose(rr.wsum.ravel(), ws, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(rr.out.reshape(npix, 5), want, rtol=1e-10, atol=1e-12)
    lit = ws > 0
    assert lit.mean() > 0.5 and (~lit).any()
    np.testing.assert_allclose(rr.out.reshape(npix, 5)[lit, 4], 0.625, rtol=1e-13)
    assert np.all(rr.nb.ravel()[lit] >= 1) and np.all(rr.bw >= 0)


def test_render_bound_shape():
    """The render bound is finite where a pixel's certain weight dominates,
    infinite where nothing blends, and grows with the weights' deviation."""
    sc = _random_small_scene(12)
    attr = np.random.default_rng(6).standard_normal((sc.n, 3)).astype(np.float32)
    rr = oracle.render_view(sc, 0, attr)
    amax = np.abs(attr).max(axis=0)
    b = oracle.render_bound(rr, amax)
    assert np.all(np.isinf(b[rr.wsum == 0]))
    lit = rr.wsum > 1e-3
    assert np.all(np.isfinite(b[lit])) and np.median(b[lit] / amax) < 1e-4
    rr2 = oracle.RenderResult(rr.out, rr.wsum, rr.bw * 10 + 1e-9, rr.nb)
    assert np.all(oracle.render_bound(rr2, amax)[lit] > b[lit])


def make_scene_small():
    from synthetic import make_scene
    return make_scene("plain_bf16_200k", n=20000, views=dict(n=1))
