"""Pins for the oracle's FP32 error model (rounding mass r, decision mass U).

The parity bars of the GPU tests are |W_gpu - W_oracle| <= r + U (plus the
summation of the per-pixel weights), with r and U derived by the oracle from
an operation count of an FP32 evaluation (see the header of
``oracle/slag_oracle.c``).  These tests check the derivation against an
actual FP32 evaluation done on the CPU -- the oracle's FP32 re-walk of the
same per-pixel lists, which expands the exponent about the 8x8 block centre
like a tile rasterizer -- and check that U is zero away from every threshold
and non-zero next to one.

Paper: Method, "Semantic Embedding" (the rasterizer's per-pixel weights of
the contributing Gaussians, and the aggregation sums over each mask).
"""
import math

import numpy as np
import pytest

import oracle
from conftest import make_custom_scene
from synthetic import make_scene


def _compare(sc, v):
    r64 = oracle.lift_view(sc, v)
    r32 = oracle.lift_view(sc, v, fp32=True)
    k64 = r64.g.astype(np.int64) << 32 | r64.s.astype(np.int64)
    k32 = r32.g.astype(np.int64) << 32 | r32.s.astype(np.int64)
    allk = np.union1d(k64, k32)
    W64, W32, B, U = (np.zeros(allk.size) for _ in range(4))
    i64 = np.searchsorted(allk, k64)
    W64[i64] = r64.w
    U[i64] = r64.u
    B[:] = oracle.SUM_ABS
    B[i64] = oracle.weight_bound(r64.w, r64.u, r64.r)
    W32[np.searchsorted(allk, k32)] = r32.w
    err = np.abs(W32 - W64)
    return err, B, U, W64, W32, r64


@pytest.mark.parametrize("case", ["plain_fp32_2k", "plain_bf16_200k[2 views]", "hires_1280x960"])
def test_fp32_rewalk_stays_within_the_error_bound(case):
    """Every triple of an FP32 walk lies within its bound r + U (+ summation)
    of the FP64 walk, and triples with U = 0 match in membership exactly.  The
    high-resolution case stresses the screen-mean rounding (means far from
    the origin)."""
    if case == "plain_fp32_2k":
        sc, views = make_scene("plain_fp32_2k"), range(4)
    elif case.startswith("plain_bf16_200k"):
        sc, views = make_scene("plain_bf16_200k", views=dict(n=2)), range(2)
    else:
        sc = make_scene("uneven_1m", n=60000, views=dict(n=1, res_list=[(1280, 960)]))
        views = range(1)
    worst = worst_strict = 0.0
    for v in views:
        err, B, U, W64, W32, r64 = _compare(sc, v)
        ratio = err / B
        assert ratio.max() <= 1.0, (case, v, ratio.max())
        strict = U == 0
        assert np.array_equal(W64[strict] > 0, W32[strict] > 0)
        worst = max(worst, float(ratio.max()))
        worst_strict = max(worst_strict, float(ratio[strict].max()))
    # the bound is not vacuous: the rounding part is a few times the error seen
    assert worst_strict > 1e-3
    print(f"{case}: max error / bound {worst:.3g} (U = 0 triples: {worst_strict:.3g})")


def test_error_bound_is_tight_enough_to_matter():
    """The rounding mass is a small relative bound (not a blanket tolerance):
    on the 200k-scene recipe its median is below 2e-4 of the weight and the
    decision mass touches only a few percent of the triples."""
    sc = make_scene("plain_bf16_200k", views=dict(n=1))
    r = oracle.lift_view(sc, 0)
    pos = r.w > 0
    rel = r.r[pos] / r.w[pos]
    assert np.median(rel) < 2e-4 and rel.max() < 5e-3
    assert np.mean(r.u > 0) < 0.05


def _one_gaussian(o, cx=32.0, cy=32.0):
    """An axis-aligned Gaussian at depth 3 on the axis, per-pixel segments."""
    cam = dict(fx=51.2, fy=51.2, cx=cx, cy=cy, R=np.eye(3), t=np.zeros(3), width=64, height=64)
    ids = np.arange(64 * 64, dtype=np.int32).reshape(64, 64)
    f = np.random.default_rng(0).standard_normal((64 * 64, 4)).astype(np.float32)
    return make_custom_scene([0, 0, 3.0], [0.12, 0.12, 0.1], [1, 0, 0, 0], [o], [cam], [ids], f)


def test_decision_mass_is_zero_away_from_thresholds_and_set_next_to_one():
    """U > 0 exactly where a decision lies inside its error band.  With the
    opacity chosen so that alpha at one pixel centre is 1/255 (1 + 2e-7), well
    inside the band of an FP32 evaluation, that pixel's triple carries U > 0;
    every pixel whose alpha is farther than 1e-4 (relative) from 1/255 has
    U = 0; and a single Gaussian never approaches the stop threshold."""
    base = _one_gaussian(0.5)
    mu, cov, con, _ = oracle.project64_view(base, 0)
    # pixel centre (38.5, 32.5), 6.5 px right of the mean
    dx, dy = 38.5 - mu[0, 0], 32.5 - mu[0, 1]
    q = con[0, 0] * dx * dx + 2 * con[0, 1] * dx * dy + con[0, 2] * dy * dy
    o = np.float32(math.exp(0.5 * q) / 255.0 * (1.0 + 2e-7))
    assert 0.1 < o < 1.0
    sc = _one_gaussian(float(o))
    r = oracle.lift_view(sc, 0, pixels=True)
    yy, xx = np.divmod(r.s, 64)
    px, py = xx + 0.5, yy + 0.5
    ddx, ddy = px - mu[0, 0], py - mu[0, 1]
    a = float(sc.opacity[0]) * np.exp(-0.5 * (con[0, 0] * ddx ** 2 + 2 * con[0, 1] * ddx * ddy +
                                              con[0, 2] * ddy ** 2))
    planted = (xx == 38) & (yy == 32)
    assert planted.sum() == 1 and abs(a[planted][0] * 255 - 1) < 1e-6
    assert r.u[planted][0] > 0
    far = np.abs(a * 255 - 1) > 1e-4
    assert far.sum() > 50 and np.all(r.u[far] == 0)
    assert np.all(r.r[r.w > 0] > 0)
    # moving the opacity well away from the threshold clears the mass
    r2 = oracle.lift_view(_one_gaussian(float(o) * 1.01), 0)
    assert np.all(r2.u == 0)


def test_transmittance_bound_covers_the_fp32_walk(oracle_2k, scene_2k):
    """The final transmittance of the FP32 walk lies within rho of the FP64
    one at every pixel with no decision in its band."""
    for v in range(scene_2k.n_views):
        r32 = oracle.lift_view(scene_2k, v, pixels=True, fp32=True)
        r64 = oracle_2k.views[v]
        ok = r64.rho >= 0
        assert ok.mean() > 0.99
        err = np.abs(r32.T[ok] - r64.T[ok])
        assert np.all(err <= r64.rho[ok] * r64.T[ok] + 2.0 ** -24), (err / r64.T[ok]).max()


@pytest.mark.parametrize("case", ["plain_fp32_2k", "plain_bf16_200k[2 views]"])
def test_embedding_bound_covers_the_fp32_walk(case):
    """Embeddings contracted from the FP32 re-walk's weights stay within the
    propagated embedding bound of the FP64 lift (the aggregation equation
    perturbed by the weight errors), Gaussian by Gaussian."""
    if case == "plain_fp32_2k":
        sc = make_scene("plain_fp32_2k")
    else:
        sc = make_scene("plain_bf16_200k", views=dict(n=2))
    views = list(range(sc.n_views))
    ref = oracle.lift(sc)
    r32 = [oracle.lift_view(sc, v, fp32=True) for v in views]
    W32 = oracle.weight_matrix(sc, views, r32)
    F = sc.feats_f64()
    den32 = np.asarray(W32.sum(axis=1)).ravel()
    num32 = np.asarray(W32 @ F)
    fmax = float(np.linalg.norm(F, axis=1).max())
    bound, vanish = oracle.embedding_bound(ref, fmax, sc.n_views,
                                           bf16_split=sc.feat_dtype == "bf16")
    ok = (ref.den > 0) & ~vanish & (den32 > 0)
    E32 = num32[ok] / den32[ok, None]
    err = np.linalg.norm(E32 - ref.E[ok], axis=1)
    assert np.all(err <= bound[ok]), (err / bound[ok]).max()
    assert ok.sum() > 0.9 * (ref.den > 0).sum()
    print(f"{case}: max error / bound {(err / bound[ok]).max():.3g}")
