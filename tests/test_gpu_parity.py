"""GPU parity: the HIP lift (through the C ABI) against the FP64 CPU oracle.

Bars (see the oracle's header for the decision-margin mass U):
  * tile lists (tile, FP32 depth bits, Gaussian) bit-exact with the oracle's
    FP32 decision path;
  * per-view weights W_v[g, s]: |W_gpu - W_orc| <= 1e-3 (W_orc + U) + U + 1e-9,
    and exact membership of every (view, Gaussian, segment) triple with U = 0.
    The relative part: the kernel evaluates alpha from the FP32 conic; a
    relative conic error delta moves alpha by about q delta / 2, and q reaches
    2 ln(255 o) ~ 11 at the 1/255 cut, while T carries the errors of earlier
    alphas, so single weights can be off by a few 1e-4 relative (2.4e-4 seen
    on a 1280x960 view of the 1M-Gaussian scene); the flipped-decision mass U
    carries the same relative error;
  * embeddings: cosine >= 0.9999 for every Gaussian with non-zero weight
    (Gaussians whose weight is more than 0.5% decision-margin mass are
    reported, not compared), zero rows exactly where the oracle's are zero.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from synthetic import make_scene

pytestmark = pytest.mark.gpu

RTOL_W = 1e-3
COS_MIN = 0.9999


def _say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


def _lifter(scene, flags=0, max_views=0):
    import paper_2505_08124_amd as slag
    L = slag.Lifter(0, None, max_views, flags | slag.SLAG_FLAG_KEEP_DEBUG)
    L.set_scene(scene)
    return L


def _gpu_triples(L, v):
    g, s, w = L.weights(v)
    key = g.astype(np.int64) * (1 << 32) + s.astype(np.int64)
    uk, inv = np.unique(key, return_inverse=True)
    ws = np.zeros(uk.size)
    np.add.at(ws, inv, w.astype(np.float64))
    return uk, ws


def check_view_weights(L, scene, v, ores):
    """Compare one view's W with the oracle's triples."""
    gk, gw = _gpu_triples(L, v)
    ok = ores.g.astype(np.int64) * (1 << 32) + ores.s.astype(np.int64)
    allk = np.union1d(gk, ok)
    Wg = np.zeros(allk.size)
    Wo = np.zeros(allk.size)
    U = np.zeros(allk.size)
    Wg[np.searchsorted(allk, gk)] = gw
    io = np.searchsorted(allk, ok)
    Wo[io] = ores.w
    U[io] = ores.u
    err = np.abs(Wg - Wo)
    bad = err > RTOL_W * (Wo + U) + U + 1e-9
    assert not bad.any(), (
        f"view {v}: {bad.sum()} weight mismatches, e.g. key {allk[bad][:5]} gpu {Wg[bad][:5]} "
        f"oracle {Wo[bad][:5]} U {U[bad][:5]}")
    strict = U == 0
    assert np.array_equal(Wg[strict] > 0, Wo[strict] > 0)
    return int(((Wg > 0) != (Wo > 0)).sum()), int((U > 0).sum())


def check_embeddings(E, den, ref):
    nz = ref.den > 0
    assert np.array_equal(den > 0, nz) or np.all(ref.U[(den > 0) != nz] > 0)
    # the denominator is a sum of W entries: same bar as the weights
    err = np.abs(den[nz].astype(np.float64) - ref.den[nz])
    assert np.all(err <= RTOL_W * (ref.den[nz] + ref.U[nz]) + ref.U[nz] + 1e-9), (err / ref.den[nz]).max()
    margin = ref.U[nz] / ref.den[nz]
    Eg = E[nz].astype(np.float64)
    Eo = ref.E[nz]
    cos = np.sum(Eg * Eo, 1) / (np.linalg.norm(Eg, axis=1) * np.linalg.norm(Eo, axis=1) + 1e-300)
    comp = margin <= 5e-3
    assert cos[comp].min() >= COS_MIN, (cos[comp].min(), np.argmin(cos[comp]))
    assert np.all(E[~nz] == 0)
    return float(cos[comp].min()), float(np.abs(Eg - Eo).max())


def check_tile_lists(L, scene, v):
    t, z, g = L.tile_lists(v)
    rt, rz, rg = oracle.sorted_keys(scene, v, 16, 16)
    assert t.size == rt.size, (t.size, rt.size)
    assert np.array_equal(t.astype(np.int64), rt)
    assert np.array_equal(z, rz)
    assert np.array_equal(g.astype(np.int64), rg.astype(np.int64))


# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def lift_2k(scene_2k):
    import paper_2505_08124_amd as slag
    _say("plain_fp32_2k: lift (count mode)")
    L = _lifter(scene_2k, flags=slag.SLAG_FLAG_COUNT)
    L.lift()
    E, den = L.embeddings()
    return L, E, den


def test_tile_lists_bit_exact_2k(scene_2k, lift_2k):
    L, _, _ = lift_2k
    for v in range(scene_2k.n_views):
        _say("tile lists view", v)
        check_tile_lists(L, scene_2k, v)


def test_weights_match_oracle_2k(scene_2k, oracle_2k, lift_2k):
    L, _, _ = lift_2k
    for v in range(scene_2k.n_views):
        _say("weights view", v)
        flips, nunc = check_view_weights(L, scene_2k, v, oracle_2k.views[v])
        _say(f"  membership flips {flips}, triples with margin mass {nunc}")


def test_embeddings_match_oracle_2k(oracle_2k, lift_2k):
    _, E, den = lift_2k
    cmin, emax = check_embeddings(E, den, oracle_2k)
    _say(f"min cosine {cmin:.9f}, max abs err {emax:.3g}")


def test_counts_match_oracle_2k(oracle_2k, lift_2k):
    L, _, _ = lift_2k
    st = L.stats()
    unc = sum(r.n_uncertain for r in oracle_2k.views)
    assert abs(st["n_contrib"] - oracle_2k.n_contrib) <= unc
    assert abs(st["n_tests"] - oracle_2k.n_tests) <= unc + st["n_contrib"] // 1000
    assert st["n_tile_tests"] >= st["n_tests"]


def test_repeat_bitwise_and_batching(scene_2k, lift_2k):
    """Two lifts are bitwise equal (no float atomics).  One view per launch
    gives bitwise-equal weight sums (same order) and embeddings equal to FP32
    rounding (the matrix-core chunks group the products differently)."""
    L, E, den = lift_2k
    L.lift()
    E2, den2 = L.embeddings()
    assert np.array_equal(E, E2) and np.array_equal(den, den2)
    _say("one view per launch")
    L1 = _lifter(scene_2k, max_views=1)
    L1.lift()
    E3, den3 = L1.embeddings()
    assert np.array_equal(den, den3)
    np.testing.assert_allclose(E3, E, rtol=1e-5, atol=1e-6)


def test_permutation_equivariance_gpu(scene_2k, lift_2k):
    _, E, den = lift_2k
    perm = np.random.default_rng(1).permutation(scene_2k.n)
    sc = dataclasses.replace(scene_2k, means=scene_2k.means[perm], scales=scene_2k.scales[perm],
                             quats=scene_2k.quats[perm], opacity=scene_2k.opacity[perm])
    L = _lifter(sc)
    L.lift()
    Ep, denp = L.embeddings()
    inv = np.argsort(perm)
    assert np.array_equal(Ep[inv], E) and np.array_equal(denp[inv], den)


def _other_gpu_work():
    import torch
    x = torch.randn(1 << 20, device="cuda")
    float((x * x).sum().item())
    torch.cuda.synchronize()


def test_graph_replay_matches_eager(scene_2k, lift_2k):
    """With graph replay the first lift runs eagerly and captures; every
    later replay (with unrelated GPU work and synchronisations in between)
    gives the eager result bitwise; changing an input re-runs eagerly."""
    import paper_2505_08124_amd as slag
    _, E_ref, den_ref = lift_2k
    L = _lifter(scene_2k, flags=slag.SLAG_FLAG_GRAPH | slag.SLAG_FLAG_PROFILE)
    L.lift()
    E0, den0 = L.embeddings()
    assert np.array_equal(E0, E_ref) and np.array_equal(den0, den_ref)
    for i in range(3):
        _other_gpu_work()
        L.lift()
        E, den = L.embeddings()
        _say("replay", i, "ms", round(L.stats()["ms_total"], 4))
        assert np.array_equal(E, E0) and np.array_equal(den, den0)
    check_tile_lists(L, scene_2k, 1)
    # new features: the next lift is eager again and matches a fresh context
    rng = np.random.default_rng(9)
    F2 = rng.standard_normal(scene_2k.feats.shape).astype(np.float32)
    slag.slag_set_features(L.ctx, F2, slag.SLAG_F32)
    L.lift()
    E1, _ = L.embeddings()
    L.lift()
    E2, _ = L.embeddings()
    sc2 = dataclasses.replace(scene_2k, feats=F2)
    L2 = _lifter(sc2)
    L2.lift()
    E3, _ = L2.embeddings()
    assert np.array_equal(E1, E3) and np.array_equal(E2, E3)


def _ragged_scene():
    """Ragged image sizes (partial tiles), background, a view with per-pixel
    noise ids (many segments per tile: several compositing passes)."""
    sc = make_scene("uneven_1m", n=6000,
                    views=dict(n=3, res_list=[(100, 75), (61, 47), (130, 90)]),
                    segments=dict(lo=5, hi=30))
    ids = [i.copy() for i in sc.ids]
    rng = np.random.default_rng(4)
    ids[0][rng.random(ids[0].shape) < 0.15] = -1
    k = int(sc.nseg[1])
    ids[1] = rng.integers(-1, k, size=ids[1].shape).astype(np.int32)
    return dataclasses.replace(sc, ids=ids)


def test_ragged_views_and_many_segments():
    import paper_2505_08124_amd as slag
    sc = _ragged_scene()
    _say("ragged: oracle")
    ref = oracle.lift(sc)
    _say("ragged: gpu")
    L = _lifter(sc, flags=slag.SLAG_FLAG_GRAPH)
    L.lift()
    E, den = L.embeddings()
    _other_gpu_work()
    L.lift()
    Er, denr = L.embeddings()
    assert np.array_equal(E, Er) and np.array_equal(den, denr)
    for v in range(sc.n_views):
        check_tile_lists(L, sc, v)
        check_view_weights(L, sc, v, ref.views[v])
    check_embeddings(E, den, ref)


def test_autotune_is_bitwise_neutral():
    """Tuning runs every compositing variant per image size and keeps the
    fastest; results equal the untuned lift bitwise, before and after."""
    import paper_2505_08124_amd as slag
    sc = _ragged_scene()
    L0 = _lifter(sc)
    L0.lift()
    E0, den0 = L0.embeddings()
    L = _lifter(sc, flags=slag.SLAG_FLAG_AUTOTUNE)
    L.lift()
    E1, den1 = L.embeddings()
    L.lift()
    E2, den2 = L.embeddings()
    tun = slag.slag_get_tuning(L.ctx)
    _say("tuning", tun)
    assert len(tun) == 3 and all(len(t["ms"]) == 4 for t in tun)
    assert np.array_equal(E0, E1) and np.array_equal(E0, E2)
    assert np.array_equal(den0, den1) and np.array_equal(den0, den2)


def test_uneven_resolutions_one_launch():
    sc = make_scene("uneven_1m", n=40000, views=dict(n=6))
    _say("uneven: oracle")
    ref = oracle.lift(sc)
    _say("uneven: gpu")
    L = _lifter(sc)
    L.lift()
    E, den = L.embeddings()
    for v in range(sc.n_views):
        check_tile_lists(L, sc, v)
        check_view_weights(L, sc, v, ref.views[v])
    check_embeddings(E, den, ref)


def test_empty_and_degenerate():
    import paper_2505_08124_amd as slag
    sc = make_scene("plain_fp32_2k", n=50)
    # no Gaussians
    e = dataclasses.replace(sc, means=sc.means[:0], scales=sc.scales[:0], quats=sc.quats[:0],
                            opacity=sc.opacity[:0])
    L = _lifter(e)
    L.lift()
    E, den = L.embeddings()
    assert E.shape == (0, sc.dim)
    # every pixel background: all weights zero, E = 0
    bg = dataclasses.replace(sc, ids=[np.full_like(i, -1) for i in sc.ids])
    L = _lifter(bg)
    L.lift()
    E, den = L.embeddings()
    assert np.all(E == 0) and np.all(den == 0)
    # everything behind the cameras
    far = dataclasses.replace(sc, means=(sc.means * 0 + np.float32([0, 0, 100])).astype(np.float32))
    L = _lifter(far)
    L.lift()
    E, den = L.embeddings()
    ref = oracle.lift(far)
    assert np.array_equal(den > 0, ref.den > 0)
    # invalid input is rejected at upload
    with pytest.raises(slag.SlagError):
        L2 = slag.Lifter(0)
        L2.set_scene(dataclasses.replace(sc, ids=[i + 100 for i in sc.ids]))


def _tie_scene():
    """Cameras looking along +z (camera depth = world z, exactly): half the
    Gaussians on one plane (one long run of equal depth per view), a block on
    three repeated depths, 100 pairs of equal depth (short runs), the rest
    distinct; stored in a shuffled order."""
    from conftest import make_custom_scene
    rng = np.random.default_rng(77)
    n = 3000
    z = rng.uniform(3.0, 9.0, n).astype(np.float32)
    z[: n // 2] = 4.0                                    # a plane facing the cameras
    z[n // 2: n // 2 + 300] = rng.choice(np.float32([5.0, 5.5, 6.25]), 300)
    short = rng.choice(np.arange(n // 2 + 300, n), 200, replace=False)
    z[short[:100]] = z[short[100:]]                      # pairs of equal depth
    xy = rng.uniform(-1.0, 1.0, (n, 2)).astype(np.float32) * z[:, None] * np.float32([0.6, 0.45])
    means = np.concatenate([xy, z[:, None]], 1)
    perm = rng.permutation(n)                            # the caller's order
    means = means[perm]
    scales = rng.uniform(0.01, 0.06, (n, 3)).astype(np.float32)
    quats = rng.normal(size=(n, 4)).astype(np.float32)
    opacity = rng.uniform(0.2, 0.95, n).astype(np.float32)
    W, H = 160, 120
    cams = [dict(fx=120.0, fy=120.0, cx=80.0, cy=60.0, t=[0.0, 0.0, 0.0], width=W, height=H),
            dict(fx=120.0, fy=120.0, cx=80.0, cy=60.0, t=[0.25, 0.0, 0.5], width=W, height=H)]
    yy, xx = np.mgrid[0:H, 0:W]
    ids = [((xx // 40) + 4 * (yy // 60)).astype(np.int32), ((xx // 32) % 5).astype(np.int32)]
    feats = rng.normal(size=(8 + 5, 64)).astype(np.float32)
    sc = make_custom_scene(means, scales, quats, opacity, cams, ids, feats, name="depth_ties")
    return sc


def test_depth_ties_follow_gaussian_index():
    """Exact depth ties, in runs of every length, are broken by the caller's
    Gaussian index (the library stores Gaussians in Morton order, so its own
    order differs).  Tile lists must equal the oracle's bit for bit."""
    sc = _tie_scene()
    L = _lifter(sc)
    L.lift()
    for v in range(2):
        _say("depth ties: tile lists view", v)
        check_tile_lists(L, sc, v)
    E, den = L.embeddings()
    ref = oracle.lift(sc)
    cmin, _ = check_embeddings(E, den, ref)
    _say(f"depth ties: min cosine {cmin:.9f}")
    # graph replay (the captured lift includes the long-run path) gives the
    # eager result bitwise, with unrelated GPU work between replays
    import paper_2505_08124_amd as slag
    Lg = _lifter(sc, flags=slag.SLAG_FLAG_GRAPH)
    for i in range(3):
        Lg.lift()
        Eg, deng = Lg.embeddings()
        assert np.array_equal(Eg, E) and np.array_equal(deng, den), i
        _other_gpu_work()
    check_tile_lists(Lg, sc, 1)


# --------------------------------------------------------------- full sizes

def test_full_size_plain_bf16_200k():
    """The benchmark's scene at full size, all 100 views in one launch (the
    benchmark's configuration): every view's tile lists and W_v for sampled
    views against the oracle, and the embeddings of every Gaussian against
    the full FP64 oracle lift."""
    import paper_2505_08124_amd as slag
    sc = make_scene("plain_bf16_200k")
    _say("200k: gpu lift as timed (graph replay, no debug exports)")
    with slag.Lifter(0, flags=slag.SLAG_FLAG_GRAPH) as L0:
        L0.set_scene(sc, device_tensors=True)
        L0.lift()
        Ee, dene = L0.embeddings()
        L0.lift()
        E0, den0 = L0.embeddings()
    assert np.array_equal(Ee, E0) and np.array_equal(dene, den0)
    _say("200k: gpu lift with debug exports")
    L = _lifter(sc)
    L.lift()
    E, den = L.embeddings()
    assert np.array_equal(E, E0) and np.array_equal(den, den0)
    _say("200k: oracle lift of all views")
    ref = oracle.lift(sc)
    for v in (0, 37, 99):
        _say("200k: view", v)
        check_tile_lists(L, sc, v)
        check_view_weights(L, sc, v, ref.views[v])
    cmin, emax = check_embeddings(E, den, ref)
    _say(f"200k: min cosine {cmin:.9f}, max abs err {emax:.3g}")
    L.close()


def test_full_size_uneven_1m_sampled_views():
    """1M Gaussians, 300 views of three resolutions in one launch: tile lists
    and W_v of one sampled view per resolution against the oracle; splitting
    the views over two launches leaves den bitwise unchanged."""
    sc = make_scene("uneven_1m")
    res = [(int(c["width"]), int(c["height"])) for c in sc.cams]
    picks = [res.index(r) for r in [(320, 240), (640, 480), (1280, 960)]]
    _say("1m: gpu lift, one launch")
    L = _lifter(sc)
    L.lift()
    E, den = L.embeddings()
    st = L.stats()
    _say(f"1m: pairs {st['n_visible_pairs']}, intersections {st['n_intersections']}")
    assert st["n_batches"] == 1
    for v in picks:
        _say("1m: view", v, res[v])
        check_tile_lists(L, sc, v)
        check_view_weights(L, sc, v, oracle.lift_view(sc, v))
    L.close()
    nz = den > 0
    # convex combinations of the feature rows as uploaded (BF16 rows are unit
    # norm only to within 2^-9)
    fmax = np.linalg.norm(sc.feats_f64(), axis=1).max()
    assert np.all(np.linalg.norm(E[nz], axis=1) <= fmax * (1 + 1e-5))
    assert np.all(E[~nz] == 0)
    _say("1m: two launches of 150 views")
    L2 = _lifter(sc, max_views=150)
    L2.lift()
    E2, den2 = L2.embeddings()
    assert L2.stats()["n_batches"] == 2
    assert np.array_equal(den, den2)
    np.testing.assert_allclose(E2, E, rtol=1e-5, atol=1e-6)
    L2.close()
