"""GPU parity: the HIP lift (through the C ABI) against the FP64 CPU oracle.

Bars, all derived by the oracle from an operation count of the FP32
evaluation (``oracle/slag_oracle.c``, pinned against an FP32 re-walk on the
CPU in ``tests/test_oracle_error_model.py``), none fitted to observed errors:
  * tile lists (tile, FP32 depth bits, Gaussian) bit-exact with the oracle's
    FP32 decision path;
  * per-view weights W_v[g, s]: |W_gpu - W_orc| <= r + U + summation, with r
    the rounding mass and U the decision mass of the triple; exact membership
    of every (view, Gaussian, segment) triple with U = 0;
  * den within the sum of its triples' bounds plus the per-view FP32 sums;
  * embeddings: ||E_gpu - E_orc|| <= the propagated bound
    (oracle.embedding_bound) for every Gaussian, and cosine >= 0.9999 for
    every Gaussian whose bound guarantees it; a Gaussian whose bound does not
    (its weight is mostly decisions inside their FP32 band: alpha within
    rounding of 1/255 over most of its footprint) may fall below 0.9999 only
    within its bound, and such Gaussians are capped at 0.1 % of those with
    weight; both counts, and the weight share of the uncertified ones, are
    recorded; zero rows exactly where the oracle's den is 0 and no decision
    could make it positive.
Each check appends one JSON line of statistics to $SLAG_PARITY_LOG when set.
"""
import dataclasses
import json
import os
import sys

import numpy as np
import pytest

import oracle
from synthetic import make_scene

pytestmark = pytest.mark.gpu

COS_MIN = 0.9999
U32 = 2.0 ** -24
MAX_UNCOMPARED = 1e-3      # fraction of Gaussians below COS_MIN (each uncertified by its bound)


def _say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


def _record(**kv):
    path = os.environ.get("SLAG_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(kv) + "\n")


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


def check_view_weights(L, scene, v, ores, tag=""):
    """Compare one view's W with the oracle's triples."""
    gk, gw = _gpu_triples(L, v)
    ok = ores.g.astype(np.int64) * (1 << 32) + ores.s.astype(np.int64)
    allk = np.union1d(gk, ok)
    Wg = np.zeros(allk.size)
    Wo = np.zeros(allk.size)
    U = np.zeros(allk.size)
    bar = np.full(allk.size, oracle.SUM_ABS)
    Wg[np.searchsorted(allk, gk)] = gw
    io = np.searchsorted(allk, ok)
    Wo[io] = ores.w
    U[io] = ores.u
    bar[io] = oracle.weight_bound(ores.w, ores.u, ores.r)
    err = np.abs(Wg - Wo)
    bad = err > bar
    assert not bad.any(), (
        f"view {v}: {bad.sum()} weight mismatches, e.g. key {allk[bad][:5]} gpu {Wg[bad][:5]} "
        f"oracle {Wo[bad][:5]} bar {bar[bad][:5]} U {U[bad][:5]}")
    strict = U == 0
    assert np.array_equal(Wg[strict] > 0, Wo[strict] > 0)
    pos = strict & (Wo > 0)
    rel = err[pos] / Wo[pos]
    st = dict(check="weights", case=tag, view=int(v), triples=int(allk.size),
              frac_decision_mass=float(np.mean(U > 0)), max_err_over_bar=float((err / bar).max()),
              max_rel_err=float(rel.max()) if rel.size else 0.0,
              median_rel_bar=float(np.median(bar[pos] / Wo[pos])) if rel.size else 0.0,
              membership_flips=int(((Wg > 0) != (Wo > 0)).sum()))
    _record(**st)
    return st["membership_flips"], int((U > 0).sum())


def check_embeddings(E, den, ref, scene, tag=""):
    """E and den against the oracle's lift, with the propagated bounds."""
    fmax = float(np.linalg.norm(scene.feats_f64(), axis=1).max()) if scene.feats.size else 1.0
    bound, vanish = oracle.embedding_bound(ref, fmax, scene.n_views,
                                           bf16_split=scene.feat_dtype == "bf16")
    nz = ref.den > 0
    gz = den > 0
    # zero rows: exactly the oracle's, unless a decision in band could change that
    differ = gz != nz
    assert np.all(vanish[differ] | ((ref.den[differ] == 0) & (ref.U[differ] > 0))), differ.sum()
    assert np.all(E[~gz] == 0)
    # den: its triples' bounds plus the per-view FP32 sums
    derr = np.abs(den.astype(np.float64) - ref.den)
    dbar = ref.B + scene.n_views * U32 * ref.den + oracle.SUM_ABS
    assert np.all(derr <= dbar), (derr / dbar).max()
    cmp = nz & ~vanish
    Eg = E[cmp].astype(np.float64)
    Eo = ref.E[cmp]
    eerr = np.linalg.norm(Eg - Eo, axis=1)
    no = np.linalg.norm(Eo, axis=1)
    cos = np.sum(Eg * Eo, 1) / (np.linalg.norm(Eg, axis=1) * no + 1e-300)
    # a bound b on ||dE|| gives 1 - cos <= (b / |E|)^2 / 2
    implied = bound[cmp] <= np.sqrt(2.0 * (1.0 - COS_MIN)) * no
    ngz = max(int(nz.sum()), 1)
    below = cos < COS_MIN
    st = dict(check="embeddings", case=tag, gaussians=int(nz.sum()),
              min_cos=float(cos.min()) if cos.size else 1.0,
              min_cos_bound_implied=float(cos[implied].min()) if implied.any() else 1.0,
              frac_not_implied=float(1.0 - implied.sum() / ngz),
              n_not_implied=int(nz.sum() - implied.sum()),
              weight_share_not_implied=float(ref.den[cmp][~implied].sum() / ref.den[nz].sum())
              if nz.any() else 0.0,
              n_cos_below=int(below.sum()), frac_cos_below=float(below.sum() / ngz),
              max_abs_err=float(eerr.max()) if eerr.size else 0.0,
              max_err_over_bound=float((eerr / bound[cmp]).max()) if eerr.size else 0.0,
              median_bound=float(np.median(bound[cmp])) if eerr.size else 0.0,
              max_den_rel_err=float((derr[nz] / ref.den[nz]).max()) if nz.any() else 0.0)
    _record(**st)
    assert np.all(eerr <= bound[cmp]), (eerr / bound[cmp]).max()
    assert not np.any(below & implied), cos[implied].min()
    assert st["frac_cos_below"] <= MAX_UNCOMPARED, st
    return st["min_cos"], st["max_abs_err"]


def check_tile_lists(L, scene, v, tile=16):
    t, z, g = L.tile_lists(v)
    rt, rz, rg = oracle.sorted_keys(scene, v, tile, tile)
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
        flips, nunc = check_view_weights(L, scene_2k, v, oracle_2k.views[v], "plain_fp32_2k")
        _say(f"  membership flips {flips}, triples with margin mass {nunc}")


def test_embeddings_match_oracle_2k(scene_2k, oracle_2k, lift_2k):
    _, E, den = lift_2k
    cmin, emax = check_embeddings(E, den, oracle_2k, scene_2k, "plain_fp32_2k")
    _say(f"min cosine {cmin:.9f}, max abs err {emax:.3g}")


def test_counts_match_oracle_2k(oracle_2k, lift_2k):
    L, _, _ = lift_2k
    st = L.stats()
    unc = sum(r.n_uncertain for r in oracle_2k.views)
    assert abs(st["n_contrib"] - oracle_2k.n_contrib) <= unc
    assert abs(st["n_tests"] - oracle_2k.n_tests) <= unc + st["n_contrib"] // 1000
    assert st["n_tile_tests"] >= st["n_tests"]


def check_pixels(L, scene, v, ores, tag=""):
    """Per-pixel invariant of front-to-back compositing (the rasterizer's
    weights telescope): sum_k w_kp = 1 - T_final(p), in FP32 to (2 n + 2) u
    for a pixel of n blends; T_final >= 1e-4; and T_final within the oracle's
    transmittance bound wherever no decision of the pixel lay in its band."""
    import paper_2505_08124_amd as slag
    T = slag.slag_get_debug(L.ctx, slag.SLAG_DEBUG_PIXEL_T_FINAL, v).astype(np.float64)
    ws = slag.slag_get_debug(L.ctx, slag.SLAG_DEBUG_PIXEL_WSUM, v).astype(np.float64)
    n = slag.slag_get_debug(L.ctx, slag.SLAG_DEBUG_PIXEL_COUNT, v).astype(np.float64)
    H, W = scene.ids[v].shape
    assert T.size == ws.size == n.size == H * W
    T, ws, n = T.reshape(H, W), ws.reshape(H, W), n.reshape(H, W)
    inv = np.abs(ws + T - 1.0)
    assert np.all(inv <= (2 * n + 2) * U32), inv.max()
    assert T.min() >= np.float32(1e-4)
    ok = ores.rho >= 0
    terr = np.abs(T - ores.T)
    assert np.all(terr[ok] <= ores.rho[ok] * ores.T[ok] + U32), (terr[ok] / ores.T[ok]).max()
    _record(check="pixels", case=tag, view=int(v), max_invariant_err=float(inv.max()),
            max_T_rel_err=float((terr[ok] / ores.T[ok]).max()), frac_in_band=float(1 - ok.mean()),
            min_T=float(T.min()), max_blends=int(n.max()))
    return float(inv.max())


def test_pixel_invariant_2k(scene_2k, oracle_2k, lift_2k):
    L, _, _ = lift_2k
    for v in range(scene_2k.n_views):
        e = check_pixels(L, scene_2k, v, oracle_2k.views[v], "plain_fp32_2k")
        _say(f"view {v}: max |sum w + T - 1| = {e:.3g}")


def test_debug_exports_are_consistent(scene_2k, lift_2k):
    """KEYS, TILE_RANGES, W_VIEW and COUNTERS of slag_get_debug agree with the
    per-call exports and the statistics."""
    import paper_2505_08124_amd as slag
    L, _, _ = lift_2k
    t, z, g = L.tile_lists(1)
    keys = slag.slag_get_debug(L.ctx, slag.SLAG_DEBUG_KEYS, 1)
    assert np.array_equal(keys, np.stack([t, z, g], 1))
    rng = slag.slag_get_debug(L.ctx, slag.SLAG_DEBUG_TILE_RANGES, 1)
    W = int(scene_2k.cams[1]["width"])
    assert rng.shape[0] == ((W + 15) // 16) * ((int(scene_2k.cams[1]["height"]) + 15) // 16)
    for k in range(rng.shape[0]):
        s, e = rng[k]
        assert np.all(t[s:e] == k)
    assert rng[-1, 1] == t.size and np.all(rng[1:, 0] == rng[:-1, 1])
    wv = slag.slag_get_debug(L.ctx, slag.SLAG_DEBUG_W_VIEW, 1)
    g2, s2, w2 = L.weights(1)
    assert np.array_equal(wv[:, 0], g2) and np.array_equal(wv[:, 1], s2)
    assert np.array_equal(wv[:, 2].view(np.float32), w2)
    cnt = slag.slag_get_debug(L.ctx, slag.SLAG_DEBUG_COUNTERS)
    st = L.stats()
    assert list(cnt[:3]) == [st["n_contrib"], st["n_tests"], st["n_tile_tests"]]
    assert cnt[3] == 0 and st["n_lost"] == 0


def test_bf16_output_is_rounded_fp32(scene_2k, lift_2k):
    """slag_get_embeddings with SLAG_BF16 returns the round-to-nearest-even
    bfloat16 of the FP32 result, to host and device memory."""
    import torch
    import paper_2505_08124_amd as slag
    from synthetic import f32_to_bf16_bits
    L, E, den = lift_2k
    hb = np.empty(E.shape, np.uint16)
    slag.slag_get_embeddings(L.ctx, hb)
    assert np.array_equal(hb, f32_to_bf16_bits(E))
    db = torch.empty(E.shape, dtype=torch.bfloat16, device="cuda")
    dd = torch.empty(den.shape, dtype=torch.float32, device="cuda")
    slag.slag_get_embeddings(L.ctx, db, dd)
    torch.cuda.synchronize()
    assert np.array_equal(db.view(torch.int16).cpu().numpy().view(np.uint16), hb)
    assert np.array_equal(dd.cpu().numpy(), den)


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
        check_view_weights(L, sc, v, ref.views[v], "ragged")
    check_embeddings(E, den, ref, sc, "ragged")


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
    assert len(tun) == 3 and all(len(t["ms"]) == slag.slag_variant_count() for t in tun)
    assert np.array_equal(E0, E1) and np.array_equal(E0, E2)
    assert np.array_equal(den0, den1) and np.array_equal(den0, den2)
    # tuned inside a lift that records a graph, then replayed
    L = _lifter(sc, flags=slag.SLAG_FLAG_AUTOTUNE | slag.SLAG_FLAG_GRAPH)
    for _ in range(3):
        L.lift()
        E3, den3 = L.embeddings()
        assert np.array_equal(E0, E3) and np.array_equal(den0, den3)
        _other_gpu_work()
    assert len(slag.slag_get_tuning(L.ctx)) == 3
    L.close()


@pytest.mark.parametrize("lpp,tile", [(1, 16), (2, 16), (1, 8)])
def test_every_compositing_variant_is_bitwise_equal(lpp, tile):
    """Every compositing variant (register budget, group padding, one
    workgroup per tile or a persistent grid taking tiles from a queue),
    forced through the composite_variant option, gives the default lift's
    bits, eagerly and on graph replays (the queue counter is reset inside the
    graph).  Three image sizes composited in one launch, 12,600 tiles: far
    more than the persistent grid, so its workgroups take many tiles each."""
    import paper_2505_08124_amd as slag
    sc = make_scene("uneven_1m", n=40000, views=dict(n=6))
    if lpp == 2:
        sc = _overlap_scene(sc)
    L0 = slag.Lifter(0, labels_per_pixel=lpp, tile_size=tile)
    L0.set_scene(sc)
    L0.lift()
    E0, den0 = L0.embeddings()
    L0.close()
    assert den0.max() > 0
    for v in range(slag.slag_variant_count()):
        _say(f"variant {v} ({slag.lib().slag_variant_name(v).decode()}), labels {lpp}, tile {tile}")
        L = slag.Lifter(0, flags=slag.SLAG_FLAG_GRAPH, labels_per_pixel=lpp,
                        composite_variant=v + 1, tile_size=tile)
        L.set_scene(sc)
        for rep in range(3):
            L.lift()
            E, den = L.embeddings()
            assert np.array_equal(E, E0) and np.array_equal(den, den0), (v, rep)
            _other_gpu_work()
        L.close()
    with pytest.raises(slag.SlagError):
        slag.Lifter(0, composite_variant=slag.slag_variant_count() + 1)
    with pytest.raises(slag.SlagError):
        slag.Lifter(0, composite_variant=-1)


def test_tuning_cache_file(tmp_path, monkeypatch):
    """SLAG_TUNE_CACHE: the tuned sizes are written after tuning and read by
    the next context (which then tunes nothing and lifts the same bits);
    lines of another device kind are kept, unreadable lines dropped."""
    import paper_2505_08124_amd as slag
    sc = _ragged_scene()
    path = tmp_path / "tune.txt"
    foreign = "slag-tune other/1 6 10 10 0 1 2 3 4 5 6"
    path.write_text("not a tuning line\n" + foreign + "\n")
    monkeypatch.setenv("SLAG_TUNE_CACHE", str(path))
    L = _lifter(sc, flags=slag.SLAG_FLAG_AUTOTUNE)
    assert slag.slag_get_tuning(L.ctx) == []
    L.lift()
    E1, den1 = L.embeddings()
    t1 = slag.slag_get_tuning(L.ctx)
    L.close()
    assert len(t1) == 3
    lines = path.read_text().splitlines()
    _say("tuning cache", lines)
    assert foreign in lines and "not a tuning line" not in lines
    assert len(lines) == 4 and all(ln.startswith("slag-tune ") for ln in lines)
    L2 = _lifter(sc, flags=slag.SLAG_FLAG_AUTOTUNE)
    assert slag.slag_get_tuning(L2.ctx) == t1          # read from the file
    L2.lift()
    E2, den2 = L2.embeddings()
    assert slag.slag_get_tuning(L2.ctx) == t1          # nothing tuned again
    assert np.array_equal(E1, E2) and np.array_equal(den1, den2)
    L2.close()
    assert path.read_text().splitlines() == lines
    monkeypatch.delenv("SLAG_TUNE_CACHE")
    L3 = _lifter(sc, flags=slag.SLAG_FLAG_AUTOTUNE)
    assert slag.slag_get_tuning(L3.ctx) == []
    L3.close()


@pytest.mark.parametrize("case", ["plain_fp32_2k", "ragged", "overlap"])
def test_tile_size_8_and_independence(case):
    """8 x 8 tiles (one wave per tile): tile lists bit-exact with the oracle's
    key mirror at 8 x 8, W_v of every view and E against the oracle; and the
    result does not depend on the tile size (the oracle has no tiles, and a
    wave blends the same 8 x 8 pixel block with the same exponent expansion
    at either size): the same (Gaussian, segment) sets, weights, den and E
    equal to the 16 x 16 lift's up to the order of the FP32 sums."""
    import paper_2505_08124_amd as slag
    lpp = 1
    if case == "plain_fp32_2k":
        sc = make_scene("plain_fp32_2k")
    elif case == "ragged":
        sc = _ragged_scene()
    else:
        sc = _overlap_scene(make_scene("plain_fp32_2k"))
        lpp = 2
    ref = oracle.lift(sc)
    out = {}
    for tile in (8, 16):
        L = slag.Lifter(0, flags=slag.SLAG_FLAG_KEEP_DEBUG, labels_per_pixel=lpp, tile_size=tile)
        L.set_scene(sc)
        L.lift()
        E, den = L.embeddings()
        trip = []
        for v in range(sc.n_views):
            check_tile_lists(L, sc, v, tile)
            check_view_weights(L, sc, v, ref.views[v], f"tile{tile}_{case}")
            trip.append(_gpu_triples(L, v))
        check_embeddings(E, den, ref, sc, f"tile{tile}_{case}")
        out[tile] = (E, den, trip)
        L.close()
    (E8, d8, t8), (E16, d16, t16) = out[8], out[16]
    for v in range(sc.n_views):
        (k8, w8), (k16, w16) = t8[v], t16[v]
        assert np.array_equal(k8, k16), v                  # same contributing sets
        np.testing.assert_allclose(w8, w16, rtol=1e-5, atol=1e-12)
    assert np.array_equal(d8 > 0, d16 > 0)
    np.testing.assert_allclose(d8, d16, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(E8, E16, rtol=1e-5, atol=1e-6)
    _say(f"tile 8 vs 16 ({case}): max |dE| {np.abs(E8 - E16).max():.3g}, "
         f"max rel d(den) {(np.abs(d8 - d16) / np.maximum(d16, 1e-30)).max():.3g}")


@pytest.mark.parametrize("D,dtype", [(128, "f32"), (256, "bf16"), (1024, "bf16"), (1024, "f32")])
def test_feature_sizes_match_oracle(D, dtype):
    """Feature sizes beyond those of the benchmark workloads (64 to 1024 are
    taken; BF16 768 and 1024 run the walk and the chunk multiply as two
    kernels) against the FP64 oracle, with the ragged tiles of the 2,000-
    Gaussian scene: E within the propagated bound, den within its bar."""
    sc = make_scene("plain_fp32_2k", features=dict(D=D, dtype=dtype))
    ref = oracle.lift(sc)
    L = _lifter(sc)
    L.lift()
    E, den = L.embeddings()
    assert E.shape == (sc.n, D)
    cmin, emax = check_embeddings(E, den, ref, sc, f"d{D}_{dtype}")
    _say(f"D = {D} {dtype}: min cosine {cmin:.9f}, max abs err {emax:.3g}")
    L.close()


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
        check_view_weights(L, sc, v, ref.views[v], "uneven_40k")
    check_embeddings(E, den, ref, sc, "uneven_40k")


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
    cmin, _ = check_embeddings(E, den, ref, sc, "depth_ties")
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
        check_view_weights(L, sc, v, ref.views[v], "plain_bf16_200k")
    _say("200k: counting lift, per-pixel outputs of sampled views")
    Lc = _lifter(sc, flags=slag.SLAG_FLAG_COUNT)
    Lc.lift()
    for v in (5, 61):
        check_pixels(Lc, sc, v, oracle.lift_view(sc, v, pixels=True), "plain_bf16_200k")
    Lc.close()
    cmin, emax = check_embeddings(E, den, ref, sc, "plain_bf16_200k")
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
        check_view_weights(L, sc, v, oracle.lift_view(sc, v), "uneven_1m")
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


CUSTOM = dict(alpha_max=0.9, alpha_min=0.02, t_min=0.01, dilation=0.5, near_z=0.5, guard=1.1)


@pytest.mark.parametrize("case", ["plain_fp32_2k", "ragged"])
def test_custom_constants_match_oracle(case):
    """Non-default rasterizer constants (slag_options) against the oracle run
    with the same constants: tile lists bit-exact, W_v within the bounds,
    embeddings within the bound; the result differs from the default lift."""
    import paper_2505_08124_amd as slag
    sc = make_scene("plain_fp32_2k") if case == "plain_fp32_2k" else _ragged_scene()
    K = {k: float(np.float32(v)) for k, v in CUSTOM.items()}
    L = slag.Lifter(0, flags=slag.SLAG_FLAG_KEEP_DEBUG, **K)
    L.set_scene(sc)
    L.lift()
    E, den = L.embeddings()
    with oracle.constants(**{k: np.float32(v) for k, v in K.items()}):
        ref = oracle.lift(sc)
        for v in range(sc.n_views):
            _say(f"custom constants {case}: view {v}")
            check_tile_lists(L, sc, v)
            check_view_weights(L, sc, v, ref.views[v], "custom_" + case)
    check_embeddings(E, den, ref, sc, "custom_" + case)
    L.close()
    L0 = _lifter(sc)
    L0.lift()
    E0, den0 = L0.embeddings()
    L0.close()
    assert not np.array_equal(den0, den)


def test_invalid_options_are_rejected():
    import paper_2505_08124_amd as slag
    for bad in (dict(alpha_min=0.5, alpha_max=0.4), dict(t_min=1.5), dict(dilation=-1.0),
                dict(deterministic=2)):
        with pytest.raises(slag.SlagError) as ei:
            slag.Lifter(0, **bad)
        assert ei.value.status == slag.SLAG_E_INVALID_ARG, bad
    for bad_tile in (4, 12, 32):
        with pytest.raises(slag.SlagError) as ei:
            slag.Lifter(0, tile_size=bad_tile)
        assert ei.value.status == slag.SLAG_E_NOT_SUPPORTED
    slag.Lifter(0, tile_size=16, deterministic=1).close()
    slag.Lifter(0, tile_size=8).close()


@pytest.mark.parametrize("max_views,chunk", [(0, 512), (0, 208), (2, 1024), (0, 4096)])
def test_chunked_lift_equals_lift(scene_2k, lift_2k, max_views, chunk):
    """The lift streamed to host memory in chunks of Gaussians (the paper's
    iterated aggregation for outputs that do not fit on the GPU) equals the
    one-piece lift bit for bit, in one or several view launches, FP32 and
    BF16 output."""
    import paper_2505_08124_amd as slag
    from synthetic import f32_to_bf16_bits
    L0 = _lifter(scene_2k, max_views=max_views)
    L0.lift()
    E0, den0 = L0.embeddings()
    L0.close()
    L = slag.Lifter(0, None, max_views)
    L.set_scene(scene_2k)
    E = np.full(E0.shape, np.nan, np.float32)
    den = np.full(den0.shape, np.nan, np.float32)
    slag.slag_lift_chunked(L.ctx, chunk, E, den)
    assert np.array_equal(E, E0) and np.array_equal(den, den0)
    Eb = np.zeros(E0.shape, np.uint16)
    slag.slag_lift_chunked(L.ctx, chunk, Eb)
    assert np.array_equal(Eb, f32_to_bf16_bits(E0))
    if max_views:
        assert L.stats()["n_batches"] == 2
    with pytest.raises(slag.SlagError):
        slag.slag_lift_chunked(L.ctx, 100, E)         # not a multiple of 16
    L.close()


def _overlap_scene(base, n_extra=9, frac=0.6, seed=11):
    """base with a second mask layer: a 3x3 grid of masks over a random
    ~60 % of each view's pixels, overlapping the first layer's segments."""
    rng = np.random.default_rng(seed)
    ids, nseg, rows = [], [], []
    off = base.seg_offsets
    F = base.feats
    for v in range(base.n_views):
        i0 = base.ids[v]
        H, W = i0.shape
        yy, xx = np.mgrid[0:H, 0:W]
        grid = (3 * yy // H) * 3 + (3 * xx // W)
        k0 = int(base.nseg[v])
        l1 = np.where(rng.random((H, W)) < frac, k0 + grid, -1).astype(np.int32)
        ids.append(np.stack([i0, l1], axis=-1))
        nseg.append(k0 + n_extra)
        extra = rng.standard_normal((n_extra, F.shape[1])).astype(np.float32)
        extra /= np.linalg.norm(extra, axis=1, keepdims=True)
        rows.append(np.concatenate([F[off[v]:off[v + 1]], extra.astype(F.dtype)]))
    return dataclasses.replace(base, ids=ids, nseg=np.array(nseg, np.int32),
                               feats=np.ascontiguousarray(np.concatenate(rows)))


@pytest.mark.parametrize("case", ["plain_fp32_2k", "uneven_40k"])
def test_overlapping_masks_match_oracle(case):
    """Pixels in two masks give their weights to both (paper: masks M_j are
    per-object binary masks, and the aggregation sums over every mask and its
    pixels): tile lists, W_v and embeddings against the oracle."""
    import paper_2505_08124_amd as slag
    base = make_scene("plain_fp32_2k") if case == "plain_fp32_2k" else \
        make_scene("uneven_1m", n=40000, views=dict(n=3))
    sc = _overlap_scene(base)
    L = slag.Lifter(0, flags=slag.SLAG_FLAG_KEEP_DEBUG, labels_per_pixel=2)
    L.set_scene(sc)
    L.lift()
    E, den = L.embeddings()
    ref = oracle.lift(sc)
    for v in range(sc.n_views):
        _say(f"overlapping masks {case}: view {v}")
        check_tile_lists(L, sc, v)
        check_view_weights(L, sc, v, ref.views[v], "overlap_" + case)
    check_embeddings(E, den, ref, sc, "overlap_" + case)
    L.close()


def test_empty_second_label_layer_is_bitwise_neutral(scene_2k, lift_2k):
    """labels_per_pixel = 2 with the second layer empty equals the one-label
    lift bit for bit; a repeated label in one pixel is rejected."""
    import paper_2505_08124_amd as slag
    _, E0, den0 = lift_2k
    ids2 = [np.stack([i, np.full_like(i, -1)], axis=-1) for i in scene_2k.ids]
    sc = dataclasses.replace(scene_2k, ids=ids2)
    L = slag.Lifter(0, labels_per_pixel=2)
    L.set_scene(sc)
    L.lift()
    E, den = L.embeddings()
    assert np.array_equal(E, E0) and np.array_equal(den, den0)
    bad = np.stack([scene_2k.ids[0], scene_2k.ids[0]], axis=-1)
    with pytest.raises(slag.SlagError):
        slag.slag_set_segments_multi(L.ctx, 0, bad, int(scene_2k.nseg[0]))
    with pytest.raises(slag.SlagError):
        slag.slag_set_segments_multi(L.ctx, 0, np.stack([bad] * 2, -1).reshape(64, 64, 4),
                                     int(scene_2k.nseg[0]))      # more layers than the option
    L.close()


@pytest.mark.parametrize("case,tile", [("plain_fp32_2k", 16), ("ragged", 16), ("ragged", 8)])
def test_kernel_weights_match_oracle(case, tile):
    """weight_mode = 1, the paper's weight equation (the Gaussian kernel
    exp(-q/2) of each Gaussian the front-to-back walk blends): W_v and the
    embeddings against the oracle run in the same mode; differs from the
    blend-weight lift."""
    import paper_2505_08124_amd as slag
    sc = make_scene("plain_fp32_2k") if case == "plain_fp32_2k" else _ragged_scene()
    L = slag.Lifter(0, flags=slag.SLAG_FLAG_KEEP_DEBUG | slag.SLAG_FLAG_AUTOTUNE, weight_mode=1,
                    tile_size=tile)
    L.set_scene(sc)
    L.lift()
    E, den = L.embeddings()
    with oracle.constants(weight_mode=1.0):
        ref = oracle.lift(sc)
    tag = f"kernel_{case}" + ("" if tile == 16 else f"_tile{tile}")
    for v in range(sc.n_views):
        check_tile_lists(L, sc, v, tile)
        check_view_weights(L, sc, v, ref.views[v], tag)
    check_embeddings(E, den, ref, sc, tag)
    L.close()
    L0 = _lifter(sc)
    L0.lift()
    _, den0 = L0.embeddings()
    L0.close()
    assert not np.array_equal(den0, den)
