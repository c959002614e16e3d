"""GPU parity on the large aerial workload (4M Gaussians in 200 clusters over
10 x 10 x 3, 1000 nadir views of 1024x768 on a lawnmower path, 100-200
segments per view, D = 768 BF16 features), in the launch configuration the
benchmark times, and on small D = 768 scenes the oracle lifts completely.

The full workload needs more than one launch (32-bit pair indices cap a
launch at 2^31 / N views); the views of the last launch keep their debug
exports, so sampled views there are checked against the oracle one by one
(tile lists bit-exact, W_v within the derived bounds); the embeddings of the
full lift are checked by properties that hold at any size (convex hull of
the feature rows, zero rows exactly where nothing weighs in, invariance of
den to the view plan), and the embeddings of all 4M Gaussians over a sample
of views against the FP64 oracle lift of those views.
"""
import sys

import numpy as np
import pytest

import oracle
from synthetic import make_scene

from test_gpu_parity import check_embeddings, check_tile_lists, check_view_weights

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-stress]", *a, flush=True)
    sys.stdout.flush()


def test_d768_small_scene_full_parity():
    """D = 768 BF16 contraction (12 column tiles per wave) against the full
    FP64 oracle lift: 40k Gaussians of the aerial recipe, 6 views."""
    import paper_2505_08124_amd as slag
    sc = make_scene("stress_4m", n=40000, views=dict(n=6))
    assert sc.dim == 768 and sc.feat_dtype == "bf16"
    _say("d768 small: oracle")
    ref = oracle.lift(sc)
    _say("d768 small: gpu")
    L = slag.Lifter(0, flags=slag.SLAG_FLAG_KEEP_DEBUG)
    L.set_scene(sc)
    L.lift()
    E, den = L.embeddings()
    for v in range(sc.n_views):
        check_tile_lists(L, sc, v)
        check_view_weights(L, sc, v, ref.views[v], "stress_d768_40k")
    cmin, emax = check_embeddings(E, den, ref, sc, "stress_d768_40k")
    _say(f"d768 small: min cosine {cmin:.9f}, max abs err {emax:.3g}")
    L.close()


@pytest.mark.parametrize("max_views,chunk", [(0, 0), (2, 0), (2, 4096), (0, 1024)])
def test_d768_split_contraction_across_launches(max_views, chunk):
    """At D = 768 the contraction runs as a walk per view launch (chunk
    lists appended to one buffer, grown and the walk re-run when the first
    guess is too small) and one chunk multiply after the last launch. With
    the same view plan, the graph replay and the chunked output give the
    eager lift's bits; across plans (one launch against three) den is
    bitwise equal (per-view sums in view order) and E equal to FP32
    rounding (the chunks group the columns differently)."""
    import paper_2505_08124_amd as slag
    sc = make_scene("stress_4m", n=40000, views=dict(n=6))

    def plain(mv):
        L0 = slag.Lifter(0, max_views_per_launch=mv)
        L0.set_scene(sc)
        L0.lift()
        out = L0.embeddings()
        nb = L0.stats()["n_batches"]
        L0.close()
        return out, nb

    (E0, den0), nb = plain(max_views)
    assert nb == (3 if max_views else 1)
    L = slag.Lifter(0, max_views_per_launch=max_views, flags=slag.SLAG_FLAG_GRAPH)
    L.set_scene(sc)
    if chunk:
        E = np.full(E0.shape, np.nan, np.float32)
        den = np.full(den0.shape, np.nan, np.float32)
        slag.slag_lift_chunked(L.ctx, chunk, E, den)
    else:
        L.lift()
        E, den = L.embeddings()
        L.lift()                               # graph replay
        E2, den2 = L.embeddings()
        assert np.array_equal(E2, E) and np.array_equal(den2, den)
    L.close()
    assert np.array_equal(den, den0) and np.array_equal(E, E0)
    if max_views:
        (E1, den1), _ = plain(0)
        assert np.array_equal(den1, den0)
        np.testing.assert_allclose(E0, E1, rtol=1e-5, atol=1e-6)


def test_replan_when_a_launch_would_overflow():
    """A launch whose tile intersections or part slots exceed the cap is
    re-planned with fewer views per launch; the result equals the one-launch
    lift (den bitwise: per-view sums in view order; E to FP32 rounding).
    Four symmetric ring views each hold about a quarter of the entries, so a
    cap of 40 % of the totals fits one view per launch and not two."""
    import paper_2505_08124_amd as slag
    sc = make_scene("plain_fp32_2k")
    L1 = slag.Lifter(0)
    L1.set_scene(sc)
    L1.lift()
    E1, den1 = L1.embeddings()
    s1 = L1.stats()
    assert s1["n_batches"] == 1
    cap = int(0.4 * max(s1["n_intersections"], s1["n_part_slots"]))
    L2 = slag.Lifter(0, max_launch_entries=cap, flags=slag.SLAG_FLAG_GRAPH)
    L2.set_scene(sc)
    L2.lift()
    E2, den2 = L2.embeddings()
    s2 = L2.stats()
    _say(f"replan: cap {cap}, {s2['n_batches']} launches")
    assert s2["n_batches"] >= 3
    assert s2["n_intersections"] == s1["n_intersections"]
    assert np.array_equal(den1, den2)
    np.testing.assert_allclose(E2, E1, rtol=1e-5, atol=1e-6)
    # the graph of the re-planned lift replays the same result
    L2.lift()
    E3, den3 = L2.embeddings()
    assert np.array_equal(E3, E2) and np.array_equal(den3, den2)
    # one view that does not fit cannot be split further
    L3 = slag.Lifter(0, max_launch_entries=16)
    L3.set_scene(sc)
    with pytest.raises(slag.SlagError) as ei:
        L3.lift()
    assert ei.value.status == slag.SLAG_E_CAPACITY
    for L in (L1, L2, L3):
        L.close()


@pytest.fixture(scope="module")
def stress_scene():
    _say("stress_4m: generating the scene")
    return make_scene("stress_4m")


def test_full_size_stress_4m(stress_scene):
    """4M Gaussians, 1000 views of 1024x768, D = 768: the lift as timed (graph
    replay, automatic view plan), sampled views of its last launch against
    the oracle, properties of the full result, and den unchanged by a plan of
    250-view launches."""
    import paper_2505_08124_amd as slag
    sc = stress_scene
    assert sc.n == 4_000_000 and sc.n_views == 1000 and sc.dim == 768
    _say("stress_4m: lift as timed (graph replay)")
    L0 = slag.Lifter(0, flags=slag.SLAG_FLAG_GRAPH)
    L0.set_scene(sc, device_tensors=True)
    L0.lift()
    Ee, dene = L0.embeddings()
    L0.lift()
    E0, den0 = L0.embeddings()
    st0 = L0.stats()
    L0.close()
    assert np.array_equal(Ee, E0) and np.array_equal(dene, den0)
    _say(f"stress_4m: {st0['n_batches']} launches, pairs {st0['n_visible_pairs']}, "
         f"intersections {st0['n_intersections']}, part slots {st0['n_part_slots']}")
    assert st0["n_batches"] >= 2
    # properties of the full result
    nz = den0 > 0
    fmax = np.linalg.norm(sc.feats_f64(), axis=1).max()
    assert np.all(np.isfinite(E0))
    assert np.all(E0[~nz] == 0)
    norms = np.linalg.norm(E0[nz].astype(np.float64), axis=1)
    assert np.all(norms <= fmax * (1 + 1e-5)), norms.max()
    _say(f"stress_4m: {int(nz.sum())} Gaussians with weight")
    # sampled views of the last launch, with debug exports
    _say("stress_4m: lift with debug exports")
    L = slag.Lifter(0, flags=slag.SLAG_FLAG_KEEP_DEBUG)
    L.set_scene(sc, device_tensors=True)
    L.lift()
    E, den = L.embeddings()
    assert np.array_equal(E, E0) and np.array_equal(den, den0)
    for v in (sc.n_views - 1, sc.n_views - 230, sc.n_views - 415):
        _say("stress_4m: oracle view", v)
        ores = oracle.lift_view(sc, v)
        check_tile_lists(L, sc, v)
        check_view_weights(L, sc, v, ores, "stress_4m")
    L.close()
    _say("stress_4m: 250 views per launch")
    L2 = slag.Lifter(0, max_views_per_launch=250)
    L2.set_scene(sc, device_tensors=True)
    L2.lift()
    E2, den2 = L2.embeddings()
    assert L2.stats()["n_batches"] == 4
    L2.close()
    assert np.array_equal(den2, den0)
    np.testing.assert_allclose(E2, E0, rtol=1e-5, atol=1e-6)


def test_stress_4m_embeddings_on_sampled_views(stress_scene):
    """All 4M Gaussians lifted over 4 sampled views (two lawnmower rows
    apart), D = 768 BF16: embeddings against the FP64 oracle lift of the same
    views, within the propagated bound and cosine >= 0.9999 where the bound
    implies it."""
    import paper_2505_08124_amd as slag
    views = [0, 333, 666, 999]
    sub = stress_scene.subset_views(views)
    _say("stress_4m sample: oracle")
    ref = oracle.lift(sub)
    _say("stress_4m sample: gpu")
    L = slag.Lifter(0)
    L.set_scene(sub, device_tensors=True)
    L.lift()
    E, den = L.embeddings()
    L.close()
    cmin, emax = check_embeddings(E, den, ref, sub, "stress_4m_4views")
    _say(f"stress_4m sample: min cosine {cmin:.9f}, max abs err {emax:.3g}")
