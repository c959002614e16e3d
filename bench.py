#!/usr/bin/env python3
"""Throughput of the segment-embedding lift on one MI355X.

One step = one full lift (tile segment tables, projection, depth sort,
binning, tile sort, compositing with masking, contraction and normalisation)
of the headline workload: 4M Gaussians in 200 clusters over 10 x 10 x 3,
1000 nadir views of 1024x768 on a lawnmower path, 100-200 segments per view,
D = 768 BF16 features (the large aerial scene of the paper's experiments,
synthetic), with every input resident in HBM before the timed region.

Prints one JSON line: views/s (value), Gaussian-pixel contributions/s, the
dominant kernel's achieved rate against its roofline (from HIP events on the
library's stream), per-stage algorithmic lower bounds, the accuracy of the
lift against the FP64 oracle on sampled views, the smaller workloads and the
learned codec as secondary sections, and the FP64 CPU oracle's rate on a
bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lift views/s + Gaussian-pixel contribs/s at 1 GPU"
HEADLINE = "stress_4m"
TILE_SIZE = 16   # tile edge of the measured lifts (--tile-size)
DESC = {
    "stress_4m": "4M Gaussians from 200 clusters over 10x10x3, 1000 nadir views 1024x768 on a "
                 "lawnmower path, 100-200 Voronoi segments/view, D=768 BF16 object-vocabulary "
                 "features",
    "uneven_1m": "1M Gaussians, 300 views of 320x240/640x480/1280x960 in one launch, 50-150 "
                 "segments/view, D=512 BF16 object-vocabulary features",
    "plain_bf16_200k": "200k Gaussians in 20 anisotropic clusters, 100 spiral views 512x384, "
                       "40-80 Voronoi segments/view + ~10% background, D=512 BF16 features",
    "plain_fp32_2k": "2,000 Gaussians, 4 ring views 64x64, 8 Voronoi segments/view, D=64 FP32 "
                     "features",
}

# Peaks of one MI355X (vendor figures; 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz)
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12      # lane-operations per second (non-packed)
MFMA_BF16_PEAK_TFLOPS = 2500.0
# VALU work per (pixel, Gaussian) support test of the blend: quadratic form
# about 7, exp about 5 (a multiply and the transcendental at four slots),
# clamp/test 2, transmittance update/test 2 = 16 slot-operations.  The kernel
# issues 19 slots per test (2 sub, 5 mul/fma, clamp, exp2 at 4, mul + min,
# compare, fma, compare, mul, select); both fractions are reported, the
# first one is the headline.
OPS_PER_TEST = 16
SLOTS_PER_TEST = 19


def _log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {"k_composite": "k_raster.hip", "contraction": "k_contract.hip"}
TRAFFIC_FILES = {"k_composite": "composite_traffic_{}.txt", "contraction": "contract_traffic_{}.txt"}


def kernel_source_hash(kernel: str = "k_composite") -> str:
    p = os.path.join(ROOT, "paper_2505_08124_amd", "csrc", KERNEL_SOURCES[kernel])
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic(workload: str, kernel: str = "k_composite"):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel source and this workload; else
    None."""
    p = os.path.join(ROOT, "profiles", TRAFFIC_FILES[kernel].format(workload))
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and not line.startswith(("|", "#", " ", "`")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash(kernel) or kv.get("workload") != workload:
        return None
    try:
        return int(float(kv["bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def stage_bounds(scene, st, stage_ms, n_tests):
    """Per-stage algorithmic lower bounds (ms) from the work the method must
    do, each against the bound of its stage: HBM at 8 TB/s for the data
    movement stages, the VALU lane-op peak for compositing."""
    N, V, D = scene.n, scene.n_views, scene.dim
    P = scene.pixels()
    S = int(scene.nseg.sum())
    pairs, ni = st["n_visible_pairs"], st["n_intersections"]
    nnz = st["n_weights"]
    nb = st["n_batches"]
    fb = 2 if scene.feat_dtype == "bf16" else 4
    by = {
        # 4 B of segment id per pixel read, 2 B per tile-table entry (about one per tile)
        "tile_segments": 4.0 * P,
        # 44 B per Gaussian per launch read, 32 B record per visible pair written
        "project": 44.0 * N * nb + 32.0 * pairs,
        # one read and one write of an 8 B key + 4 B value per pair
        "depth_sort": 24.0 * pairs,
        # 32 B read per visible pair, 12 B written per intersection
        "bin": 32.0 * pairs + 12.0 * ni,
        # one read and one write of key + value per intersection
        "tile_sort": 24.0 * ni,
        # 8 B per non-zero partial read, feature table once, E and den written
        "contract": 8.0 * nnz + fb * S * D + 4.0 * (D + 1) * N,
    }
    out = {}
    lb_total = 0.0
    for k, b in by.items():
        lb = b / (HBM_PEAK_GBS * 1e9) * 1e3
        out[k] = dict(bound="hbm", bytes=int(b), lb_ms=round(lb, 4),
                      ms=round(stage_ms.get(k, 0.0), 4),
                      frac=round(lb / stage_ms[k], 4) if stage_ms.get(k) else None)
        lb_total += lb
    if n_tests:
        lb = n_tests * OPS_PER_TEST / (VALU_PEAK_TOPS * 1e12) * 1e3
        out["composite"] = dict(bound="alu", ops=int(n_tests * OPS_PER_TEST), lb_ms=round(lb, 4),
                                ms=round(stage_ms.get("composite", 0.0), 4),
                                frac=round(lb / stage_ms["composite"], 4)
                                if stage_ms.get("composite") else None)
        lb_total += lb
    return out, lb_total


def measure(slag, torch, scene, steps, warmup, count=True, stage_steps=3, eager=False):
    """Time K back-to-back lifts (graph replays) on one default-priority
    stream with HIP events, then per-stage times from eager profiled lifts.
    Returns a dict of measurements (and the embeddings of the timed lift)."""
    V = scene.n_views
    res = {"feature_dim": scene.dim, "feat_bf16": scene.feat_dtype == "bf16"}
    if count:
        # contributions, in-box tests and non-zero weights: a separate counting
        # lift (not timed)
        with slag.Lifter(0, flags=slag.SLAG_FLAG_COUNT | slag.SLAG_FLAG_KEEP_DEBUG,
                         tile_size=TILE_SIZE) as Lc:
            Lc.set_scene(scene, device_tensors=True)
            Lc.lift()
            st = Lc.stats()
        res.update(n_contrib=st["n_contrib"], n_tests=st["n_tests"],
                   n_tile_tests=st["n_tile_tests"], n_weights=st["n_weights"])
        _log(f"{scene.name}: contributions {st['n_contrib']}, in-box tests {st['n_tests']}, "
             f"tile tests {st['n_tile_tests']}, non-zero weights {st['n_weights']}")
    flags = slag.SLAG_FLAG_PROFILE | slag.SLAG_FLAG_AUTOTUNE | (0 if eager else slag.SLAG_FLAG_GRAPH)
    stream = torch.cuda.Stream()
    L = slag.Lifter(0, stream=stream.cuda_stream, flags=flags, tile_size=TILE_SIZE)
    t_up = time.perf_counter()
    L.set_scene(scene, device_tensors=True)
    torch.cuda.synchronize()
    res["upload_s"] = round(time.perf_counter() - t_up, 3)
    for _ in range(max(warmup, 1)):
        L.lift()
    L.embeddings()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        L.lift()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev_ms = ev0.elapsed_time(ev1) / steps
    ms = (t1 - t0) * 1e3 / steps
    E, den = L.embeddings()
    assert np.isfinite(E).all()
    info = L.stats()
    res["tuning"] = slag.slag_get_tuning(L.ctx)
    L.close()
    res.update(ms_step=ms, ms_hip_events=ev_ms, views_per_s=V / (ms * 1e-3),
               n_visible_pairs=info["n_visible_pairs"], n_intersections=info["n_intersections"],
               n_part_slots=info["n_part_slots"], n_batches=info["n_batches"])
    _log(f"{scene.name}: step {ms:.3f} ms wall, {ev_ms:.3f} ms HIP events "
         f"({'eager' if eager else 'graph replay'}), {info['n_batches']} launch(es)")
    # per-stage times: HIP events the library records on its stream around
    # each stage of eager lifts of the same scene, right after the timed
    # replays (events recorded by graph nodes cannot be timed on this
    # runtime); their sum is checked against the replayed step
    stage_ms = {}
    tot = 0.0
    with slag.Lifter(0, flags=slag.SLAG_FLAG_PROFILE | slag.SLAG_FLAG_AUTOTUNE,
                     tile_size=TILE_SIZE) as Lp:
        Lp.set_scene(scene, device_tensors=True)
        Lp.lift()
        Lp.stats()
        for _ in range(stage_steps):
            Lp.lift()
            stp = Lp.stats()
            tot += stp["ms_total"]
            for k, v in stp["ms_stage"].items():
                stage_ms[k] = stage_ms.get(k, 0.0) + v
    res["stage_ms"] = {k: v / stage_steps for k, v in stage_ms.items()}
    res["stage_ms_eager_total"] = tot / stage_steps
    _log(f"{scene.name}: stage ms", json.dumps({k: round(v, 4) for k, v in res["stage_ms"].items()}))
    if count:
        res["contribs_per_s"] = res["n_contrib"] / (ms * 1e-3)
        st = dict(n_visible_pairs=res["n_visible_pairs"], n_intersections=res["n_intersections"],
                  n_weights=res["n_weights"], n_batches=res["n_batches"])
        res["stages"], lb = stage_bounds(scene, st, res["stage_ms"], res["n_tests"])
        res["lift_lb_ms"] = lb
        res["lift_roofline_frac"] = lb / ms
    return res, E, den


def search_and_render(slag, torch, scene, E, reps=3):
    """The search over the lifted embeddings (device-resident, the query
    side of the paper) and the render-back of one view, timed on the GPU.
    A count-only search reads the embedding table once (HBM-bound: its GB/s
    against 8 TB/s); a top-k search adds a per-query sort of the n scores."""
    dev = torch.from_numpy(E).cuda()
    rng = np.random.default_rng(7)
    F = scene.feats_f64()
    gb = E.shape[0] * E.shape[1] * 4 / 1e9
    search = []
    with slag.Lifter(0) as L:
        for q, k in ((1, 0), (16, 0), (1, 10), (16, 10)):
            rows = F[rng.choice(F.shape[0], q, replace=False)].astype(np.float32)
            Q = torch.from_numpy(np.ascontiguousarray(rows)).cuda()
            torch.cuda.synchronize()
            slag.slag_query(L.ctx, dev, Q, 0.28, k)      # first call sizes the workspace
            t0 = time.perf_counter()
            for _ in range(reps):
                cnt, _, _ = slag.slag_query(L.ctx, dev, Q, 0.28, k)
            ms = (time.perf_counter() - t0) / reps * 1e3
            row = dict(queries=q, k=k, threshold=0.28, ms=round(ms, 3),
                       count_first=int(cnt[0]))
            if k == 0:
                row.update(emb_gb=round(gb, 3), gbs=round(gb / (ms * 1e-3), 1),
                           frac=round(gb / (ms * 1e-3) / HBM_PEAK_GBS, 4))
            search.append(row)
        _log("search:", json.dumps(search))
    del dev
    # render-back of 16 channels into view 0 (projection, sorts and the
    # compositing of one view, then one pass of k_render)
    render = None
    with slag.Lifter(0) as L:
        L.set_scene(scene, device_tensors=True)
        C = 16
        attr = torch.from_numpy(np.ascontiguousarray(E[:, :C])).cuda()
        H, W = int(scene.cams[0]["height"]), int(scene.cams[0]["width"])
        out = torch.empty((H, W, C), dtype=torch.float32, device="cuda")
        ws = torch.empty((H, W), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        slag.slag_render(L.ctx, 0, attr, out, ws)
        t0 = time.perf_counter()
        for _ in range(reps):
            slag.slag_render(L.ctx, 0, attr, out, ws)
        ms = (time.perf_counter() - t0) / reps * 1e3
        render = dict(view=0, width=W, height=H, channels=C, ms=round(ms, 3),
                      lit_fraction=round(float((ws > 0).float().mean().item()), 4))
        _log("render:", json.dumps(render))
    return search, render


def kernel_rooflines(res, workload):
    """Roofline of the two heaviest stages per launch: k_composite (VALU:
    in-box tests x 16 operations, and the 19 issue slots the kernel spends per
    test) and the contraction (HBM: 8 B per non-zero partial, the feature
    table once, E and den written; k_contract_mfma, which at D >= 768 BF16
    walks only and hands chunks to k_contract_chunks), each from its stage
    time over the launches of one step, and which of them dominates."""
    out = {}
    nl = int(res.get("n_batches") or 1)
    comp = res["stage_ms"].get("composite", 0.0)
    ncomp = nl   # one compositing launch per view launch, all image sizes together
    if res.get("n_tests") and comp > 0:
        ach = res["n_tests"] * OPS_PER_TEST / (comp * 1e-3) / 1e12
        ach19 = res["n_tests"] * SLOTS_PER_TEST / (comp * 1e-3) / 1e12
        out["k_composite"] = dict(
            kernel="k_composite", bound="alu", achieved=round(ach, 4), peak=round(VALU_PEAK_TOPS, 3),
            unit="Tops/s", frac=round(ach / VALU_PEAK_TOPS, 4),
            traffic=measured_traffic(workload, "k_composite"), ops_per_test=OPS_PER_TEST,
            frac_issued_slots=round(ach19 / VALU_PEAK_TOPS, 4), slots_per_test=SLOTS_PER_TEST,
            launches_per_step=ncomp, tests_per_launch=int(res["n_tests"] / ncomp),
            avg_launch_ms=round(comp / ncomp, 4))
    con = res["stage_ms"].get("contract", 0.0)
    st = res.get("stages") or {}
    if "contract" in st and con > 0:
        b = st["contract"]["bytes"]
        ach = b / (con * 1e-3) / 1e9
        split = res.get("feature_dim", 0) >= 768 and res.get("feat_bf16", False)
        out["contraction"] = dict(
            kernel="k_contract_mfma + k_contract_chunks" if split else "k_contract_mfma",
            bound="hbm", achieved=round(ach, 2), peak=HBM_PEAK_GBS,
            unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
            traffic=measured_traffic(workload, "contraction"), launches_per_step=nl,
            bytes_per_launch=int(b / nl), avg_launch_ms=round(con / nl, 4))
    if not out:
        return None, out
    dom = max(out, key=lambda k: res["stage_ms"]["composite" if k == "k_composite" else "contract"])
    return dict(out[dom], dominant_stage=max(res["stage_ms"], key=res["stage_ms"].get)), out


def accuracy_and_cpu(slag, scene, views, budget_s):
    """The FP64 oracle lift of sampled views (timed: the CPU baseline) and the
    GPU lift of the same views (all Gaussians), compared per Gaussian:
    minimum cosine, maximum absolute error, and the propagated error bound."""
    import oracle
    sub = scene.subset_views(views)
    t0 = time.perf_counter()
    ref = oracle.lift(sub)
    dt = time.perf_counter() - t0
    with slag.Lifter(0) as L:
        L.set_scene(sub, device_tensors=True)
        L.lift()
        E, den = L.embeddings()
    F = sub.feats_f64()
    fmax = float(np.linalg.norm(F, axis=1).max()) if F.size else 1.0
    bound, vanish = oracle.embedding_bound(ref, fmax, sub.n_views,
                                           bf16_split=sub.feat_dtype == "bf16")
    nz = ref.den > 0
    cmp = nz & ~vanish & (den > 0)
    a, b = E[cmp].astype(np.float64), ref.E[cmp]
    err = np.linalg.norm(a - b, axis=1)
    na, nb_ = np.linalg.norm(a, axis=1), np.linalg.norm(b, axis=1)
    cos = np.sum(a * b, 1) / (na * nb_ + 1e-300)
    implied = bound[cmp] <= np.sqrt(2.0 * 1e-4) * nb_
    acc = dict(views=[int(v) for v in views], gaussians=int(nz.sum()),
               min_cos=float(cos.min()) if cos.size else None,
               frac_cos_ge_09999=float((cos >= 0.9999).mean()) if cos.size else None,
               max_abs_err=float(err.max()) if err.size else None,
               max_err_over_bound=float((err / bound[cmp]).max()) if err.size else None,
               median_bound=float(np.median(bound[cmp])) if err.size else None,
               frac_bound_implies_09999=float(implied.mean()) if cos.size else None,
               zero_rows_agree=bool(np.array_equal(den > 0, nz)),
               reference="FP64 oracle (per-pixel full depth sort, no tiles)")
    cpu = dict(value=len(views) / dt, unit="views/s", cores=oracle.max_threads(), kind="oracle",
               cpu_model=cpu_model(),
               sample=f"views {list(views)} of the {scene.n_views}-view workload (all "
                      f"{scene.n} Gaussians; per-view W_v in FP64 + contraction), {dt:.1f} s wall; "
                      f"the whole workload extrapolates linearly in views (the lift is additive "
                      f"over views) to {scene.n_views * dt / len(views):.0f} s",
               extrapolated_workload_s=round(scene.n_views * dt / len(views), 1))
    # the same oracle on one thread, whole 2,000-Gaussian workload (4 views of 64x64)
    from synthetic import make_scene
    small = make_scene("plain_fp32_2k")
    t0 = time.perf_counter()
    oracle.lift(small, nthreads=1)
    dt1 = time.perf_counter() - t0
    cpu["single_thread_plain_fp32_2k"] = dict(value=round(small.n_views / dt1, 3), unit="views/s",
                                              threads=1, seconds=round(dt1, 3))
    return acc, cpu


def codec_section(args, slag, torch, eval_scene, k, hidden, steps, train_recipe, train_over):
    """The learned codec: train on the plain lifts of three seeded scenes of
    the evaluation scene's recipe (GPU kernels), then time the plain and the
    codec lift of the evaluation scene (graph replays) and compare the
    codec's embeddings with the plain ones.  Besides the mean cosine, the
    weight-weighted mean (each Gaussian weighted by its total weight den) and
    the ceiling any k-dim code of this feature model faces: a segment's
    feature is its object's word plus noise spread over all D dimensions, and
    a code that carries words cannot carry that noise, so a Gaussian's best
    cosine is about |P E| / |E|, P the projection onto the span of the
    vocabulary (few segments: little averaging of the noise)."""
    from synthetic import make_scene, vocabulary_words
    from synthetic.codec_inputs import init_params
    d = eval_scene.dim
    t0 = time.perf_counter()
    L = slag.Lifter(0, flags=slag.SLAG_FLAG_GRAPH | slag.SLAG_FLAG_PROFILE | slag.SLAG_FLAG_AUTOTUNE)
    slag.slag_codec_init(L.ctx, d, hidden, k, slag.SLAG_BF16, init_params(d, hidden, k, seed=1040))
    seeds = (1041, 1042, 1043) if train_recipe != "stress_4m" else (1051, 1052, 1053)
    for sd in seeds:
        _log("codec: training scene", train_recipe, sd)
        sc = make_scene(train_recipe, seed=sd, **train_over)
        L.set_scene(sc, device_tensors=True)
        L.lift()
        slag.slag_codec_add_lift_rows(L.ctx, 100_000, sd)
        del sc
    nseg, nrows, nnz = slag.slag_codec_pool_size(L.ctx)
    t1 = time.perf_counter()
    hist = slag.slag_codec_train(L.ctx, steps=steps, batch_rows=8192, lr=1e-3)
    t2 = time.perf_counter()
    _log(f"codec: trained {steps} steps on {nrows} rows in {t2 - t1:.1f} s, "
         f"loss {hist[:5].mean():.4f} -> {hist[-20:].mean():.4f}")
    sc = eval_scene
    L.set_scene(sc, device_tensors=True)
    V = sc.n_views

    def timed(fn, reps):
        fn()
        fn()
        torch.cuda.synchronize()
        ms = 0.0
        for _ in range(reps):
            fn()
            ms += L.stats()["ms_total"]
        return ms / reps

    ms_plain = timed(L.lift, args.codec_reps)
    tuning = slag.slag_get_tuning(L.ctx)
    E_plain, den = L.embeddings()
    ms_codec = timed(L.lift_codec, args.codec_reps)
    E_codec, _ = L.embeddings()
    L.close()
    # the decode's share (eager, per-stage events): lift-to-codes = codec lift - decode
    with slag.Lifter(0, flags=slag.SLAG_FLAG_PROFILE) as Lp:
        slag.slag_codec_init(Lp.ctx, d, hidden, k, slag.SLAG_BF16, init_params(d, hidden, k, seed=1040))
        Lp.set_scene(sc, device_tensors=True)
        Lp.lift_codec()
        Lp.stats()
        Lp.lift_codec()
        st = Lp.stats()["ms_stage"]
    dec_ms = st.get("decode", 0.0)
    nz = den > 0
    a, b = E_plain[nz].astype(np.float64), E_codec[nz].astype(np.float64)
    na = np.linalg.norm(a, axis=1)
    cos = np.sum(a * b, 1) / (na * np.linalg.norm(b, axis=1) + 1e-300)
    Wd = vocabulary_words(d)
    Q, _ = np.linalg.qr(Wd.T)                     # orthonormal basis of the vocabulary's span
    ceil = np.linalg.norm(a @ Q, axis=1) / (na + 1e-300)
    wts = den[nz].astype(np.float64)
    out = dict(workload=sc.name, desc=DESC.get(sc.name, sc.name),
               k=k, hidden=hidden, precision="bf16",
               plain_views_per_s=round(V / (ms_plain * 1e-3), 2),
               codec_views_per_s=round(V / (ms_codec * 1e-3), 2),
               plain_ms=round(ms_plain, 3), codec_ms=round(ms_codec, 3),
               lift_to_codes_ms=round(ms_codec - dec_ms, 3), decode_ms=round(dec_ms, 3),
               speedup=round(ms_plain / ms_codec, 4),
               speedup_to_codes=round(ms_plain / max(ms_codec - dec_ms, 1e-9), 4),
               cos_mean=round(float(cos.mean()), 5), cos_p1=round(float(np.percentile(cos, 1)), 5),
               cos_median=round(float(np.median(cos)), 5),
               cos_mean_weight_weighted=round(float(np.sum(cos * wts) / np.sum(wts)), 5),
               cos_min=round(float(cos.min()), 5),
               frac_cos_ge_099=round(float((cos >= 0.99).mean()), 5),
               ceiling_mean=round(float(ceil.mean()), 5),
               ceiling_weight_weighted=round(float(np.sum(ceil * wts) / np.sum(wts)), 5),
               cos_over_ceiling_mean=round(float(np.mean(cos / np.maximum(ceil, 1e-12))), 5),
               tuning=tuning,
               train=dict(recipe=train_recipe, overrides=train_over, scenes=list(seeds), rows=nrows,
                          segments=nseg, weights=nnz, steps=steps, batch_rows=8192,
                          seconds=round(t2 - t1, 2), loss_first=round(float(hist[:5].mean()), 5),
                          loss_last=round(float(hist[-20:].mean()), 5),
                          setup_seconds=round(t1 - t0, 1)))
    _log("codec:", json.dumps(out))
    return out


def _round(d):
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(DESC))
    ap.add_argument("--cpu-views", type=int, default=4,
                    help="views of the workload the CPU oracle lifts (baseline + accuracy; 0 = skip)")
    ap.add_argument("--no-count", action="store_true", help="skip the counting lift")
    ap.add_argument("--eager", action="store_true", help="time eager lifts instead of graph replays")
    ap.add_argument("--no-secondary", action="store_true", help="skip the smaller workloads")
    ap.add_argument("--no-codec", action="store_true", help="skip the codec section")
    ap.add_argument("--no-search", action="store_true",
                    help="skip the search and render-back timings")
    ap.add_argument("--tile-size", type=int, default=16, choices=[8, 16],
                    help="binning and compositing tile edge of the timed lifts")
    ap.add_argument("--codec-steps", type=int, default=4000)
    ap.add_argument("--codec-k", type=int, default=16, help="code size (16, 32, 48 or 64)")
    ap.add_argument("--codec-hidden", type=int, default=256)
    ap.add_argument("--codec-reps", type=int, default=5)
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="also run one plain device copy of BYTES (read) + BYTES (write), "
                         "to scale hardware traffic counters")
    args = ap.parse_args()
    global TILE_SIZE
    TILE_SIZE = args.tile_size
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library lifts on a "
              "single GPU and does not shard across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "no GPU"
    import paper_2505_08124_amd as slag
    from synthetic import make_scene

    if args.copy_calib > 0:
        # elementwise kernel reading and writing exactly copy_calib bytes
        x = torch.ones(args.copy_calib // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        _log(f"copy calibration: {args.copy_calib} bytes read and written")
        del x, y

    wl = args.workload
    _log("generating scene", wl)
    t0 = time.perf_counter()
    scene = make_scene(wl)
    _log(f"generated in {time.perf_counter() - t0:.1f} s")
    V, N, D = scene.n_views, scene.n, scene.dim
    res, E_head, _ = measure(slag, torch, scene, args.steps, args.warmup, count=not args.no_count,
                        stage_steps=3 if scene.n >= 1_000_000 else args.steps, eager=args.eager)
    roof, kernels = kernel_rooflines(res, wl)

    accuracy = cpu = None
    if args.cpu_views > 0:
        k = min(args.cpu_views, V)
        views = sorted(set(int(round(i * (V - 1) / max(k - 1, 1))) for i in range(k)))
        _log(f"CPU oracle on views {views} (baseline and accuracy)")
        accuracy, cpu = accuracy_and_cpu(slag, scene, views, 0)
        _log("accuracy:", json.dumps(accuracy))

    search = render = None
    if not args.no_search:
        search, render = search_and_render(slag, torch, scene, E_head)
    del E_head

    codec_stress = None
    if not args.no_codec and wl == "stress_4m":
        codec_stress = codec_section(args, slag, torch, scene, 32, 256, args.codec_steps, "stress_4m",
                                     dict(n=1_000_000, views=dict(n=200)))
    del scene

    secondary = []
    uneven = None
    if not args.no_secondary:
        for w in ("plain_bf16_200k", "uneven_1m", "plain_fp32_2k"):
            if w == wl:
                continue
            _log("secondary workload", w)
            sc = make_scene(w)
            if w == "uneven_1m":
                uneven = sc
            r, _, _ = measure(slag, torch, sc, max(args.steps, 10), args.warmup,
                              stage_steps=5 if sc.n >= 1_000_000 else 10)
            ro, rk = kernel_rooflines(r, w)
            secondary.append(dict(
                workload=w, desc=DESC[w], n_gaussians=sc.n, n_views=sc.n_views,
                feature_dim=sc.dim, feature_dtype=sc.feat_dtype,
                views_per_s=round(r["views_per_s"], 2), ms_per_step=round(r["ms_step"], 4),
                contribs_per_s=round(r["contribs_per_s"], 1), n_contrib=r["n_contrib"],
                composite_frac=rk["k_composite"]["frac"] if "k_composite" in rk else None,
                contract_frac=rk["contraction"]["frac"] if "contraction" in rk else None,
                lift_roofline_frac=round(r["lift_roofline_frac"], 4),
                stage_ms={k: round(v, 4) for k, v in r["stage_ms"].items()},
                launches=r["n_batches"]))
            del sc

    codec = None
    if not args.no_codec:
        if uneven is None:
            uneven = make_scene("uneven_1m")
        codec = codec_section(args, slag, torch, uneven, args.codec_k, args.codec_hidden,
                              args.codec_steps, "codec_train", {})

    ms = res["ms_step"]
    out = {
        "metric": METRIC,
        "value": round(V / (ms * 1e-3), 2),
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if wl != "plain_fp32_2k" else "f32",
        "data": "synthetic",
        "config": {"workload": wl, "desc": DESC[wl], "n_gaussians": N, "n_views": V,
                   "feature_dim": D, "tile_size": TILE_SIZE, "parallelism": "single GPU"},
        "contribs_per_s": round(res["contribs_per_s"], 1) if "contribs_per_s" in res else None,
        "n_contrib": res.get("n_contrib"),
        "n_visible_pairs": res["n_visible_pairs"],
        "n_intersections": res["n_intersections"],
        "n_weights": res.get("n_weights"),
        "launches": res["n_batches"],
        "ms_per_step_hip_events": round(res["ms_hip_events"], 4),
        "launch": "eager" if args.eager else "hip graph replay",
        "upload_s": res["upload_s"],
        "tuning": res["tuning"],
        "stage_ms": {k: round(v, 4) for k, v in res["stage_ms"].items()},
        "roofline": roof,
        "kernel_roofline": kernels,
        "stage_roofline": res.get("stages"),
        "lift_roofline_frac": round(res["lift_roofline_frac"], 4) if "lift_roofline_frac" in res
        else None,
        "accuracy": accuracy,
        "secondary": secondary,
        "codec": codec,
        "codec_headline": codec_stress,
        "search": search,
        "render": render,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
