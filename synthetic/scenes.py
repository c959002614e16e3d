"""Seeded scene generator.

Every array is drawn from NumPy's PCG64 streams derived from one integer seed,
so a (config, seed, overrides) triple always yields identical bytes.

Conventions shared with the library's C interface:
  * Gaussians are given with *linear* scales and *activated* opacity; the
    log-normal scales and logistic opacities of the workload recipes are
    converted here in float64 and rounded once to float32.
  * Quaternions are (w, x, y, z), drawn uniformly on the unit 3-sphere.
  * Cameras follow the OpenCV axes (x right, y down, z forward); R, t map
    world to camera; the principal point is the image centre.
  * Segment ids are int32, row-major H x W, -1 marks background pixels.
  * Features are a [sum_v n_seg_v, D] table, view-major; BF16 tables are kept
    as uint16 bit patterns (round-to-nearest-even from float32).

The workload recipes (sizes and distributions) stand in for the paper's
scenes: a room-scale scene of about 2M Gaussians seen from ~250 views, and an
aerial scene of 38M Gaussians seen from 1657 views (Experiments section).
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional

import numpy as np
from scipy.spatial import cKDTree

camera_dtype = np.dtype([
    ("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"),
    ("R", "<f4", (9,)), ("t", "<f4", (3,)),
    ("width", "<i4"), ("height", "<i4"),
])
assert camera_dtype.itemsize == 72


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); return bits."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    means: np.ndarray        # [N,3] f32
    scales: np.ndarray       # [N,3] f32 (linear)
    quats: np.ndarray        # [N,4] f32 (w,x,y,z)
    opacity: np.ndarray      # [N]   f32 in (0,1)
    cams: np.ndarray         # [V] camera_dtype
    ids: List[np.ndarray]    # V x [H,W] int32
    nseg: np.ndarray         # [V] int32
    feat_dtype: str          # "f32" | "bf16"
    feats: np.ndarray        # [S,D] f32, or uint16 bf16 bits
    meta: Dict

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_views(self) -> int:
        return int(self.cams.shape[0])

    @property
    def dim(self) -> int:
        return int(self.feats.shape[1])

    @property
    def seg_offsets(self) -> np.ndarray:
        off = np.zeros(self.n_views + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.nseg.astype(np.int64))
        return off

    def feats_f64(self) -> np.ndarray:
        """Feature table widened exactly to float64."""
        if self.feat_dtype == "bf16":
            return bf16_bits_to_f32(self.feats).astype(np.float64)
        return self.feats.astype(np.float64)

    def pixels(self) -> int:
        return int(sum(int(c["width"]) * int(c["height"]) for c in self.cams))

    def subset_views(self, views) -> "Scene":
        """The same scene restricted to the given views (feature rows follow)."""
        views = [int(v) for v in views]
        off = self.seg_offsets
        rows = np.concatenate([np.arange(off[v], off[v + 1]) for v in views]) if views else \
            np.zeros(0, dtype=np.int64)
        return Scene(self.name + "[sub]", self.seed, self.means, self.scales, self.quats,
                     self.opacity, self.cams[views].copy(), [self.ids[v] for v in views],
                     self.nseg[views].copy(), self.feat_dtype,
                     np.ascontiguousarray(self.feats[rows]), dict(self.meta))


# ----------------------------------------------------------------------------
# cameras

def _look_at(pos, target, up=(0.0, 0.0, 1.0)):
    pos = np.asarray(pos, np.float64)
    f = np.asarray(target, np.float64) - pos
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    r = np.cross(f, up)
    if np.linalg.norm(r) < 1e-6:          # looking along the up axis
        r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])               # rows: x right, y down, z forward
    t = -R @ pos
    return R, t


def _camera(R, t, w, h, focal_ratio):
    c = np.zeros((), dtype=camera_dtype)
    c["fx"] = c["fy"] = focal_ratio * w
    c["cx"] = 0.5 * w
    c["cy"] = 0.5 * h
    c["R"] = np.asarray(R, np.float64).reshape(9).astype(np.float32)
    c["t"] = np.asarray(t, np.float64).astype(np.float32)
    c["width"] = w
    c["height"] = h
    return c


def _views_ring(n, radius, res, focal_ratio, rng):
    cams = []
    for i in range(n):
        a = 2.0 * math.pi * i / n
        R, t = _look_at((radius * math.cos(a), radius * math.sin(a), 0.0), (0, 0, 0))
        cams.append(_camera(R, t, res[0], res[1], focal_ratio))
    return cams


def _views_spiral(n, radius, res, focal_ratio, rng, turns=2.0, z0=-1.0, z1=1.0):
    cams = []
    for i in range(n):
        a = 2.0 * math.pi * turns * i / n
        z = z0 + (z1 - z0) * (i / max(n - 1, 1))
        R, t = _look_at((radius * math.cos(a), radius * math.sin(a), z), (0, 0, 0))
        cams.append(_camera(R, t, res[0], res[1], focal_ratio))
    return cams


def _views_fibonacci(n, radius, res_list, focal_ratio, rng):
    # resolution classes: n/len(res_list) views each, shuffled
    k = len(res_list)
    cls = np.repeat(np.arange(k), int(math.ceil(n / k)))[:n]
    cls = rng.permutation(cls)
    golden = math.pi * (3.0 - math.sqrt(5.0))
    cams = []
    for i in range(n):
        zc = 1.0 - 2.0 * (i + 0.5) / n
        rxy = math.sqrt(max(0.0, 1.0 - zc * zc))
        phi = golden * i
        pos = (radius * rxy * math.cos(phi), radius * rxy * math.sin(phi), radius * zc)
        R, t = _look_at(pos, (0, 0, 0))
        w, h = res_list[int(cls[i])]
        cams.append(_camera(R, t, w, h, focal_ratio))
    return cams


def _views_lawnmower(rows, cols, extent, height, res, focal_ratio, rng):
    cams = []
    ys = np.linspace(0.0, extent, rows + 2)[1:-1]
    xs = np.linspace(0.0, extent, cols + 2)[1:-1]
    for r, y in enumerate(ys):
        xx = xs if r % 2 == 0 else xs[::-1]
        for x in xx:
            pos = (x, y, height)
            R, t = _look_at(pos, (x, y, height - 1.0), up=(0.0, 1.0, 0.0))
            cams.append(_camera(R, t, res[0], res[1], focal_ratio))
    return cams


# ----------------------------------------------------------------------------
# Gaussians

def _random_rotations(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _rot_from_quat64(q):
    w, x, y, z = q.T
    return np.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=1).reshape(-1, 3, 3)


def _gaussians(rng, spec, n):
    kind = spec["kind"]
    labels = None
    if kind == "uniform":
        lo, hi = spec["lo"], spec["hi"]
        means = rng.uniform(lo, hi, size=(n, 3))
        centres = None
        sig = None
    elif kind == "clusters":
        k = spec["k"]
        lo = np.asarray(spec["centre_lo"], np.float64)
        hi = np.asarray(spec["centre_hi"], np.float64)
        centres = rng.uniform(lo, hi, size=(k, 3))
        sig = rng.uniform(spec["sigma"][0], spec["sigma"][1],
                          size=(k, 3) if spec.get("aniso", False) else (k, 1))
        sig = np.broadcast_to(sig, (k, 3))
        rots = _rot_from_quat64(_random_rotations(rng, k)) if spec.get("aniso", False) else \
            np.broadcast_to(np.eye(3), (k, 3, 3))
        labels = np.repeat(np.arange(k), int(math.ceil(n / k)))[:n]
        z = rng.standard_normal((n, 3)) * sig[labels]
        means = centres[labels] + np.einsum("nij,nj->ni", rots[labels], z)
    else:
        raise ValueError(kind)
    ls_mu, ls_sd = spec["log_scale"]
    scales = np.exp(rng.normal(ls_mu, ls_sd, size=(n, 3)))
    quats = _random_rotations(rng, n)
    op_mu, op_sd = spec["opacity_logit"]
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(op_mu, op_sd, size=n)))
    return (means.astype(np.float32), scales.astype(np.float32), quats.astype(np.float32),
            opacity.astype(np.float32), centres, labels, sig)


# ----------------------------------------------------------------------------
# segments

def _voronoi_seeds(rng, w, h, n_seg, bg_frac):
    """Seed points of a view's Voronoi cells (the extra background cells last)."""
    n_bg = int(round(n_seg * bg_frac / max(1e-9, 1.0 - bg_frac))) if bg_frac > 0 else 0
    return np.column_stack([rng.uniform(0, w, n_seg + n_bg), rng.uniform(0, h, n_seg + n_bg)])


def _voronoi_map(seeds, w, h, n_seg, workers=-1):
    """Cell of every pixel centre (ties to the lower seed); background cells -1."""
    tree = cKDTree(seeds)
    uu, vv = np.meshgrid(np.arange(w) + 0.5, np.arange(h) + 0.5)
    _, idx = tree.query(np.column_stack([uu.ravel(), vv.ravel()]), workers=workers)
    idx = idx.astype(np.int32).reshape(h, w)
    if seeds.shape[0] > n_seg:
        idx[idx >= n_seg] = -1
    return idx


def _voronoi_ids(rng, w, h, n_seg, bg_frac):
    seeds = _voronoi_seeds(rng, w, h, n_seg, bg_frac)
    return _voronoi_map(seeds, w, h, n_seg), seeds[:n_seg]


def _pixel_rays(cam):
    """Camera centre and unit world-space directions of every pixel centre's
    ray ([H, W, 3]), from the pinhole model (OpenCV axes)."""
    W, H = int(cam["width"]), int(cam["height"])
    R = cam["R"].astype(np.float64).reshape(3, 3)
    t = cam["t"].astype(np.float64)
    C = -R.T @ t
    u, v = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dc = np.stack([(u - float(cam["cx"])) / float(cam["fx"]), (v - float(cam["cy"])) / float(cam["fy"]),
                   np.ones_like(u)], axis=-1)
    d = dc @ R                      # R^T d_cam, row-wise
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return C, d


def _object_map_box(cam, centres, lo, hi):
    """Object under each pixel of a solid box of Gaussians partitioned into
    the Voronoi cells of `centres`: the cell of the point where the pixel's
    ray enters the box; -1 where the ray misses it.  No compositing."""
    C, d = _pixel_rays(cam)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - C) / d
        t2 = (hi - C) / d
    tn = np.nanmax(np.minimum(t1, t2), axis=-1)
    tf = np.nanmin(np.maximum(t1, t2), axis=-1)
    hit = (tn <= tf) & (tf > 0)
    tn = np.maximum(tn, 0.0)
    obj = np.full(hit.shape, -1, np.int64)
    if hit.any():
        pts = C + tn[hit][:, None] * d[hit]
        _, idx = cKDTree(centres).query(pts, workers=-1)
        obj[hit] = idx
    return obj


def _object_map_spheres(cam, centres, radii):
    """Object under each pixel of a scene of Gaussian clusters, each taken as
    a sphere around its centre: the first sphere the pixel's ray enters; -1
    where it enters none.  Each sphere is tested only inside the pixel box of
    its projection.  No compositing."""
    W, H = int(cam["width"]), int(cam["height"])
    C, d = _pixel_rays(cam)
    best = np.full((H, W), np.inf)
    obj = np.full((H, W), -1, np.int64)
    u, v, z = _project_points(cam, centres)
    f = max(float(cam["fx"]), float(cam["fy"]))
    for o in range(centres.shape[0]):
        r = radii[o]
        if z[o] + r <= 1e-3:
            continue                                    # behind the camera
        if z[o] - r > 1e-3:
            rp = f * r / (z[o] - r) + 2.0
            x0, x1 = int(max(0, np.floor(u[o] - rp))), int(min(W, np.ceil(u[o] + rp)))
            y0, y1 = int(max(0, np.floor(v[o] - rp))), int(min(H, np.ceil(v[o] + rp)))
            if x0 >= x1 or y0 >= y1:
                continue
        else:
            x0, x1, y0, y1 = 0, W, 0, H
        dd = d[y0:y1, x0:x1]
        oc = C - centres[o]
        b = dd @ oc
        disc = b * b - (oc @ oc - r * r)
        tt = -b - np.sqrt(np.maximum(disc, 0.0))
        hit = (disc >= 0) & (tt > 0) & (tt < best[y0:y1, x0:x1])
        best[y0:y1, x0:x1][hit] = tt[hit]
        obj[y0:y1, x0:x1][hit] = o
    return obj


def _segments_on_objects(cells, obj):
    """Segments = the (2D cell, object) parts of a view: each Voronoi cell
    split along the object boundaries; pixels without an object are
    background (-1).  Returns the id map and each segment's object."""
    key = cells.astype(np.int64) * (1 << 20) + obj
    valid = obj >= 0
    uk, inv = np.unique(key[valid], return_inverse=True)
    ids = np.full(cells.shape, -1, np.int32)
    ids[valid] = inv.astype(np.int32)
    return ids, (uk % (1 << 20)).astype(np.int64)


# ----------------------------------------------------------------------------
# features

def _unit_rows(x):
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def _project_points(cam, pts):
    R = cam["R"].astype(np.float64).reshape(3, 3)
    t = cam["t"].astype(np.float64)
    pc = pts @ R.T + t
    z = pc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam["fx"] * pc[:, 0] / z + cam["cx"]
        v = cam["fy"] * pc[:, 1] / z + cam["cy"]
    return u, v, z


def vocabulary_words(D: int, n_words: int = 64, seed: int = 7) -> np.ndarray:
    """The global unit words of the object-vocabulary feature model [n_words][D]
    (float64)."""
    return _unit_rows(np.random.default_rng(seed).standard_normal((n_words, D)))


def _features_of_objects(rng, spec, D, seg_obj, n_obj):
    """Object vocabulary: every object takes one of the global words (seed
    word_seed); a segment's feature is its object's word plus noise."""
    words = vocabulary_words(D, spec.get("n_words", 64), spec.get("word_seed", 7))
    obj_word = rng.integers(0, words.shape[0], size=n_obj) if n_obj > words.shape[0] else \
        rng.permutation(words.shape[0])[:n_obj]
    lab = np.concatenate(seg_obj) if seg_obj else np.zeros(0, np.int64)
    noise = rng.standard_normal((lab.size, D)) / math.sqrt(D)
    return _unit_rows(words[obj_word[lab]] + spec.get("noise", 0.25) * noise), lab


def _features(rng, spec, D, nseg, seeds_per_view, cams, obj_centres):
    model = spec["model"]
    S = int(nseg.sum())
    if model == "iid":
        return _unit_rows(rng.standard_normal((S, D))), None
    # object vocabulary: each segment takes the word of the object whose
    # projected centre lies nearest to the segment's seed point
    words = _unit_rows(np.random.default_rng(spec.get("word_seed", 7)).standard_normal(
        (spec.get("n_words", 64), D)))
    n_obj = obj_centres.shape[0]
    obj_word = rng.integers(0, words.shape[0], size=n_obj) if n_obj > words.shape[0] else \
        rng.permutation(words.shape[0])[:n_obj]
    rows, labels = [], []
    for v, cam in enumerate(cams):
        u, vv, z = _project_points(cam, obj_centres)
        front = z > 1e-3
        seeds = seeds_per_view[v]
        if front.any():
            d2 = (seeds[:, 0:1] - u[None, front]) ** 2 + (seeds[:, 1:2] - vv[None, front]) ** 2
            lab = np.flatnonzero(front)[np.argmin(d2, axis=1)]
        else:
            lab = np.zeros(seeds.shape[0], dtype=np.int64)
        noise = rng.standard_normal((seeds.shape[0], D)) / math.sqrt(D)
        rows.append(_unit_rows(words[obj_word[lab]] + spec.get("noise", 0.25) * noise))
        labels.append(lab)
    return np.concatenate(rows, axis=0), np.concatenate(labels)


# ----------------------------------------------------------------------------
# recipes

CONFIGS: Dict[str, Dict] = {
    # 2,000 Gaussians, 4 ring views 64x64, 8 Voronoi segments/view, D=64 FP32
    "plain_fp32_2k": dict(
        seed=101, n=2000,
        gauss=dict(kind="uniform", lo=-1.0, hi=1.0, log_scale=(-3.0, 0.3), opacity_logit=(0.0, 1.0)),
        views=dict(kind="ring", n=4, radius=3.0, res=(64, 64), focal_ratio=0.8),
        segments=dict(lo=8, hi=8, bg_frac=0.0),
        features=dict(D=64, dtype="f32", model="iid")),
    # 200k Gaussians in 20 anisotropic clusters, 100 spiral views 512x384,
    # 40-80 segments/view + ~10% background, D=512 BF16
    "plain_bf16_200k": dict(
        seed=102, n=200_000,
        gauss=dict(kind="clusters", k=20, centre_lo=(-1, -1, -1), centre_hi=(1, 1, 1),
                   sigma=(0.05, 0.3), aniso=True, log_scale=(-4.5, 0.5), opacity_logit=(0.0, 1.0)),
        views=dict(kind="spiral", n=100, radius=3.0, res=(512, 384), focal_ratio=0.8),
        segments=dict(lo=40, hi=80, bg_frac=0.1),
        features=dict(D=512, dtype="bf16", model="iid")),
    # 1M Gaussians, 300 views of three resolutions, 50-150 segments/view,
    # D=512 BF16 object-vocabulary features
    "uneven_1m": dict(
        seed=103, n=1_000_000,
        gauss=dict(kind="uniform", lo=-1.0, hi=1.0, log_scale=(-5.0, 0.6), opacity_logit=(0.5, 1.5)),
        views=dict(kind="fibonacci", n=300, radius=3.0,
                   res_list=[(320, 240), (640, 480), (1280, 960)], focal_ratio=0.8),
        segments=dict(lo=50, hi=150, bg_frac=0.0, kind="objects"),
        features=dict(D=512, dtype="bf16", model="vocab", n_objects=48)),
    # 4M Gaussians from 200 clusters over 10x10x3, 1000 nadir views 1024x768
    "stress_4m": dict(
        seed=105, n=4_000_000,
        gauss=dict(kind="clusters", k=200, centre_lo=(0, 0, -3), centre_hi=(10, 10, 0),
                   sigma=(0.1, 0.5), aniso=False, log_scale=(-5.0, 0.7), opacity_logit=(0.5, 1.5)),
        views=dict(kind="lawnmower", rows=25, cols=40, extent=10.0, height=2.0,
                   res=(1024, 768), focal_ratio=0.8),
        segments=dict(lo=100, hi=200, bg_frac=0.0, kind="objects"),
        features=dict(D=768, dtype="bf16", model="vocab", objects="clusters")),
}
CONFIGS["codec_train"] = dict(CONFIGS["uneven_1m"], seed=1041)


def _merge(base: Dict, over: Dict) -> Dict:
    out = dict(base)
    for k, v in over.items():
        if isinstance(v, dict) and isinstance(out.get(k), dict):
            out[k] = _merge(out[k], v)
        else:
            out[k] = v
    return out


def make_scene(name: str, seed: Optional[int] = None, **over) -> Scene:
    """Build a scene from a recipe name plus nested overrides.

    Example: ``make_scene("plain_bf16_200k", n=20000, views=dict(n=4))``.
    """
    spec = _merge(CONFIGS[name], over)
    seed = spec["seed"] if seed is None else int(seed)
    ss = np.random.SeedSequence(seed)
    r_gauss, r_view, r_seg, r_feat = [np.random.default_rng(s) for s in ss.spawn(4)]
    n = int(spec["n"])
    means, scales, quats, opacity, centres, labels, csig = _gaussians(r_gauss, spec["gauss"], n)

    vs = spec["views"]
    kind = vs["kind"]
    if kind == "ring":
        cams = _views_ring(vs["n"], vs["radius"], vs["res"], vs["focal_ratio"], r_view)
    elif kind == "spiral":
        cams = _views_spiral(vs["n"], vs["radius"], vs["res"], vs["focal_ratio"], r_view)
    elif kind == "fibonacci":
        cams = _views_fibonacci(vs["n"], vs["radius"], [tuple(r) for r in vs["res_list"]],
                                vs["focal_ratio"], r_view)
    elif kind == "lawnmower":
        cams = _views_lawnmower(vs["rows"], vs["cols"], vs["extent"], vs["height"], vs["res"],
                                vs["focal_ratio"], r_view)
        if "n" in vs:
            cams = cams[: vs["n"]]
    elif kind == "list":
        cams = [_camera(np.asarray(c["R"]).reshape(3, 3), c["t"], c["res"][0], c["res"][1],
                        c.get("focal_ratio", 0.8)) for c in vs["cams"]]
    else:
        raise ValueError(kind)
    cams = np.array(cams, dtype=camera_dtype)

    sg = spec["segments"]
    fs = spec["features"]
    D = int(fs["D"])
    obj = None
    if fs["model"] == "vocab":
        if fs.get("objects") == "clusters" and centres is not None:
            obj = centres
        else:
            obj = np.random.default_rng(seed + 7919).uniform(-1, 1, size=(fs.get("n_objects", 48), 3))
    # objects of the scene geometry (vocabulary model with per-pixel object
    # segments): cells of a solid box, or spheres of 2.2 sigma around the
    # cluster centres (about where a ray through a cluster becomes opaque)
    on_objects = fs["model"] == "vocab" and sg.get("kind", "voronoi") == "objects"
    # all random draws first, in view order; the per-pixel maps are then
    # built view by view on a thread pool (same bytes whatever the threads)
    draws = []
    for v, c in enumerate(cams):
        k = int(r_seg.integers(sg["lo"], sg["hi"] + 1))
        draws.append((k, _voronoi_seeds(r_seg, int(c["width"]), int(c["height"]), k,
                                        sg.get("bg_frac", 0.0))))

    def view_maps(v):
        c = cams[v]
        k, seeds = draws[v]
        m = _voronoi_map(seeds, int(c["width"]), int(c["height"]), k, workers=1)
        so = None
        if on_objects:
            if fs.get("objects") == "clusters" and centres is not None:
                om = _object_map_spheres(c, obj, 2.2 * csig[:, 0])
            else:
                om = _object_map_box(c, obj, spec["gauss"]["lo"], spec["gauss"]["hi"])
            m, so = _segments_on_objects(m, om)
        return m, so

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        maps = list(ex.map(view_maps, range(len(cams))))
    ids, seeds_pv, seg_obj = [], [], []
    nseg = np.zeros(len(cams), dtype=np.int32)
    for v in range(len(cams)):
        m, so = maps[v]
        ids.append(m)
        seeds_pv.append(draws[v][1][: draws[v][0]])
        if on_objects:
            seg_obj.append(so)
            nseg[v] = so.size
        else:
            nseg[v] = draws[v][0]

    if on_objects:
        F64, seg_labels = _features_of_objects(r_feat, fs, D, seg_obj, obj.shape[0])
    else:
        F64, seg_labels = _features(r_feat, fs, D, nseg, seeds_pv, cams, obj)
    F32 = F64.astype(np.float32)
    feats = f32_to_bf16_bits(F32) if fs["dtype"] == "bf16" else F32
    meta = dict(spec=spec, seg_labels=seg_labels, gauss_labels=labels)
    return Scene(name, seed, means, scales, quats, opacity, cams, ids, nseg, fs["dtype"],
                 np.ascontiguousarray(feats), meta)
