"""Plain FP64 CPU oracle for the loss-free embedding lift.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the GPU library (the two only read the same synthetic
scenes).

Split of work:
  * ``slag_oracle.c`` -- per view: projection, per-pixel depth-sorted walk,
    masking and the per-(Gaussian, segment) weight sums W_v (FP64), plus an
    FP32 evaluation of the integer decisions (depth order, culling, box).
  * this module -- the aggregation equation of the Method section:
    E_k = sum_i sum_j W_i[k, j] E_ij / sum_i sum_j W_i[k, j], computed as one
    sparse-times-dense product in FP64 (a library matmul), with E_k = 0 where
    the denominator is 0.
"""
from __future__ import annotations

import contextlib
import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slag_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the C half of the oracle with gcc (FP64, OpenMP, no contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
               "-fPIC", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Counts(ctypes.Structure):
    _fields_ = [("n_contrib", ctypes.c_int64), ("n_tests", ctypes.c_int64),
                ("n_visible", ctypes.c_int64), ("n_uncertain", ctypes.c_int64)]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.orc_lift_view.restype = P
        L.orc_lift_view.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, P, P, P, ctypes.POINTER(_Counts),
                                    ctypes.POINTER(ctypes.c_int64)]
        L.orc_view_fetch.argtypes = [P, P, P, P, P, P]
        L.orc_view_free.argtypes = [P]
        L.orc_mirror_view.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P]
        L.orc_project64_view.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_constants.argtypes = [P]
        L.orc_set_constants.restype = None
        L.orc_render_view.restype = ctypes.c_int32
        L.orc_render_view.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int32,
                                      ctypes.c_int32, P, P, P, P]
        _lib_handle = L
    return _lib_handle


CONSTANT_NAMES = ("alpha_max", "alpha_min", "t_min", "dilation", "near_z", "guard",
                  "weight_mode")


@contextlib.contextmanager
def constants(**kw):
    """Run the oracle with non-default rasterizer constants (the library's
    options of the same names; each given as the float the library receives,
    0 or absent = the 3D Gaussian splatting default; weight_mode = 1: kernel
    weights exp(-q/2) instead of alpha T), restoring the defaults
    afterwards."""
    bad = set(kw) - set(CONSTANT_NAMES)
    if bad:
        raise ValueError(f"unknown constants {sorted(bad)}")
    c = np.array([kw.get(k, 0.0) for k in CONSTANT_NAMES], np.float32)
    L = _lib()
    L.orc_set_constants(_p(c))
    try:
        yield
    finally:
        L.orc_set_constants(_p(np.zeros(len(CONSTANT_NAMES), np.float32)))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def max_threads() -> int:
    return int(_lib().orc_max_threads())


@dataclasses.dataclass
class ViewResult:
    g: np.ndarray          # int32 Gaussian index
    s: np.ndarray          # int32 view-local segment id
    w: np.ndarray          # float64 W_v[g, s]
    u: np.ndarray          # float64 decision mass for the triple (flips within the error bound)
    r: np.ndarray          # float64 rounding mass: bound on an FP32 walk's deviation from w
    n_contrib: int         # accepted blends (all pixels)
    n_tests: int           # box-candidate evaluations before termination
    n_visible: int
    n_uncertain: int       # decisions that lay inside their error band
    T: Optional[np.ndarray] = None      # [H, W] final transmittance
    wsum: Optional[np.ndarray] = None   # [H, W] sum of blend weights
    rho: Optional[np.ndarray] = None    # [H, W] bound on T's relative FP32 error (-1: a decision
                                        # of the pixel lay inside its band)


def lift_view(scene, v: int, mode: str = "box", pixels: bool = False,
              nthreads: int = 0, fp32: bool = False) -> ViewResult:
    """W_v for one view (paper: rasterize, mask, sum over the view's pixels).

    fp32=True runs the FP32 re-walk of the same per-pixel lists (test
    infrastructure for the error model; its r and u are zero)."""
    L = _lib()
    cam = np.ascontiguousarray(scene.cams[v:v + 1])
    ids = _c(scene.ids[v], np.int32)
    # one label per pixel ([H, W]) or several ([H, W, L]: overlapping masks,
    # -1 where a pixel lies in fewer)
    H, W = ids.shape[:2]
    nlab = ids.shape[2] if ids.ndim == 3 else 1
    T = np.empty((H, W), np.float64) if pixels else None
    ws = np.empty((H, W), np.float64) if pixels else None
    rho = np.empty((H, W), np.float64) if pixels else None
    cnt = _Counts()
    nt = ctypes.c_int64(0)
    means, scales = _c(scene.means, np.float32), _c(scene.scales, np.float32)
    quats, opac = _c(scene.quats, np.float32), _c(scene.opacity, np.float32)
    m = (0 if mode == "brute" else 1) | (2 if fp32 else 0)
    h = L.orc_lift_view(scene.n, _p(means), _p(scales), _p(quats), _p(opac), _p(cam), _p(ids),
                        nlab, m, int(nthreads), _p(T), _p(ws), _p(rho), ctypes.byref(cnt),
                        ctypes.byref(nt))
    if not h:
        raise MemoryError("oracle view lift failed")
    k = nt.value
    g = np.empty(k, np.int32)
    s = np.empty(k, np.int32)
    w = np.empty(k, np.float64)
    u = np.empty(k, np.float64)
    r = np.empty(k, np.float64)
    L.orc_view_fetch(h, _p(g), _p(s), _p(w), _p(u), _p(r))
    L.orc_view_free(h)
    return ViewResult(g, s, w, u, r, cnt.n_contrib, cnt.n_tests, cnt.n_visible, cnt.n_uncertain,
                      T, ws, rho)


@dataclasses.dataclass
class RenderResult:
    out: np.ndarray        # [H, W, C] float64 sum w a / sum w (0 where nothing blends)
    wsum: np.ndarray       # [H, W] float64 sum of the weights
    bw: np.ndarray         # [H, W] float64 bound on the FP32 weights' total deviation
    nb: np.ndarray         # [H, W] int32 contributions (taken or possibly taken)


def render_view(scene, v: int, attr: np.ndarray, nthreads: int = 0) -> RenderResult:
    """Render per-Gaussian attributes into view v with the lift's weights
    (Method, the rendering equation: the attributes alpha-composited front to
    back with the same alpha T (or kernel) weights the lift sums, normalised
    by their sum; no masking)."""
    L = _lib()
    a = _c(attr, np.float32)
    if a.ndim != 2 or a.shape[0] != scene.n:
        raise ValueError("attr must be [N, C]")
    C = a.shape[1]
    cam = np.ascontiguousarray(scene.cams[v:v + 1])
    H, W = int(cam["height"][0]), int(cam["width"][0])
    out = np.empty((H, W, C), np.float64)
    ws = np.empty((H, W), np.float64)
    bw = np.empty((H, W), np.float64)
    nb = np.empty((H, W), np.int32)
    means, scales = _c(scene.means, np.float32), _c(scene.scales, np.float32)
    quats, opac = _c(scene.quats, np.float32), _c(scene.opacity, np.float32)
    if L.orc_render_view(scene.n, _p(means), _p(scales), _p(quats), _p(opac), _p(cam), _p(a), C,
                         int(nthreads), _p(out), _p(ws), _p(bw), _p(nb)) != 0:
        raise MemoryError("oracle render failed")
    return RenderResult(out, ws, bw, nb)


def render_bound(rr: RenderResult, amax: np.ndarray) -> np.ndarray:
    """Bound on |out_fp32 - out| per pixel and channel for a front-to-back
    FP32 accumulation of w a and w (one rounding per term) followed by one
    reciprocal and one product.  amax [C]: max |attr| per channel.  With
    eD = Bw + m u (D + Bw) and eN = amax (Bw + m u (D + Bw)), m = nb + 1:
      |N'/D' - N/D| <= (eN + |out| eD) / (D - eD)   (+ 4 u of the result);
    inf where D <= eD (nothing certain blends at the pixel)."""
    u = 2.0 ** -24
    D = rr.wsum[..., None]
    Bw = rr.bw[..., None]
    m = rr.nb[..., None].astype(np.float64) + 1.0
    eD = Bw + m * u * (D + Bw)
    eN = np.asarray(amax, np.float64)[None, None, :] * eD
    o = np.abs(rr.out)
    with np.errstate(divide="ignore", invalid="ignore"):
        b = np.where(D > eD, (eN + o * eD) / (D - eD), np.inf)
    return b + 4.0 * u * (o + b)


@dataclasses.dataclass
class LiftResult:
    num: np.ndarray        # [N, D] float64
    den: np.ndarray        # [N] float64
    E: np.ndarray          # [N, D] float64, 0 where den == 0
    U: np.ndarray          # [N] float64 decision mass per Gaussian
    R: np.ndarray          # [N] float64 rounding mass per Gaussian
    B: np.ndarray          # [N] float64 bound on |W| deviations (rounding + decisions + sums)
    nnz: np.ndarray        # [N] int64 (view, segment) terms per Gaussian
    views: List[ViewResult]
    n_contrib: int
    n_tests: int


def weight_matrix(scene, views: List[int], results: List[ViewResult], field: str = "w"):
    """Stack the per-view triples into one sparse [N, S_total] matrix."""
    off = scene.seg_offsets
    rows, cols, vals = [], [], []
    for v, r in zip(views, results):
        rows.append(r.g.astype(np.int64))
        cols.append(off[v] + r.s.astype(np.int64))
        vals.append(getattr(r, field) if field != "bound" else weight_bound(r.w, r.u, r.r))
    if rows:
        rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    else:
        rows = cols = np.zeros(0, np.int64)
        vals = np.zeros(0, np.float64)
    return sp.csr_matrix((vals, (rows, cols)), shape=(scene.n, int(off[-1])))


# Summation in the GPU path: a (pair, tile, segment) sum adds up to 256 pixel
# weights through a 6-level wave tree and 3 cross-wave adds in FP32 (at most
# 9 roundings of the running sum), and is accumulated in fixed point with 2^-40
# truncation per entry (at most 2^10 tile entries per triple).
SUM_REL = 16 * 2.0 ** -24
SUM_ABS = 2.0 ** -30


def weight_bound(w, u, r):
    """Bound on |W_fp32 - W_fp64| for one triple: rounding mass, decision mass
    (with its own rounding) and the summation of the per-pixel weights."""
    return r + u * (1.0 + 2.0 ** -20) + SUM_REL * w + SUM_ABS


def lift(scene, views: Optional[List[int]] = None, mode: str = "box",
         nthreads: int = 0, pixels: bool = False) -> LiftResult:
    """The lifted embeddings of the aggregation equation, in FP64."""
    views = list(range(scene.n_views)) if views is None else [int(v) for v in views]
    res = [lift_view(scene, v, mode=mode, nthreads=nthreads, pixels=pixels) for v in views]
    Wm = weight_matrix(scene, views, res)
    F = scene.feats_f64()
    num = np.asarray(Wm @ F)
    den = np.asarray(Wm.sum(axis=1)).ravel()
    E = np.zeros_like(num)
    nz = den > 0
    E[nz] = num[nz] / den[nz, None]
    U = np.asarray(weight_matrix(scene, views, res, "u").sum(axis=1)).ravel()
    R = np.asarray(weight_matrix(scene, views, res, "r").sum(axis=1)).ravel()
    Bm = weight_matrix(scene, views, res, "bound")
    B = np.asarray(Bm.sum(axis=1)).ravel()
    nnz = np.diff(Bm.indptr).astype(np.int64)
    return LiftResult(num, den, E, U, R, B, nnz, res, sum(r.n_contrib for r in res),
                      sum(r.n_tests for r in res))


def embedding_bound(ref: LiftResult, fmax: float, n_views: int, bf16_split: bool = True):
    """Per-Gaussian bound on ||E_fp32 - E_fp64||_2 (0 where den = 0), and the
    mask of Gaussians whose weight could vanish (den <= B).

    With W perturbed by dW (|dW_s| <= b_s, sum b_s = B): E' - E =
    sum_s dW_s (F_s - E) / (den + sum dW), and ||F_s - E|| <= fmax + ||E||
    (triangle inequality), so ||E' - E|| <= (fmax + ||E||) B / (den - B).
    The contraction adds the hi/lo split of W (2^-18 relative), FP32
    accumulation of the products (at most nnz + 64 roundings of partial sums
    bounded by fmax den) and the per-view FP32 sums of den (n_views
    roundings); the division adds one rounding."""
    u = 2.0 ** -24
    den, B = ref.den, ref.B
    ok = den > B
    out = np.zeros_like(den)
    split = 2.0 ** -18 if bf16_split else 0.0
    d = np.where(ok, den - B, 1.0)
    e_w = (fmax + np.linalg.norm(ref.E, axis=1)) * B / d
    e_c = fmax * (split + (ref.nnz + 64 + n_views) * u) * den / d
    out[ok] = (e_w + e_c)[ok] + u * np.linalg.norm(ref.E[ok], axis=1)
    return out, ~ok & (den > 0)


# ----------------------------------------------------------------------------
# FP32 decisions: visibility, depth keys, tile membership

@dataclasses.dataclass
class MirrorView:
    vis: np.ndarray     # uint8: 1 visible, 2 in front but off-screen, 0 culled
    z32: np.ndarray     # float32 camera depth
    box: np.ndarray     # int32 [N, 4] pixel box x0, x1, y0, y1 (valid where vis == 1)
    mu: np.ndarray      # float32 [N, 2]
    cov: np.ndarray     # float32 [N, 3]


def mirror_view(scene, v: int) -> MirrorView:
    L = _lib()
    n = scene.n
    cam = np.ascontiguousarray(scene.cams[v:v + 1])
    vis = np.zeros(n, np.uint8)
    z = np.zeros(n, np.float32)
    box = np.zeros((n, 4), np.int32)
    mu = np.zeros((n, 2), np.float32)
    cov = np.zeros((n, 3), np.float32)
    L.orc_mirror_view(n, _p(_c(scene.means, np.float32)), _p(_c(scene.scales, np.float32)),
                      _p(_c(scene.quats, np.float32)), _p(cam), _p(vis), _p(z), _p(box),
                      _p(mu), _p(cov))
    return MirrorView(vis, z, box, mu, cov)


def project64_view(scene, v: int):
    """FP64 screen mean, covariance (with dilation), conic and camera depth."""
    L = _lib()
    n = scene.n
    cam = np.ascontiguousarray(scene.cams[v:v + 1])
    mu = np.zeros((n, 2))
    cov = np.zeros((n, 3))
    con = np.zeros((n, 3))
    zc = np.zeros(n)
    L.orc_project64_view(n, _p(_c(scene.means, np.float32)), _p(_c(scene.scales, np.float32)),
                         _p(_c(scene.quats, np.float32)), _p(_c(scene.opacity, np.float32)),
                         _p(cam), _p(mu), _p(cov), _p(con), _p(zc))
    return mu, cov, con, zc


def sorted_keys(scene, v: int, tile_w: int, tile_h: int, mv: Optional[MirrorView] = None):
    """Reference tile lists of one view: (tile, depth bits, Gaussian) rows in
    the order a front-to-back tile rasterizer must visit them -- ascending tile
    (row-major tile index), then ascending FP32 depth, then Gaussian index."""
    mv = mirror_view(scene, v) if mv is None else mv
    W = int(scene.cams[v]["width"])
    ntx = (W + tile_w - 1) // tile_w
    g = np.flatnonzero(mv.vis == 1)
    b = mv.box[g]
    tx0, tx1 = b[:, 0] // tile_w, b[:, 1] // tile_w
    ty0, ty1 = b[:, 2] // tile_h, b[:, 3] // tile_h
    cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
    tot = int(cnt.sum())
    gi = np.repeat(g, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    k = np.arange(tot) - start
    w = np.repeat(tx1 - tx0 + 1, cnt)
    tx = np.repeat(tx0, cnt) + k % w
    ty = np.repeat(ty0, cnt) + k // w
    tile = (ty * ntx + tx).astype(np.int64)
    zb = mv.z32[gi].view(np.uint32).astype(np.int64)
    order = np.lexsort((gi, zb, tile))
    return tile[order], zb[order].astype(np.uint32), gi[order].astype(np.int32)
