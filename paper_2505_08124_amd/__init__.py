"""MI355X (gfx950) lift of per-view segment embeddings into per-Gaussian embeddings.

Thin ctypes binding of ``include/slag.h``: the functions below carry the C
names and only marshal arguments; every step of the lift runs in the HIP
library ``lib/libslag.so``.  There is no fallback: if the library is missing
or no GPU is present, calls raise.

Arrays may be NumPy arrays (host memory) or torch tensors on a GPU (device
memory, passed by pointer); PyTorch only provides device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libslag.so")

SLAG_OK, SLAG_E_INVALID_ARG, SLAG_E_OUT_OF_MEMORY, SLAG_E_DEVICE, SLAG_E_STATE, \
    SLAG_E_CAPACITY, SLAG_E_NOT_SUPPORTED = range(7)
SLAG_HOST, SLAG_DEVICE = 0, 1
SLAG_QUERY_SCRATCH_BYTES = 128 << 20      # include/slag_query.h
SLAG_F32, SLAG_BF16 = 0, 1
SLAG_FLAG_PROFILE, SLAG_FLAG_COUNT, SLAG_FLAG_KEEP_DEBUG, SLAG_FLAG_GRAPH, SLAG_FLAG_AUTOTUNE = \
    1, 2, 4, 8, 16
SLAG_DEBUG_KEYS, SLAG_DEBUG_TILE_RANGES, SLAG_DEBUG_W_VIEW, SLAG_DEBUG_PIXEL_T_FINAL, \
    SLAG_DEBUG_PIXEL_WSUM, SLAG_DEBUG_PIXEL_COUNT, SLAG_DEBUG_COUNTERS = range(7)

STATUS_NAMES = {0: "SLAG_OK", 1: "SLAG_E_INVALID_ARG", 2: "SLAG_E_OUT_OF_MEMORY",
                3: "SLAG_E_DEVICE", 4: "SLAG_E_STATE", 5: "SLAG_E_CAPACITY",
                6: "SLAG_E_NOT_SUPPORTED"}


class slag_camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class slag_options(ctypes.Structure):
    _fields_ = [("max_views_per_launch", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("max_launch_entries", ctypes.c_int64),
                ("alpha_max", ctypes.c_float), ("alpha_min", ctypes.c_float),
                ("t_min", ctypes.c_float), ("dilation", ctypes.c_float),
                ("near_z", ctypes.c_float), ("guard", ctypes.c_float),
                ("tile_size", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("labels_per_pixel", ctypes.c_int32), ("weight_mode", ctypes.c_int32),
                ("composite_variant", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class slag_stats(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int64), ("n_batches", ctypes.c_int64),
                ("n_visible_pairs", ctypes.c_int64), ("n_intersections", ctypes.c_int64),
                ("n_part_slots", ctypes.c_int64), ("n_weights", ctypes.c_int64),
                ("n_contrib", ctypes.c_int64), ("n_tests", ctypes.c_int64),
                ("n_tile_tests", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("ms_stage", ctypes.c_double * 16), ("n_stages", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_lost", ctypes.c_int64)]


class slag_tuning(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("n_variants", ctypes.c_int32), ("ms", ctypes.c_float * 8)]


class slag_train_cfg(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch_rows", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("reserved", ctypes.c_int64 * 4)]


EXPORTS = ["slag_create", "slag_destroy", "slag_last_error", "slag_set_gaussians",
           "slag_set_cameras", "slag_set_segments", "slag_set_features", "slag_lift",
           "slag_get_embeddings", "slag_get_stats", "slag_stage_name", "slag_debug_tile_lists",
           "slag_debug_weights", "slag_get_tuning", "slag_variant_name", "slag_get_debug",
           "slag_variant_count",
           # include/slag_codec.h
           "slag_codec_init", "slag_codec_get_params", "slag_codec_clear_pool",
           "slag_codec_set_pool", "slag_codec_add_lift_rows", "slag_codec_pool_size",
           "slag_codec_loss_grad", "slag_codec_train", "slag_lift_codec", "slag_get_codes",
           # include/slag_query.h
           "slag_query", "slag_classify", "slag_query_static", "slag_lift_chunked",
           "slag_set_segments_multi", "slag_render"]

_lib_handle = None


def lib():
    """Load libslag.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2505_08124_amd.build "
                           "(there is no non-HIP fallback)")
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7 and
    # the dynamic loader serves that soname from whichever copy loads first.
    # Load PyTorch's first (when installed) so that tensors handed to the
    # library and the library's own calls share it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.slag_create.argtypes = [I32, P, ctypes.POINTER(slag_options), ctypes.POINTER(P)]
    L.slag_destroy.argtypes = [P]
    L.slag_destroy.restype = None
    L.slag_last_error.argtypes = [P]
    L.slag_last_error.restype = ctypes.c_char_p
    L.slag_set_gaussians.argtypes = [P, I64, P, P, P, P, I32]
    L.slag_set_cameras.argtypes = [P, I32, P]
    L.slag_set_segments.argtypes = [P, I32, P, I32, I32]
    L.slag_set_segments_multi.argtypes = [P, I32, P, I32, I32, I32]
    L.slag_set_features.argtypes = [P, I32, I32, P, I32]
    L.slag_lift.argtypes = [P]
    L.slag_lift_chunked.argtypes = [P, I64, P, I32, P]
    L.slag_render.argtypes = [P, I32, P, I32, I32, P, P, I32]
    L.slag_get_embeddings.argtypes = [P, P, I32, P, I32]
    L.slag_get_debug.argtypes = [P, I32, I32, P, I64, ctypes.POINTER(I64)]
    L.slag_get_stats.argtypes = [P, ctypes.POINTER(slag_stats)]
    L.slag_stage_name.argtypes = [I32]
    L.slag_stage_name.restype = ctypes.c_char_p
    L.slag_debug_tile_lists.argtypes = [P, I32, P, P, P, I64, ctypes.POINTER(I64)]
    L.slag_debug_weights.argtypes = [P, I32, P, P, P, I64, ctypes.POINTER(I64)]
    L.slag_get_tuning.argtypes = [P, ctypes.POINTER(slag_tuning), I32, ctypes.POINTER(I32)]
    L.slag_variant_name.argtypes = [I32]
    L.slag_variant_count.argtypes = []
    L.slag_variant_name.restype = ctypes.c_char_p
    L.slag_codec_init.argtypes = [P, I32, I32, I32, I32, P, I32]
    L.slag_codec_get_params.argtypes = [P, P, I32]
    L.slag_codec_clear_pool.argtypes = [P]
    L.slag_codec_set_pool.argtypes = [P, I64, P, I64, P, P, P, P, I32]
    L.slag_codec_add_lift_rows.argtypes = [P, I64, ctypes.c_uint64, ctypes.POINTER(I64)]
    L.slag_codec_pool_size.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                       ctypes.POINTER(I64)]
    L.slag_codec_loss_grad.argtypes = [P, I64, I64, ctypes.POINTER(ctypes.c_float), P, I32]
    L.slag_codec_train.argtypes = [P, ctypes.POINTER(slag_train_cfg), P]
    L.slag_lift_codec.argtypes = [P]
    L.slag_get_codes.argtypes = [P, P, I32]
    L.slag_query.argtypes = [P, I64, I32, P, I32, I32, P, I32, ctypes.c_float, I32,
                             ctypes.POINTER(I64), P, P, I32]
    L.slag_classify.argtypes = [P, I64, I32, P, I32, I32, P, I32, P, P, I32]
    L.slag_query_static.argtypes = L.slag_query.argtypes
    for f in EXPORTS:
        if f not in ("slag_destroy", "slag_last_error", "slag_stage_name", "slag_variant_name"):
            getattr(L, f).restype = I32
    _lib_handle = L
    return L


class SlagError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(ctx, st):
    if st != SLAG_OK:
        m = lib().slag_last_error(ctx)
        raise SlagError(st, m.decode() if m else "")


def _ptr(a):
    """(pointer, where) of a NumPy array or a GPU torch tensor; keeps no copy."""
    if a is None:
        return None, SLAG_HOST
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), (SLAG_DEVICE if a.is_cuda else SLAG_HOST)
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return a.ctypes.data_as(ctypes.c_void_p), SLAG_HOST


# ---------------------------------------------------------------- C names

def slag_create(device: int = 0, stream=None, max_views_per_launch: int = 0, flags: int = 0,
                max_launch_entries: int = 0, **constants):
    """constants: alpha_max, alpha_min, t_min, dilation, near_z, guard (floats),
    tile_size, deterministic, labels_per_pixel, weight_mode, composite_variant (ints);
    absent = default."""
    o = slag_options(max_views_per_launch, flags, max_launch_entries)
    for k, v in constants.items():
        if k not in ("alpha_max", "alpha_min", "t_min", "dilation", "near_z", "guard",
                     "tile_size", "deterministic", "labels_per_pixel", "weight_mode",
                     "composite_variant"):
            raise ValueError(f"unknown option {k}")
        setattr(o, k, v)
    h = ctypes.c_void_p()
    st = lib().slag_create(device, ctypes.c_void_p(stream) if stream else None, ctypes.byref(o),
                           ctypes.byref(h))
    if st != SLAG_OK:
        raise SlagError(st, "slag_create failed")
    return h


def slag_destroy(ctx):
    lib().slag_destroy(ctx)


def slag_set_gaussians(ctx, means, scales, quats, opacity):
    n = int(means.shape[0])
    pm, w = _ptr(means)
    ps, _ = _ptr(scales)
    pq, _ = _ptr(quats)
    po, _ = _ptr(opacity)
    _check(ctx, lib().slag_set_gaussians(ctx, n, pm, ps, pq, po, w))


def slag_set_cameras(ctx, cams: np.ndarray):
    cams = np.ascontiguousarray(cams)
    assert cams.dtype.itemsize == ctypes.sizeof(slag_camera)
    _check(ctx, lib().slag_set_cameras(ctx, int(cams.shape[0]), cams.ctypes.data_as(ctypes.c_void_p)))


def slag_set_segments(ctx, view: int, ids, n_seg: int):
    p, w = _ptr(ids)
    _check(ctx, lib().slag_set_segments(ctx, int(view), p, int(n_seg), w))


def slag_set_segments_multi(ctx, view: int, ids, n_seg: int):
    """ids [H][W][L]: the masks containing each pixel, -1 for unused entries."""
    p, w = _ptr(ids)
    _check(ctx, lib().slag_set_segments_multi(ctx, int(view), p, int(ids.shape[2]), int(n_seg), w))


def slag_set_features(ctx, table, dtype: int):
    p, w = _ptr(table)
    _check(ctx, lib().slag_set_features(ctx, int(table.shape[1]), int(dtype), p, w))


def slag_lift_chunked(ctx, chunk_rows: int, out, den=None):
    """Lift with the output streamed to host arrays out [N][d] (float32, or
    uint16 BF16 bits) and den [N] (float32), chunk_rows Gaussians at a time."""
    po, _ = _ptr(out)
    pd, _ = _ptr(den)
    dt = SLAG_BF16 if (out is not None and out.dtype == np.uint16) else SLAG_F32
    _check(ctx, lib().slag_lift_chunked(ctx, int(chunk_rows), po, dt, pd))


def slag_lift(ctx):
    _check(ctx, lib().slag_lift(ctx))


def slag_render(ctx, view: int, attr, out, wsum=None):
    """Render attr [N][C] (float32 array or tensor) into view `view`:
    out [H][W][C] and wsum [H][W] (float32, both host arrays or both GPU
    tensors; wsum may be None)."""
    pa, wa = _ptr(attr)
    po, wo = _ptr(out)
    pw, ww = _ptr(wsum)
    if wsum is not None and ww != wo:
        raise ValueError("out and wsum must be in the same memory")
    C = int(attr.shape[1]) if attr is not None and len(attr.shape) == 2 else 0
    if out is None or tuple(out.shape[2:]) != (C,):
        raise ValueError("out must be [H][W][C] with C = attr.shape[1]")
    _check(ctx, lib().slag_render(ctx, int(view), pa, C, wa, po, pw, wo))


def _dtype_of(a) -> int:
    """SLAG_F32 for float32 arrays/tensors, SLAG_BF16 for torch.bfloat16 tensors
    or uint16 arrays of bfloat16 bit patterns."""
    name = str(getattr(a, "dtype", ""))
    if name in ("float32", "torch.float32"):
        return SLAG_F32
    if name in ("uint16", "torch.bfloat16", "torch.uint16", "torch.int16"):
        return SLAG_BF16
    raise ValueError(f"unsupported output dtype {name}")


def slag_get_embeddings(ctx, out, den=None):
    p, w = _ptr(out)
    pd, wd = _ptr(den)
    if out is not None and den is not None and w != wd:
        raise ValueError("out and den must be in the same memory")
    dt = _dtype_of(out) if out is not None else SLAG_F32
    _check(ctx, lib().slag_get_embeddings(ctx, p, dt, pd, w if out is not None else wd))


_DEBUG_DTYPE = {SLAG_DEBUG_KEYS: (np.uint32, 3), SLAG_DEBUG_TILE_RANGES: (np.uint32, 2),
                SLAG_DEBUG_W_VIEW: (np.uint32, 3), SLAG_DEBUG_PIXEL_T_FINAL: (np.float32, 0),
                SLAG_DEBUG_PIXEL_WSUM: (np.float32, 0), SLAG_DEBUG_PIXEL_COUNT: (np.uint32, 0),
                SLAG_DEBUG_COUNTERS: (np.int64, 1)}


def slag_get_debug(ctx, what: int, view: int = 0) -> np.ndarray:
    """One debug export as a NumPy array (rows per the layout in slag.h;
    per-pixel exports come back as [H, W])."""
    n = ctypes.c_int64(0)
    _check(ctx, lib().slag_get_debug(ctx, int(what), int(view), None, 0, ctypes.byref(n)))
    buf = np.empty(max(n.value, 1), np.uint8)
    _check(ctx, lib().slag_get_debug(ctx, int(what), int(view), _ptr(buf)[0], n.value,
                                     ctypes.byref(n)))
    dt, cols = _DEBUG_DTYPE[int(what)]
    a = buf[:n.value].view(dt)
    return a.reshape(-1, cols) if cols > 1 else a


def slag_get_stats(ctx) -> dict:
    s = slag_stats()
    _check(ctx, lib().slag_get_stats(ctx, ctypes.byref(s)))
    d = {f: getattr(s, f) for f, _ in slag_stats._fields_ if f not in ("ms_stage", "reserved")}
    d["ms_stage"] = {lib().slag_stage_name(i).decode(): s.ms_stage[i] for i in range(s.n_stages)}
    return d


def slag_get_tuning(ctx) -> list:
    n = ctypes.c_int32(0)
    _check(ctx, lib().slag_get_tuning(ctx, None, 0, ctypes.byref(n)))
    arr = (slag_tuning * max(n.value, 1))()
    _check(ctx, lib().slag_get_tuning(ctx, arr, n.value, ctypes.byref(n)))
    out = []
    for t in arr[:n.value]:
        out.append(dict(width=t.width, height=t.height, variant=t.variant,
                        name=lib().slag_variant_name(t.variant).decode(),
                        ms=[round(t.ms[i], 4) for i in range(t.n_variants)]))
    return out


def slag_variant_count() -> int:
    return int(lib().slag_variant_count())


def slag_debug_tile_lists(ctx, view: int):
    n = ctypes.c_int64(0)
    _check(ctx, lib().slag_debug_tile_lists(ctx, view, None, None, None, 0, ctypes.byref(n)))
    t = np.empty(n.value, np.uint32)
    z = np.empty(n.value, np.uint32)
    g = np.empty(n.value, np.uint32)
    _check(ctx, lib().slag_debug_tile_lists(ctx, view, _ptr(t)[0], _ptr(z)[0], _ptr(g)[0], n.value,
                                            ctypes.byref(n)))
    return t, z, g


def slag_debug_weights(ctx, view: int):
    n = ctypes.c_int64(0)
    _check(ctx, lib().slag_debug_weights(ctx, view, None, None, None, 0, ctypes.byref(n)))
    g = np.empty(n.value, np.uint32)
    s = np.empty(n.value, np.uint32)
    w = np.empty(n.value, np.float32)
    _check(ctx, lib().slag_debug_weights(ctx, view, _ptr(g)[0], _ptr(s)[0], _ptr(w)[0], n.value,
                                         ctypes.byref(n)))
    return g, s, w


# ---------------------------------------------------------------- codec (slag_codec.h)

def codec_param_count(d: int, hidden: int, k: int) -> int:
    return hidden * d + hidden + k * hidden + k + hidden * k + hidden + d * hidden + d


def slag_codec_init(ctx, d: int, hidden: int, k: int, precision: int, params):
    p, w = _ptr(params)
    _check(ctx, lib().slag_codec_init(ctx, d, hidden, k, precision, p, w))


def slag_codec_get_params(ctx, out):
    p, w = _ptr(out)
    _check(ctx, lib().slag_codec_get_params(ctx, p, w))


def slag_codec_clear_pool(ctx):
    _check(ctx, lib().slag_codec_clear_pool(ctx))


def slag_codec_set_pool(ctx, feats, row_ptr, col, w, target):
    pf, where = _ptr(feats)
    _check(ctx, lib().slag_codec_set_pool(ctx, int(feats.shape[0]), pf, int(target.shape[0]),
                                          _ptr(row_ptr)[0], _ptr(col)[0], _ptr(w)[0],
                                          _ptr(target)[0], where))


def slag_codec_add_lift_rows(ctx, max_rows: int, seed: int) -> int:
    added = ctypes.c_int64(0)
    _check(ctx, lib().slag_codec_add_lift_rows(ctx, int(max_rows), int(seed), ctypes.byref(added)))
    return added.value


def slag_codec_pool_size(ctx):
    a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(ctx, lib().slag_codec_pool_size(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def slag_codec_loss_grad(ctx, row0: int, n_rows: int, grad=None) -> float:
    loss = ctypes.c_float(0.0)
    pg, w = _ptr(grad)
    _check(ctx, lib().slag_codec_loss_grad(ctx, int(row0), int(n_rows), ctypes.byref(loss), pg, w))
    return loss.value


def slag_codec_train(ctx, steps: int, batch_rows: int = 0, lr: float = 1e-3, beta1: float = 0.9,
                     beta2: float = 0.999, eps: float = 1e-8) -> np.ndarray:
    cfg = slag_train_cfg(int(steps), int(batch_rows), lr, beta1, beta2, eps)
    hist = np.zeros(max(int(steps), 1), np.float32)
    _check(ctx, lib().slag_codec_train(ctx, ctypes.byref(cfg), hist.ctypes.data_as(ctypes.c_void_p)))
    return hist[:steps]


def slag_lift_codec(ctx):
    _check(ctx, lib().slag_lift_codec(ctx))


def slag_get_codes(ctx, out):
    p, w = _ptr(out)
    _check(ctx, lib().slag_get_codes(ctx, p, w))


def slag_query(ctx, emb, queries, threshold: float = 0.0, k: int = 0, out=None,
               static: bool = False):
    """Cosine-similarity search: returns (count[Q], top_idx[Q][k], top_cos[Q][k]).
    emb [n][d] and queries [Q][d]: float32 NumPy arrays or CUDA tensors.  The
    top-k rows go to `out` = (idx, cos) when given (NumPy or CUDA tensors),
    else to new NumPy arrays.  static=True calls slag_query_static (no
    device allocation; emb must be a CUDA tensor)."""
    n, d = int(emb.shape[0]), int(emb.shape[1])
    nq = int(queries.shape[0])
    pe, we = _ptr(emb)
    pq, wq = _ptr(queries)
    cnt = np.zeros(nq, np.int64)
    if out is None:
        idx = np.empty((nq, k), np.uint32)
        cs = np.empty((nq, k), np.float32)
    else:
        idx, cs = out
    pi, wo = _ptr(idx) if k > 0 else (None, SLAG_HOST)
    pc, _ = _ptr(cs) if k > 0 else (None, SLAG_HOST)
    fn = lib().slag_query_static if static else lib().slag_query
    _check(ctx, fn(ctx, n, d, pe, we, nq, pq, wq, float(threshold), int(k),
                   cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), pi, pc, wo))
    return cnt, idx, cs


def slag_classify(ctx, emb, classes, out=None):
    """Per-Gaussian class of highest cosine: returns (label[n], best[n]);
    `out` = (label, best) tensors or arrays to write into."""
    n, d = int(emb.shape[0]), int(emb.shape[1])
    nc = int(classes.shape[0])
    pe, we = _ptr(emb)
    pq, wq = _ptr(classes)
    if out is None:
        lab = np.empty(n, np.int32)
        best = np.empty(n, np.float32)
    else:
        lab, best = out
    pl, wo = _ptr(lab)
    pb, _ = _ptr(best)
    _check(ctx, lib().slag_classify(ctx, n, d, pe, we, nc, pq, wq, pl, pb, wo))
    return lab, best


# ---------------------------------------------------------------- convenience

class Lifter:
    """One context on one device: upload a scene, lift, fetch."""

    def __init__(self, device: int = 0, stream=None, max_views_per_launch: int = 0,
                 flags: int = 0, max_launch_entries: int = 0, **constants):
        self.ctx = slag_create(device, stream, max_views_per_launch, flags, max_launch_entries,
                               **constants)
        self.n = 0
        self.d = 0

    def close(self):
        if self.ctx:
            slag_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_scene(self, scene, device_tensors: bool = False):
        """Upload a synthetic.Scene (host arrays, or torch GPU tensors if asked)."""
        if device_tensors:
            import torch
            dev = torch.device("cuda")
            tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
            means, scales, quats, opac = (tt(scene.means), tt(scene.scales), tt(scene.quats),
                                          tt(scene.opacity))
            # the library copies on its own stream: make torch's copies land first
            torch.cuda.synchronize()
        else:
            means, scales, quats, opac = scene.means, scene.scales, scene.quats, scene.opacity
        slag_set_gaussians(self.ctx, means, scales, quats, opac)
        slag_set_cameras(self.ctx, scene.cams)
        for v, ids in enumerate(scene.ids):
            ids = np.ascontiguousarray(ids, np.int32)
            if ids.ndim == 3:                 # several masks per pixel
                slag_set_segments_multi(self.ctx, v, ids, int(scene.nseg[v]))
            else:
                slag_set_segments(self.ctx, v, ids, int(scene.nseg[v]))
        dt = SLAG_BF16 if scene.feat_dtype == "bf16" else SLAG_F32
        slag_set_features(self.ctx, np.ascontiguousarray(scene.feats), dt)
        self.n = scene.n
        self.d = scene.dim

    def lift(self):
        slag_lift(self.ctx)

    def render(self, view: int, attr, cams):
        """attr [N][C] rendered into view `view` of cams (the scene's cameras):
        (out [H, W, C], wsum [H, W]) as host arrays."""
        H, W = int(cams[view]["height"]), int(cams[view]["width"])
        attr = np.ascontiguousarray(attr, np.float32)
        out = np.empty((H, W, attr.shape[1]), np.float32)
        ws = np.empty((H, W), np.float32)
        slag_render(self.ctx, view, attr, out, ws)
        return out, ws

    def embeddings(self):
        E = np.empty((self.n, self.d), np.float32)
        den = np.empty(self.n, np.float32)
        slag_get_embeddings(self.ctx, E, den)
        return E, den

    def stats(self) -> dict:
        return slag_get_stats(self.ctx)

    def lift_codec(self):
        slag_lift_codec(self.ctx)

    def codes(self, k: int):
        C = np.empty((self.n, k), np.float32)
        slag_get_codes(self.ctx, C)
        return C

    def tile_lists(self, view: int):
        return slag_debug_tile_lists(self.ctx, view)

    def weights(self, view: int):
        return slag_debug_weights(self.ctx, view)
