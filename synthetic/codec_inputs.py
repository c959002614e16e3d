"""Seeded inputs for the codec: initial network parameters and random
training pools (no codec arithmetic here; the oracle and the library both
take these as given)."""
from __future__ import annotations

import math

import numpy as np


def param_shapes(d: int, h: int, k: int):
    """Packed parameter blocks in order (row-major, out x in)."""
    return [("W1", (h, d)), ("b1", (h,)), ("W2", (k, h)), ("b2", (k,)),
            ("W3", (h, k)), ("b3", (h,)), ("W4", (d, h)), ("b4", (d,))]


def init_params(d: int, h: int, k: int, seed: int, bias_sd: float = 0.0) -> np.ndarray:
    """Weights N(0, 1/fan_in), biases N(0, bias_sd^2) (0 by default), FP32."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shp in param_shapes(d, h, k):
        if name.startswith("W"):
            out.append(rng.standard_normal(shp).ravel() / math.sqrt(shp[1]))
        else:
            out.append(bias_sd * rng.standard_normal(shp).ravel())
    return np.concatenate(out).astype(np.float32)


def random_pool(seed: int, S: int, R: int, d: int, per_row=(1, 8)):
    """Unit feature rows F [S][d], R rows of 1..8 distinct columns with
    positive weights summing to 1 (CSR), and unit targets [R][d]; FP32."""
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((S, d))
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    rp, cols, ws = [0], [], []
    for _ in range(R):
        m = int(rng.integers(per_row[0], per_row[1] + 1))
        c = np.sort(rng.choice(S, size=m, replace=False))
        w = rng.random(m) + 0.05
        cols.append(c)
        ws.append(w / w.sum())
        rp.append(rp[-1] + m)
    T = rng.standard_normal((R, d))
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    return (F.astype(np.float32), np.array(rp, np.uint32), np.concatenate(cols).astype(np.uint32),
            np.concatenate(ws).astype(np.float32), T.astype(np.float32))
