"""FP64 reference of the learned segment-feature codec.

TEST INFRASTRUCTURE ONLY: the test-suite and the benchmark's CPU leg use this
module; the product path never imports it.

The codec is not part of the paper (which argues against per-scene feature
compression); it is an extension of the lift: segment features are encoded
to k-dim codes before splatting, the lift accumulates the codes with the
same weights it would give the features (the aggregation equation applied to
codes), and each Gaussian's code is decoded back to a D-dim embedding.

Network (one hidden layer each side, tanh-form GELU):
    encoder  c = W2 gelu(W1 f + b1) + b2          D -> H -> k
    decoder  y = W4 gelu(W3 c + b3) + b4          k -> H -> D
Parameters are packed in one FP32 vector in the order
    W1[H][D], b1[H], W2[k][H], b2[k], W3[H][k], b3[H], W4[D][H], b4[D]
(row-major, out x in), the layout of the library's codec entry points.

Training is "through the mixing": a row r is a Gaussian with normalised
weights w_rj over segments col_rj (sum_j w_rj = 1) and a target embedding
t_r (the plain lift's E); its code is sum_j w_rj enc(f_{col_rj}), its output
dec(code); the loss is the mean over rows of 1 - cos(y_r, t_r).

Gradients are derived by the chain rule here, written out layer by layer,
and pinned against central finite differences by the tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


@dataclass(frozen=True)
class Dims:
    d: int
    h: int
    k: int

    def shapes(self):
        d, h, k = self.d, self.h, self.k
        return [("W1", (h, d)), ("b1", (h,)), ("W2", (k, h)), ("b2", (k,)),
                ("W3", (h, k)), ("b3", (h,)), ("W4", (d, h)), ("b4", (d,))]

    @property
    def size(self) -> int:
        return sum(int(np.prod(s)) for _, s in self.shapes())


def unpack(p: np.ndarray, dims: Dims) -> dict:
    out, o = {}, 0
    for name, shp in dims.shapes():
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    assert o == p.size
    return out


def pack(parts: dict, dims: Dims) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).ravel()
                           for name, _ in dims.shapes()])


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + GELU_A * x ** 3)))


def gelu_grad(x):
    u = GELU_C * (x + GELU_A * x ** 3)
    th = np.tanh(u)
    return 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th * th) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


def _act(x, act):
    return gelu(x) if act == "gelu" else x


def _act_grad(x, act):
    return gelu_grad(x) if act == "gelu" else np.ones_like(x)


def encode(p, dims: Dims, F, act="gelu"):
    P = unpack(np.asarray(p, np.float64), dims)
    a1 = F @ P["W1"].T + P["b1"]
    h1 = _act(a1, act)
    return h1 @ P["W2"].T + P["b2"]


def decode(p, dims: Dims, code, act="gelu"):
    P = unpack(np.asarray(p, np.float64), dims)
    a3 = code @ P["W3"].T + P["b3"]
    h2 = _act(a3, act)
    return h2 @ P["W4"].T + P["b4"]


def mix(row_ptr, col, w, C):
    """code_r = sum_j w_rj C[col_rj] (one row per Gaussian)."""
    R = row_ptr.size - 1
    out = np.zeros((R, C.shape[1]))
    for r in range(R):
        a, b = int(row_ptr[r]), int(row_ptr[r + 1])
        if b > a:
            out[r] = w[a:b].astype(np.float64) @ C[col[a:b]]
    return out


def loss_and_grad(p, dims: Dims, F, row_ptr, col, w, target, act="gelu"):
    """Mean over rows of 1 - cos(dec(mix(enc(F))), target) and its gradient
    with respect to the packed parameters (FP64)."""
    P = unpack(np.asarray(p, np.float64), dims)
    F = np.asarray(F, np.float64)
    t = np.asarray(target, np.float64)
    R = row_ptr.size - 1
    # forward
    a1 = F @ P["W1"].T + P["b1"]
    h1 = _act(a1, act)
    C = h1 @ P["W2"].T + P["b2"]
    code = mix(row_ptr, col, w, C)
    a3 = code @ P["W3"].T + P["b3"]
    h2 = _act(a3, act)
    y = h2 @ P["W4"].T + P["b4"]
    ny = np.linalg.norm(y, axis=1)
    nt = np.linalg.norm(t, axis=1)
    dot = np.sum(y * t, axis=1)
    cos = dot / (ny * nt)
    loss = float(np.mean(1.0 - cos))
    # backward: d(1 - cos)/dy = -(t / (|y||t|) - cos y / |y|^2), averaged
    dy = -(t / (ny * nt)[:, None] - (cos / (ny * ny))[:, None] * y) / R
    G = {}
    G["W4"] = dy.T @ h2
    G["b4"] = dy.sum(0)
    da3 = (dy @ P["W4"]) * _act_grad(a3, act)
    G["W3"] = da3.T @ code
    G["b3"] = da3.sum(0)
    dcode = da3 @ P["W3"]
    dC = np.zeros_like(C)
    for r in range(R):
        a, b = int(row_ptr[r]), int(row_ptr[r + 1])
        np.add.at(dC, col[a:b], w[a:b, None].astype(np.float64) * dcode[r][None, :])
    G["W2"] = dC.T @ h1
    G["b2"] = dC.sum(0)
    da1 = (dC @ P["W2"]) * _act_grad(a1, act)
    G["W1"] = da1.T @ F
    G["b1"] = da1.sum(0)
    return loss, pack(G, dims), cos


def codec_lift(p, dims: Dims, Wn, F, act="gelu"):
    """Codec lift with normalised weights Wn (a sparse or dense [N][S] matrix
    whose rows sum to 1, or to 0 for Gaussians without weight): E = dec(Wn
    enc(F)), and E = 0 for rows without weight."""
    C = encode(p, dims, np.asarray(F, np.float64), act)
    code = Wn @ C
    E = decode(p, dims, code, act)
    rs = np.asarray(Wn.sum(axis=1)).ravel()
    E[rs == 0] = 0.0
    return E, code


def pca_fit(E, k):
    """Mean and top-k principal directions of the rows of E."""
    E = np.asarray(E, np.float64)
    mu = E.mean(0)
    _, _, Vt = np.linalg.svd(E - mu, full_matrices=False)
    return mu, Vt[:k]


def pca_params(mu, V, dims: Dims):
    """A linear codec (identity activations) that is the PCA projection:
    enc(f) = V (f - mu), dec(c) = V^T c + mu, with H = k, W3 = I."""
    d, h, k = dims.d, dims.h, dims.k
    assert h == k == V.shape[0] and d == V.shape[1]
    parts = dict(W1=V, b1=-V @ mu, W2=np.eye(k), b2=np.zeros(k), W3=np.eye(k),
                 b3=np.zeros(k), W4=V.T, b4=mu)
    return pack(parts, dims)


def cosine_rows(A, B):
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    return np.sum(A * B, 1) / (np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1) + 1e-300)
