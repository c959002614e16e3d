"""Plain FP64 cosine-similarity search (paper, Method, "Query processing for
inference": query vectors are matched against the per-Gaussian embeddings
by cosine similarity; Experiments: a threshold on the cosine, the best
matching Gaussians as the query response, and the class of highest cosine
per Gaussian).

TEST INFRASTRUCTURE ONLY: used by the test-suite; shares no code with the
GPU library.  Everything is the definition written out: cosines by a
library matrix product in FP64, counts by comparison, top-k by a stable
sort (ties by ascending index), classes by argmax (ties to the lower class).
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def cosines(E, Q):
    """cos[q][g] = E_g . Q_q / (|E_g| |Q_q|) in FP64; -inf where E_g = 0."""
    E = np.asarray(E, np.float64)
    Q = np.asarray(Q, np.float64)
    ne = np.linalg.norm(E, axis=1)
    nq = np.linalg.norm(Q, axis=1)
    dots = Q @ E.T
    out = np.full(dots.shape, -np.inf)
    live = ne > 0
    out[:, live] = dots[:, live] / (nq[:, None] * ne[None, live])
    return out


def count_above(cos, thr):
    return (cos >= thr).sum(axis=1).astype(np.int64)


def topk(cos, k):
    """Per query the k largest cosines, best first, ties by ascending index;
    (idx [Q][k], cos [Q][k]), rows padded with (0xFFFFFFFF, -inf) past the
    scored Gaussians."""
    nq, n = cos.shape
    idx = np.full((nq, k), 0xFFFFFFFF, np.uint64)
    val = np.full((nq, k), -np.inf)
    order_idx = np.arange(n)
    for q in range(nq):
        o = np.lexsort((order_idx, -cos[q]))[:k]
        o = o[np.isfinite(cos[q][o])]
        idx[q, : o.size] = o
        val[q, : o.size] = cos[q][o]
    return idx, val


def classify(cos):
    """Per Gaussian the class of highest cosine (ties to the lower class),
    -1 where the Gaussian has no score; and that cosine."""
    lab = np.argmax(cos, axis=0).astype(np.int64)      # first maximum: lower class on ties
    best = cos[lab, np.arange(cos.shape[1])]
    lab[~np.isfinite(best)] = -1
    return lab, best


def fp32_cos_bound(d: int) -> float:
    """Bound on |cos_fp32 - cos_fp64| for an FP32 evaluation: the dot
    product and the sum of squares of d terms each carry at most d u of
    relative error (first order, any summation order); normalising the
    query (sum of squares, square root, reciprocal, products) adds d u / 2 +
    3 u per element, the row's inverse norm as much again, and the final
    product u: |cos| <= 1 gives 2 d u + 8 u."""
    return (2 * d + 8) * U32
