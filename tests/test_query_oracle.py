"""Pins of the FP64 cosine-similarity search oracle (paper, Method, "Query
processing for inference"): closed forms, invariances, brute force on tiny
inputs, and its FP32 error bound against an FP32 evaluation on the CPU."""
import math

import numpy as np

from oracle import query as oq
from synthetic.query_inputs import queries, query_table


def test_closed_form_in_a_plane():
    """Rows (a, b, 0, ...) against the query e0: cos = a / sqrt(a^2 + b^2)."""
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(50), rng.standard_normal(50)
    E = np.zeros((50, 8))
    E[:, 0], E[:, 1] = a, b
    q = np.zeros((1, 8))
    q[0, 0] = 2.5
    c = oq.cosines(E, q)[0]
    np.testing.assert_allclose(c, a / np.sqrt(a * a + b * b), rtol=1e-15)
    # the second axis at 90 degrees
    q2 = np.zeros((1, 8))
    q2[0, 1] = 1.0
    np.testing.assert_allclose(oq.cosines(E, q2)[0], b / np.sqrt(a * a + b * b), rtol=1e-15)


def test_scale_invariance_and_zero_rows():
    E, W = query_table(1, 300, 32)
    Q = queries(2, W, 3)
    c = oq.cosines(E, Q)
    c2 = oq.cosines(E * np.float32(8.0), Q * np.float32(0.25))   # exact scalings
    zero = np.linalg.norm(E, axis=1) == 0
    assert zero.any()
    assert np.all(np.isneginf(c[:, zero]))
    np.testing.assert_allclose(c[:, ~zero], c2[:, ~zero], rtol=1e-15, atol=1e-15)
    assert np.all(np.abs(c[:, ~zero]) <= 1 + 1e-12)


def test_topk_count_and_classes_by_brute_force():
    """Tiny tables with exact ties: top-k, counts and classes against plain
    Python loops over the definition."""
    rng = np.random.default_rng(5)
    E = rng.integers(-2, 3, (40, 4)).astype(np.float64)     # many equal cosines
    Q = rng.integers(-2, 3, (3, 4)).astype(np.float64)
    Q[np.linalg.norm(Q, axis=1) == 0, 0] = 1.0
    c = oq.cosines(E, Q)
    k = 12
    idx, val = oq.topk(c, k)
    for q in range(3):
        pairs = []
        for g in range(40):
            nE = math.sqrt(sum(x * x for x in E[g]))
            if nE == 0:
                continue
            s = sum(E[g, i] * Q[q, i] for i in range(4)) / (nE * math.sqrt(sum(x * x for x in Q[q])))
            pairs.append((-s, g))
        pairs.sort()
        want = [g for _, g in pairs[:k]]
        assert list(idx[q, : len(want)]) == want
        assert oq.count_above(c, 0.3)[q] == sum(1 for s, _ in pairs if -s >= 0.3)
    lab, best = oq.classify(c)
    for g in range(40):
        col = c[:, g]
        if not np.isfinite(col).any():
            assert lab[g] == -1
        else:
            assert lab[g] == min(i for i in range(3) if col[i] == col.max())


def test_fp32_bound_covers_an_fp32_evaluation():
    """An FP32 evaluation of the same cosines (NumPy float32 arithmetic,
    queries normalised first as the library does) stays within
    fp32_cos_bound(d) of the FP64 cosines."""
    for d in (64, 768):
        E, W = query_table(11, 2000, d)
        Q = queries(12, W, 5)
        c64 = oq.cosines(E, Q)
        qn = Q / np.sqrt(np.sum(Q * Q, axis=1, dtype=np.float32))[:, None]
        dots = (E @ qn.T).T.astype(np.float32)
        ne = np.sqrt(np.sum(E * E, axis=1, dtype=np.float32))
        live = ne > 0
        c32 = dots[:, live] * (np.float32(1) / ne[live])[None, :]
        err = np.abs(c32.astype(np.float64) - c64[:, live])
        assert err.max() <= oq.fp32_cos_bound(d), (d, err.max())
        assert err.max() > 0
