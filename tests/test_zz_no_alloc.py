"""slag_query_static (no device allocation; static work area per GPU)
against slag_query, through the C ABI: identical results, bit for bit, on
two calls in a row (the second smaller, so stale contents of the shared area
must not leak into it), with host and device outputs; sizes beyond the
static area are rejected with SLAG_E_CAPACITY.  Runs alone in a fresh
process or after the other GPU tests."""
import numpy as np
import pytest

from synthetic.query_inputs import queries, query_table

pytestmark = pytest.mark.gpu


def _both(L, Et, Q, thr, k):
    import paper_2505_08124_amd as slag
    a = slag.slag_query(L.ctx, Et, Q, thr, k)
    b = slag.slag_query(L.ctx, Et, Q, thr, k, static=True)
    return a, b


def test_static_query_equals_allocating_query():
    import torch
    import paper_2505_08124_amd as slag
    L = slag.Lifter(0)
    # first call: 50k x 512, 5 queries, k = 2000
    E, W = query_table(21, 50000, 512)
    Q = queries(22, W, 5)
    Et = torch.from_numpy(E).cuda()
    (c1, i1, s1), (c2, i2, s2) = _both(L, Et, Q, 0.28, 2000)
    assert np.array_equal(c1, c2) and np.array_equal(i1, i2) and np.array_equal(s1, s2)
    assert c1.sum() > 0 and np.all(i1[:, 0] != 0xFFFFFFFF)
    # second call, smaller: 3001 x 256, 2 queries, k = 40, device outputs
    E2, W2 = query_table(23, 3001, 256)
    Q2 = torch.from_numpy(queries(24, W2, 2)).cuda()
    Et2 = torch.from_numpy(E2).cuda()
    ia = torch.empty((2, 40), dtype=torch.int32, device="cuda")
    ca = torch.empty((2, 40), dtype=torch.float32, device="cuda")
    ib = torch.empty((2, 40), dtype=torch.int32, device="cuda")
    cb = torch.empty((2, 40), dtype=torch.float32, device="cuda")
    na, _, _ = slag.slag_query(L.ctx, Et2, Q2, 0.1, 40, out=(ia, ca))
    nb, _, _ = slag.slag_query(L.ctx, Et2, Q2, 0.1, 40, out=(ib, cb), static=True)
    torch.cuda.synchronize()
    assert np.array_equal(na, nb)
    assert torch.equal(ia, ib) and torch.equal(ca, cb)
    # counts only (k = 0) needs no sort area
    n0, _, _ = slag.slag_query(L.ctx, Et, Q, 0.28, 0, static=True)
    assert np.array_equal(n0, c1)
    # too large for the static area: rejected, and the allocating call still works
    big_n = (slag.SLAG_QUERY_SCRATCH_BYTES // (16 * 64)) + 1024
    Eb = torch.zeros((big_n, 16), dtype=torch.float32, device="cuda")
    Eb[:, 0] = 1.0
    Qb = np.ones((64, 16), np.float32)
    with pytest.raises(slag.SlagError) as ei:
        slag.slag_query(L.ctx, Eb, Qb, 0.5, 1, static=True)
    assert ei.value.status == slag.SLAG_E_CAPACITY
    # host embeddings are refused (the static variant copies nothing in)
    with pytest.raises(slag.SlagError) as ei:
        slag.slag_query(L.ctx, E2, queries(24, W2, 2), 0.5, 1, static=True)
    assert ei.value.status == slag.SLAG_E_INVALID_ARG
    L.close()
