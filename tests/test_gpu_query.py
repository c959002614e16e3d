"""GPU parity of the cosine-similarity search (include/slag_query.h) against
the FP64 oracle (oracle/query.py), through the C ABI.

The scores are FP32 on the GPU and FP64 in the oracle, and they decide
integers (which Gaussians pass the threshold, which are the best k, which
class wins), so near-ties may go either way.  Both sides are compared where
the result is unique, and the rest is checked for validity, with the
oracle's FP32 error bound eps = fp32_cos_bound(d):
  * every returned cosine is within eps of the oracle's cosine of the
    returned Gaussian, and the returned rows are sorted best first (ties by
    index, exactly, on the GPU's own scores);
  * the returned set holds every Gaussian whose cosine beats the oracle's
    k-th best by more than 2 eps, and nothing worse than it by more than
    2 eps;
  * counts differ from the oracle's by at most the number of Gaussians within
    eps of the threshold;
  * classes equal the oracle's wherever the best class leads the second by
    more than 2 eps.
Paper: Method, "Query processing for inference" (cosine similarity search
over the embedding tensor).
"""
import numpy as np
import pytest

from oracle import query as oq
from synthetic.query_inputs import queries, query_table

pytestmark = pytest.mark.gpu


def _ctx():
    import paper_2505_08124_amd as slag
    return slag.Lifter(0)


def check_topk(E, Q, idx, cs, k, d):
    eps = oq.fp32_cos_bound(d)
    c64 = oq.cosines(E, Q)
    n = E.shape[0]
    for q in range(Q.shape[0]):
        row = c64[q]
        scored = np.isfinite(row)
        kk = min(k, int(scored.sum()))
        gi = idx[q, :kk].astype(np.int64)
        assert np.all(idx[q, kk:] == 0xFFFFFFFF) and np.all(np.isneginf(cs[q, kk:]))
        assert np.all(gi < n) and np.unique(gi).size == kk
        assert np.all(np.abs(cs[q, :kk].astype(np.float64) - row[gi]) <= eps)
        # best first on the GPU's own scores, ties by index
        v = cs[q, :kk]
        assert np.all((v[:-1] > v[1:]) | ((v[:-1] == v[1:]) & (gi[:-1] < gi[1:])))
        if kk == 0:
            continue
        kth = np.sort(row[scored])[::-1][kk - 1]
        must = np.flatnonzero(row > kth + 2 * eps)
        assert np.isin(must, gi).all()
        assert np.all(row[gi] >= kth - 2 * eps)


@pytest.mark.parametrize("n,d,nq,k", [(20011, 64, 1, 100), (12345, 512, 3, 1000),
                                      (4099, 768, 17, 4099), (777, 16, 64, 5)])
def test_query_matches_oracle(n, d, nq, k):
    import paper_2505_08124_amd as slag
    E, W = query_table(100 + d, n, d)
    Q = queries(200 + d, W, nq)
    thr = 0.28
    L = _ctx()
    cnt, idx, cs = slag.slag_query(L.ctx, E, Q, thr, k)
    c64 = oq.cosines(E, Q)
    eps = oq.fp32_cos_bound(d)
    want = oq.count_above(c64, thr)
    near = (np.abs(c64 - thr) <= eps).sum(axis=1)
    assert np.all(np.abs(cnt - want) <= near), (cnt, want, near)
    check_topk(E, Q, idx, cs, k, d)
    # device inputs and outputs give the same bits; repeated calls are equal
    import torch
    Et = torch.from_numpy(E).cuda()
    Qt = torch.from_numpy(Q).cuda()
    it = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    ct = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    cnt2, _, _ = slag.slag_query(L.ctx, Et, Qt, thr, k, out=(it, ct))
    torch.cuda.synchronize()
    assert np.array_equal(cnt2, cnt)
    assert np.array_equal(it.cpu().numpy().view(np.uint32), idx)
    assert np.array_equal(ct.cpu().numpy(), cs)
    L.close()


def test_query_counts_only_and_edges():
    import paper_2505_08124_amd as slag
    E, W = query_table(7, 5000, 128)
    Q = queries(8, W, 4)
    L = _ctx()
    cnt, _, _ = slag.slag_query(L.ctx, E, Q, -2.0, 0)
    assert np.all(cnt == (np.linalg.norm(E, axis=1) > 0).sum())   # every scored Gaussian
    cnt, _, _ = slag.slag_query(L.ctx, E, Q, 2.0, 0)
    assert np.all(cnt == 0)
    # a zero query is rejected; k > n is rejected
    with pytest.raises(slag.SlagError):
        slag.slag_query(L.ctx, E, np.zeros((1, 128), np.float32), 0.0, 1)
    with pytest.raises(slag.SlagError):
        slag.slag_query(L.ctx, E[:3], Q, 0.0, 4)
    # all rows zero: no scores, top-k rows padded
    Z = np.zeros((100, 128), np.float32)
    cnt, idx, cs = slag.slag_query(L.ctx, Z, Q, -2.0, 10)
    assert np.all(cnt == 0) and np.all(idx == 0xFFFFFFFF) and np.all(np.isneginf(cs))
    L.close()


@pytest.mark.parametrize("n,d,nc", [(30001, 512, 19), (999, 768, 64), (64, 16, 1)])
def test_classify_matches_oracle(n, d, nc):
    import paper_2505_08124_amd as slag
    E, W = query_table(300 + nc, n, d, n_words=max(nc, 2))
    C = queries(400 + nc, W, nc, noise=0.3)
    L = _ctx()
    lab, best = slag.slag_classify(L.ctx, E, C)
    L.close()
    c64 = oq.cosines(E, C)
    lab64, best64 = oq.classify(c64)
    eps = oq.fp32_cos_bound(d)
    scored = lab64 >= 0
    assert np.array_equal(lab < 0, ~scored)
    assert np.all(np.isneginf(best[~scored]))
    srt = np.sort(c64[:, scored], axis=0)
    gap = srt[-1] - srt[-2] if nc > 1 else np.full(int(scored.sum()), np.inf)
    clear = gap > 2 * eps
    assert np.array_equal(lab[scored][clear], lab64[scored][clear])
    assert np.all(np.abs(best[scored].astype(np.float64) - best64[scored]) <= eps)
    # a near tie may go either way, but only to a class within 2 eps of the best
    amb = ~clear
    if amb.any():
        cols = np.flatnonzero(scored)[amb]
        assert np.all(c64[lab[cols], cols] >= best64[cols] - 2 * eps)
