"""Pins for the FP64 codec reference (CPU only): analytic gradients against
central finite differences, the GELU's defining identities and its distance
to the exact (erf) GELU, and the linear special case whose codec lift has a
closed form (a PCA codec commutes with the weighted average)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import codec as cd
from synthetic.codec_inputs import init_params


def _pool(rng, S, R, d, per_row=(1, 6)):
    F = rng.standard_normal((S, d))
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    rp = [0]
    cols, ws = [], []
    for _ in range(R):
        m = int(rng.integers(per_row[0], per_row[1] + 1))
        c = rng.choice(S, size=m, replace=False)
        w = rng.random(m) + 0.05
        cols.append(c)
        ws.append(w / w.sum())
        rp.append(rp[-1] + m)
    row_ptr = np.array(rp, np.uint32)
    col = np.concatenate(cols).astype(np.uint32)
    w = np.concatenate(ws)
    T = rng.standard_normal((R, d))
    return F, row_ptr, col, w, T


@pytest.mark.parametrize("act", ["gelu", "linear"])
def test_gradient_matches_central_differences(act):
    """Every parameter's analytic derivative equals the central difference
    of the loss to 1e-7 (relative to the gradient's scale): a dropped term,
    a wrong sign or a transposed product in the backward pass fails."""
    rng = np.random.default_rng(3)
    dims = cd.Dims(d=7, h=5, k=3)
    F, rp, col, w, T = _pool(rng, S=9, R=6, d=dims.d)
    p = init_params(dims.d, dims.h, dims.k, seed=5).astype(np.float64)
    p += 0.1 * rng.standard_normal(p.size)      # non-zero biases too
    loss, g, _ = cd.loss_and_grad(p, dims, F, rp, col, w, T, act=act)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp, _, _ = cd.loss_and_grad(p + e, dims, F, rp, col, w, T, act=act)
        lm, _, _ = cd.loss_and_grad(p - e, dims, F, rp, col, w, T, act=act)
        num[i] = (lp - lm) / (2 * h)
    scale = np.abs(g).max()
    assert np.abs(num - g).max() <= 1e-7 * max(scale, 1.0), np.abs(num - g).max()
    assert 0.0 <= loss <= 2.0


def test_gelu_identities_and_erf_distance():
    """gelu(x) - gelu(-x) = x; gelu(0) = 0; the tanh form stays within 5e-4
    of x Phi(x) (its published accuracy); gelu' is the derivative."""
    x = np.linspace(-8, 8, 4001)
    assert np.allclose(cd.gelu(x) - cd.gelu(-x), x, atol=1e-14)
    assert cd.gelu(np.array([0.0]))[0] == 0.0
    phi = 0.5 * (1 + np.vectorize(math.erf)(x / math.sqrt(2)))
    assert np.abs(cd.gelu(x) - x * phi).max() < 5e-4
    h = 1e-6
    fd = (cd.gelu(x + h) - cd.gelu(x - h)) / (2 * h)
    assert np.abs(fd - cd.gelu_grad(x)).max() < 1e-8


def test_mixing_reproduces_rows_and_is_linear():
    rng = np.random.default_rng(4)
    C = rng.standard_normal((5, 3))
    rp = np.arange(6, dtype=np.uint32)
    col = np.array([4, 0, 3, 1, 2], np.uint32)
    assert np.array_equal(cd.mix(rp, col, np.ones(5), C), C[col])
    F, rp, col, w, _ = _pool(rng, S=8, R=4, d=3)
    A, B = rng.standard_normal((8, 3)), rng.standard_normal((8, 3))
    assert np.allclose(cd.mix(rp, col, w, 2 * A - B), 2 * cd.mix(rp, col, w, A) - cd.mix(rp, col, w, B))


def test_pca_codec_lift_is_the_projection_of_the_plain_embedding():
    """With identity activations and PCA weights the codec is linear, so the
    weighted average of codes is the code of the weighted average: the codec
    lift equals mu + V^T V (E - mu) for E the plain lift (rows summing to 1),
    and 0 for Gaussians without weight."""
    rng = np.random.default_rng(6)
    S, N, d, k = 30, 50, 12, 4
    F = rng.standard_normal((S, d))
    Wd = rng.random((N, S)) * (rng.random((N, S)) < 0.2)
    Wd[:3] = 0.0                                      # Gaussians without weight
    rs = Wd.sum(1)
    Wn = np.divide(Wd, rs[:, None], out=np.zeros_like(Wd), where=rs[:, None] > 0)
    E = Wn @ F
    mu, V = cd.pca_fit(E[3:], k)
    dims = cd.Dims(d=d, h=k, k=k)
    p = cd.pca_params(mu, V, dims)
    Ec, code = cd.codec_lift(p, dims, sp.csr_matrix(Wn), F, act="linear")
    ref = mu + (E - mu) @ V.T @ V
    assert np.allclose(Ec[3:], ref[3:], atol=1e-12)
    assert np.all(Ec[:3] == 0)
    assert np.allclose(code[3:], (E[3:] - mu) @ V.T, atol=1e-12)


def test_exact_subspace_gives_zero_loss():
    """Features in a k-dim subspace through the origin: the PCA codec of the
    pool's targets reproduces every target, so the loss is 0 (cos = 1)."""
    rng = np.random.default_rng(8)
    d, k = 10, 3
    basis = np.linalg.qr(rng.standard_normal((d, k)))[0].T
    F = rng.standard_normal((20, k)) @ basis
    _, rp, col, w, _ = _pool(rng, S=20, R=15, d=d)
    T = cd.mix(rp, col, w, F)
    mu, V = cd.pca_fit(T, k)
    dims = cd.Dims(d=d, h=k, k=k)
    loss, _, cos = cd.loss_and_grad(cd.pca_params(mu, V, dims), dims, F, rp, col, w, T,
                                    act="linear")
    assert loss < 1e-12 and np.all(cos > 1 - 1e-12)
