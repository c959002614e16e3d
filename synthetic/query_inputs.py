"""Seeded inputs for the cosine-similarity search: an embedding table shaped
like a lift's output (rows near one of a few unit "words", some rows mixing
two words, some rows zero for Gaussians without weight, exact duplicate rows
for ties) and query vectors (the words themselves, plus noise).  No search
arithmetic here; the oracle and the library both take these as given."""
from __future__ import annotations

import math

import numpy as np


def query_table(seed: int, n: int, d: int, n_words: int = 16, zero_frac: float = 0.05,
                dup_frac: float = 0.02):
    """(E [n][d] float32, words [n_words][d] float32)."""
    rng = np.random.default_rng(seed)
    words = rng.standard_normal((n_words, d))
    words /= np.linalg.norm(words, axis=1, keepdims=True)
    a = rng.integers(0, n_words, n)
    b = rng.integers(0, n_words, n)
    mix = np.where(rng.random(n) < 0.3, rng.random(n), 0.0)[:, None]
    E = (1.0 - mix) * words[a] + mix * words[b] + 0.3 * rng.standard_normal((n, d)) / math.sqrt(d)
    E *= rng.uniform(0.2, 1.0, (n, 1))           # lifted embeddings are not unit length
    E[rng.random(n) < zero_frac] = 0.0
    nd = int(dup_frac * n)
    if nd and n > 1:
        src = rng.integers(0, n, nd)
        dst = rng.integers(0, n, nd)
        E[dst] = E[src]
    return E.astype(np.float32), words.astype(np.float32)


def queries(seed: int, words: np.ndarray, nq: int, noise: float = 0.1):
    """nq query vectors: words (cycled) plus Gaussian noise, float32."""
    rng = np.random.default_rng(seed)
    d = words.shape[1]
    Q = words[np.arange(nq) % words.shape[0]] + noise * rng.standard_normal((nq, d)) / math.sqrt(d)
    return Q.astype(np.float32)
