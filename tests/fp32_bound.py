"""Elementwise check of FP32-accumulated products against the decoded
oracle (test helper, no GPU).

For an output row i, every path of roundings into y_i meets at most
K = n (column terms) + the ranks and the number of the leaves covering row
i + 8 (product, s_b, alpha, the update) roundings, so for any order of
summation |y_i - y_dec_i| <= gamma_K (|A^| |x|)_i with gamma_K = K u / (1 - K u),
u = 2^-24, where A^ holds the factors as stored.  The oracle computes the
sampled rows exactly from the leaves covering them (blocks_in_rows).
"""

import numpy as np

import oracle

U32 = 2.0 ** -24


def sample_rows(n: int, leaves: int, seed: int) -> np.ndarray:
    """Whole 64-row clusters of rows plus the first and last row."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(max(1, n // 64), min(leaves, max(1, n // 64)), replace=False)
    rows = [np.array([0, n - 1])] + [np.arange(64 * l, min(n, 64 * l + 64)) for l in pick]
    return np.unique(np.concatenate(rows))


def check_rows(H, X, Y, rows, sigma_dtype=oracle.F32):
    """Y (n x r, the GPU result for X) at ``rows`` against the decoded
    oracle within gamma_K (|A^| |X|); returns (max err / scale, relative
    error vs the decoded oracle, relative error vs the unrounded factors)."""
    X = np.asarray(X, dtype=np.float64).reshape(H.n, -1)
    Y = np.asarray(Y, dtype=np.float64).reshape(H.n, -1)
    blk = oracle.blocks_in_rows(H, rows)
    dec = oracle.decoded_factors(H, sigma_dtype=sigma_dtype, blocks=blk)
    ref = oracle.hmvm_multi(H, X, factors=dec, blocks=blk)[rows]
    truth = oracle.hmvm_multi(H, X, blocks=blk)[rows]
    absf = [(np.abs(a), None if b is None else np.abs(b), None if s is None else np.abs(s)) for a, b, s in dec]
    scale = oracle.hmvm_multi(H, np.abs(X), factors=absf, blocks=blk)[rows]
    K = H.n + int(np.sum(np.where(np.asarray(H.adm)[blk] != 0, np.asarray(H.rank)[blk], 0))) + int(blk.size) + 8
    gam = K * U32 / (1 - K * U32)
    err = np.abs(Y[rows] - ref)
    assert np.all(err <= gam * scale), float(np.max(err / np.maximum(gam * scale, 1e-300)))
    worst = float(np.max(err / np.maximum(scale, 1e-300)))
    rel_dec = float(np.linalg.norm(Y[rows] - ref) / np.linalg.norm(ref))
    rel_truth = float(np.linalg.norm(Y[rows] - truth) / np.linalg.norm(truth))
    return worst, rel_dec, rel_truth
