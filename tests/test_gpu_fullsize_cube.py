"""Full-size batched products of the uniform-cube exponential-kernel matrix
(leaf 64, eta 2, eps 1e-6, FP32 factors) with 32 Gaussian right-hand sides
through hm_mvm_batch, in the launch configurations the benchmark and the
tuner use (they change no bit).

The oracle cannot afford all n rows for 32 right-hand sides, so it computes
sampled rows exactly: y at a row is the sum over the leaves whose row cluster
contains it (blocks_in_rows), with the factors rounded to FP32 as stored
(decoded oracle) and unrounded (FP64 truth).  Whole leaf clusters of rows are
sampled, plus the first and last row.  Bars: elementwise within the rigorous
FP32 bound gamma_K (|A^| |X|) of the decoded oracle, and a relative error of
at most 1e-6 against both the decoded oracle and the FP64 truth.

n = 2^18 always runs (seconds of host construction).  n = 2^20 needs about
140 GB of host memory and minutes of host construction; it runs when the
host has that memory available (MemAvailable), and is skipped with the
measured value otherwise.
"""

import sys

import numpy as np
import pytest

import hmgen
import oracle
from paper_2308_10960_amd import hm, DeviceHMatrix, tune

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
CUBE1M_HOST_BYTES = 180e9         # factors (137 GB FP64) plus construction and oracle working memory


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def mem_available() -> float:
    with open("/proc/meminfo") as f:
        for line in f:
            if line.startswith("MemAvailable:"):
                return float(line.split()[1]) * 1024
    return 0.0


def check_cube(n: int, R: int = 32, leaves_sampled: int = 12):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say(f"building cube n={n}")
    H = hmgen.build_preset("cube1m", n=n)
    say("built", H.stats())
    D = DeviceHMatrix(H, hm.HM_F32, max_nrhs=R)
    say("uploaded", D.info["store_bytes"], "work", D.work_bytes)
    Xh = hmgen.gaussian_block(H.n, R, seed=hmgen.presets.SEED_RHS).astype(np.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(Xh.T)).cuda()
    outs = {}
    for c in tune.BATCH_CANDIDATES:
        hm.hm_matrix_set_launch(D.handle, c)
        Yd = torch.zeros_like(Xd)
        hm.hm_mvm_batch(D.handle, R, 1.0, Xd, H.n, Yd, H.n, D.work, D.work.numel())
        torch.cuda.synchronize()
        outs[c] = Yd.cpu().numpy().T
        say("gpu done", c)
    Y = outs[tune.BATCH_CANDIDATES[0]]
    for c in tune.BATCH_CANDIDATES[1:]:
        np.testing.assert_array_equal(outs[c], Y)
    assert np.all(np.isfinite(Y))
    D.close()
    del Xd, Yd

    rng = np.random.default_rng(11)
    leaves = rng.choice(H.n // 64, leaves_sampled, replace=False)
    rows = np.unique(np.concatenate([[0, H.n - 1]] + [np.arange(64 * l, 64 * l + 64) for l in leaves]))
    blk = oracle.blocks_in_rows(H, rows)
    say(f"oracle on {rows.size} rows, {blk.size} leaves")
    X = Xh.astype(np.float64)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F32, blocks=blk)
    ref = oracle.hmvm_multi(H, X, factors=dec, blocks=blk)[rows]
    truth = oracle.hmvm_multi(H, X, blocks=blk)[rows]
    absf = [(np.abs(a), None if b is None else np.abs(b), s) for a, b, s in dec]
    scale = oracle.hmvm_multi(H, np.abs(X), factors=absf, blocks=blk)[rows]
    Ys = Y[rows]
    # rigorous elementwise FP32 bound: K bounds the roundings on any path into
    # a sampled output (n column terms, the ranks and the number of the
    # leaves that cover its row, 8 for product, s_b, alpha and the update)
    K = H.n + int(np.sum(np.where(H.adm[blk] != 0, H.rank[blk], 0))) + int(blk.size) + 8
    gam = K * U32 / (1 - K * U32)
    assert np.all(np.abs(Ys - ref) <= gam * scale)
    rel_dec = np.linalg.norm(Ys - ref) / np.linalg.norm(ref)
    rel_truth = np.linalg.norm(Ys - truth) / np.linalg.norm(truth)
    worst = float(np.max(np.abs(Ys - ref) / scale))
    say(f"cube n={n}: rel vs decoded {rel_dec:.3e}, rel vs FP64 truth {rel_truth:.3e}, "
        f"max err/scale {worst:.3e}")
    assert rel_dec <= 1e-6
    assert rel_truth <= 1e-6


def test_cube256k_batched_sampled_rows():
    check_cube(1 << 18)


def test_cube1m_batched_sampled_rows():
    avail = mem_available()
    if avail < CUBE1M_HOST_BYTES:
        pytest.skip(f"n=2^20 cube needs ~{CUBE1M_HOST_BYTES / 1e9:.0f} GB of host memory; "
                    f"MemAvailable is {avail / 1e9:.1f} GB")
    check_cube(1 << 20)
