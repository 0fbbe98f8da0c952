"""GPU parity of the byte-aligned storage formats of Sec. 3.2 (truncated
FP64: DFL; adaptive exponent: AFLP; FP32's exponent: BFL) with FP64
accumulation, through the C-ABI, one format per matrix or block, or chosen per column (APLR, Sec. 3.3).

The kernels decode DFL exactly to FP64, so the product must match the oracle
evaluated on the DFL-rounded factors to the FP64 bar (relative 2-norm error
<= 1e-12, elementwise <= 1e-13 of the summand scale).  Against the unrounded
FP64 product the error is the storage rounding, stated and bounded by the
format's unit roundoff.  Layouts: one format everywhere (DFL32, DFL40 with
partials at n = 16384, DFL48), dense blocks in DFL48 and FP64 beside
low-rank DFL32, and FP32 storage (BFL at 4 bytes) under FP64 accumulation;
AFLP per block (sphere4k_aflp), and AFLP of every width beside DFL32 and
FP64 in column groups with partials at n = 16384; both schedules,
persistent grids and a graph replay; the full n = 2^18 sizes at eps 1e-6
(DFL32; APLR; AFLP) and 1e-8 (DFL40; APLR; AFLP).
"""

import os
import sys

import numpy as np
import pytest

import hmgen
import oracle
from paper_2308_10960_amd import hm, DeviceHMatrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
MANT = {hm.HM_DFL32: 20, hm.HM_DFL40: 28, hm.HM_DFL48: 36}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(hm.LIB_PATH), "libhm.so must be built before the GPU tests"


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def run(D, x, y0=None, alpha=1.0):
    xd = D.vector(x)
    yd = D.vector(y0) if y0 is not None else D.vector()
    D.mvm(xd, yd, alpha)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.float64)


def abs_bound(H, x, factors):
    fac = [(np.abs(np.asfortranarray(a)), None if b is None else np.abs(np.asfortranarray(b)),
            None if s is None else np.abs(np.asarray(s))) for a, b, s in factors]
    return oracle.hmvm(H, np.abs(x), factors=fac)


AFLP = {hm.HM_AFLP16: 2, hm.HM_AFLP24: 3, hm.HM_AFLP32: 4, hm.HM_AFLP40: 5, hm.HM_AFLP48: 6}
BFL_MANT = {hm.HM_BFL24: 15, hm.HM_BFL40: 31, hm.HM_BFL48: 39, hm.HM_F32: 23}


def aflp_bound(H):
    """4 x the largest relative rounding error of H's data blocks: 2^-m for
    an AFLP block of m mantissa bits (|v - fl(v)| <= 2^-(m+1) (|v| + 2^k)
    with 2^k <= |v|), the unit roundoff for DFL / FP64."""
    worst = 2.0 ** -53
    for i in range(H.nblocks):
        a, b, _ = H.factors(i)
        c0 = 0
        for g in range(int(H.ngroups[i])):
            dt = int(H.group_dtype[i, g])
            kc = int(H.group_cols[i, g]) if H.adm[i] else a.shape[1]
            for F in (a, b):
                if F is None or kc == 0:
                    continue
                blk = F[:, c0:c0 + kc]
                if dt in AFLP:
                    worst = max(worst, 2.0 ** -oracle.aflp_params(blk, AFLP[dt])[2])
                elif dt in BFL_MANT:
                    worst = max(worst, 2.0 ** -(BFL_MANT[dt] + 1))
                elif dt in MANT:
                    worst = max(worst, 2.0 ** -(MANT[dt] + 1))
            c0 += kc
    return 4 * worst


def layout(name):
    """(H, bound on the relative error against the unrounded FP64 product:
    4 x the largest unit roundoff of its formats, or for APLR eps) for a
    named DFL or AFLP layout."""
    if name == "aflp":
        H = hmgen.build_preset("sphere4k_aflp")
        return H, aflp_bound(H)
    if name == "aflp_any_16k":
        # AFLP of every width beside DFL32 and FP64, in up to 4 column
        # groups per block, at n = 16384 (partials)
        H = hmgen.build_preset("sphere4k", n=16384, eps=1e-10)
        _groups(H, [hm.HM_F64, hm.HM_DFL32, hm.HM_AFLP16, hm.HM_AFLP24, hm.HM_AFLP32, hm.HM_AFLP40,
                    hm.HM_AFLP48], np.random.default_rng(4))
        return H, aflp_bound(H)
    if name == "bfl40":
        H = hmgen.build_preset("sphere4k_bfl")
        return H, 4 * 2.0 ** -32
    if name == "bfl_any_16k":
        # BFL of every width beside DFL40, AFLP32, FP32 and FP64 in column
        # groups, at n = 16384 (partials)
        H = hmgen.build_preset("sphere4k", n=16384, eps=1e-10)
        _groups(H, [hm.HM_F64, hm.HM_BFL24, hm.HM_BFL40, hm.HM_BFL48, hm.HM_DFL40, hm.HM_AFLP32, hm.HM_F32],
                np.random.default_rng(8))
        return H, aflp_bound(H)
    if name == "aflp_zeros":
        H, _ = layout("aflp")
        _plant_zeros(H)
        return H, aflp_bound(H)
    if name == "aplr":
        # per-column formats from DFL16 to FP64, every block within eps / 2
        H = hmgen.build_preset("sphere4k_aplr")
        return H, hmgen.preset("sphere4k_aplr")["eps"]
    if name == "dfl_mix":
        H = hmgen.build_preset("sphere4k")
        H.set_uniform_dtype(hm.HM_DFL32)
        dense = np.flatnonzero(H.adm == 0)
        H.group_dtype[dense, 0] = hm.HM_DFL48
        H.group_dtype[dense[::3], 0] = hm.HM_F64
        return H, 4 * 2.0 ** -(MANT[hm.HM_DFL32] + 1)
    if name == "bfl32":
        # BFL at 4 bytes (8 exponent bits, 23 mantissa bits) is FP32 storage
        H = hmgen.build_preset("sphere4k")
        H.set_uniform_dtype(hm.HM_F32)
        return H, 4 * 2.0 ** -24
    dt = {"dfl32": hm.HM_DFL32, "dfl40_16k": hm.HM_DFL40, "dfl48": hm.HM_DFL48}[name]
    H = hmgen.build_preset("sphere4k", n=16384 if name.endswith("16k") else None)
    H.set_uniform_dtype(dt)
    return H, 4 * 2.0 ** -(MANT[dt] + 1)


def check(y, ref, scale, what):
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    say(f"{what}: relative error vs decoded oracle {rel:.3e}")
    assert rel <= F64_TOL
    assert np.all(np.abs(y - ref) <= 1e-13 * scale + 1e-300)


@pytest.mark.parametrize("name", ["dfl32", "dfl40_16k", "dfl48", "dfl_mix", "bfl32", "aplr", "aflp",
                                  "aflp_any_16k", "aflp_zeros", "bfl40", "bfl_any_16k"])
def test_dfl_parity(name):
    H, bound = layout(name)
    say("layout", name, "n", H.n)
    D = DeviceHMatrix(H, hm.HM_F64)
    if name.endswith("_16k"):
        assert D.info["n_partials"] > 0
    x = hmgen.uniform_vector(H.n)
    y0 = hmgen.uniform_vector(H.n, seed=9)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F64)
    ref = oracle.hmvm(H, x, y0, alpha=0.75, factors=dec)
    scale = 0.75 * abs_bound(H, x, dec) + np.abs(y0)
    base = {}
    for sched in (0, 1):
        for unroll in (4, 8):
            c = f"schedule={sched} unroll={unroll} order=1 persist=0"
            hm.hm_matrix_set_launch(D.handle, c)
            y = run(D, x, y0, 0.75)
            check(y, ref, scale, f"{name} {c}")
            base.setdefault(sched, y)
        for ps in (1, 2):
            c = f"schedule={sched} unroll=8 order=0 persist={ps}"
            say(c)
            hm.hm_matrix_set_launch(D.handle, c)
            np.testing.assert_array_equal(run(D, x, y0, 0.75), base[sched])
    # column tiles on a workgroup each and on a wave each (persistent too)
    for colw in (0, 2):
        hm.hm_matrix_set_launch(D.handle, f"schedule=0 unroll=8 order=1 persist=0 colw={colw}")
        y = run(D, x, y0, 0.75)
        check(y, ref, scale, f"{name} colw={colw}")
        hm.hm_matrix_set_launch(D.handle, "persist=2")
        np.testing.assert_array_equal(run(D, x, y0, 0.75), y)
    hm.hm_matrix_set_launch(D.handle, "persist=0 colw=1")
    # storage rounding against the unrounded FP64 product, bounded by the
    # unit roundoff of the formats (two rounded factors per low-rank term)
    truth = oracle.hmvm(H, x)
    y = run(D, x)
    rel_truth = np.linalg.norm(y - truth) / np.linalg.norm(truth)
    say(f"{name}: relative error vs unrounded FP64 {rel_truth:.3e} (bound {bound:.2e})")
    assert rel_truth <= bound
    D.close()


@pytest.mark.parametrize("name", ["dfl_mix", "aflp_any_16k"])
def test_dfl_graph_replay(name):
    """A captured single-RHS product of a DFL / AFLP store replays bit for
    bit like the eager call, also with eager work between the replays."""
    H, _ = layout(name)
    D = DeviceHMatrix(H, hm.HM_F64)
    x = hmgen.uniform_vector(H.n)
    xd = D.vector(x)
    yd = D.vector()
    D.mvm(xd, yd, 1.0)
    torch.cuda.synchronize()
    eager = yd.clone()
    g = hm.hm_graph_create(D.handle, 1, 1.0, xd, H.n, yd, H.n, D.work, D.work.numel())
    try:
        for r in range(3):
            yd.zero_()
            torch.cuda.synchronize()
            hm.hm_graph_launch(g, torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert torch.equal(yd, eager), f"replay {r}"
            run(D, x)                                   # eager work in between
    finally:
        hm.hm_graph_destroy(g)
    D.close()


def test_aflp_batch_equals_single():
    """hm_mvm_batch on an AFLP store (FP64 accumulation: right-hand sides
    one by one) gives each column bit for bit as hm_mvm does."""
    H, _ = layout("aflp")
    D = DeviceHMatrix(H, hm.HM_F64, max_nrhs=3)
    X = np.stack([hmgen.uniform_vector(H.n, seed=20 + j) for j in range(3)])
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.zeros_like(Xd)
    hm.hm_mvm_batch(D.handle, 3, 0.5, Xd, H.n, Yd, H.n, D.work, D.work.numel())
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    for j in range(3):
        y = run(D, X[j], alpha=0.5)
        np.testing.assert_array_equal(Y[j], y)
    D.close()


@pytest.mark.parametrize("name", ["sphere256k_dfl", "sphere256k_e8_dfl", "sphere256k_aplr",
                                  "sphere256k_e8_aplr", "sphere256k_aflp", "sphere256k_e8_aflp",
                                  "sphere256k_e8_bfl"])
def test_dfl_full_size(name):
    say("building", name)
    H = hmgen.build_preset(name)
    say("built", H.stats())
    if name.endswith("_dfl"):
        assert np.all(H.group_dtype[:, 0] == {"sphere256k_dfl": hm.HM_DFL32,
                                              "sphere256k_e8_dfl": hm.HM_DFL40}[name])
    if name.endswith("_bfl"):
        assert np.all(H.group_dtype[:, 0] == hm.HM_BFL40)
    D = DeviceHMatrix(H, hm.HM_F64)
    say("uploaded", D.info["store_bytes"])
    x = hmgen.uniform_vector(H.n)
    y = run(D, x)
    say("gpu done; oracle")
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F64)
    ref = oracle.hmvm(H, x, factors=dec)
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    truth = oracle.hmvm(H, x)
    rel_truth = np.linalg.norm(y - truth) / np.linalg.norm(truth)
    say(f"{name}: relative error vs decoded oracle {rel:.3e}, vs unrounded FP64 {rel_truth:.3e}")
    assert rel <= F64_TOL
    idx = np.random.default_rng(0).choice(H.n, 2000, replace=False)
    scale = abs_bound(H, x, dec)
    assert np.all(np.abs(y[idx] - ref[idx]) <= 1e-13 * scale[idx])
    eps = hmgen.preset(name)["eps"]
    assert rel_truth <= eps
    D.close()


def _plant_zeros(H, seed=6):
    """Exact zeros in the factors (the AFLP zero code): 10% of the entries
    of every fifth block, one whole dense block and one whole V_b."""
    rng = np.random.default_rng(seed)
    dense = np.flatnonzero(H.adm == 0)
    lowr = np.flatnonzero((H.adm != 0) & (H.rank > 0))
    for i in range(0, H.nblocks, 5):
        for F in H.factors(i)[:2]:
            if F is not None and F.size:
                F[rng.random(F.shape) < 0.1] = 0.0
    H.factors(int(dense[3]))[0][:] = 0.0
    H.factors(int(lowr[7]))[1][:] = 0.0


def _groups(H, fmts, rng):
    """Every low-rank block split into up to 4 column groups with formats
    drawn from fmts (dense blocks one format each)."""
    H.set_uniform_dtype(fmts[0])
    for i in range(H.nblocks):
        if not H.adm[i]:
            H.group_dtype[i, 0] = fmts[rng.integers(len(fmts))]
            continue
        k = int(H.rank[i])
        if k == 0:
            continue
        ng = int(rng.integers(1, min(4, k) + 1))
        cuts = np.sort(rng.choice(np.arange(1, k), ng - 1, replace=False)) if ng > 1 else np.array([], int)
        sizes = np.diff(np.concatenate([[0], cuts, [k]]))
        H.ngroups[i] = ng
        H.group_cols[i, :] = 0
        H.group_cols[i, :ng] = sizes
        H.group_dtype[i, :] = 0
        H.group_dtype[i, :ng] = [fmts[j] for j in rng.integers(len(fmts), size=ng)]


def _random_layout(seed):
    """Random per-group formats (all seventeen with FP64 accumulation, the
    16/32-bit IEEE ones with FP32) and a random column-tile shape, n = 16384."""
    rng = np.random.default_rng(seed)
    H = hmgen.build_preset("sphere4k_mixed", n=16384)
    acc = hm.HM_F64 if seed % 2 else hm.HM_F32
    fmts = ([hm.HM_F64, hm.HM_F32, hm.HM_F16, hm.HM_BF16, hm.HM_DFL16, hm.HM_DFL24, hm.HM_DFL32,
             hm.HM_DFL40, hm.HM_DFL48, hm.HM_AFLP16, hm.HM_AFLP24, hm.HM_AFLP32, hm.HM_AFLP40, hm.HM_AFLP48,
             hm.HM_BFL24, hm.HM_BFL40, hm.HM_BFL48]
            if acc == hm.HM_F64 else [hm.HM_F32, hm.HM_F16, hm.HM_BF16])
    _groups(H, fmts, rng)
    return H, acc, int(rng.integers(64, 513)), int(rng.integers(8, 65))


@pytest.mark.parametrize("seed", [11, 12])
def test_random_layouts(seed):
    """The kernels on random format mixes and tile shapes: FP64 accumulation
    to the FP64 bar against the oracle on the rounded factors, both
    schedules; FP32 accumulation within the rigorous FP32 bound, single and
    batched (32 right-hand sides)."""
    from test_gpu_parity import fp32_depth
    H, acc, chunk, tile = _random_layout(seed)
    say("seed", seed, "acc", acc, "chunk", chunk, "tile", tile)
    D = DeviceHMatrix(H, acc, max_nrhs=32 if acc == hm.HM_F32 else 1, chunk_rows=chunk, tile_groups=tile)
    x = hmgen.uniform_vector(H.n)
    if acc == hm.HM_F32:
        x = x.astype(np.float32).astype(np.float64)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F64 if acc == hm.HM_F64 else oracle.F32)
    ref = oracle.hmvm(H, x, factors=dec)
    scale = abs_bound(H, x, dec)
    if acc == hm.HM_F64:
        for sched in (0, 1):
            hm.hm_matrix_set_launch(D.handle, f"schedule={sched}")
            check(run(D, x), ref, scale, f"random seed {seed} schedule {sched}")
    else:
        K = fp32_depth(H)
        gam = K * 2.0 ** -24 / (1 - K * 2.0 ** -24)
        y = run(D, x)
        assert np.all(np.abs(y - ref) <= gam * scale)
        R = 32
        X = np.stack([hmgen.uniform_vector(H.n, seed=40 + j).astype(np.float32) for j in range(R)])
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.zeros_like(Xd)
        hm.hm_mvm_batch(D.handle, R, 1.0, Xd, H.n, Yd, H.n, D.work, D.work.numel())
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy().astype(np.float64)
        for j in (0, 17, 31):
            xj = X[j].astype(np.float64)
            rj = oracle.hmvm(H, xj, factors=dec)
            assert np.all(np.abs(Y[j] - rj) <= gam * abs_bound(H, xj, dec)), j
        say(f"random seed {seed}: FP32 single and batched within gamma_K")
    D.close()
