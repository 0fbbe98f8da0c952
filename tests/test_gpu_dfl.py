"""GPU parity of the byte-aligned truncated FP64 storage formats (DFL,
Sec. 3.2) with FP64 accumulation, through the C-ABI, one format per matrix
or chosen per column (APLR, Sec. 3.3).

The kernels decode DFL exactly to FP64, so the product must match the oracle
evaluated on the DFL-rounded factors to the FP64 bar (relative 2-norm error
<= 1e-12, elementwise <= 1e-13 of the summand scale).  Against the unrounded
FP64 product the error is the storage rounding, stated and bounded by the
format's unit roundoff.  Layouts: one format everywhere (DFL32, DFL40 with
partials at n = 16384, DFL48), dense blocks in DFL48 and FP64 beside
low-rank DFL32, and FP32 storage (BFL at 4 bytes) under FP64 accumulation;
both schedules, persistent grids and a graph replay; the
full n = 2^18 sizes at eps 1e-6 (DFL32; APLR) and 1e-8 (DFL40; APLR).
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


def layout(name):
    """(H, bound on the relative error against the unrounded FP64 product:
    4 x the largest unit roundoff of its formats, or for APLR eps) for a
    named DFL layout."""
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


@pytest.mark.parametrize("name", ["dfl32", "dfl40_16k", "dfl48", "dfl_mix", "bfl32", "aplr"])
def test_dfl_parity(name):
    H, bound = layout(name)
    say("layout", name, "n", H.n)
    D = DeviceHMatrix(H, hm.HM_F64)
    if name == "dfl40_16k":
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
    # storage rounding against the unrounded FP64 product, bounded by the
    # unit roundoff of the formats (two rounded factors per low-rank term)
    truth = oracle.hmvm(H, x)
    y = run(D, x)
    rel_truth = np.linalg.norm(y - truth) / np.linalg.norm(truth)
    say(f"{name}: relative error vs unrounded FP64 {rel_truth:.3e} (bound {bound:.2e})")
    assert rel_truth <= bound
    D.close()


def test_dfl_graph_replay():
    """A captured single-RHS product of a DFL store replays bit for bit like
    the eager call, also with eager work between the replays."""
    H, _ = layout("dfl_mix")
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


@pytest.mark.parametrize("name", ["sphere256k_dfl", "sphere256k_e8_dfl", "sphere256k_aplr",
                                  "sphere256k_e8_aplr"])
def test_dfl_full_size(name):
    say("building", name)
    H = hmgen.build_preset(name)
    say("built", H.stats())
    if name.endswith("_dfl"):
        assert np.all(H.group_dtype[:, 0] == {"sphere256k_dfl": hm.HM_DFL32,
                                              "sphere256k_e8_dfl": hm.HM_DFL40}[name])
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
