"""hm_mvm_noalloc: the single-right-hand-side product with the library's fixed
device workspace instead of a caller workspace.

Through the C-ABI it must give the result of hm_mvm bit for bit (same
kernels, same launch parameters) on consecutive calls, the second on a
smaller matrix, so the fixed array still holds the first call's partial
sums and t entries when the second runs; both also agree with the oracle
to the FP64 bar.  FP64 and FP32 (mixed-storage) accumulation are covered.
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


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(hm.LIB_PATH), "libhm.so must be built before the GPU tests"


def _pair(H, acc):
    """(hm_mvm result, hm_mvm_noalloc result) on the same x and y0."""
    D = DeviceHMatrix(H, acc)
    assert D.info["work_bytes_per_rhs"] <= hm.HM_NOALLOC_SCRATCH_BYTES
    x = D.vector(hmgen.uniform_vector(H.n, seed=1))
    y0 = hmgen.uniform_vector(H.n, seed=9)
    ya, yb = D.vector(y0), D.vector(y0)
    say(f"n={H.n} acc={acc}: hm_mvm, then hm_mvm_noalloc")
    hm.hm_mvm(D.handle, 0.5, x, ya, D.work, D.work.numel())
    hm.hm_mvm_noalloc(D.handle, 0.5, x, yb)
    torch.cuda.synchronize()
    out = ya.cpu().numpy().astype(np.float64), yb.cpu().numpy().astype(np.float64)
    D.close()
    return out, y0


def test_noalloc_equals_mvm_on_consecutive_calls():
    # first call on the larger matrix, second on a smaller one: the fixed
    # array still holds the first call's entries beyond the second's
    for name, n in (("sphere4k", 16384), ("sphere4k", 4096)):
        H = hmgen.build_preset(name, n=n)
        (ya, yb), y0 = _pair(H, hm.HM_F64)
        np.testing.assert_array_equal(yb, ya)
        ref = oracle.hmvm(H, hmgen.uniform_vector(H.n, seed=1), y0, alpha=0.5)
        rel = np.linalg.norm(yb - ref) / np.linalg.norm(ref)
        say(f"n={n}: bitwise equal to hm_mvm, relative error vs oracle {rel:.3e}")
        assert rel <= 1e-12


def test_noalloc_fp32_accumulation():
    H = hmgen.build_preset("sphere4k_mixed", n=8192)
    (ya, yb), _ = _pair(H, hm.HM_F32)
    np.testing.assert_array_equal(yb, ya)


def test_noalloc_rejects_bad_arguments():
    H = hmgen.build_preset("sphere4k")
    D = DeviceHMatrix(H, hm.HM_F64)
    x = D.vector(hmgen.uniform_vector(H.n))
    with pytest.raises(hm.HMError) as e:
        hm.hm_mvm_noalloc(D.handle, 1.0, x, x)          # x aliases y
    assert e.value.status == hm.HM_EINVAL
    with pytest.raises(hm.HMError) as e:
        hm.hm_mvm_noalloc(D.handle, 1.0, None, x)
    assert e.value.status == hm.HM_EINVAL
    D.close()
