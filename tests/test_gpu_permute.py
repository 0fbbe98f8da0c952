"""GPU test of hm_permute: vectors between the caller's index order and
cluster order (the generator's permutation), both directions, FP64 and
FP32, several vectors with padded leading dimensions; out-of-range entries
are not dereferenced."""

import os
import sys

import numpy as np
import pytest

import hmgen
from paper_2308_10960_amd import hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(hm.LIB_PATH), "libhm.so must be built before the GPU tests"


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype", [hm.HM_F64, hm.HM_F32])
def test_permute_round_trip(dtype):
    H = hmgen.build_preset("sphere4k")
    n, nvec, ld = H.n, 3, H.n + 5
    perm = np.ascontiguousarray(H.perm, dtype=np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    tdt = torch.float64 if dtype == hm.HM_F64 else torch.float32
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (nvec, ld))
    Xd = torch.from_numpy(X).to(tdt).cuda()
    Pd = torch.from_numpy(perm).cuda()
    Cd = torch.full((nvec, ld), -7.0, dtype=tdt, device="cuda")
    say("gather", dtype, n, nvec)
    hm.hm_permute(Pd, n, dtype, 0, nvec, Xd, ld, Cd, ld)
    torch.cuda.synchronize()
    C = Cd.cpu().numpy()
    Xr = Xd.cpu().numpy()
    np.testing.assert_array_equal(C[:, :n], Xr[:, perm])           # into cluster order
    assert np.all(C[:, n:] == -7.0)                                 # padding untouched
    Bd = torch.full((nvec, ld), -7.0, dtype=tdt, device="cuda")
    hm.hm_permute(Pd, n, dtype, 1, nvec, Cd, ld, Bd, ld)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Bd.cpu().numpy()[:, :n], Xr[:, :n])   # and back
    # an entry outside [0, n): gather writes NaN there, scatter skips it
    bad = perm.copy()
    bad[17] = n
    Pb = torch.from_numpy(bad).cuda()
    hm.hm_permute(Pb, n, dtype, 0, 1, Xd, ld, Cd, ld)
    Sd = torch.full((1, ld), -7.0, dtype=tdt, device="cuda")
    hm.hm_permute(Pb, n, dtype, 1, 1, Xd, ld, Sd, ld)
    torch.cuda.synchronize()
    C = Cd.cpu().numpy()[0]
    assert np.isnan(C[17]) and np.array_equal(np.delete(C[:n], 17), np.delete(Xr[0, perm], 17))
    S = Sd.cpu().numpy()[0]
    assert S[perm[17]] == -7.0                                      # that position got nothing
    with pytest.raises(hm.HMError):
        hm.hm_permute(Pd, n, hm.HM_F16, 0, 1, Xd, ld, Cd, ld)
    with pytest.raises(hm.HMError):
        hm.hm_permute(Pd, n, dtype, 2, 1, Xd, ld, Cd, ld)
