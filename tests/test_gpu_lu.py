"""GPU H-LU with accumulated updates (include/hm_lu.h) against the oracle
(oracle/hlu.py) and against what the factorisation must satisfy.

* n = 1024 (sphere and cube, eps 1e-6 and 1e-8, FP64 and DFL-compressed
  leaves): every leaf of L and U against the oracle's, as the matrix the
  leaf represents (its factors are unique only up to the truncation's
  choices); the ranks equal the oracle's on almost all leaves; the backward
  error |A - L U|_F / |A|_F within 5 eps (the oracle's pin) and
  ||I - A (L U)^-1||_2 within a factor 1.5 of the oracle's;
* the GPU triangular solves against dense triangular solves with the
  GPU's own factors;
* n = 4096 sphere: the solve's residual |A x - b| / |b| through the oracle's
  FP64 H-matrix-vector product, and the times of factorisation and solve;
* error paths: a second factorisation, a solve before it, a bad format.
"""

import sys
import time

import numpy as np
import pytest
from scipy.linalg import solve_triangular

import hmgen
import oracle
from hmgen import hmatrix as hmm
from oracle import hlu
from paper_2308_10960_amd import hm
from paper_2308_10960_amd.lu import DeviceHLU

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def build(geometry, n, eps):
    pts = hmgen.fibonacci_sphere(n) if geometry == "sphere" else hmgen.cube_points(n, 0)
    kern = hmm.KERNEL_LAPLACE if geometry == "sphere" else hmm.KERNEL_EXP
    return hmm.build_hmatrix(pts, kern, eps=eps)


def assemble(H, leaf_matrix):
    """Dense L and U from leaf matrices indexed like H's leaves."""
    tr = H.tree()
    n = H.n
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(H.nblocks):
        r = slice(int(H.rb[i]), int(H.re[i]))
        c = slice(int(H.cb[i]), int(H.ce[i]))
        M = leaf_matrix(i)
        if tr["tau"][i] == tr["sigma"][i]:
            L[r, c] += np.tril(M, -1)
            U[r, c] = np.triu(M)
        elif H.rb[i] > H.cb[i]:
            L[r, c] = M
        else:
            U[r, c] = M
    return L, U


@pytest.mark.parametrize("geometry,eps,compress", [("sphere", 1e-6, False), ("cube", 1e-6, False),
                                                   ("sphere", 1e-8, False), ("cube", 1e-6, True),
                                                   ("cube", 1e-8, True)])
def test_parity_1024(geometry, eps, compress):
    H = build(geometry, 1024, eps)
    dt = hmm.dfl_format(eps) if compress else None
    say(f"{geometry} n=1024 eps={eps} dtype={dt}")
    A = hlu.assemble_h(H)
    t = time.perf_counter()
    F = hlu.HLU(H, eps, dt=dt).factor()
    t_or = time.perf_counter() - t
    G = DeviceHLU(H)
    t = time.perf_counter()
    st = G.factor(eps, dt if dt is not None else hm.HM_F64)
    t_gpu = time.perf_counter() - t
    say(f"oracle {t_or:.2f}s ({F.truncations} truncations), GPU {t_gpu:.3f}s {st}")
    assert st["truncations"] == F.truncations
    tr = H.tree()
    worst, nrank_diff, nlr = 0.0, 0, 0
    for i in range(H.nblocks):
        key = (int(tr["tau"][i]), int(tr["sigma"][i]))
        Mo = F.leaf_matrix(*key)
        Mg = G.leaf(i)
        if H.adm[i]:
            Ug, _ = hm.hm_lu_leaf(G.handle, i, int(G.m[i]), int(G.nn[i]), False)
            nrank_diff += int(Ug.shape[1] != F.leaf[key][1].shape[1])
            nlr += 1
        worst = max(worst, np.linalg.norm(Mg - Mo) / max(np.linalg.norm(A[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]]),
                                                          1e-300))
    say(f"low-rank leaves whose rank differs from the oracle's: {nrank_diff} of {nlr}")
    assert nrank_diff <= 0.02 * nlr
    Lo, Uo = F.assemble()
    Lg, Ug = assemble(H, G.leaf)
    dL = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo)
    dU = np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo)
    back_g = np.linalg.norm(A - Lg @ Ug) / np.linalg.norm(A)
    back_o = np.linalg.norm(A - Lo @ Uo) / np.linalg.norm(A)
    e_g, e_o = hlu.lu_error(A, Lg, Ug), hlu.lu_error(A, Lo, Uo)
    say(f"|L_gpu - L_or| {dL:.2e}, |U_gpu - U_or| {dU:.2e}, worst leaf diff / |A_b| {worst:.2e}; "
        f"backward error GPU {back_g:.2e} oracle {back_o:.2e}; ||I - A (LU)^-1|| GPU {e_g:.3e} oracle {e_o:.3e}")
    assert back_g <= 5 * eps
    assert e_g <= 1.5 * e_o + 1e-12
    assert dL <= 10 * eps and dU <= 10 * eps


def test_solve_matches_dense_triangular_solves():
    H = build("sphere", 1024, 1e-6)
    G = DeviceHLU(H)
    G.factor(1e-6)
    Lg, Ug = assemble(H, G.leaf)
    rng = np.random.default_rng(3)
    B = rng.standard_normal((5, H.n))
    X = torch.from_numpy(B.copy()).cuda()
    G.solve(X)
    got = X.cpu().numpy().T
    want = solve_triangular(Ug, solve_triangular(Lg, B.T, lower=True, unit_diagonal=True), lower=False)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    say(f"solve vs dense triangular solves with the GPU factors: {rel:.2e}")
    assert rel <= 1e-11


def test_larger_sphere_solve_residual():
    n, eps = 4096, 1e-6
    H = build("sphere", n, eps)
    G = DeviceHLU(H)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = G.factor(eps)
    t_f = time.perf_counter() - t
    b = np.random.default_rng(5).standard_normal(n)
    X = torch.from_numpy(b.copy()).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    G.solve(X)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t
    x = X.cpu().numpy()
    r = np.linalg.norm(oracle.hmvm(H, x) - b) / np.linalg.norm(b)
    say(f"n={n}: factor {t_f:.2f}s, solve {t_s * 1e3:.1f}ms, {st}; residual |A x - b| / |b| = {r:.2e}")
    assert r <= 0.05


def test_error_paths():
    H = build("cube", 1024, 1e-6)
    G = DeviceHLU(H)
    X = torch.zeros((1, H.n), dtype=torch.float64, device="cuda")
    with pytest.raises(hm.HMError) as e:
        G.solve(X)
    assert e.value.status == hm.HM_ESTATE
    with pytest.raises(hm.HMError) as e:
        G.factor(1e-6, hm.HM_F32)
    assert e.value.status == hm.HM_EDTYPE
    G.factor(1e-6)
    with pytest.raises(hm.HMError) as e:
        G.factor(1e-6)
    assert e.value.status == hm.HM_ESTATE
