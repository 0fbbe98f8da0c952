"""Pins of the H-LU oracle (oracle/hlu.py) against what the mathematics
fixes, not against the oracle itself:

* an H-matrix whose leaves are all dense (admissibility never met) has an
  H-LU that is the block LU of a dense matrix; with eps at rounding level
  the truncated sums of the updates are exact, so L U must equal A to
  rounding, with L unit lower and U upper triangular (the unpivoted LU is
  unique, so this characterises it);
* with low-rank leaves and a tiny eps the same holds to 1e-11;
* at eps in {1e-4, 1e-6, 1e-8} the backward error |A - L U|_F / |A|_F stays
  within a small multiple of eps, and (L U)^-1 solves A x = b with the
  residual that ||I - A (L U)^-1||_2 allows;
* with compression of the final leaves and accumulators in FP64 the error
  of the factorisation on the well-conditioned cube matrix equals the
  uncompressed one (Sec. 4.1);
* Alg. 1's rank rule: the smallest rank meeting the Frobenius tail bound;
* planted mistakes (a sign, a dropped Schur update, a transposed solve) fail
  the exactness pin.
"""

import numpy as np
import pytest

import hmgen
from hmgen import hmatrix as hmm
from oracle import hlu


def build(geometry, n, eps, eta=2.0):
    pts = hmgen.fibonacci_sphere(n) if geometry == "sphere" else hmgen.cube_points(n, 0)
    kern = hmm.KERNEL_LAPLACE if geometry == "sphere" else hmm.KERNEL_EXP
    return hmm.build_hmatrix(pts, kern, eps=eps, eta=eta)


def check_structure(L, U):
    n = L.shape[0]
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) == 1.0)
    assert np.all(np.tril(U, -1) == 0)
    assert np.all(np.abs(np.diag(U)) > 0)


@pytest.mark.parametrize("geometry", ["sphere", "cube"])
def test_all_dense_is_block_lu(geometry):
    H = build(geometry, 1024, 1e-6, eta=1e-9)
    assert not np.any(H.adm)
    A = hlu.assemble_h(H)
    F = hlu.HLU(H, 1e-15).factor()
    L, U = F.assemble()
    check_structure(L, U)
    err = np.linalg.norm(A - L @ U) / np.linalg.norm(A)
    assert err <= 1e-13, err


@pytest.mark.parametrize("geometry", ["sphere", "cube"])
def test_tiny_eps_exact(geometry):
    H = build(geometry, 1024, 1e-12)
    assert np.any(H.adm)
    A = hlu.assemble_h(H)
    F = hlu.HLU(H, 1e-14).factor()
    L, U = F.assemble()
    check_structure(L, U)
    err = np.linalg.norm(A - L @ U) / np.linalg.norm(A)
    assert err <= 1e-11, err


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
@pytest.mark.parametrize("geometry", ["sphere", "cube"])
def test_backward_error_scales_with_eps(geometry, eps):
    H = build(geometry, 1024, eps)
    A = hlu.assemble_h(H)
    F = hlu.HLU(H, eps).factor()
    L, U = F.assemble()
    check_structure(L, U)
    back = np.linalg.norm(A - L @ U) / np.linalg.norm(A)
    assert 0.02 * eps <= back <= 5 * eps, back
    fwd = hlu.lu_error(A, L, U)
    b = np.random.default_rng(1).standard_normal(H.n)
    x = F.solve(b)[:, 0]
    assert np.linalg.norm(A @ x - b) <= 1.01 * fwd * np.linalg.norm(b) + 1e-12


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_compressed_cube_equals_uncompressed(eps):
    H = build("cube", 1024, eps)
    A = hlu.assemble_h(H)
    L, U = hlu.HLU(H, eps).factor().assemble()
    Lc, Uc = hlu.HLU(H, eps, dt=hmm.dfl_format(eps)).factor().assemble()
    e, ec = hlu.lu_error(A, L, U), hlu.lu_error(A, Lc, Uc)
    assert 0.8 * e <= ec <= 1.25 * e, (e, ec)


def test_trunc_rank_rule():
    rng = np.random.default_rng(0)
    U = rng.standard_normal((60, 12)) * np.logspace(0, -9, 12)
    V = rng.standard_normal((50, 12))
    M = U @ V.T
    S = np.linalg.svd(M, compute_uv=False)
    for eps in [1e-2, 1e-4, 1e-6]:
        W, X = hlu.truncate(U, V, eps)
        k = W.shape[1]
        assert np.linalg.norm(M - W @ X.T) <= eps * np.linalg.norm(M) * (1 + 1e-10)
        # one rank less misses the bound (SVD of the product, computed directly)
        assert np.sqrt(np.sum(S[k - 1:] ** 2)) > eps * np.linalg.norm(M)
    assert hlu.trunc_rank(np.zeros(4), 1e-6) == 0


class _SignFlip(hlu.HLU):
    def apply(self, t, s, acc):
        if acc is not None:
            acc = (acc[0], -acc[1]) + tuple(acc[2:])
        super().apply(t, s, acc)


class _NoSchur(hlu.HLU):
    def lu(self, t, acc=None, pend=None):
        acc, pend = self.gather(t, t, acc, pend or [])
        if self.is_leaf(t, t):
            return super().lu(t, acc, [])
        t0, t1 = self.sons[t]
        sub = self.split(t, t, acc, pend)
        self.lu(t0, *sub[0, 0])
        self.solve_l(t0, t1, *sub[0, 1])
        self.solve_u(t1, t0, *sub[1, 0])
        self.lu(t1, *sub[1, 1])                              # Schur update dropped


class _TransposedSolve(hlu.HLU):
    def solve_upper_t(self, s, Z):
        D = self.leaf.get((s, s))
        if D is not None:
            from scipy.linalg import solve_triangular
            return solve_triangular(D[1], Z, lower=False)    # U^-1 instead of U^-T
        return super().solve_upper_t(s, Z)


@pytest.mark.parametrize("cls", [_SignFlip, _NoSchur, _TransposedSolve])
def test_planted_mistakes_fail(cls):
    H = build("sphere", 1024, 1e-12)
    A = hlu.assemble_h(H)
    try:
        L, U = cls(H, 1e-14).factor().assemble()
        err = np.linalg.norm(A - L @ U) / np.linalg.norm(A)
    except (ValueError, np.linalg.LinAlgError):                # the mistake blew up the factors
        err = np.inf
    assert not err <= 1e-6
