"""Pins that tie the oracle to something other than itself.

P1 brute force: |y_H - A x| <= 2 eps |A|_F |x| (Eq. (1) per block) and the
   per-block bound, with A assembled densely from the points in numpy.
P2 placement: dense assembly of the stored blocks then a numpy gemv.
P3 special cases: all-dense partitions equal A @ x; a separable kernel
   (exact rank one) equals f (g^T x).
P5 kernel identity: the Matern covariance of Sec. 5.1 at nu = 1/2 is exp(-d/l).
P7 linearity, y += semantics, x = 0.
P8 physics: Laplace on the unit sphere with x = 1 has row sums ~ n/(4 pi).
Plus: the decoded (mixed-precision) oracle stays within the block-relative
storage accuracy, and planted mistakes are caught by these pins.  P1 and P2
also run on matrices whose low-rank leaves keep s (W diag(s) X^T, Sec. 3.3),
so the oracle's s step is pinned: s applied twice, a neighbouring column's s
or s ignored each break them.
"""

import math

import numpy as np
import pytest
from scipy.special import gamma, kv

import hmgen
import oracle
from hmgen import hmatrix as hm


def dense_kernel(H):
    """The kernel matrix in cluster order, assembled in numpy from the points."""
    P = H.points_cluster_order()
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    if H.kernel == hm.KERNEL_LAPLACE:
        np.fill_diagonal(d, 1.0)
        A = 1.0 / (4 * math.pi * d)
        np.fill_diagonal(A, 1.0 / (4 * math.pi * H.kparams[0]))
    elif H.kernel == hm.KERNEL_EXP:
        A = np.exp(-d / H.kparams[0])
        A[np.diag_indices_from(A)] += H.kparams[1]
    else:
        A = np.outer(1 + P[:, 0], np.exp(P[:, 1]))
    return A


def assemble(H, factors=None):
    """Dense H-matrix from the block table (placement check)."""
    A = np.zeros((H.n, H.n))
    for i in range(H.nblocks):
        a, b, s = factors[i] if factors is not None else H.factors(i)
        if not H.adm[i]:
            blk = a
        else:
            blk = (a * s) @ b.T if s is not None else a @ b.T
        A[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]] += blk
    return A


@pytest.fixture(scope="module")
def sphere4k():
    return hmgen.build_preset("sphere4k")


@pytest.fixture(scope="module")
def cube4k():
    return hmgen.build_preset("cube4k")


@pytest.mark.parametrize("which", ["sphere4k", "cube4k"])
def test_p1_brute_force_bound(which, request):
    H = request.getfixturevalue(which)
    A = dense_kernel(H)
    x = hmgen.uniform_vector(H.n)
    y = oracle.hmvm(H, x)
    err = np.linalg.norm(y - A @ x)
    assert err <= 2 * H.eps * np.linalg.norm(A) * np.linalg.norm(x)
    worst = 0.0
    for i in np.flatnonzero(H.adm):
        U, V, _ = H.factors(i)
        Ab = A[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]]
        worst = max(worst, np.linalg.norm(Ab - U @ V.T) / np.linalg.norm(Ab))
    assert worst <= 2 * H.eps
    # dense leaves hold the kernel (to the last bit of libm vs numpy exp/sqrt)
    for i in np.flatnonzero(H.adm == 0)[:200]:
        D, _, _ = H.factors(i)
        np.testing.assert_allclose(D, A[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]], rtol=5e-16, atol=0)


def test_p2_dense_assembly(sphere4k):
    H = sphere4k
    At = assemble(H)
    x = hmgen.uniform_vector(H.n, seed=7)
    ref = At @ x
    y = oracle.hmvm(H, x)
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref) * 10


@pytest.mark.parametrize("mode", ["eta0", "one_leaf"])
def test_p3_all_dense_equals_gemv(mode):
    pts = hmgen.fibonacci_sphere(1024)
    if mode == "eta0":
        H = hm.build_hmatrix(pts, hm.KERNEL_LAPLACE, leaf=32, eta=0.0)
        assert H.nblocks > 1
    else:
        H = hm.build_hmatrix(pts, hm.KERNEL_LAPLACE, leaf=2048)
        assert H.nblocks == 1
    assert not H.adm.any()
    A = dense_kernel(H)
    x = hmgen.uniform_vector(H.n)
    y = oracle.hmvm(H, x)
    ref = A @ x
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref) * 10


def test_p3_separable_kernel():
    pts = hmgen.cube_points(3000, seed=11)
    H = hm.build_hmatrix(pts, hm.KERNEL_SEPARABLE, leaf=16, eps=1e-10)
    P = H.points_cluster_order()
    f, g = 1 + P[:, 0], np.exp(P[:, 1])
    x = hmgen.uniform_vector(H.n, seed=3)
    ref = f * (g @ x)
    y = oracle.hmvm(H, x)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


def test_p5_matern_half_is_exponential():
    # C(d) = s2 2^(1-nu)/Gamma(nu) (sqrt(2 nu) d / l)^nu K_nu(sqrt(2 nu) d / l)
    nu, ell, s2 = 0.5, 0.1, 1.0
    d = np.linspace(1e-4, 2.0, 2000)
    z = math.sqrt(2 * nu) * d / ell
    C = s2 * 2 ** (1 - nu) / gamma(nu) * z ** nu * kv(nu, z)
    np.testing.assert_allclose(C, np.exp(-d / ell), rtol=1e-12, atol=1e-300)


def test_p7_linearity_and_update_semantics(sphere4k):
    H = sphere4k
    x = hmgen.uniform_vector(H.n, seed=1)
    z = hmgen.uniform_vector(H.n, seed=2)
    y0 = hmgen.uniform_vector(H.n, seed=9)
    a, b = 0.7, -1.3
    lhs = oracle.hmvm(H, a * x + b * z)
    rhs = a * oracle.hmvm(H, x) + b * oracle.hmvm(H, z)
    assert np.linalg.norm(lhs - rhs) <= 1e-14 * np.linalg.norm(lhs) * 10
    np.testing.assert_array_equal(oracle.hmvm(H, np.zeros(H.n), y0), y0)     # x = 0
    with_y0 = oracle.hmvm(H, x, y0, alpha=2.5)
    np.testing.assert_allclose(with_y0 - y0, 2.5 * oracle.hmvm(H, x), rtol=0, atol=1e-12)


def test_p8_sphere_row_sums(sphere4k):
    H = sphere4k
    y = oracle.hmvm(H, np.ones(H.n))
    ratio = y / (H.n / (4 * math.pi))
    assert np.all(np.abs(ratio - 1) < 0.05)


def test_multi_rhs_is_columnwise(sphere4k):
    H = sphere4k
    X = hmgen.gaussian_block(H.n, 5)
    Y = oracle.hmvm_multi(H, X)
    for c in range(5):
        np.testing.assert_array_equal(Y[:, c], oracle.hmvm(H, X[:, c]))


def test_sampled_rows_from_covering_leaves(sphere4k):
    """Rows of y from the leaves that cover them: against the densely
    assembled matrix at those rows (P2), and bit for bit the full sum there
    (same leaves in the same order); the subset is exactly the leaves that
    touch a sampled row."""
    H = sphere4k
    rng = np.random.default_rng(5)
    rows = np.concatenate([[0, H.n - 1], rng.choice(H.n, 40, replace=False)])
    blk = oracle.blocks_in_rows(H, rows)
    touch = [i for i in range(H.nblocks) if np.any((rows >= H.rb[i]) & (rows < H.re[i]))]
    np.testing.assert_array_equal(blk, touch)
    assert 0 < blk.size < H.nblocks
    X = hmgen.gaussian_block(H.n, 3)
    part = oracle.hmvm_multi(H, X, blocks=blk)
    full = oracle.hmvm_multi(H, X)
    np.testing.assert_array_equal(part[rows], full[rows])
    At = assemble(H)
    ref = At[rows] @ X
    assert np.linalg.norm(part[rows] - ref) <= 1e-13 * np.linalg.norm(ref)
    dec_all = oracle.decoded_factors(H, sigma_dtype=oracle.F64)
    dec_sub = oracle.decoded_factors(H, sigma_dtype=oracle.F64, blocks=blk)
    for q, i in enumerate(blk):
        np.testing.assert_array_equal(dec_sub[q][0], dec_all[i][0])
    np.testing.assert_array_equal(oracle.hmvm(H, X[:, 0], factors=dec_sub, blocks=blk)[rows],
                                  oracle.hmvm(H, X[:, 0], factors=dec_all)[rows])


def test_decoded_oracle_within_storage_accuracy():
    H = hmgen.build_preset("sphere4k_mixed")
    tol = hmgen.presets.MIXED_TOL / 2
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F32)
    worst = 0.0
    for i in range(H.nblocks):
        a, b, s = H.factors(i)
        da, db, ds = dec[i]
        if not H.adm[i]:
            exact, stored = a, da
        else:
            exact, stored = (a * s) @ b.T, (da * ds) @ db.T
        e = np.linalg.norm(exact - stored) / np.linalg.norm(exact)
        worst = max(worst, e)
        assert e <= tol * (1 + 1e-6)
        assert np.linalg.norm(exact - stored) <= H.store_err_bound[i] * (1 + 1e-6) + 1e-300
    assert worst > tol / 20          # formats were actually lowered
    x = hmgen.uniform_vector(H.n)
    y_truth = oracle.hmvm(H, x)
    y_dec = oracle.hmvm(H, x, factors=dec)
    rel = np.linalg.norm(y_dec - y_truth) / np.linalg.norm(y_truth)
    assert 0 < rel <= 1e-6


def test_planted_mistakes_are_caught():
    """Each plausible oracle mistake (dropped block, wrong sign, transposed
    factors, shifted column index) breaks P3's separable-kernel pin."""
    pts = hmgen.cube_points(1500, seed=4)
    H = hm.build_hmatrix(pts, hm.KERNEL_SEPARABLE, leaf=16, eps=1e-10)
    P = H.points_cluster_order()
    ref_fn = lambda x: (1 + P[:, 0]) * (np.exp(P[:, 1]) @ x)
    x = hmgen.uniform_vector(H.n, seed=8)
    ref = ref_fn(x)
    base = [tuple(None if v is None else np.asfortranarray(v) for v in H.factors(i))
            for i in range(H.nblocks)]
    ok = oracle.hmvm(H, x, factors=base)
    assert np.linalg.norm(ok - ref) <= 1e-12 * np.linalg.norm(ref)
    lr = np.flatnonzero(H.adm)
    sq = [i for i in lr if H.re[i] - H.rb[i] == H.ce[i] - H.cb[i]]
    assert sq

    def broken(mutate):
        f = [tuple(None if v is None else v.copy(order="F") for v in t) for t in base]
        mutate(f)
        y = oracle.hmvm(H, x, factors=f)
        return np.linalg.norm(y - ref) / np.linalg.norm(ref)

    def drop(f):
        i = int(lr[0])
        f[i] = (np.zeros_like(f[i][0], order="F"), f[i][1], None)

    def sign(f):
        i = int(np.flatnonzero(H.adm == 0)[0])
        f[i] = (np.asfortranarray(-f[i][0]), None, None)

    def transpose(f):
        i = int(sq[0])
        f[i] = (f[i][1].copy(order="F"), f[i][0].copy(order="F"), None)

    for mut in (drop, sign, transpose):
        assert broken(mut) > 1e-6
    # a shifted column window (off-by-one in E_sigma) on one dense block
    bad = hm.HMatrix(**{k: getattr(H, k) for k in (
        "n", "points", "kernel", "kparams", "leaf", "eta", "eps", "keep_sigma", "perm", "rb",
        "re", "adm", "rank", "a_ptr", "b_ptr", "s_ptr")}, cb=H.cb.copy(), ce=H.ce.copy())
    i = int(np.flatnonzero((H.adm == 0) & (H.cb > 0))[0])
    bad.cb[i] -= 1
    bad.ce[i] -= 1
    y = oracle.hmvm(bad, x)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) > 1e-6


# ---------------------------------------------------------------- the sigma step
# Low-rank leaves kept in the form W diag(s) X^T (Sec. 3.3): the oracle scales
# t = X^T x by s before applying W.  These pins run on matrices built with s
# kept, so that a mistake in that step (s applied twice, a neighbouring
# column's s, s ignored) moves the result far outside every bound.

@pytest.fixture(scope="module")
def sphere4k_sigma():
    pts = hmgen.fibonacci_sphere(4096)
    return hm.build_hmatrix(pts, hm.KERNEL_LAPLACE, leaf=64, eta=2.0, eps=1e-6, keep_sigma=True)


def _sigma_spread(H):
    """Largest ratio between neighbouring singular values of one leaf, and
    the largest |log s|: a pin on the s step is only as sharp as these."""
    spread, scale = 1.0, 0.0
    for i in np.flatnonzero(H.adm):
        _, _, s = H.factors(i)
        if s.size > 1:
            spread = max(spread, float(np.max(s[:-1] / s[1:])))
        if s.size:
            scale = max(scale, float(np.max(np.abs(np.log(s)))))
    return spread, scale


def test_p1_brute_force_bound_sigma_form(sphere4k_sigma):
    """P1 on a matrix whose low-rank leaves carry s: the product is within
    2 eps |A|_F |x| of the dense kernel matrix, and every leaf's
    W diag(s) X^T within 2 eps of its block."""
    H = sphere4k_sigma
    assert H.keep_sigma
    spread, scale = _sigma_spread(H)
    assert spread > 10 and scale > 3          # s far from 1 and far from its neighbours
    A = dense_kernel(H)
    x = hmgen.uniform_vector(H.n)
    y = oracle.hmvm(H, x)
    assert np.linalg.norm(y - A @ x) <= 2 * H.eps * np.linalg.norm(A) * np.linalg.norm(x)
    worst = 0.0
    for i in np.flatnonzero(H.adm):
        W, X, s = H.factors(i)
        Ab = A[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]]
        worst = max(worst, np.linalg.norm(Ab - (W * s) @ X.T) / np.linalg.norm(Ab))
        # W and X are orthonormal (Alg. 1), so s carries the whole scale
        np.testing.assert_allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-12)
        np.testing.assert_allclose(X.T @ X, np.eye(X.shape[1]), atol=1e-12)
    assert worst <= 2 * H.eps


@pytest.mark.parametrize("name", ["sphere4k_mixed", "sphere4k_aplr"])
def test_p2_dense_assembly_sigma_form(name):
    """P2 on the mixed-precision and APLR matrices (s kept): the densely
    assembled matrix times x equals the oracle, both for the unrounded
    factors and for the decoded ones the parity tests use."""
    H = hmgen.build_preset(name)
    assert H.keep_sigma
    sig = oracle.F32 if name.endswith("mixed") else oracle.F64
    dec = oracle.decoded_factors(H, sigma_dtype=sig)
    x = hmgen.uniform_vector(H.n, seed=7)
    for factors in (None, dec):
        ref = assemble(H, factors) @ x
        y = oracle.hmvm(H, x, factors=factors)
        assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    # the decoded s really differs from the unrounded one (FP32) where it should
    if sig == oracle.F32:
        i = int(np.flatnonzero(H.adm)[0])
        assert np.any(dec[i][2] != H.factors(i)[2])


def test_planted_sigma_mistakes_are_caught(sphere4k_sigma):
    """An oracle that applies s twice, takes the neighbouring column's s or
    ignores s computes the correct product of mutated s; each such product
    breaks P1's bound and P2's assembly of the true factors."""
    H = sphere4k_sigma
    A = dense_kernel(H)
    x = hmgen.uniform_vector(H.n, seed=8)
    ref = assemble(H) @ x
    bound = 2 * H.eps * np.linalg.norm(A) * np.linalg.norm(x)
    base = [tuple(None if v is None else np.array(v, order="F") for v in H.factors(i))
            for i in range(H.nblocks)]
    assert np.linalg.norm(oracle.hmvm(H, x, factors=base) - ref) <= 1e-13 * np.linalg.norm(ref)

    def with_sigma(fn):
        return [t if t[2] is None else (t[0], t[1], np.ascontiguousarray(fn(t[2]))) for t in base]

    mistakes = {
        "twice": lambda s: s * s,
        "next column": lambda s: np.roll(s, -1),
        "previous column": lambda s: np.roll(s, 1),
        "ignored": lambda s: np.ones_like(s),
    }
    for what, fn in mistakes.items():
        y = oracle.hmvm(H, x, factors=with_sigma(fn))
        assert np.linalg.norm(y - A @ x) > bound, what
        assert np.linalg.norm(y - ref) > 1e-3 * np.linalg.norm(ref), what
