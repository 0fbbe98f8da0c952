"""Construction (input generator) invariants: Definitions of Sec. 2.1,
admissibility of Sec. 5.1, Algorithm 1, ACA exactness on a separable kernel."""

import ctypes as C

import numpy as np
import pytest

import hmgen
from hmgen import hmatrix as hm
from hmgen.hmatrix import truncate


def _clusters(H):
    L = hm.lib()
    h = C.c_void_p(H.handle)
    nc = L.hmg_num_clusters(h)
    b, e = np.empty(nc, np.int64), np.empty(nc, np.int64)
    s0, s1, lv = (np.empty(nc, np.int32) for _ in range(3))
    box = np.empty(6 * nc)
    L.hmg_get_clusters(h, b, e, s0, s1, lv, box)
    return b, e, s0, s1, box.reshape(nc, 6)


@pytest.fixture(scope="module")
def sphere4k():
    return hmgen.build_preset("sphere4k")


def test_cluster_tree_definition(sphere4k):
    H = sphere4k
    assert np.array_equal(np.sort(H.perm), np.arange(H.n))       # bijection
    b, e, s0, s1, box = _clusters(H)
    assert b[0] == 0 and e[0] == H.n                              # root = I
    P = H.points_cluster_order()
    for c in range(b.shape[0]):
        if s0[c] < 0:
            assert 0 < e[c] - b[c] <= H.leaf
        else:                                                     # sons partition the parent
            assert e[c] - b[c] > H.leaf
            assert b[s0[c]] == b[c] and e[s0[c]] == b[s1[c]] and e[s1[c]] == e[c]
        pts = P[b[c]:e[c]]
        assert np.all(pts >= box[c, :3]) and np.all(pts <= box[c, 3:])


def test_block_tree_tiles_product_exactly(sphere4k):
    H = sphere4k
    cover = np.zeros((H.n, H.n), np.int8)
    for i in range(H.nblocks):
        cover[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]] += 1
    assert cover.min() == 1 and cover.max() == 1


def test_admissibility_of_leaves(sphere4k):
    H = sphere4k
    b, e, s0, s1, box = _clusters(H)
    start = {int(b[c]) * (H.n + 1) + int(e[c]): c for c in range(b.shape[0])}

    def cl(lo, hi):
        return start[int(lo) * (H.n + 1) + int(hi)]

    def diam(c):
        return np.linalg.norm(box[c, 3:] - box[c, :3])

    def dist(c, d):
        gap = np.maximum(0, np.maximum(box[d, :3] - box[c, 3:], box[c, :3] - box[d, 3:]))
        return np.linalg.norm(gap)

    for i in range(H.nblocks):
        t, s = cl(H.rb[i], H.re[i]), cl(H.cb[i], H.ce[i])
        dd = dist(t, s)
        adm = dd > 0 and min(diam(t), diam(s)) <= H.eta * dd
        assert bool(H.adm[i]) == adm
        if not adm:
            assert s0[t] < 0 or s0[s] < 0          # inadmissible leaves sit at a leaf cluster


def test_truncation_eckart_young():
    rng = np.random.default_rng(5)
    m, n, r = 300, 200, 20
    Q1, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s = 10.0 ** -np.linspace(0, 9, r)
    # hand the factors over in a non-orthogonal form: U = Q1 diag(s) G, V = Q2 G^-T
    G = rng.standard_normal((r, r)) + 4 * np.eye(r)
    U = Q1 @ np.diag(s) @ G
    V = Q2 @ np.linalg.inv(G).T
    eps = 1e-5
    W, S, X = truncate(U, V, eps)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])                # tail[k] = |s[k:]|
    k_expected = int(np.argmax(tail <= eps * np.linalg.norm(s))) if (tail <= eps * np.linalg.norm(s)).any() else r
    assert W.shape[1] == k_expected
    np.testing.assert_allclose(S, s[:k_expected], rtol=1e-9)
    np.testing.assert_allclose(W.T @ W, np.eye(k_expected), atol=1e-12)
    np.testing.assert_allclose(X.T @ X, np.eye(k_expected), atol=1e-12)
    err = np.linalg.norm(U @ V.T - W @ np.diag(S) @ X.T)
    np.testing.assert_allclose(err, tail[k_expected], rtol=1e-4)


def test_aca_exact_on_separable_kernel():
    pts = hmgen.fibonacci_sphere(2048)
    H = hm.build_hmatrix(pts, hm.KERNEL_SEPARABLE, leaf=32, eps=1e-8)
    lr = H.adm != 0
    assert lr.any()
    assert np.all(H.rank[lr] == 1)
    P = H.points_cluster_order()
    for i in np.flatnonzero(lr)[:50]:
        U, V, _ = H.factors(i)
        A = np.outer(1 + P[H.rb[i]:H.re[i], 0], np.exp(P[H.cb[i]:H.ce[i], 1]))
        assert np.linalg.norm(A - U @ V.T) <= 1e-13 * np.linalg.norm(A)


def test_precision_groups_are_well_formed():
    H = hmgen.build_preset("sphere4k_mixed")
    lr = H.adm != 0
    assert np.all(H.group_cols[lr].sum(1) == H.rank[lr])
    assert np.all(H.ngroups >= 1)
    for i in range(H.nblocks):
        g = int(H.ngroups[i])
        dts = list(H.group_dtype[i][:g])
        assert len(set(dts)) == g                             # one group per format
        assert all(d in (hm.DT_F32, hm.DT_F16, hm.DT_BF16) for d in dts)
    used = set(H.group_dtype[lr, 0])
    assert hm.DT_F32 in used
    # FP16 carries the trailing singular vectors of many blocks
    has16 = [hm.DT_F16 in H.group_dtype[i][:H.ngroups[i]] for i in np.flatnonzero(lr)]
    assert np.mean(has16) > 0.5


def test_aplr_dfl_selection_meets_block_budget():
    """APLR over the DFL formats (Sec. 3.3): every block's storage error,
    recomputed with the oracle's own DFL rounding on the dense block, is
    within tol ||M_b||_F; groups are contiguous, at most 4, widening towards
    the large singular values; the budget is not met trivially (narrow
    formats are used)."""
    import oracle
    H = hmgen.build_preset("sphere4k_aplr")
    tol = hmgen.preset("sphere4k_aplr")["eps"] / 2
    width = [hm.DT_DFL16, hm.DT_DFL24, hm.DT_DFL32, hm.DT_DFL40, hm.DT_DFL48, hm.DT_F64]
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F64)
    used = set()
    for i in range(H.nblocks):
        a, b, s = H.factors(i)
        da, db, ds = dec[i]
        g = int(H.ngroups[i])
        dts = [int(d) for d in H.group_dtype[i][:g]]
        used |= set(dts)
        assert all(d in width for d in dts)
        if not H.adm[i]:
            assert g == 1
            M, Md = np.asarray(a), np.asarray(da)
        else:
            if int(H.rank[i]) == 0:
                continue
            assert H.group_cols[i][:g].sum() == H.rank[i] and g <= 4
            assert [width.index(d) for d in dts] == sorted((width.index(d) for d in dts), reverse=True)
            np.testing.assert_array_equal(ds, s)                 # s kept in FP64
            M = (np.asarray(a) * s) @ np.asarray(b).T
            Md = (np.asarray(da) * ds) @ np.asarray(db).T
        assert np.linalg.norm(M - Md) <= tol * np.linalg.norm(M) * (1 + 1e-9), i
    assert {hm.DT_DFL16, hm.DT_DFL24} <= used


def test_fill_in_shares_equals_fill_at_once(capsys):
    """Filling the leaves in 16 shares (with progress lines) gives the same
    ranks and factors, bit for bit, as one fill."""
    pts = hmgen.cube_points(3000, 0)
    H1 = hm.build_hmatrix(pts, hm.KERNEL_EXP, eps=1e-6, progress=False)
    H2 = hm.build_hmatrix(pts, hm.KERNEL_EXP, eps=1e-6, progress=True)
    assert capsys.readouterr().out.count("filled share") == 16
    np.testing.assert_array_equal(H1.rank, H2.rank)
    for i in range(H1.nblocks):
        for f1, f2 in zip(H1.factors(i), H2.factors(i)):
            if f1 is None:
                assert f2 is None
            else:
                np.testing.assert_array_equal(f1, f2)
