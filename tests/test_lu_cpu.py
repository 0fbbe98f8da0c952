"""Host-side validation of hm_lu_create (include/hm_lu.h), which runs before
any device call: a block tree that the leaves do not tile, a repeated leaf,
a diagonal leaf that is low rank or too large, a bad rank, a broken cluster
tree.  No GPU needed."""

import numpy as np
import pytest

import hmgen
from hmgen import hmatrix as hmm
from paper_2308_10960_amd import hm


@pytest.fixture(scope="module")
def small():
    return hmm.build_hmatrix(hmgen.fibonacci_sphere(1024), hmm.KERNEL_LAPLACE, eps=1e-6)


def args(H):
    tr = H.tree()
    kind = (np.asarray(H.adm) != 0).astype(np.int32)
    rank = np.where(kind == 1, H.rank, 0).astype(np.int32)
    return dict(begin=tr["begin"].copy(), end=tr["end"].copy(), son0=tr["son0"].copy(), son1=tr["son1"].copy(),
                tau=tr["tau"].astype(np.int32), sigma=tr["sigma"].astype(np.int32), kind=kind, rank=rank,
                a_ptrs=np.asarray(H.a_ptr, np.uint64).copy(), b_ptrs=np.asarray(H.b_ptr, np.uint64).copy())


def create(a, arena=1 << 30):
    return hm.hm_lu_create(a["begin"], a["end"], a["son0"], a["son1"], a["tau"], a["sigma"], a["kind"], a["rank"],
                           a["a_ptrs"], a["b_ptrs"], arena)


def expect(status, a):
    with pytest.raises(hm.HMError) as e:
        create(a)
    assert e.value.status == status, str(e.value)


def drop(a, i):
    return {k: (np.delete(v, i) if k in ("tau", "sigma", "kind", "rank", "a_ptrs", "b_ptrs") else v)
            for k, v in a.items()}


def test_missing_leaf(small):
    expect(hm.HM_EPARTITION, drop(args(small), 7))


def test_repeated_leaf(small):
    a = args(small)
    a["tau"][3], a["sigma"][3] = a["tau"][4], a["sigma"][4]
    expect(hm.HM_EPARTITION, a)


def test_leaf_above_the_tree(small):
    a = args(small)                   # a leaf on a block above other leaves: (son 0, son 1) of the root
    extra = {"tau": a["son0"][0], "sigma": a["son1"][0], "kind": 0, "rank": 0}
    for k in ("tau", "sigma", "kind", "rank"):
        a[k] = np.append(a[k], extra[k]).astype(np.int32)
    for k in ("a_ptrs", "b_ptrs"):
        a[k] = np.append(a[k], a[k][0]).astype(np.uint64)
    expect(hm.HM_EPARTITION, a)


def test_low_rank_diagonal(small):
    a = args(small)
    d = int(np.flatnonzero(a["tau"] == a["sigma"])[0])
    a["kind"][d] = 1
    expect(hm.HM_ESHAPE, a)


def test_bad_rank(small):
    a = args(small)
    i = int(np.flatnonzero(a["kind"] == 1)[0])
    a["rank"][i] = 10 ** 6
    expect(hm.HM_ESHAPE, a)


def test_broken_cluster_tree(small):
    a = args(small)
    c = int(np.flatnonzero(a["son0"] >= 0)[0])
    a["son1"][c] = -1
    expect(hm.HM_EINVAL, a)
    a = args(small)
    a["end"][a["son0"][c]] -= 1                            # sons no longer split the cluster
    expect(hm.HM_EINVAL, a)


def test_diagonal_leaf_too_large():
    H = hmm.build_hmatrix(hmgen.fibonacci_sphere(512), hmm.KERNEL_LAPLACE, eps=1e-6, leaf=128)
    a = args(H)
    expect(hm.HM_ESHAPE, a)
