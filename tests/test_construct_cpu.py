"""Host side of the GPU construction (include/hm_construct.h), no GPU:
region layout and the synchronous argument checks, which reject a call
before anything touches the device."""

import numpy as np
import pytest

from paper_2308_10960_amd import hm


def _blocks(spec):
    b = np.zeros(len(spec), hm.CBLOCK_DTYPE)
    for i, (rb, cb, m, n, adm, cap) in enumerate(spec):
        b[i] = (rb, cb, m, n, adm, cap, 0, 0)
    return b


def test_layout_regions_follow_each_other():
    b = _blocks([(0, 0, 40, 30, 0, 0), (0, 40, 64, 200, 1, 0), (64, 0, 300, 500, 1, 17), (0, 0, 5, 3, 1, 0)])
    out_d, scr_d = hm.hm_construct_layout(b)
    assert list(b["cap"]) == [0, 64, 17, 3]
    align2 = lambda v: (v + 1) // 2 * 2
    o = [align2(40 * 30), align2((64 + 200) * 64 + 64), align2((300 + 500) * 17 + 17), align2((5 + 3) * 3 + 3)]
    s = [0, align2((64 + 200) * 64 + (64 + 7) // 8), align2((300 + 500) * 17 + (300 + 7) // 8),
         align2((5 + 3) * 3 + 1)]
    assert list(b["out"]) == list(np.cumsum([0] + o[:-1]))
    assert list(b["scr"]) == list(np.cumsum([0] + s[:-1]))
    assert out_d == sum(o) and scr_d == sum(s)
    big = _blocks([(0, 0, 1000, 1000, 1, 0)])
    hm.hm_construct_layout(big)
    assert big["cap"][0] == hm.HM_CONSTRUCT_MAX_RANK


@pytest.mark.parametrize("spec", [[(0, 0, 0, 4, 0, 0)], [(0, 0, 4, 4, 2, 0)], [(0, 0, 4, 8, 1, 5)],
                                  [(0, 0, 400, 400, 1, hm.HM_CONSTRUCT_MAX_RANK + 1)]])
def test_layout_rejects_bad_leaves(spec):
    with pytest.raises(hm.HMError) as e:
        hm.hm_construct_layout(_blocks(spec))
    assert e.value.status == hm.HM_EINVAL


def _call(blocks, n_points=100, kernel=hm.HM_KERNEL_LAPLACE, params=(0.1, 0.0), eps=1e-6, out=10 ** 6,
          scr=10 ** 6, desc=4096):
    # fake device addresses: every case below fails validation before any use
    hm.hm_construct(0x1000, n_points, blocks, 0x2000, desc, kernel, params, eps / 10, eps, False,
                    0x3000, out, 0x4000, scr, 0x5000)


@pytest.mark.parametrize("case", ["outside", "kernel", "param", "eps", "desc", "region", "cap"])
def test_construct_rejects_before_launch(case):
    b = _blocks([(0, 0, 40, 30, 0, 0), (40, 0, 60, 40, 1, 0)])
    hm.hm_construct_layout(b)
    kw = {}
    if case == "outside":
        b["rb"][1] = 50                      # rows 50 .. 109 of 100 points
    elif case == "kernel":
        kw["kernel"] = 7
    elif case == "param":
        kw["params"] = (0.0, 0.0)
    elif case == "eps":
        kw["eps"] = 0.0
    elif case == "desc":
        kw["desc"] = 8
    elif case == "region":
        kw["out"] = 8 * int(b["out"][1])        # the second leaf's output does not fit
    elif case == "cap":
        b["cap"][1] = 41
    with pytest.raises(hm.HMError) as e:
        _call(b, **kw)
    assert e.value.status in (hm.HM_EINVAL, hm.HM_ENOMEM)
