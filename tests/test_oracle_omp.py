"""The all-cores timing variant of the oracle (OpenMP over ranges of rows,
t_b per block first) is bitwise the plain single-threaded oracle for any
thread count and any cut of the rows: every output entry receives the same
additions in the same order.  It is what the CPU baseline times on all
cores; the plain loop stays the pinned oracle."""

import numpy as np
import pytest

import hmgen
import oracle


@pytest.mark.parametrize("name,n", [("sphere4k", 4096), ("sphere4k_mixed", 8192), ("cube4k", 4096),
                                    ("sphere4k_e8_mixed", 4096)])
def test_omp_variant_bitwise_equal(name, n):
    H = hmgen.build_preset(name, n=n)
    x = hmgen.uniform_vector(H.n, seed=3)
    y0 = hmgen.uniform_vector(H.n, seed=4)
    ref = oracle.hmvm(H, x, y0, alpha=-0.7)
    for nthreads, rows in [(1, 64), (2, 1), (3, 17), (8, 64), (4, 100000)]:
        y, used = oracle.hmvm_omp(H, x, y0, alpha=-0.7, nthreads=nthreads, rows_per_task=rows)
        assert used == nthreads
        np.testing.assert_array_equal(y, ref)
    if H.keep_sigma:
        dec = oracle.decoded_factors(H, sigma_dtype=oracle.F32)
        y, _ = oracle.hmvm_omp(H, x, factors=dec, nthreads=4)
        np.testing.assert_array_equal(y, oracle.hmvm(H, x, factors=dec))


def test_omp_variant_planted_mistake_differs():
    """A planted mistake in the inputs (one block's s doubled) changes the
    all-cores result the same way as the plain one: both compute the same
    function of the factors, not a cached value."""
    H = hmgen.build_preset("sphere4k_mixed")
    x = hmgen.uniform_vector(H.n, seed=5)
    base = [tuple(None if v is None else np.array(v, order="F") for v in H.factors(i))
            for i in range(H.nblocks)]
    i = int(np.flatnonzero(H.adm)[0])
    bad = list(base)
    bad[i] = (base[i][0], base[i][1], base[i][2] * 2)
    y_ok, _ = oracle.hmvm_omp(H, x, factors=base, nthreads=4)
    y_bad, _ = oracle.hmvm_omp(H, x, factors=bad, nthreads=4)
    np.testing.assert_array_equal(y_bad, oracle.hmvm(H, x, factors=bad))
    assert np.linalg.norm(y_bad - y_ok) > 0
