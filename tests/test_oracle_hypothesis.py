"""Property tests on small random geometries: the block tree tiles I x J,
the oracle meets the brute-force bound (P1) and matches dense assembly (P2)."""

import numpy as np
from hypothesis import given, settings, strategies as st, HealthCheck

import hmgen
import oracle
from hmgen import hmatrix as hm
from test_oracle_pins import dense_kernel, assemble


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(n=st.integers(64, 900), leaf=st.integers(8, 64), eta=st.sampled_from([0.5, 1.0, 2.0]),
       geo=st.sampled_from(["sphere", "cube"]), kern=st.sampled_from(["laplace", "exp"]),
       seed=st.integers(0, 1000))
def test_random_geometries(n, leaf, eta, geo, kern, seed):
    pts = hmgen.fibonacci_sphere(n) if geo == "sphere" else hmgen.cube_points(n, seed)
    k = hm.KERNEL_LAPLACE if kern == "laplace" else hm.KERNEL_EXP
    eps = 1e-6
    H = hm.build_hmatrix(pts, k, leaf=leaf, eta=eta, eps=eps, length=0.2)
    cover = np.zeros((n, n), np.int16)
    for i in range(H.nblocks):
        cover[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]] += 1
    assert cover.min() == 1 and cover.max() == 1
    A = dense_kernel(H)
    x = hmgen.uniform_vector(n, seed=seed)
    y = oracle.hmvm(H, x)
    assert np.linalg.norm(y - A @ x) <= 2 * eps * np.linalg.norm(A) * np.linalg.norm(x)
    ref = assemble(H) @ x
    assert np.linalg.norm(y - ref) <= 1e-13 * max(np.linalg.norm(ref), 1e-300)
