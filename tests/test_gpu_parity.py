"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

FP64 path: relative 2-norm error <= 1e-12 against the oracle (plus an
elementwise bound), at n = 4096 and at the full n = 2^18 sizes (eps 1e-6 and
1e-8, the configuration the benchmark times).  Mixed storage with FP32
accumulation: against the decoded oracle within the rigorous FP32 summation
bound, and against the unrounded FP64 oracle within 1e-6.  Edge cases:
all-dense and single-block partitions, tiny and non-square tilings, y0 / alpha
handling, x = 0, determinism, linearity, batched right-hand sides.
"""

import os
import sys

import numpy as np
import pytest

import hmgen
import oracle
from hmgen import hmatrix as hmm
from paper_2308_10960_amd import hm, DeviceHMatrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(hm.LIB_PATH), "libhm.so must be built before the GPU tests"


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def run(D, x, y0=None, alpha=1.0):
    xd = D.vector(x)
    yd = D.vector(y0) if y0 is not None else D.vector()
    D.mvm(xd, yd, alpha)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.float64)


def abs_bound(H, x, factors=None):
    """|A| |x| with |U| |V|^T for low-rank blocks: scale of the summands."""
    fac = []
    for i in range(H.nblocks):
        a, b, s = factors[i] if factors is not None else H.factors(i)
        fac.append((np.abs(np.asfortranarray(a)), None if b is None else np.abs(np.asfortranarray(b)),
                    None if s is None else np.abs(np.asarray(s))))
    return oracle.hmvm(H, np.abs(x), factors=fac)


def fp32_depth(H):
    """Bound on the number of roundings on any path into one output entry:
    y_i sums, over the leaves covering row i, their dense row or U_i t with
    t_l = sum_j V_jl x_j; every path meets at most n column terms, the
    ranks of the low-rank leaves covering row i, one addition per leaf and
    a few roundings of its own (product, s_b, alpha, the update of y: 8).
    gamma_K (|A| |x|) then bounds the error for any order of summation."""
    n = H.n
    acc = np.zeros(n + 1)
    lr = np.asarray(H.adm) != 0
    np.add.at(acc, np.asarray(H.rb), np.where(lr, H.rank, 0) + 1)
    np.add.at(acc, np.asarray(H.re), -(np.where(lr, H.rank, 0) + 1))
    return int(n + np.cumsum(acc)[:n].max()) + 8


def check_f64(y, ref, scale, tol=F64_TOL):
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    say(f"relative error {rel:.3e}")
    assert rel <= tol
    assert np.all(np.abs(y - ref) <= 1e-13 * scale + 1e-300)


@pytest.fixture(scope="module")
def sphere4k():
    return hmgen.build_preset("sphere4k")


def test_sphere4k_f64(sphere4k):
    H = sphere4k
    say("sphere4k f64")
    D = DeviceHMatrix(H, hm.HM_F64)
    x = hmgen.uniform_vector(H.n)
    y0 = hmgen.uniform_vector(H.n, seed=9)
    ref = oracle.hmvm(H, x)
    y = run(D, x)
    check_f64(y, ref, abs_bound(H, x))
    # y += alpha A x with nonzero y0
    ref2 = oracle.hmvm(H, x, y0, alpha=-0.625)
    y2 = run(D, x, y0, alpha=-0.625)
    check_f64(y2, ref2, 0.625 * abs_bound(H, x) + np.abs(y0))
    # x = 0 leaves y unchanged, bit for bit
    y3 = run(D, np.zeros(H.n), y0)
    np.testing.assert_array_equal(y3, y0)
    # determinism: repeated calls agree bit for bit
    for _ in range(3):
        np.testing.assert_array_equal(run(D, x), y)
    # linearity
    z = hmgen.uniform_vector(H.n, seed=4)
    lin = run(D, 2.0 * x - 3.0 * z)
    assert np.linalg.norm(lin - (2 * y - 3 * run(D, z))) <= 1e-13 * np.linalg.norm(lin)
    D.close()


@pytest.mark.parametrize("window", [None, 4096, 65536])
def test_store_upload_matches_host_packing(sphere4k, window, monkeypatch):
    """The device store equals the host packing byte for byte, also when the
    upload streams the factor data in many small windows (the window grows
    to the largest packing job where that is larger); for AFLP the data
    blocks' parameters, derived once, serve every window."""
    if window is not None:
        monkeypatch.setenv("HM_UPLOAD_WINDOW_BYTES", str(window))
    for name, H, acc in [("sphere4k", sphere4k, hm.HM_F64),
                         ("sphere4k_mixed", hmgen.build_preset("sphere4k_mixed"), hm.HM_F32),
                         ("sphere4k_aflp", hmgen.build_preset("sphere4k_aflp"), hm.HM_F64)]:
        say("upload", name, window)
        D = DeviceHMatrix(H, acc)
        buf = np.zeros(D.info["store_bytes"], np.uint8)
        hm.hm_pack_host(D.plan, H.a_ptr, H.b_ptr, H.s_ptr if H.keep_sigma else None, buf)
        dev = D.store.cpu().numpy()
        np.testing.assert_array_equal(dev, buf)
        D.close()


@pytest.mark.parametrize("case", ["eta0", "one_block", "tiny5", "tiny1"])
def test_degenerate_partitions(case):
    say("degenerate", case)
    if case == "eta0":
        H = hmm.build_hmatrix(hmgen.fibonacci_sphere(1000), hmm.KERNEL_LAPLACE, leaf=32, eta=0.0)
    elif case == "one_block":
        H = hmm.build_hmatrix(hmgen.fibonacci_sphere(300), hmm.KERNEL_LAPLACE, leaf=512)
    elif case == "tiny5":
        H = hmm.build_hmatrix(hmgen.cube_points(5, 1), hmm.KERNEL_EXP, leaf=2)
    else:
        H = hmm.build_hmatrix(hmgen.cube_points(1, 1), hmm.KERNEL_EXP, leaf=64)
    H.set_uniform_dtype(hmm.DT_F64)
    D = DeviceHMatrix(H, hm.HM_F64)
    x = hmgen.uniform_vector(H.n, seed=2)
    check_f64(run(D, x), oracle.hmvm(H, x), abs_bound(H, x))
    D.close()
    # the same partition in the byte-aligned formats (FP64 accumulation):
    # 2-byte AFLP (data blocks down to one value) and 3-byte DFL
    for dt in (hm.HM_AFLP16, hm.HM_DFL24):
        H.set_uniform_dtype(dt)
        D = DeviceHMatrix(H, hm.HM_F64)
        dec = oracle.decoded_factors(H, sigma_dtype=oracle.F64)
        check_f64(run(D, x), oracle.hmvm(H, x, factors=dec), abs_bound(H, x, dec))
        D.close()
    # the same partition in FP32 storage through the batched (MFMA) path
    H.set_uniform_dtype(hmm.DT_F32)
    D = DeviceHMatrix(H, hm.HM_F32, max_nrhs=3)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F32)
    X = hmgen.gaussian_block(H.n, 3).astype(np.float32).astype(np.float64)
    Y = _batch(D, X)
    ref = oracle.hmvm_multi(H, X, factors=dec)
    K = fp32_depth(H)
    gam = K * U32 / (1 - K * U32)
    for c in range(3):
        assert np.all(np.abs(Y[:, c] - ref[:, c]) <= gam * abs_bound(H, X[:, c], dec) + 1e-30), c
    D.close()


def test_ragged_leaf_sizes_and_eta():
    """Several tiles per panel, ragged panel heights, and a ragged tail."""
    for n, leaf, eta in [(3001, 37, 1.0), (2500, 64, 0.5), (4099, 16, 2.0)]:
        say("ragged", n, leaf, eta)
        H = hmm.build_hmatrix(hmgen.cube_points(n, 7), hmm.KERNEL_EXP, leaf=leaf, eta=eta, eps=1e-7)
        H.set_uniform_dtype(hmm.DT_F64)
        D = DeviceHMatrix(H, hm.HM_F64)
        x = hmgen.uniform_vector(n, seed=3)
        check_f64(run(D, x), oracle.hmvm(H, x), abs_bound(H, x))
        D.close()


def test_batched_rhs_equal_single(sphere4k):
    H = sphere4k
    D = DeviceHMatrix(H, hm.HM_F64, max_nrhs=5)
    X = hmgen.gaussian_block(H.n, 5)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()      # (r, n) = column-major n x r
    Yd = torch.zeros_like(Xd)
    hm.hm_mvm_batch(D.handle, 5, 1.0, Xd, H.n, Yd, H.n, D.work, D.work.numel())
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().T
    ref = oracle.hmvm_multi(H, X)
    for c in range(5):
        np.testing.assert_array_equal(Y[:, c], run(D, X[:, c]))
        check_f64(Y[:, c], ref[:, c], abs_bound(H, X[:, c]))
    D.close()


@pytest.mark.parametrize("name", ["sphere256k", "sphere256k_e8"])
def test_full_size_f64(name):
    say("building", name)
    H = hmgen.build_preset(name)
    say("built", H.stats())
    D = DeviceHMatrix(H, hm.HM_F64)
    say("uploaded", D.info["store_bytes"])
    x = hmgen.uniform_vector(H.n)
    y = run(D, x)
    say("gpu done; oracle")
    ref = oracle.hmvm(H, x)
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    say(f"{name}: relative error {rel:.3e}")
    assert rel <= F64_TOL
    # elementwise on a sample of rows, against the summand scale
    idx = np.random.default_rng(0).choice(H.n, 2000, replace=False)
    scale = abs_bound(H, x)
    assert np.all(np.abs(y[idx] - ref[idx]) <= 1e-13 * scale[idx])
    D.close()


def _mixed(H, name, launch=None):
    D = DeviceHMatrix(H, hm.HM_F32)
    if launch:
        say(name, launch)
        hm.hm_matrix_set_launch(D.handle, launch)
    x64 = hmgen.uniform_vector(H.n)
    x = x64.astype(np.float32).astype(np.float64)        # the vector the GPU sees
    y = run(D, x)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F32)
    ref_dec = oracle.hmvm(H, x, factors=dec)
    truth = oracle.hmvm(H, x)
    # rigorous FP32 summation bound: |err| <= gamma_K * (|A_dec| |x|)
    K = fp32_depth(H)
    gam = K * U32 / (1 - K * U32)
    scale = abs_bound(H, x, dec)
    err = np.abs(y - ref_dec)
    say(f"{name}: max err/scale {np.max(err / scale):.3e}, "
        f"rel vs decoded {np.linalg.norm(y - ref_dec) / np.linalg.norm(ref_dec):.3e}, "
        f"rel vs truth {np.linalg.norm(y - truth) / np.linalg.norm(truth):.3e}")
    assert np.all(err <= gam * scale)
    assert np.linalg.norm(y - truth) / np.linalg.norm(truth) <= 1e-6
    D.close()


def block_norms(H):
    """Frobenius norm of every stored block (|s| for low-rank blocks kept as
    W diag(s) X^T with orthonormal W, X)."""
    out = np.zeros(H.nblocks)
    for i in range(H.nblocks):
        a, _, s = H.factors(i)
        out[i] = np.linalg.norm(s) if H.adm[i] else np.linalg.norm(a)
    return out


def check_store_budget(H, tol):
    """Every block's storage error bound within tol of its own norm."""
    nrm = block_norms(H)
    ratio = np.where(nrm > 0, H.store_err_bound / np.maximum(nrm, 1e-300), 0.0)
    say(f"max storage error / block norm {ratio.max():.3e} (budget {tol:.1e})")
    assert ratio.max() <= tol


def test_mixed_sphere4k():
    H = hmgen.build_preset("sphere4k_mixed")
    _mixed(H, "sphere4k_mixed")
    for colw in (0, 2):                  # column tiles a workgroup / a wave each
        _mixed(H, "sphere4k_mixed", f"colw={colw}")


def test_mixed_full_size():
    say("building sphere256k_mixed")
    H = hmgen.build_preset("sphere256k_mixed")
    check_store_budget(H, hmgen.presets.MIXED_TOL / 2)
    _mixed(H, "sphere256k_mixed")


@pytest.mark.parametrize("name", ["sphere4k_e8_mixed", "sphere256k_e8_mixed"])
def test_mixed_fp64_accumulation(name):
    """The eps = 1e-8 matrix with FP64 kept only for the dense (near-field)
    blocks, s and the accumulation of y, and the low-rank column groups in
    FP32 / FP16 / BF16: the FP64 bar against the oracle on the decoded
    factors, and the stated 1e-6 against the unrounded FP64 matrix."""
    say("building", name)
    H = hmgen.build_preset(name)
    dense = H.adm == 0
    assert np.all(H.group_dtype[dense, 0] == hm.HM_F64)
    lr = np.flatnonzero(~dense)
    used = np.concatenate([H.group_dtype[i, :H.ngroups[i]] for i in lr])
    assert set(np.unique(used).tolist()) <= {hm.HM_F32, hm.HM_F16, hm.HM_BF16}
    check_store_budget(H, hmgen.presets.MIXED_TOL / 2)
    D = DeviceHMatrix(H, hm.HM_F64)
    say("uploaded", D.info["store_bytes"], D.info["bytes_by_dtype"][:4])
    x = hmgen.uniform_vector(H.n)
    y = run(D, x)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F64)
    ref = oracle.hmvm(H, x, factors=dec)
    truth = oracle.hmvm(H, x)
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    rel_truth = np.linalg.norm(y - truth) / np.linalg.norm(truth)
    say(f"{name}: relative error vs decoded oracle {rel:.3e}, vs unrounded FP64 {rel_truth:.3e}")
    assert rel <= F64_TOL
    idx = np.random.default_rng(0).choice(H.n, min(H.n, 2000), replace=False)
    scale = abs_bound(H, x, dec)
    assert np.all(np.abs(y[idx] - ref[idx]) <= 1e-13 * scale[idx])
    assert rel_truth <= 1e-6
    D.close()


def _batch(D, X, alpha=1.0, Y0=None):
    Xd = torch.from_numpy(np.ascontiguousarray(X.T.astype(np.float32))).cuda()
    Yd = torch.zeros_like(Xd) if Y0 is None else torch.from_numpy(
        np.ascontiguousarray(Y0.T.astype(np.float32))).cuda()
    r = X.shape[1]
    hm.hm_mvm_batch(D.handle, r, alpha, Xd, X.shape[0], Yd, X.shape[0], D.work, D.work.numel())
    torch.cuda.synchronize()
    return Yd.cpu().numpy().T.astype(np.float64)


@pytest.mark.parametrize("name", ["sphere4k_mixed", "cube4k"])
def test_batched_f32_mfma(name):
    """FP32 batched product on the matrix cores: every column within the
    rigorous FP32 bound of the decoded oracle; a column's result does not
    depend on the other columns of the batch (bitwise); ragged batch sizes
    across the 32- and 64-column groups."""
    H = hmgen.build_preset(name)
    D = DeviceHMatrix(H, hm.HM_F32, max_nrhs=70)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F32)
    X = hmgen.gaussian_block(H.n, 70).astype(np.float32).astype(np.float64)
    Y0 = hmgen.gaussian_block(H.n, 70, seed=7).astype(np.float32).astype(np.float64)
    Y = _batch(D, X, -0.5, Y0)
    ref = oracle.hmvm_multi(H, X, Y0, alpha=-0.5, factors=dec)
    K = fp32_depth(H)
    gam = K * U32 / (1 - K * U32)
    worst = 0.0
    for c in range(70):
        scale = 0.5 * abs_bound(H, X[:, c], dec) + np.abs(Y0[:, c])
        err = np.abs(Y[:, c] - ref[:, c])
        worst = max(worst, float(np.max(err / scale)))
        assert np.all(err <= gam * scale), c
    say(f"{name} batch max err/scale {worst:.3e}")
    # batch independence: the same right-hand side in other batches
    for r, pick in [(1, [5]), (7, [5, 0, 69, 33, 2, 40, 11]), (33, list(range(33))), (64, list(range(64)))]:
        Yb = _batch(D, X[:, pick], -0.5, Y0[:, pick])
        for q, c in enumerate(pick):
            np.testing.assert_array_equal(Yb[:, q], Y[:, c])
    # XCD-contiguous row-panel order: same sums, padding workgroups idle
    hm.hm_matrix_set_launch(D.handle, "order=1")
    np.testing.assert_array_equal(_batch(D, X, -0.5, Y0), Y)
    # FP32 column tiles as 16-byte groups: each column's MFMA chain is the same
    hm.hm_matrix_set_launch(D.handle, "colb=1")
    np.testing.assert_array_equal(_batch(D, X, -0.5, Y0), Y)
    D.close()


@pytest.mark.parametrize("fmt", [hm.HM_F16, hm.HM_BF16])
def test_uniform_16bit_formats(fmt):
    """Every block stored in one 16-bit format (so every column tile has one
    format: the FP16 and BF16 tile kernels of both paths): single and
    batched products against the decoded oracle within the rigorous FP32
    bound, batch independence bitwise."""
    H = hmgen.build_preset("sphere4k_mixed")
    H.set_uniform_dtype(fmt)
    dec = oracle.decoded_factors(H, sigma_dtype=oracle.F32)
    K = fp32_depth(H)
    gam = K * U32 / (1 - K * U32)
    D = DeviceHMatrix(H, hm.HM_F32, max_nrhs=40)
    x = hmgen.uniform_vector(H.n).astype(np.float32).astype(np.float64)
    y = run(D, x)
    ref = oracle.hmvm(H, x, factors=dec)
    assert np.all(np.abs(y - ref) <= gam * abs_bound(H, x, dec))
    X = hmgen.gaussian_block(H.n, 40).astype(np.float32).astype(np.float64)
    Y = _batch(D, X, 0.5)
    refX = oracle.hmvm_multi(H, X, alpha=0.5, factors=dec)
    for c in (0, 17, 39):
        assert np.all(np.abs(Y[:, c] - refX[:, c]) <= gam * 0.5 * abs_bound(H, X[:, c], dec)), c
    np.testing.assert_array_equal(_batch(D, X[:, [17]], 0.5)[:, 0], Y[:, 17])
    say(f"format {fmt}: rel {np.linalg.norm(y - ref) / np.linalg.norm(ref):.2e}")
    D.close()


def test_launch_variants_and_tune_cache(sphere4k, tmp_path):
    """Every schedule/unroll meets parity; unroll depth never changes a bit;
    the tune cache written by the tuner is read back by hm_build_plan."""
    from paper_2308_10960_amd import tune
    H = sphere4k
    D = DeviceHMatrix(H, hm.HM_F64)
    x = hmgen.uniform_vector(H.n)
    ref = oracle.hmvm(H, x)
    scale = abs_bound(H, x)
    out = {}
    for c in tune.CANDIDATES:
        hm.hm_matrix_set_launch(D.handle, c)
        assert hm.hm_matrix_get_launch(D.handle) == c + " chunk=512 tile=64 colb=0 tmix=0 colw=1"
        out[c] = run(D, x)
        check_f64(out[c], ref, scale)
    # within one schedule, unroll depth, order and persistence change no bit
    for c in tune.CANDIDATES:
        first = next(d for d in tune.CANDIDATES if d.split()[0] == c.split()[0])
        np.testing.assert_array_equal(out[c], out[first])
    with pytest.raises(hm.HMError):
        hm.hm_matrix_set_launch(D.handle, "schedule=7")
    xd, yd = D.vector(x), D.vector()
    best, times = tune.tune(D, lambda: D.mvm(xd, yd), reps=3, warmup=1)
    assert best in tune.CANDIDATES and set(times) == set(tune.CANDIDATES)
    key = hm.hm_matrix_tune_key(D.handle)
    path = str(tmp_path / "tune.txt")
    tune.write_cache(path, key, "schedule=1 unroll=8 order=0 persist=2")
    tune.write_cache(path, "acc9-fmt0-n2^0", "schedule=0 unroll=4")
    D2 = DeviceHMatrix(H, hm.HM_F64, tune_cache=path)
    assert hm.hm_matrix_get_launch(D2.handle) == "schedule=1 unroll=8 order=0 persist=2 chunk=512 tile=64 colb=0 tmix=0 colw=1"
    D2.close()
    # a tuned tile shape: parity, and the shape is the plan's (set_launch
    # accepts only the plan's own)
    tune.write_cache(path, key, "schedule=0 unroll=8 order=1 persist=0 chunk=128 tile=16")
    D3 = DeviceHMatrix(H, hm.HM_F64, tune_cache=path)
    assert hm.hm_matrix_get_launch(D3.handle) == "schedule=0 unroll=8 order=1 persist=0 chunk=128 tile=16 colb=0 tmix=0 colw=1"
    assert D3.info["n_col_tiles"] > D.info["n_col_tiles"]
    check_f64(run(D3, x), ref, scale)
    hm.hm_matrix_set_launch(D3.handle, "unroll=4 chunk=128 tile=16")
    with pytest.raises(hm.HMError):
        hm.hm_matrix_set_launch(D3.handle, "chunk=512")
    D3.close()
    D.close()


@pytest.fixture(scope="module")
def sphere64k():
    return hmgen.build_preset("sphere256k", n=65536)


def test_persistent_grids_loop(sphere64k):
    """Persistent grids small enough that every workgroup loops over several
    row panels and column tiles give the plain launch's result bit for bit,
    in both schedules and both panel orders; parity against the oracle."""
    H = sphere64k
    D = DeviceHMatrix(H, hm.HM_F64)
    info = D.info
    assert info["n_row_panels"] > 4 * 256 and info["n_col_tiles"] > 4 * 256
    x = hmgen.uniform_vector(H.n)
    y0 = hmgen.uniform_vector(H.n, seed=9)
    ref = oracle.hmvm(H, x, y0, alpha=0.75)
    scale = 0.75 * abs_bound(H, x) + np.abs(y0)
    for sched in (0, 1):
        hm.hm_matrix_set_launch(D.handle, f"schedule={sched} order=0 persist=0")
        base = run(D, x, y0, 0.75)
        check_f64(base, ref, scale)
        for order in (0, 1):
            for ps in (1, 2, 8):
                c = f"schedule={sched} order={order} persist={ps}"
                say(c)
                hm.hm_matrix_set_launch(D.handle, c)
                np.testing.assert_array_equal(run(D, x, y0, 0.75), base)
    D.close()


@pytest.mark.parametrize("chunk", [512, 64])
def test_column_tile_wave_modes(sphere64k, chunk, tmp_path):
    """Column tiles on a workgroup each (colw=0), on a wave each (colw=2)
    or chosen per launch class (colw=1, built in), with 512- and 64-row
    column chunks: parity with the oracle in each mode, and persistent grids,
    where every wave loops over several tiles, give the plain launch's
    result bit for bit."""
    from paper_2308_10960_amd import tune
    H = sphere64k
    D = DeviceHMatrix(H, hm.HM_F64)
    key = hm.hm_matrix_tune_key(D.handle)
    D.close()
    path = str(tmp_path / "tune.txt")
    tune.write_cache(path, key, f"schedule=0 unroll=8 order=1 persist=0 chunk={chunk} tile=64")
    D = DeviceHMatrix(H, hm.HM_F64, tune_cache=path)
    assert D.info["n_col_tiles"] > 4 * 256           # persist=1: every wave loops
    x = hmgen.uniform_vector(H.n)
    y0 = hmgen.uniform_vector(H.n, seed=9)
    ref = oracle.hmvm(H, x, y0, alpha=0.75)
    scale = 0.75 * abs_bound(H, x) + np.abs(y0)
    for colw in (0, 1, 2):
        hm.hm_matrix_set_launch(D.handle, f"colw={colw} persist=0")
        say(f"chunk={chunk} colw={colw}")
        base = run(D, x, y0, 0.75)
        check_f64(base, ref, scale)
        for ps in (1, 2):
            hm.hm_matrix_set_launch(D.handle, f"persist={ps}")
            np.testing.assert_array_equal(run(D, x, y0, 0.75), base)
    D.close()


def _graph_replays(D, make_args, eager, replays=3):
    """Replays of a captured product equal the eager call bit for bit, with
    eager work and synchronisation between the replays."""
    X, Y, Y0, ld = make_args()
    Ye = Y0.clone()
    eager(X, Ye)
    torch.cuda.synchronize()
    g = hm.hm_graph_create(D.handle, X.shape[0] if X.dim() == 2 else 1, -0.5, X, ld, Y, ld,
                           D.work, D.work.numel())
    other = Y0.clone()
    stream = torch.cuda.current_stream()
    try:
        for r in range(replays):
            Y.copy_(Y0)
            hm.hm_graph_launch(g, stream)
            torch.cuda.synchronize()
            assert torch.equal(Y, Ye), f"replay {r}"
            eager(X, other)                      # eager work between replays
            torch.cuda.synchronize()
    finally:
        hm.hm_graph_destroy(g)


def test_graph_single_rhs(sphere4k):
    H = sphere4k
    D = DeviceHMatrix(H, hm.HM_F64)
    for params in ("schedule=0 order=1 persist=0", "schedule=1 order=0 persist=1"):
        hm.hm_matrix_set_launch(D.handle, params)

        def make():
            x = D.vector(hmgen.uniform_vector(H.n))
            y0 = D.vector(hmgen.uniform_vector(H.n, seed=9))
            return x, torch.empty_like(y0), y0, H.n

        _graph_replays(D, make, lambda x, y: D.mvm(x, y, -0.5))
    with pytest.raises(hm.HMError) as e:          # argument checks as in hm_mvm
        x = D.vector()
        hm.hm_graph_create(D.handle, 1, 1.0, x, H.n, x, H.n, D.work, D.work.numel())
    assert e.value.status == hm.HM_EINVAL
    D.close()


def test_graph_batch_f32():
    H = hmgen.build_preset("sphere4k_mixed")
    D = DeviceHMatrix(H, hm.HM_F32, max_nrhs=40)

    def make():
        Xh = hmgen.gaussian_block(H.n, 40).astype(np.float32)
        X = torch.from_numpy(np.ascontiguousarray(Xh.T)).cuda()
        Y0 = torch.from_numpy(np.ascontiguousarray(
            hmgen.gaussian_block(H.n, 40, seed=7).astype(np.float32).T)).cuda()
        return X, torch.empty_like(Y0), Y0, H.n

    def eager(X, Y):
        hm.hm_mvm_batch(D.handle, 40, -0.5, X, H.n, Y, H.n, D.work, D.work.numel())

    _graph_replays(D, make, eager)
    D.close()
