"""GPU tests of the request loop (hm_server_create / hm_submit / hm_wait).

* Every request's result in a random mix equals the same request served
  alone, bit for bit, and the decoded oracle within the FP32 bound.
* A tiny arena makes requests wait for memory instead of failing.
* A request that can never fit fails with HM_ENOMEM; the loop keeps serving.
* The test hook HM_SERVER_FAULT_EVERY fails whole batches with HM_EDEVICE
  from the host side; other requests still complete.
* hm_wait times out with HM_ETIMEOUT; unknown tickets give HM_ESTATE.
"""

import os

import numpy as np
import pytest

import hmgen
import oracle
from fp32_bound import check_rows, sample_rows
from paper_2308_10960_amd import hm, DeviceHMatrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def mats():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Hs = [hmgen.build_preset("sphere4k_mixed"), hmgen.build_preset("cube4k")]
    Ds = [DeviceHMatrix(H, hm.HM_F32, max_nrhs=16) for H in Hs]
    yield Hs, Ds
    for D in Ds:
        D.close()


def _server(Ds, arena_bytes, nstreams=2):
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    s = hm.hm_server_create([D.handle for D in Ds], arena, arena_bytes, streams)
    return s, arena, streams


def _requests(Hs, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        m = int(rng.integers(len(Hs)))
        r = int(rng.integers(1, 9))
        X = np.asfortranarray(rng.standard_normal((Hs[m].n, r)).astype(np.float32))
        reqs.append((m, r, X))
    return reqs


def _submit_all(s, reqs):
    outs, tickets = [], []
    for m, r, X in reqs:
        Y = np.zeros((X.shape[0], r), np.float32, order="F")
        outs.append(Y)
        tickets.append(hm.hm_submit(s, m, r, X, X.shape[0], Y, Y.shape[0]))
    return outs, tickets


def test_mix_equals_alone_and_oracle(mats):
    Hs, Ds = mats
    reqs = _requests(Hs, 40, 0)
    s, arena, _ = _server(Ds, 256 << 20, nstreams=3)
    outs, tickets = _submit_all(s, reqs)
    for t in tickets:
        assert hm.hm_wait(s, t, 60_000_000) == hm.HM_OK
    p50, p99, mps = hm.hm_server_stats(s)
    assert 0 < p50 <= p99 and mps > 0
    hm.hm_server_destroy(s)
    # each request alone on a fresh server: bitwise equal; every row within
    # the elementwise FP32 bound of the decoded oracle
    s1, arena1, _ = _server(Ds, 256 << 20, nstreams=1)
    for (m, r, X), Y in zip(reqs[:12], outs[:12]):
        Ya, ta = _submit_all(s1, [(m, r, X)])
        assert hm.hm_wait(s1, ta[0], 60_000_000) == hm.HM_OK
        np.testing.assert_array_equal(Ya[0], Y)
        worst, rel_dec, rel_truth = check_rows(Hs[m], X, Y, np.arange(Hs[m].n))
        assert rel_truth <= 1e-6
    hm.hm_server_destroy(s1)


def test_mix_equals_alone_full_size():
    """Served mix on an n = 2^18 mixed-precision matrix (requests of up to 64
    right-hand sides, batched with each other) and a small one: every
    result equals the same request served alone, bit for bit, and sampled
    rows are within the elementwise FP32 bound of the decoded oracle and
    1e-6 of the unrounded FP64 product."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Hs = [hmgen.build_preset("sphere256k_mixed"), hmgen.build_preset("sphere4k_mixed")]
    Ds = [DeviceHMatrix(H, hm.HM_F32, max_nrhs=64) for H in Hs]
    rng = np.random.default_rng(21)
    reqs = []
    for r in (64, 1, 37, 13, 64, 5):
        reqs.append((0, r, np.asfortranarray(rng.standard_normal((Hs[0].n, r)).astype(np.float32))))
        r2 = int(rng.integers(1, 17))
        reqs.append((1, r2, np.asfortranarray(rng.standard_normal((Hs[1].n, r2)).astype(np.float32))))
    s, arena, _ = _server(Ds, 8 << 30, nstreams=3)
    outs, tickets = _submit_all(s, reqs)
    for t in tickets:
        assert hm.hm_wait(s, t, 120_000_000) == hm.HM_OK
    hm.hm_server_destroy(s)
    s1, arena1, _ = _server(Ds, 8 << 30, nstreams=1)
    rows = sample_rows(Hs[0].n, 6, 5)
    for (m, r, X), Y in zip(reqs, outs):
        Ya, ta = _submit_all(s1, [(m, r, X)])
        assert hm.hm_wait(s1, ta[0], 120_000_000) == hm.HM_OK
        np.testing.assert_array_equal(Ya[0], Y)
        if m == 0:
            worst, rel_dec, rel_truth = check_rows(Hs[0], X, Y, rows)
            print(f"[gpu-test] n=2^18 r={r}: max err/scale {worst:.3e}, rel vs decoded {rel_dec:.3e}, "
                  f"vs truth {rel_truth:.3e}", flush=True)
            assert rel_truth <= 1e-6
    hm.hm_server_destroy(s1)
    for D in Ds:
        D.close()


def test_pinned_client_buffers(mats):
    """Requests whose X and Y are page-locked (copied by the device without
    staging, with their leading dimensions) give bitwise the results of the
    same requests in pageable buffers."""
    Hs, Ds = mats
    reqs = _requests(Hs, 10, 4)
    s, arena, _ = _server(Ds, 256 << 20, nstreams=2)
    outs, tickets = _submit_all(s, reqs)
    pin_in, pin_out, pin_t = [], [], []             # the buffers stay alive until their tickets end
    for m, r, X in reqs:
        n = Hs[m].n
        ld = n + 37                                    # leading dimensions above n
        Xp = torch.empty((r, ld), dtype=torch.float32, pin_memory=True).numpy()
        Xp[:, :n] = X.T
        Yp = torch.zeros((r, ld), dtype=torch.float32, pin_memory=True).numpy()
        pin_in.append(Xp)
        pin_out.append(Yp)
        pin_t.append(hm.hm_submit(s, m, r, Xp, ld, Yp, ld))
    for t in tickets + pin_t:
        assert hm.hm_wait(s, t, 60_000_000) == hm.HM_OK
    hm.hm_server_destroy(s)
    for (m, r, X), Y, Yp in zip(reqs, outs, pin_out):
        np.testing.assert_array_equal(Yp[:, :Hs[m].n].T, Y)
        assert np.all(Yp[:, Hs[m].n:] == 0)             # nothing written past n


def test_tiny_arena_queues(mats):
    Hs, Ds = mats
    reqs = _requests(Hs, 12, 1)
    # room for one request of at most 8 right-hand sides at a time
    need = max(4096 * 8 * 4 * 2 + 32 * D.info["work_bytes_per_rhs"] + 4096 for D in Ds)
    s, arena, _ = _server(Ds, need, nstreams=2)
    outs, tickets = _submit_all(s, reqs)
    for t in tickets:
        assert hm.hm_wait(s, t, 60_000_000) == hm.HM_OK
    hm.hm_server_destroy(s)
    s2, arena2, _ = _server(Ds, 256 << 20, nstreams=2)
    outs2, t2 = _submit_all(s2, reqs)
    for t in t2:
        assert hm.hm_wait(s2, t, 60_000_000) == hm.HM_OK
    for a, b in zip(outs, outs2):
        np.testing.assert_array_equal(a, b)
    hm.hm_server_destroy(s2)


def test_oversized_request_fails_and_loop_continues(mats):
    Hs, Ds = mats
    small = 32 * Ds[0].info["work_bytes_per_rhs"] + 2 * 4096 * 4 + 4096
    s, arena, _ = _server(Ds, small)            # fits 1 right-hand side, not 16 (64-slot workspace)
    X = np.ones((4096, 16), np.float32, order="F")
    Y = np.zeros_like(X)
    t = hm.hm_submit(s, 0, 16, X, 4096, Y, 4096)
    assert hm.hm_wait(s, t, 60_000_000) == hm.HM_ENOMEM
    X1 = np.ones((4096, 1), np.float32, order="F")
    Y1 = np.zeros_like(X1)
    t1 = hm.hm_submit(s, 0, 1, X1, 4096, Y1, 4096)
    assert hm.hm_wait(s, t1, 60_000_000) == hm.HM_OK
    assert np.abs(Y1).sum() > 0
    hm.hm_server_destroy(s)


def test_injected_batch_failure(mats, monkeypatch):
    Hs, Ds = mats
    monkeypatch.setenv("HM_SERVER_FAULT_EVERY", "3")
    s, arena, _ = _server(Ds, 256 << 20, nstreams=1)
    monkeypatch.delenv("HM_SERVER_FAULT_EVERY")
    reqs = [(0, 1, np.asfortranarray(np.ones((4096, 1), np.float32))) for _ in range(9)]
    results = []
    for m, r, X in reqs:                      # one at a time: one batch per request
        outs, t = _submit_all(s, [(m, r, X)])
        results.append(hm.hm_wait(s, t[0], 60_000_000))
    assert results.count(hm.HM_EDEVICE) == 3
    assert results.count(hm.HM_OK) == 6
    hm.hm_server_destroy(s)


def test_wait_timeout_and_unknown_ticket(mats):
    """A ticket queued behind 31 others on one slot whose arena holds one
    batch at a time is still pending right after submission: hm_wait with
    timeout 0 returns HM_ETIMEOUT (and hm_poll reports it not done).  A
    ticket reported done is released: asking again gives HM_ESTATE."""
    Hs, Ds = mats
    D = Ds[1]
    one = 2 * 4096 * 16 * 4 + 64 * D.info["work_bytes_per_rhs"] + 4096
    s, arena, _ = _server(Ds, one, nstreams=1)
    X = np.asfortranarray(np.ones((4096, 16), np.float32))
    Ys = [np.zeros_like(X) for _ in range(32)]
    ts = [hm.hm_submit(s, 1, 16, X, 4096, Y, 4096) for Y in Ys]
    with pytest.raises(hm.HMError) as e:
        hm.hm_wait(s, ts[-1], 0)
    assert e.value.status == hm.HM_ETIMEOUT
    done, _ = hm.hm_poll(s, ts[-1])
    assert not done
    for t in ts:
        assert hm.hm_wait(s, t, 60_000_000) == hm.HM_OK
    for Y in Ys[1:]:
        np.testing.assert_array_equal(Y, Ys[0])
    # released after being reported
    with pytest.raises(hm.HMError) as e:
        hm.hm_poll(s, ts[0])
    assert e.value.status == hm.HM_ESTATE
    with pytest.raises(hm.HMError) as e:
        hm.hm_wait(s, ts[-1], 0)
    assert e.value.status == hm.HM_ESTATE
    with pytest.raises(hm.HMError) as e:
        hm.hm_poll(s, 10 ** 9)
    assert e.value.status == hm.HM_ESTATE
    # hm_poll reporting done also releases
    t = hm.hm_submit(s, 0, 1, X, 4096, Ys[0], 4096)
    while True:
        done, res = hm.hm_poll(s, t)
        if done:
            break
    assert res == hm.HM_OK
    with pytest.raises(hm.HMError) as e:
        hm.hm_wait(s, t, 0)
    assert e.value.status == hm.HM_ESTATE
    hm.hm_server_destroy(s)
