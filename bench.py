#!/usr/bin/env python3
"""Benchmark of the H-matrix-vector product on one MI355X.

Default workload: Fibonacci-sphere Laplace matrix, n = 2^18, leaf 64, eta 2,
ACA + SVD recompression at eps = 1e-6, plain FP64 storage and accumulation,
one right-hand side (synthetic, seeded).  A step is one full product
y += A x (column tiles, partial reduction, row panels) with the matrix and
the vectors resident in HBM.  Prints one JSON line.

value = algorithmic bytes per product / time per product (effective GB/s);
the algorithmic bytes are the stored factor bytes plus x read once and y
read and written once.  The roofline entry is for the kernel with the
largest measured time, timed with HIP events on its own stream over the
timed region.  cpu_baseline times the CPU oracle (single thread) on full
products of the same matrix.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# per-call kernel phases reported by hm_profile_end: single RHS (hm_mvm) and
# batched (hm_mvm_batch) schedules
KERNELS = {0: ["k_col", "k_reduce", "k_row"], 1: ["k_p1", "k_reduce", "k_p2"]}
KERNELS_BATCH = ["k_xpose+k_col_b", "k_reduce_b", "k_row_b"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(H, info, vs, R=1, schedule=0):
    """Algorithmic bytes each kernel must move in one product of R
    right-hand sides (factors once, vectors and partial sums per column)."""
    m = (H.re - H.rb).astype(np.float64)
    nb = (H.ce - H.cb).astype(np.float64)
    dense = H.adm == 0
    sz = np.array([8, 4, 2, 2, 4, 5, 6, 2, 3, 2, 3, 4, 5, 6, 3, 5, 6], np.float64)   # bytes per value, by format
    d_bytes = float((m * nb * sz[H.group_dtype[:, 0]])[dense].sum())
    gcols = H.group_cols.astype(np.float64)
    gbytes = (gcols * sz[H.group_dtype]).sum(1)          # bytes per row of U / V
    u_bytes = float((m * gbytes)[~dense].sum())
    v_bytes = float((nb * gbytes)[~dense].sum())
    n = float(H.n)
    n_t, n_p = float(info["n_t"]), float(info["n_partials"])
    sig = n_t * vs if getattr(H, "keep_sigma", False) else 0.0
    if R == 1 and schedule == 0:
        return {
            "k_col": v_bytes + vs * (n + n_p),
            "k_reduce": vs * (n_p + n_t) + sig,
            "k_row": d_bytes + u_bytes + vs * (n + n_t + 2 * n),
        }
    if R == 1:
        return {
            # dense row-panel sections and column tiles: D and V bytes, x, y read+write,
            # partial sums written
            "k_p1": d_bytes + v_bytes + vs * (n + 2 * n + n_p),
            "k_reduce": vs * (n_p + n_t) + sig,
            # U sections: U bytes, t, y read+write
            "k_p2": u_bytes + vs * (n_t + 2 * n),
        }
    return {
        # X transposed (read + write) then V bytes, X rows, partials written
        "k_xpose+k_col_b": v_bytes + R * vs * (2 * n + n + n_p),
        "k_reduce_b": R * vs * (n_p + n_t) + sig,
        # D and U bytes, X and t rows, Y read+write
        "k_row_b": d_bytes + u_bytes + R * vs * (n + n_t + 2 * n),
    }


# launch parameters chosen by the autotuner (bench.py --tune), per kind of matrix
TUNE_CACHE = os.path.join(ROOT, "paper_2308_10960_amd", "tune_cache.txt")

BATCH_KERNELS = ("k_xpose", "k_col_b", "k_reduce_b", "k_row_b")


def kernels_source_hash(kernel="k_row"):
    """Hash of the sources a kernel is built from (the single- or the
    multi-right-hand-side kernel file, the shared device header, the store
    layout)."""
    batch = any(k in kernel for k in BATCH_KERNELS)
    h = hashlib.sha256()
    for f in ("hm_kernels_batch.hip" if batch else "hm_kernels.hip", "hm_device.hpp", "hm_layout.hpp"):
        with open(os.path.join(ROOT, "paper_2308_10960_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None.  workload: the
    preset name, with _n<n> when the size is overridden and _r<R> for R
    right-hand sides (profiles/traffic_<kernel>_<workload>.json); a phase
    of several launches (k_col over tile classes) holds their sum."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernels_source_hash(kernel):
        return None
    return d.get("bytes_per_launch")


# the 8 resident matrices of the request loop: sphere-Laplace and cube-exp
# kernels, n from 2^14 to 2^20 (the n = 2^20 cube, 111 s of host construction
# and 137 GB of host memory, is replaced by its n = 2^18 instance)
SERVE_SET = [("sphere", 16384), ("cube", 16384), ("sphere", 65536), ("cube", 65536),
             ("sphere", 262144), ("cube", 131072), ("sphere", 1048576), ("cube", 262144)]


def serve_bench(args, torch, hmgen, hm, DeviceHMatrix):
    """Request loop under Poisson arrivals: 8 resident mixed-precision
    matrices, requests of 1-64 right-hand sides, matrix chosen uniformly.
    First a closed-loop burst measures the saturation rate; then open-loop
    Poisson streams at 0.5, 0.8 and 0.95 x that rate give p50 / p99 latency
    (the 0.8 point is the headline)."""
    sizes, Ds = [], []
    for geo, n in SERVE_SET:
        name = "sphere4k_mixed" if geo == "sphere" else "cube4k"
        H = hmgen.build_preset(name, n=n, dtype="mixed")
        cache = None if args.no_tune_cache or not os.path.exists(args.tune_cache) else args.tune_cache
        Ds.append(DeviceHMatrix(H, hm.HM_F32, max_nrhs=64, tune_cache=cache))
        torch.cuda.synchronize()
        sizes.append(H.n)
        log(f"serve: built {geo} n={n} in {H.build_seconds:.1f}s, store {Ds[-1].info['store_bytes'] / 1e9:.2f} GB")
        del H                                     # the host factors are no longer needed
    arena_bytes = args.serve_arena_gb << 30
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    streams = [torch.cuda.Stream() for _ in range(args.serve_streams)]
    rng = np.random.default_rng(hmgen.presets.SEED_REQUESTS)
    # right-hand sides: one N(0,1) pool of 64 columns per matrix; a request of
    # r columns reads the first r (a contiguous column-major slice).  Client
    # buffers are page-locked (allocated pinned), so the request loop copies
    # them to and from the device without staging.
    def pinned(n):
        return torch.empty((64, n), dtype=torch.float32, pin_memory=True).numpy().T   # (n, 64), column-major

    pool = []
    for n in sizes:
        buf = pinned(n)
        buf[:] = rng.standard_normal((n, 64)).astype(np.float32)
        pool.append(buf)

    # results: a ring of OUT_RING output buffers per matrix; a request reuses
    # the buffer of the request OUT_RING places before it on the same
    # matrix, after waiting for that one (host memory stays bounded)
    OUT_RING = 16
    outbuf = [[None] * OUT_RING for _ in sizes]

    def make(count):
        reqs = []
        for _ in range(count):
            m = int(rng.integers(len(sizes)))
            r = int(rng.integers(1, 65))
            reqs.append((m, r, pool[m][:, :r]))
        return reqs

    def run(reqs, rate):
        s = hm.hm_server_create([D.handle for D in Ds], arena, arena_bytes, streams)
        last = [[None] * OUT_RING for _ in sizes]
        count = [0] * len(sizes)
        res = []
        t0 = time.perf_counter()
        gaps = rng.exponential(1.0 / rate, len(reqs)) if rate else np.zeros(len(reqs))
        t_next = t0
        for (m, r, X), g in zip(reqs, gaps):
            j = count[m] % OUT_RING
            count[m] += 1
            if last[m][j] is not None:
                res.append(hm.hm_wait(s, last[m][j], 600_000_000))
            if outbuf[m][j] is None:
                outbuf[m][j] = pinned(sizes[m])
            Y = outbuf[m][j]
            t_next += g
            while time.perf_counter() < t_next:
                pass
            last[m][j] = hm.hm_submit(s, m, r, X, X.shape[0], Y, Y.shape[0])
        res += [hm.hm_wait(s, t, 600_000_000) for row in last for t in row if t is not None]
        wall = time.perf_counter() - t0
        p50, p99, mps = hm.hm_server_stats(s)
        hm.hm_server_destroy(s)
        assert len(res) == len(reqs) and all(r == hm.HM_OK for r in res), res
        rhs = sum(r for _, r, _ in reqs)
        return {"p50_us": round(p50, 1), "p99_us": round(p99, 1), "matvecs_per_s": round(rhs / wall, 1),
                "requests": len(reqs), "rhs": rhs, "wall_s": round(wall, 3)}

    run(make(32), None)                                   # warm-up
    sat = run(make(args.serve_requests), None)
    log("serve: saturation", sat)
    sweep = []
    for load in (0.5, 0.8, 0.95):
        req_rate = load * sat["matvecs_per_s"] / 32.5     # mean r of U{1..64} is 32.5
        pt = run(make(args.serve_requests), req_rate)
        pt["load"] = load
        pt["arrival_rate_per_s"] = round(req_rate, 2)
        log("serve: load", load, pt)
        sweep.append(pt)
    out = dict(next(p for p in sweep if p["load"] == 0.8))
    out["saturation_matvecs_per_s"] = sat["matvecs_per_s"]
    out["sweep"] = sweep
    out["matrices"] = [f"{g}-n{n}" for g, n in SERVE_SET]
    out["arena_gb"] = args.serve_arena_gb
    out["streams"] = args.serve_streams
    for D in Ds:
        D.close()
    return out


def host_threads() -> int:
    """Host cores this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(env)) if env.isdigit() and int(env) > 0 else n


def cpu_baseline(H, xh, alg_bytes, seconds):
    """The CPU oracle timed on full single-RHS products of the same matrix:
    the plain single-threaded loop (the pinned oracle, as it stands) until
    ``seconds`` have passed and at least 3 runs, then its all-cores variant
    (bitwise the same result) for at least 3 runs; medians."""
    import oracle
    single = []
    while len(single) < 3 or sum(single) < seconds:
        a = time.perf_counter()
        oracle.hmvm(H, xh)
        single.append(time.perf_counter() - a)
    nthreads = host_threads()
    multi, used = [], 0
    while len(multi) < 3 or sum(multi) < seconds / 4:
        a = time.perf_counter()
        _, used = oracle.hmvm_omp(H, xh, nthreads=nthreads)
        multi.append(time.perf_counter() - a)
    t1, tn = float(np.median(single)), float(np.median(multi))
    return {"value": round(alg_bytes / t1 / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "seconds_per_matvec": round(t1, 4), "runs": len(single),
            "sample": f"median of {len(single)} full single-RHS products of the same n={H.n} matrix, "
                      "single-threaded FP64 oracle",
            "all_cores": {"value": round(alg_bytes / tn / 1e9, 3), "unit": "GB/s", "cores": used,
                          "affinity_cpus": len(os.sched_getaffinity(0)),
                          "seconds_per_matvec": round(tn, 4), "runs": len(multi),
                          "sample": f"median of {len(multi)} full products, the oracle's all-cores variant "
                                    "(OpenMP over row ranges, bitwise the single-threaded result)"}}


FP64_PEAK_TFLOPS = 78.6


def lu_bench(args, torch, hmgen, hm):
    """The H-LU factorisation with accumulated updates of the workload's
    kernel matrix (sphere or cube, its eps) at n = --n (default 4096): the
    GPU's time per factorisation over --steps fresh objects, the truncation
    kernel's arithmetic rate against the FP64 peak, and the oracle's time on
    the same matrix (one run, on all host cores numpy uses)."""
    from paper_2308_10960_amd.lu import DeviceHLU
    p = hmgen.preset(args.workload)
    n = args.n or 4096
    pts = hmgen.fibonacci_sphere(n) if p["geometry"] == "sphere" else hmgen.cube_points(n, 0)
    kern = hmgen.hmatrix.KERNEL_LAPLACE if p["kernel"] == "laplace" else hmgen.hmatrix.KERNEL_EXP
    H = hmgen.hmatrix.build_hmatrix(pts, kern, eps=p["eps"])
    dt = hm.HM_F64 if args.lu_dtype == "f64" else hmgen.dfl_format(p["eps"])
    log(f"H-LU of {p['geometry']} n={n} eps={p['eps']}: {H.nblocks} leaves, final leaves in {args.lu_dtype}")
    steps = max(1, min(args.steps, 5))
    times, st = [], None
    for q in range(steps + 1):                         # the first is a warm-up
        G = DeviceHLU(H)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = G.factor(p["eps"], dt)
        t1 = time.perf_counter()
        G.close()
        if q > 0:
            times.append(t1 - t0)
        log(f"factorisation {q}: {t1 - t0:.3f}s")
    G = DeviceHLU(H)
    prof = G.factor(p["eps"], dt, profile=True)
    G.close()
    sec = float(np.median(times))
    per = prof["trunc_flops"] / max(prof["timed_truncations"], 1)
    avg_ms = prof["trunc_ms"] / max(prof["timed_truncations"], 1)
    achieved = per / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    log("statistics", st, "profiled", prof)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import hlu as ohlu
        t0 = time.perf_counter()
        ohlu.HLU(H, p["eps"], dt=None if dt == hm.HM_F64 else dt).factor()
        cs = time.perf_counter() - t0
        cpu = {"value": round(cs, 3), "unit": "s", "cores": host_threads(), "kind": "oracle",
               "sample": f"one factorisation of the same n={n} matrix by the numpy oracle (oracle/hlu.py)"}
        log("oracle factorisation: %.2fs" % cs)
    out = {"metric": "H-LU factorisation time (accumulated updates)", "value": round(sec, 4), "unit": "s",
           "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": round(sec * 1e3, 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"hlu {p['geometry']}-{p['kernel']} n={n} eps={p['eps']} leaves {args.lu_dtype}",
                      "n": n, "eps": p["eps"], "leaves": int(H.nblocks), "kernels": st["kernels"],
                      "truncations": st["truncations"], "max_rank": st["max_rank"],
                      "stored_bytes": st["stored_bytes"], "arena_peak": st["arena_peak"]},
           "roofline": {"bound": "alu", "kernel": "k_trunc", "achieved": round(achieved, 4),
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 6),
                        "traffic": None, "flops_per_launch": per, "avg_ms": round(avg_ms, 4),
                        "share_of_factor_time": round(prof["trunc_ms"] / 1e3 / sec, 3) if sec > 0 else None},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sphere256k")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides per product (> 1: hm_mvm_batch; reported separately)")
    ap.add_argument("--n", type=int, default=0, help="override the workload size (not the default line)")
    ap.add_argument("--dtype", default=None,
                    help="override the workload's storage (f64, f32, mixed, mixed64, dfl, aplr, aflp, bfl)")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner on this matrix before the timed region and store its "
                         "choice in the tune cache (default: read the cache, no tuning)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="tune cache to read (and, with --tune, to update)")
    ap.add_argument("--no-tune-cache", action="store_true",
                    help="ignore the tune cache: built-in launch parameters")
    ap.add_argument("--launch", default="",
                    help="launch parameters applied after the tune cache (e.g. 'colb=1'); not the default line")
    ap.add_argument("--build", choices=("host", "gpu"), default="host",
                    help="construct the matrix's leaves on the host (default) or on the GPU (ACA and the "
                         "truncation of Algorithm 1 in HIP kernels); --build-compare also times the other")
    ap.add_argument("--build-compare", action="store_true",
                    help="also construct the matrix the other way and report both times")
    ap.add_argument("--no-stream-probe", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-loop measurement")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per load point")
    ap.add_argument("--serve-arena-gb", type=int, default=16)
    ap.add_argument("--serve-streams", type=int, default=8)
    ap.add_argument("--lu", action="store_true",
                    help="time the H-LU factorisation (accumulated updates) of the workload's matrix at --n "
                         "(default 4096) instead of the product, with the oracle's factorisation beside it")
    ap.add_argument("--lu-dtype", default="f64", help="storage of the final L and U leaves: f64 or dfl")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(sharding the row panels over GPUs, with one all-gather of x, is designed but not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import hmgen
    from paper_2308_10960_amd import hm, DeviceHMatrix

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    if args.copy_gib > 0:
        nbytes = int(args.copy_gib * 2 ** 30) // 16 * 16
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "launches": max(1, args.steps)}), flush=True)
        return
    if args.lu:
        lu_bench(args, torch, hmgen, hm)
        return
    p = hmgen.preset(args.workload)
    if args.dtype:
        p["dtype"] = args.dtype
    log("building", args.workload, p, "leaves on the", args.build)
    from paper_2308_10960_amd import construct

    def make_matrix(where):
        filler = (lambda T: construct.fill_gpu(T)) if where == "gpu" else None
        return hmgen.build_preset(args.workload, n=args.n or None, dtype=p["dtype"], filler=filler)

    H = make_matrix(args.build)
    st = H.stats()
    log("built in %.1fs: %s" % (H.build_seconds, st))
    build_info = {"leaves_on": args.build, "seconds": round(H.build_seconds, 3),
                  "host_threads": hmgen.hmatrix.default_threads()}
    if args.build == "gpu":
        build_info["gpu"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in H.fill_stats.items()}
    if args.build_compare:
        other = "host" if args.build == "gpu" else "gpu"
        H2 = make_matrix(other)
        build_info[f"{other}_seconds"] = round(H2.build_seconds, 3)
        d = np.abs(H.rank.astype(np.int64) - H2.rank.astype(np.int64))
        build_info["rank_diff_max"] = int(d.max())
        build_info["rank_diff_leaves"] = int((d > 0).sum())
        del H2
    log("construction", build_info)
    # the byte-aligned formats and the eps = 1e-8 mixed storage accumulate in FP64
    mixed = p["dtype"] not in ("f64", "dfl", "aplr", "aflp", "bfl", "mixed64")
    acc = hm.HM_F32 if mixed else hm.HM_F64
    storage = p["dtype"]
    if storage == "dfl":
        storage = hmgen.hmatrix.DT_NAMES[hmgen.dfl_format(p["eps"])]
    elif storage == "aplr":
        storage = "aplr-dfl"
    elif storage == "aflp":
        storage = "aflp-per-block"
    elif storage == "bfl":
        storage = hmgen.hmatrix.DT_NAMES[hmgen.bfl_format(p["eps"])]
    elif storage == "mixed64":
        storage = "mixed-f64acc (dense f64, low-rank f32/f16/bf16)"
    vs = 4 if mixed else 8
    stream = torch.cuda.Stream()
    cache = None if args.no_tune_cache or not os.path.exists(args.tune_cache) else args.tune_cache
    R = args.nrhs

    def build(chunk=0, tile=0, mix=0, use_cache=True):
        with torch.cuda.stream(stream):
            return DeviceHMatrix(H, acc, stream=stream, max_nrhs=R, tune_cache=cache if use_cache else None,
                                 chunk_rows=chunk, tile_groups=tile, tile_mix=mix)

    if R > 1:
        Xh = hmgen.gaussian_block(H.n, R, seed=hmgen.presets.SEED_RHS)
        X = torch.from_numpy(np.ascontiguousarray(Xh.T)).to(
            torch.float64 if acc == hm.HM_F64 else torch.float32).cuda()
        Y = torch.zeros_like(X)

    def make_step(D):
        """One product of D and its vectors (x, y)."""
        if R == 1:
            xv = D.vector(hmgen.uniform_vector(H.n, seed=hmgen.presets.SEED_X))
            yv = D.vector()
            return (lambda: D.mvm(xv, yv, 1.0, stream=stream)), xv, yv
        return (lambda: hm.hm_mvm_batch(D.handle, R, 1.0, X, H.n, Y, H.n, D.work, D.work.numel(),
                                        stream)), X[0], Y

    D = build()
    step, x, y = make_step(D)
    torch.cuda.synchronize()

    key = hm.hm_matrix_tune_key(D.handle)
    if args.launch:
        hm.hm_matrix_set_launch(D.handle, args.launch)
    if args.tune:
        from paper_2308_10960_amd import tune
        best, times = tune.tune(D, step, tune.CANDIDATES if R == 1 else tune.BATCH_CANDIDATES)
        shape, shape_times = tune.tune_shape(lambda c, t, mx: build(c, t, mx, use_cache=False),
                                             lambda Dc: make_step(Dc)[0], best,
                                             variants=tune.COLW_VARIANTS if R == 1 else ("",))
        chosen = f"{best} chunk={shape[0]} tile={shape[1]} tmix={shape[2] - 1} {shape[3]}".strip()
        tune.write_cache(args.tune_cache, key, chosen)
        cache = args.tune_cache
        D.close()
        D = build()                                 # the tuned launch parameters and tile shape
        step, x, y = make_step(D)
        torch.cuda.synchronize()
        tuned = {"source": "autotuner, this run (written to the tune cache)", "key": key,
                 "chosen": chosen, "avg_ms": {k: round(v, 5) for k, v in times.items()},
                 "shape_avg_ms": {f"chunk={c} tile={t} tmix={mx - 1} {w}".strip(): round(v, 5)
                                  for (c, t, mx, w), v in shape_times.items()}}
    else:
        tuned = {"source": "tune cache" if cache else "built-in", "key": key,
                 "chosen": hm.hm_matrix_get_launch(D.handle)}
    log("launch parameters:", tuned)
    info = D.info
    log("uploaded: store %.3f GB, alg %.3f GB" % (info["store_bytes"] / 1e9, info["alg_bytes"] / 1e9))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hm.hm_profile_begin(D.handle, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_k, calls = hm.hm_profile_end(D.handle)
    assert calls == args.steps
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # factors once per product, vectors once per right-hand side
    alg = info["alg_bytes"] + (R - 1) * vs * (H.n + 2 * H.n)
    value = alg / (ms_per_step * 1e-3) / 1e9
    log("%d right-hand sides: %.1f matvecs/s" % (R, R / (ms_per_step * 1e-3)))
    log("%.4f ms/step, %.1f GB/s effective (%.1f%% of 8 TB/s)" % (ms_per_step, value, value / 80.0))

    schedule = int(hm.hm_matrix_get_launch(D.handle).split()[0].split("=")[1])
    kb = kernel_bytes(H, info, vs, R, schedule)
    names = KERNELS[schedule] if R == 1 else KERNELS_BATCH
    avg_ms = {k: ms_k[i] / calls for i, k in enumerate(names)}
    dom = max(avg_ms, key=avg_ms.get)
    achieved = kb[dom] / (avg_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": read_traffic(dom, args.workload + (f"_n{args.n}" if args.n else "") +
                                        (f"_r{R}" if R > 1 else "")),
                "alg_bytes_per_launch": kb[dom], "avg_ms": round(avg_ms[dom], 5)}
    kernels = {k: {"avg_ms": round(avg_ms[k], 5), "alg_bytes": kb[k],
                   "gbs": round(kb[k] / (avg_ms[k] * 1e-3) / 1e9, 1) if avg_ms[k] > 0 else None}
               for k in names}
    log("kernels", kernels)

    # distribution of single steps (HIP events on the product's stream)
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(args.steps)]
    for e0, e1 in pairs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    each = np.array([e0.elapsed_time(e1) for e0, e1 in pairs])
    step_ms = {"median": round(float(np.median(each)), 5),
               "p10": round(float(np.percentile(each, 10)), 5),
               "p90": round(float(np.percentile(each, 90)), 5)}
    log("step ms", step_ms)

    # the same product replayed from a HIP graph
    if R == 1:
        g = hm.hm_graph_create(D.handle, 1, 1.0, x, H.n, y, H.n, D.work, D.work.numel())
    else:
        g = hm.hm_graph_create(D.handle, R, 1.0, X, H.n, Y, H.n, D.work, D.work.numel())
    for _ in range(args.warmup):
        hm.hm_graph_launch(g, stream)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(args.steps):
        hm.hm_graph_launch(g, stream)
    g1.record(stream)
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps
    hm.hm_graph_destroy(g)
    log("graph replay: %.4f ms/step" % graph_ms)

    stream_gbs = None
    if not args.no_stream_probe:
        nbytes = 4 << 30
        buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        scratch = torch.zeros(4, dtype=torch.int32, device="cuda")
        for _ in range(3):
            hm.hm_stream_read(buf, nbytes, scratch, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            hm.hm_stream_read(buf, nbytes, scratch, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        stream_gbs = nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del buf
        log("stream-read probe: %.1f GB/s" % stream_gbs)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(H, x.cpu().numpy().astype(np.float64), info["alg_bytes"], args.cpu_seconds)
        log("cpu baseline", cpu)

    serving = None
    if not args.no_serve:
        serving = serve_bench(args, torch, hmgen, hm, DeviceHMatrix)
        log("serving", serving)

    out = {
        "metric": "H-MVM effective GB/s & % HBM peak at n=2^18 eps=1e-6; p50/p99 req latency",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"{p['geometry']}-{p['kernel']} n={H.n} eps={p['eps']} "
                               f"{storage} {R}rhs leaf64 eta2",
                   "n": H.n, "eps": p["eps"], "storage": storage, "nrhs": R,
                   "matvecs_per_s": round(R / (ms_per_step * 1e-3), 1),
                   "blocks": st["blocks"], "dense_blocks": st["dense_blocks"],
                   "lowrank_blocks": st["lowrank_blocks"], "mean_rank": round(st["mean_rank"], 2),
                   "alg_bytes": alg, "store_bytes": info["store_bytes"]},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "stream_read_gbs": round(stream_gbs, 1) if stream_gbs else None,
        "pct_of_stream_read": round(100 * value / stream_gbs, 2) if stream_gbs else None,
        "step_ms": step_ms,
        "graph_ms_per_step": round(graph_ms, 5),
        "launch": hm.hm_matrix_get_launch(D.handle),
        "tuning": tuned,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "serving": serving,
        "construction": build_info,
    }
    print(json.dumps(out), flush=True)
    D.close()


if __name__ == "__main__":
    main()
