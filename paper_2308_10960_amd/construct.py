"""GPU-side construction of an H-matrix's leaves (include/hm_construct.h).

Marshalling and batching only: the kernel entries, the adaptive cross
approximation (Sec. 5.1) and the truncation of Algorithm 1 (Sec. 2.2) run in
the library's HIP kernels.  The trees come from the host construction
(``hmgen.build_hmatrix(..., fill=False)``); the leaves are constructed on the
GPU in batches that fit a device-memory budget, packed on the device and
copied into the host tree.  Leaves the GPU cannot finish (ACA rank above the
LDS limit of the truncation, or beyond the column capacity) are filled by the
host construction, and counted.
"""

from __future__ import annotations

import time

import numpy as np

from . import hm


def _kernel_params(H):
    from hmgen.hmatrix import KERNEL_LAPLACE, KERNEL_EXP
    if H.kernel == KERNEL_LAPLACE:
        return hm.HM_KERNEL_LAPLACE, (float(H.kparams[0]), 0.0)
    if H.kernel == KERNEL_EXP:
        return hm.HM_KERNEL_EXP, (float(H.kparams[0]), float(H.kparams[1]))
    raise ValueError(f"kernel {H.kernel} has no GPU construction")


# ACA columns reserved per leaf in the first pass; leaves whose ACA needs
# more run again with HM_CONSTRUCT_MAX_RANK columns
FIRST_CAP = 48
# doubles of the page-locked staging buffer for the copies to the host (1 GiB)
STAGE = 1 << 27


def _batches(order, need, budget):
    batches, cur, acc = [], [], 0
    for b in order:
        if cur and acc + need[b] > budget:
            batches.append(np.array(cur, np.int64))
            cur, acc = [], 0
        cur.append(b)
        acc += need[b]
    if cur:
        batches.append(np.array(cur, np.int64))
    return batches


def fill_gpu(H, eps_aca: float | None = None, budget_bytes: int = 48 << 30, device: str = "cuda",
             stream=None) -> dict:
    """Construct every leaf of the tree-only H-matrix ``H`` on the GPU (ACA
    at eps_aca, default H.eps / 10, then Algorithm 1 at H.eps); returns
    statistics (seconds, batches, leaves left to the host).  The device
    memory for the leaves' regions is at most budget_bytes and half of what
    is free."""
    import torch
    t0 = time.perf_counter()
    kernel, params = _kernel_params(H)
    eps_aca = H.eps / 10 if eps_aca is None else eps_aca
    pc = torch.from_numpy(np.ascontiguousarray(H.points[H.perm], dtype=np.float64)).to(device)
    m = (H.re - H.rb).astype(np.int64)
    n = (H.ce - H.cb).astype(np.int64)
    adm = (np.asarray(H.adm) != 0).astype(np.int32)
    free, _ = torch.cuda.mem_get_info()
    budget_d = min(budget_bytes, free // 2) // 8
    host_left, gpu_s, copy_s = [], 0.0, 0.0
    nbatches, retried = 0, 0
    h_stage = None
    todo = np.argsort(-(m + n), kind="stable")             # large leaves first within a batch
    for cap_max in (FIRST_CAP, hm.HM_CONSTRUCT_MAX_RANK):
        if todo.size == 0:
            break
        cap = np.where(adm == 1, np.minimum(np.minimum(m, n), cap_max), 0)
        # device doubles per leaf: output and scratch regions (hm_construct_layout's rule)
        need = np.where(adm == 1, 2 * ((m + n) * cap + cap) + (m + 7) // 8 + 4, m * n + 2)
        batches = _batches(todo, need, max(budget_d, int(need[todo].max())))
        nbatches += len(batches)
        again = []
        d_out = d_scr = d_desc = d_rank = None
        for idx in batches:
            blk = np.zeros(idx.shape[0], hm.CBLOCK_DTYPE)
            blk["rb"], blk["cb"], blk["m"], blk["n"] = H.rb[idx], H.cb[idx], m[idx], n[idx]
            blk["adm"], blk["cap"] = adm[idx], cap[idx]
            out_d, scr_d = hm.hm_construct_layout(blk)
            nb = idx.shape[0]

            def grow(t, count, dtype):
                return t if t is not None and t.numel() >= count else torch.empty(max(count, 1), dtype=dtype,
                                                                                  device=device)
            d_out = grow(d_out, out_d, torch.float64)
            d_scr = grow(d_scr, scr_d, torch.float64)
            d_desc = grow(d_desc, nb * hm.CBLOCK_DTYPE.itemsize, torch.uint8)
            d_rank = grow(d_rank, 2 * nb, torch.int32)
            a = time.perf_counter()
            hm.hm_construct(pc, H.n, blk, d_desc, d_desc.numel(), kernel, params, eps_aca, H.eps,
                            H.keep_sigma, d_out, d_out.numel() * 8, d_scr, d_scr.numel() * 8, d_rank, stream)
            torch.cuda.synchronize()
            gpu_s += time.perf_counter() - a
            a = time.perf_counter()
            rank = d_rank[nb:2 * nb].cpu().numpy()
            ok = rank >= 0
            size = np.where(adm[idx] == 1, (m[idx] + n[idx] + 1) * np.maximum(rank, 0), m[idx] * n[idx])
            size = np.where(ok, size, 0)
            off = np.zeros(nb, np.int64)
            off[1:] = np.cumsum(size)[:-1]
            total = int(size.sum())
            d_off = torch.from_numpy(off).to(device)
            d_packed = torch.empty(max(total, 1), dtype=torch.float64, device=device)
            lib = hm.lib()
            hm._check(lib.hm_construct_pack(hm._ptr(d_desc), nb, hm._ptr(d_rank), hm._ptr(d_out),
                                            hm._ptr(d_off), hm._ptr(d_packed), d_packed.numel() * 8,
                                            hm._stream(stream)), "hm_construct_pack")
            # device -> host in chunks of whole leaves through two page-locked
            # buffers of STAGE doubles: the copy of one chunk runs while the
            # host tree takes the leaves of the other
            if h_stage is None:
                h_stage = [torch.empty(STAGE, dtype=torch.float64, pin_memory=True) for _ in range(2)]
            sel = np.flatnonzero(ok)
            kk = np.where(adm[idx] == 1, np.maximum(rank, 0), 0)
            chunks, q0 = [], 0
            while q0 < sel.size:
                q1 = q0 + 1
                c0 = off[sel[q0]]
                while q1 < sel.size and off[sel[q1]] + size[sel[q1]] - c0 <= STAGE:
                    q1 += 1
                chunks.append((q0, q1))
                q0 = q1
            pending = None
            for ci in range(len(chunks) + 1):
                if ci < len(chunks):
                    q0, q1 = chunks[ci]
                    c0 = int(off[sel[q0]])
                    c1 = int(off[sel[q1 - 1]] + size[sel[q1 - 1]])
                    if c1 - c0 > STAGE:
                        raise RuntimeError(f"a leaf of {c1 - c0} doubles exceeds the staging buffer")
                    buf = h_stage[ci % 2]
                    buf[:c1 - c0].copy_(d_packed[c0:c1], non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record()
                if pending is not None:
                    pq0, pq1, pc0, pbuf, pev = pending
                    pev.synchronize()
                    part = sel[pq0:pq1]
                    H.set_factors(idx[part], kk[part], pbuf.numpy(), off[part] - pc0, kk[part])
                pending = (q0, q1, c0, buf, ev) if ci < len(chunks) else None
            torch.cuda.synchronize()
            del d_packed, d_off
            # ACA past its columns with room to grow: again with more; the rest to the host
            more = (rank == -1) & (cap[idx] < np.minimum(np.minimum(m[idx], n[idx]), hm.HM_CONSTRUCT_MAX_RANK))
            again.extend(idx[more].tolist())
            host_left.extend(idx[~ok & ~more].tolist())
            copy_s += time.perf_counter() - a
        del d_out, d_scr, d_desc, d_rank
        torch.cuda.empty_cache()
        retried += len(again) if cap_max == FIRST_CAP else 0
        todo = np.array(again, np.int64)
    host_left.extend(todo.tolist())
    a = time.perf_counter()
    if host_left:
        H.fill_blocks(np.array(host_left, np.int64), eps_aca=eps_aca)
    host_s = time.perf_counter() - a
    return {"seconds": time.perf_counter() - t0, "gpu_seconds": gpu_s, "copy_seconds": copy_s,
            "host_fallback_seconds": host_s, "batches": nbatches, "second_pass_leaves": retried,
            "host_leaves": len(host_left), "leaves": int(H.nblocks)}


def build_hmatrix_gpu(points, kernel: int, *, leaf: int = 64, eta: float = 2.0, eps: float = 1e-6,
                      eps_aca: float | None = None, keep_sigma: bool = False, diag: float | None = None,
                      length: float = 0.1, budget_bytes: int = 24 << 30, device: str = "cuda"):
    """The H-matrix of ``kernel`` over ``points``: trees on the host
    (hmgen), leaves on the GPU.  Returns (H, statistics)."""
    import hmgen
    t0 = time.perf_counter()
    H = hmgen.build_hmatrix(points, kernel, leaf=leaf, eta=eta, eps=eps, eps_aca=eps_aca,
                            keep_sigma=keep_sigma, diag=diag, length=length, fill=False)
    tree_s = time.perf_counter() - t0
    st = fill_gpu(H, eps_aca=eps_aca, budget_bytes=budget_bytes, device=device)
    st["tree_seconds"] = tree_s
    H.build_seconds = time.perf_counter() - t0
    st["total_seconds"] = H.build_seconds
    return H, st
