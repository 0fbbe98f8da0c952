"""Device-resident H-matrix handle: plan + store + workspace in torch memory.

Marshalling helpers around the C-ABI (no arithmetic): the block table comes
from any object exposing per-block arrays rb, re, cb, ce, adm, rank, ngroups,
group_cols, group_dtype, keep_sigma and host factor pointers a_ptr, b_ptr,
s_ptr (FP64, column-major), e.g. the H-matrix construction in ``hmgen``.
"""

from __future__ import annotations

import numpy as np

from . import hm


def batch_slots(acc_dtype: int, nrhs: int) -> int:
    """Workspace slots (x work_bytes_per_rhs) hm_mvm_batch needs (see hm.h)."""
    if acc_dtype == hm.HM_F64:
        return 1
    return 32 if nrhs <= 32 else 64


def blocks_from_table(T) -> np.ndarray:
    adm = np.asarray(T.adm) != 0
    has_sigma = adm & bool(getattr(T, "keep_sigma", False))
    return hm.make_blocks(T.rb, T.re, T.cb, T.ce, adm.astype(np.int32),
                          np.where(adm, T.rank, 0), T.ngroups, T.group_cols, T.group_dtype,
                          has_sigma.astype(np.int32))


class DeviceHMatrix:
    def __init__(self, T, acc_dtype: int = hm.HM_F64, max_nrhs: int = 1, device="cuda",
                 stream=None, tune_cache: str | None = None, chunk_rows: int = 0, tile_groups: int = 0,
                 tile_mix: int = 0):
        import torch
        self.torch = torch
        self.n_rows = int(T.n)
        self.n_cols = int(T.n)
        self.acc_dtype = acc_dtype
        self.vec_torch = torch.float64 if acc_dtype == hm.HM_F64 else torch.float32
        self.max_nrhs = max_nrhs
        self.blocks = blocks_from_table(T)
        self.plan = hm.hm_build_plan(self.n_rows, self.n_cols, self.blocks, acc_dtype, max_nrhs,
                                     tune_cache, chunk_rows, tile_groups, tile_mix)
        self.info = hm.hm_plan_info(self.plan)
        self.store = torch.empty(self.info["store_bytes"], dtype=torch.uint8, device=device)
        s_ptr = T.s_ptr if getattr(T, "keep_sigma", False) else None
        self.handle = hm.hm_upload(self.plan, T.a_ptr, T.b_ptr, s_ptr, self.store,
                                   self.info["store_bytes"], stream)
        slots = batch_slots(acc_dtype, max_nrhs) if max_nrhs > 1 else 1
        self.work_bytes = max(256, self.info["work_bytes_per_rhs"] * slots)
        self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=device)
        self.device = device

    def mvm(self, x, y, alpha: float = 1.0, stream=None, work=None):
        """y += alpha * A x (device tensors of the vector dtype)."""
        w = self.work if work is None else work
        hm.hm_mvm(self.handle, alpha, x, y, w, w.numel(), stream)
        return y

    def mvm_batch(self, X, Y, alpha: float = 1.0, stream=None):
        """Y += alpha * A X for column-major X (n x r) given as a (r, n) tensor view."""
        nrhs = X.shape[1]
        hm.hm_mvm_batch(self.handle, nrhs, alpha, X, X.stride(1), Y, Y.stride(1), self.work,
                        self.work.numel(), stream)
        return Y

    def vector(self, values=None):
        torch = self.torch
        if values is None:
            return torch.zeros(self.n_rows, dtype=self.vec_torch, device=self.device)
        return torch.as_tensor(np.asarray(values)).to(self.vec_torch).to(self.device)

    def close(self):
        if getattr(self, "handle", None):
            hm.hm_matrix_destroy(self.handle)
            self.handle = None
        if getattr(self, "plan", None):
            hm.hm_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
