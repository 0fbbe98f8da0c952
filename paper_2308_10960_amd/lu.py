"""H-LU factorisation on the GPU (include/hm_lu.h): argument marshalling only.

The factorisation, the triangular solves and every truncation run in the
library's HIP kernels; this module passes the cluster tree and the leaves of
an hmgen H-matrix to ``hm_lu_create`` and wraps the handle.
"""

from __future__ import annotations

import numpy as np

from . import hm


class DeviceHLU:
    """The H-LU object of the H-matrix ``H`` on the current device.

    ``arena_bytes``: device memory for the factors and all temporaries; the
    factorisation frees its temporaries only at its end (its branches run
    on several streams), so the default is generous: the larger of 16 GiB
    and 2048 times the bytes of A's leaves, at most half of the free device
    memory."""

    def __init__(self, H, arena_bytes: int | None = None):
        tr = H.tree()
        nb = H.nblocks
        kind = (np.asarray(H.adm) != 0).astype(np.int32)
        rank = np.where(kind == 1, H.rank, 0).astype(np.int32)
        a_ptr = np.asarray(H.a_ptr, np.uint64).copy()
        b_ptr = np.asarray(H.b_ptr, np.uint64).copy()
        self._keep = []
        if H.keep_sigma:                               # U = W diag(s) for the C-ABI's U V^T
            for i in np.flatnonzero(kind == 1):
                a, _, s = H.factors(int(i))
                U = np.asfortranarray(a * s)
                self._keep.append(U)
                a_ptr[i] = U.ctypes.data
        m = (H.re - H.rb).astype(np.int64)
        n = (H.ce - H.cb).astype(np.int64)
        leaf_bytes = int(np.where(kind == 1, (m + n) * np.maximum(rank, 1), m * n).sum()) * 8
        if not arena_bytes:
            import torch
            free, _ = torch.cuda.mem_get_info()
            arena_bytes = min(max(16 << 30, 2048 * leaf_bytes), free // 2)
        self.arena_bytes = arena_bytes
        self.n = int(H.n)
        self.m, self.nn, self.kind = m, n, kind
        self.handle = hm.hm_lu_create(tr["begin"], tr["end"], tr["son0"], tr["son1"], tr["tau"], tr["sigma"],
                                      kind, rank, a_ptr, b_ptr, self.arena_bytes)
        self._keep = []

    def factor(self, eps: float, dtype: int = hm.HM_F64, stream=None, profile: bool = False) -> dict:
        """Factorises; with ``profile`` the truncation kernels are timed
        (HIP events) and their arithmetic is logged (see hm_lu_stats)."""
        hm.hm_lu_profile(self.handle, profile)
        hm.hm_lu_factor(self.handle, eps, dtype, stream)
        return hm.hm_lu_stats_get(self.handle)

    def solve(self, X, stream=None) -> None:
        """X := (L U)^-1 X in place; X a device tensor of shape (nrhs, n)
        (column-major n x nrhs) or (n,), FP64."""
        import torch
        assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous()
        nrhs = 1 if X.dim() == 1 else X.shape[0]
        hm.hm_lu_solve(self.handle, X, self.n, nrhs, stream)

    def leaf(self, i: int):
        """Leaf i of the factors as a dense matrix (host)."""
        m, n = int(self.m[i]), int(self.nn[i])
        if self.kind[i] == 0:
            return hm.hm_lu_leaf(self.handle, i, m, n, True)
        U, V = hm.hm_lu_leaf(self.handle, i, m, n, False)
        return U @ V.T

    def close(self) -> None:
        """Frees the device memory of the object."""
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            hm.hm_lu_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:          # interpreter shutdown: the library may be gone already
            pass
