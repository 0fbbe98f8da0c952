"""ctypes driver for libhmgen: builds an H-matrix and exposes its leaves.

Every vector index here is in cluster order (the order of the cluster tree's
leaves); ``perm[i]`` is the original point index at cluster position i.
"""

from __future__ import annotations

import ctypes as C
import math
import os
import time
from dataclasses import dataclass, field

import numpy as np

from .geometry import mean_nn_distance

DT_F64, DT_F32, DT_F16, DT_BF16 = 0, 1, 2, 3
DT_DFL32, DT_DFL40, DT_DFL48, DT_DFL16, DT_DFL24 = 4, 5, 6, 7, 8
DT_AFLP16, DT_AFLP24, DT_AFLP32, DT_AFLP40, DT_AFLP48 = 9, 10, 11, 12, 13
DT_BFL24, DT_BFL40, DT_BFL48 = 14, 15, 16
DT_BYTES = {DT_F64: 8, DT_F32: 4, DT_F16: 2, DT_BF16: 2, DT_DFL32: 4, DT_DFL40: 5, DT_DFL48: 6,
            DT_DFL16: 2, DT_DFL24: 3, DT_AFLP16: 2, DT_AFLP24: 3, DT_AFLP32: 4, DT_AFLP40: 5, DT_AFLP48: 6,
            DT_BFL24: 3, DT_BFL40: 5, DT_BFL48: 6}
DT_NAMES = {DT_F64: "f64", DT_F32: "f32", DT_F16: "f16", DT_BF16: "bf16",
            DT_DFL32: "dfl32", DT_DFL40: "dfl40", DT_DFL48: "dfl48", DT_DFL16: "dfl16", DT_DFL24: "dfl24",
            DT_AFLP16: "aflp16", DT_AFLP24: "aflp24", DT_AFLP32: "aflp32", DT_AFLP40: "aflp40",
            DT_AFLP48: "aflp48", DT_BFL24: "bfl24", DT_BFL40: "bfl40", DT_BFL48: "bfl48"}


def dfl_mantissa_bits(eps: float) -> int:
    """Mantissa bits m_eps for accuracy eps (Sec. 3.2 leaves the rule to the
    accuracy; read here as the least m with unit roundoff 2^-(m+1) <= eps/2,
    i.e. m = ceil(log2(1/eps)))."""
    if not 0 < eps < 1:
        raise ValueError("eps must be in (0, 1)")
    return int(math.ceil(-math.log2(eps)))


def dfl_format(eps: float) -> int:
    """DFL storage format for accuracy eps (Sec. 3.2): 1 sign + 11 exponent +
    m_eps mantissa bits, mantissa increased to a whole number of bytes; 8
    bytes is FP64 itself.  Provided: 4, 5 and 6 bytes (fewer bytes take
    DFL32, 7 bytes take FP64)."""
    nbytes = -(-(1 + 11 + dfl_mantissa_bits(eps)) // 8)
    return {4: DT_DFL32, 5: DT_DFL40, 6: DT_DFL48}.get(max(nbytes, 4), DT_F64)

def bfl_format(eps: float) -> int:
    """BFL storage format for accuracy eps (Sec. 3.2): 1 sign + 8 exponent +
    m_eps mantissa bits, the mantissa increased to whole bytes; 2 and 4
    bytes are BF16 and FP32, 3 / 5 / 6 bytes BFL24 / 40 / 48, 7 bytes take
    FP64."""
    nbytes = -(-(1 + 8 + dfl_mantissa_bits(eps)) // 8)
    return {2: DT_BF16, 3: DT_BFL24, 4: DT_F32, 5: DT_BFL40, 6: DT_BFL48}.get(nbytes, DT_F64)

KERNEL_LAPLACE, KERNEL_EXP, KERNEL_SEPARABLE = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmgen.so")

_lib = None

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run hmgen.build.build()")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.hmg_build_tree.argtypes = [_f64p, C.c_int64, C.c_int32, C.c_double, C.POINTER(vp)]
    L.hmg_build_tree.restype = C.c_int
    L.hmg_destroy.argtypes = [vp]
    L.hmg_num_clusters.argtypes = [vp]
    L.hmg_num_clusters.restype = C.c_int64
    L.hmg_num_blocks.argtypes = [vp]
    L.hmg_num_blocks.restype = C.c_int64
    L.hmg_get_perm.argtypes = [vp, _i64p]
    L.hmg_get_clusters.argtypes = [vp, _i64p, _i64p, _i32p, _i32p, _i32p, _f64p]
    L.hmg_get_blocks.argtypes = [vp, _i64p, _i64p, _i64p, _i64p, _i32p, _i32p, _i32p, _i32p]
    L.hmg_fill.argtypes = [vp, C.c_int32, _f64p, C.c_double, C.c_double, C.c_int32, C.c_int32]
    L.hmg_fill.restype = C.c_int
    L.hmg_fill_part.argtypes = [vp, C.c_int32, _f64p, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                C.c_int32, C.c_int32]
    L.hmg_fill_part.restype = C.c_int
    L.hmg_set_kernel.argtypes = [vp, C.c_int32, _f64p, C.c_int32]
    L.hmg_set_kernel.restype = C.c_int
    L.hmg_set_factors.argtypes = [vp, C.c_int64, _i64p, _i32p, C.c_void_p, _i64p, _i32p]
    L.hmg_set_factors.restype = C.c_int
    L.hmg_fill_blocks.argtypes = [vp, C.c_int64, _i64p, C.c_double, C.c_double, C.c_int32]
    L.hmg_fill_blocks.restype = C.c_int
    L.hmg_get_factor_ptrs.argtypes = [vp, _u64p, _u64p, _u64p]
    L.hmg_get_ranks.argtypes = [vp, _i32p]
    L.hmg_eval.argtypes = [vp, _i64p, _i64p, C.c_int64, _f64p]
    L.hmg_select_precision.argtypes = [vp, C.c_double, C.c_int32, _i32p, _i32p, _i32p, _f64p]
    L.hmg_select_precision.restype = C.c_int
    L.hmg_select_precision_dfl.argtypes = [vp, C.c_double, _i32p, _i32p, _i32p, _f64p]
    L.hmg_select_precision_dfl.restype = C.c_int
    L.hmg_select_aflp.argtypes = [vp, C.c_int, _i32p, _i32p, _i32p]
    L.hmg_select_aflp.restype = C.c_int
    L.hmg_round.argtypes = [_f64p, C.c_int64, C.c_int32, _f64p]
    L.hmg_truncate.argtypes = [_f64p, _f64p, C.c_int64, C.c_int64, C.c_int32, C.c_double,
                               _f64p, _f64p, _f64p]
    L.hmg_truncate.restype = C.c_int
    _lib = L
    return L


def _view(ptr: int, count: int) -> np.ndarray:
    if ptr == 0 or count == 0:
        return np.zeros(0)
    buf = (C.c_double * count).from_address(int(ptr))
    return np.ctypeslib.as_array(buf)


@dataclass
class HMatrix:
    """A constructed H-matrix: block table plus per-block FP64 factors.

    Dense leaf b: ``a`` is D_b (m x n_b, column-major).
    Low-rank leaf b: ``a`` is U_b (m x k) and ``b`` is V_b (n_b x k),
    column-major, with M_b = U_b V_b^T; when ``keep_sigma`` the form is
    W_b diag(s_b) X_b^T with ``a`` = W_b, ``b`` = X_b, ``s`` = s_b.
    """

    n: int
    points: np.ndarray
    kernel: int
    kparams: np.ndarray
    leaf: int
    eta: float
    eps: float
    keep_sigma: bool
    perm: np.ndarray = field(repr=False)
    rb: np.ndarray = field(repr=False)
    re: np.ndarray = field(repr=False)
    cb: np.ndarray = field(repr=False)
    ce: np.ndarray = field(repr=False)
    adm: np.ndarray = field(repr=False)
    rank: np.ndarray = field(repr=False)
    a_ptr: np.ndarray = field(repr=False)
    b_ptr: np.ndarray = field(repr=False)
    s_ptr: np.ndarray = field(repr=False)
    handle: int = field(repr=False, default=0)
    build_seconds: float = 0.0
    ngroups: np.ndarray | None = field(repr=False, default=None)
    group_cols: np.ndarray | None = field(repr=False, default=None)
    group_dtype: np.ndarray | None = field(repr=False, default=None)
    store_err_bound: np.ndarray | None = field(repr=False, default=None)

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.hmg_destroy(C.c_void_p(self.handle))
            self.handle = 0

    # ------------------------------------------------------------ access
    @property
    def nblocks(self) -> int:
        return int(self.rb.shape[0])

    def shape(self, i: int):
        return int(self.re[i] - self.rb[i]), int(self.ce[i] - self.cb[i])

    def factors(self, i: int):
        """numpy views (no copy) of block i's factors: (a, b, s)."""
        m, nb = self.shape(i)
        if not self.adm[i]:
            return _view(self.a_ptr[i], m * nb).reshape(nb, m).T, None, None
        k = int(self.rank[i])
        a = _view(self.a_ptr[i], m * k).reshape(k, m).T
        b = _view(self.b_ptr[i], nb * k).reshape(k, nb).T
        s = _view(self.s_ptr[i], k) if self.keep_sigma else None
        return a, b, s

    def kernel_entries(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(rows.shape[0])
        lib().hmg_eval(C.c_void_p(self.handle), rows, cols, rows.shape[0], out)
        return out

    def tree(self) -> dict:
        """The cluster tree (per cluster: begin, end, son0, son1, level;
        sons -1 at a leaf; cluster 0 is the root) and the clusters (tau,
        sigma) of every leaf of the block tree."""
        L = lib()
        h = C.c_void_p(self.handle)
        nc = L.hmg_num_clusters(h)
        beg, end = np.empty(nc, np.int64), np.empty(nc, np.int64)
        son0, son1, level = (np.empty(nc, np.int32) for _ in range(3))
        box = np.empty(6 * nc)
        L.hmg_get_clusters(h, beg, end, son0, son1, level, box)
        nb = self.nblocks
        rb, re, cb, ce = (np.empty(nb, np.int64) for _ in range(4))
        adm, tau, sig, rank = (np.empty(nb, np.int32) for _ in range(4))
        L.hmg_get_blocks(h, rb, re, cb, ce, adm, tau, sig, rank)
        return {"begin": beg, "end": end, "son0": son0, "son1": son1, "level": level, "tau": tau, "sigma": sig}

    def points_cluster_order(self) -> np.ndarray:
        return self.points[self.perm]

    # ------------------------------------------------------------ filling
    def set_factors(self, idx, rank, buf: np.ndarray, off, cap) -> None:
        """Copy factors computed elsewhere into the leaves idx (layout of
        hmg_set_factors: per leaf, D or U at buf[off], V at off + m cap, s at
        off + (m + n) cap), then refresh the ranks and factor pointers."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        rc = lib().hmg_set_factors(C.c_void_p(self.handle), idx.shape[0], idx,
                                   np.ascontiguousarray(rank, dtype=np.int32), buf.ctypes.data,
                                   np.ascontiguousarray(off, dtype=np.int64),
                                   np.ascontiguousarray(cap, dtype=np.int32))
        if rc != 0:
            raise RuntimeError("hmg_set_factors failed")
        self.refresh()

    def fill_blocks(self, idx, eps_aca: float | None = None, nthreads: int | None = None) -> None:
        """Fill the leaves idx on the host (ACA at eps_aca, default eps / 10,
        then Algorithm 1 at eps)."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        rc = lib().hmg_fill_blocks(C.c_void_p(self.handle), idx.shape[0], idx,
                                   self.eps / 10 if eps_aca is None else eps_aca, self.eps,
                                   nthreads or default_threads())
        if rc != 0:
            raise RuntimeError("hmg_fill_blocks failed")
        self.refresh()

    def refresh(self) -> None:
        """Re-read the ranks and factor pointers after the leaves changed."""
        L = lib()
        L.hmg_get_ranks(C.c_void_p(self.handle), self.rank)
        L.hmg_get_factor_ptrs(C.c_void_p(self.handle), self.a_ptr, self.b_ptr, self.s_ptr)

    # ------------------------------------------------------------ precision
    def select_precision(self, tol: float, allow_f64: bool = False, dense_f64: bool = False,
                         sigma_f64: bool = False) -> int:
        """Choose per-block storage formats (see hmg_select_precision):
        allow_f64 lets a low-rank block that FP32 cannot hold fall back to
        FP64, dense_f64 keeps the dense blocks in FP64, sigma_f64 prices the
        columns with s exact (s kept in FP64 by FP64-accumulating products).
        Returns the number of blocks that miss the budget."""
        if not self.keep_sigma:
            raise ValueError("precision selection needs keep_sigma=True")
        nb = self.nblocks
        self.ngroups = np.zeros(nb, np.int32)
        self.group_cols = np.zeros((nb, 4), np.int32)
        self.group_dtype = np.zeros((nb, 4), np.int32)
        self.store_err_bound = np.zeros(nb)
        bad = lib().hmg_select_precision(
            C.c_void_p(self.handle), tol, int(allow_f64) | 2 * int(dense_f64) | 4 * int(sigma_f64),
            self.ngroups,
            self.group_cols.reshape(-1), self.group_dtype.reshape(-1), self.store_err_bound)
        return int(bad)

    def select_precision_dfl(self, tol: float) -> int:
        """Per-column DFL formats (APLR over DFL16 ... DFL48, FP64), s kept
        in FP64 (see hmg_select_precision_dfl)."""
        if not self.keep_sigma:
            raise ValueError("precision selection needs keep_sigma=True")
        nb = self.nblocks
        self.ngroups = np.zeros(nb, np.int32)
        self.group_cols = np.zeros((nb, 4), np.int32)
        self.group_dtype = np.zeros((nb, 4), np.int32)
        self.store_err_bound = np.zeros(nb)
        bad = lib().hmg_select_precision_dfl(
            C.c_void_p(self.handle), tol, self.ngroups,
            self.group_cols.reshape(-1), self.group_dtype.reshape(-1), self.store_err_bound)
        return int(bad)

    def select_aflp(self, eps: float) -> int:
        """AFLP storage (Sec. 3.2) per block: the fewest bytes whose AFLP
        mantissa keeps m_eps = dfl_mantissa_bits(eps) bits for every data
        block of the block (see hmg_select_aflp).  Returns the number of
        blocks left in FP64."""
        nb = self.nblocks
        self.ngroups = np.zeros(nb, np.int32)
        self.group_cols = np.zeros((nb, 4), np.int32)
        self.group_dtype = np.zeros((nb, 4), np.int32)
        return int(lib().hmg_select_aflp(C.c_void_p(self.handle), dfl_mantissa_bits(eps), self.ngroups,
                                         self.group_cols.reshape(-1), self.group_dtype.reshape(-1)))

    def set_uniform_dtype(self, dt: int) -> None:
        """Store every block (all columns) in one format."""
        nb = self.nblocks
        self.ngroups = np.ones(nb, np.int32)
        self.group_cols = np.zeros((nb, 4), np.int32)
        self.group_cols[:, 0] = np.where(self.adm != 0, self.rank, 0)
        self.group_dtype = np.zeros((nb, 4), np.int32)
        self.group_dtype[:, 0] = dt

    # ------------------------------------------------------------ statistics
    def stats(self) -> dict:
        m = (self.re - self.rb).astype(np.int64)
        nb = (self.ce - self.cb).astype(np.int64)
        dense = self.adm == 0
        k = self.rank.astype(np.int64)
        d_el = int((m * nb)[dense].sum())
        lr_el = int(((m + nb) * k)[~dense].sum())
        return {
            "n": self.n, "blocks": self.nblocks, "dense_blocks": int(dense.sum()),
            "lowrank_blocks": int((~dense).sum()), "dense_elems": d_el,
            "lowrank_elems": lr_el, "max_rank": int(k.max()) if k.size else 0,
            "mean_rank": float(k[~dense].mean()) if (~dense).any() else 0.0,
            "fp64_bytes": 8 * (d_el + lr_el),
            "lowrank_not_smaller": int(((m + nb) * k >= m * nb)[~dense].sum()),
            "build_seconds": self.build_seconds,
        }


def default_threads() -> int:
    """Host threads for construction: the CPUs this process may run on,
    capped by OMP_NUM_THREADS when that is set (the CPU share of a machine
    can be smaller than what the affinity mask shows)."""
    n = len(os.sched_getaffinity(0))
    try:
        cap = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        cap = 0
    return max(1, min(n, cap) if cap > 0 else n)


def build_hmatrix(points: np.ndarray, kernel: int, *, leaf: int = 64, eta: float = 2.0,
                  eps: float = 1e-6, eps_aca: float | None = None, keep_sigma: bool = False,
                  diag: float | None = None, length: float = 0.1, nthreads: int | None = None,
                  kparams=None, progress: bool | None = None, fill: bool = True) -> HMatrix:
    """Construct the H-matrix of ``kernel`` over ``points`` (n x 3, FP64).

    kernel: KERNEL_LAPLACE (1/(4 pi r), diagonal 1/(4 pi h) with h the mean
    nearest-neighbour distance unless ``diag`` gives h), KERNEL_EXP
    (exp(-r/length), diagonal + ``diag`` (default 1e-3)), KERNEL_SEPARABLE.
    ACA runs at ``eps_aca`` (default eps/10), then Algorithm 1 at ``eps``.
    With ``progress`` (default: n >= 2^19) the leaves are filled in 16 shares
    and a line is printed after each.  With ``fill=False`` only the trees are
    built and the kernel recorded: the leaves stay empty (rank 0) until
    set_factors / fill_blocks fill them.
    """
    L = lib()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n = pts.shape[0]
    t0 = time.perf_counter()
    if kparams is None:
        if kernel == KERNEL_LAPLACE:
            h = mean_nn_distance(pts) if diag is None else float(diag)
            kparams = np.array([h, 0.0, 0.0, 0.0])
        elif kernel == KERNEL_EXP:
            kparams = np.array([length, 1e-3 if diag is None else float(diag), 0.0, 0.0])
        else:
            kparams = np.zeros(4)
    kparams = np.ascontiguousarray(kparams, dtype=np.float64)
    handle = C.c_void_p()
    rc = L.hmg_build_tree(pts.reshape(-1), n, leaf, eta, C.byref(handle))
    if rc != 0:
        raise RuntimeError(f"hmg_build_tree failed ({rc})")
    nthr = nthreads if nthreads else default_threads()
    if progress is None:
        progress = n >= 2 ** 19
    nparts = 16 if progress else 1
    if not fill:
        nparts = 0
        rc = L.hmg_set_kernel(handle, kernel, kparams, int(keep_sigma))
    for part in range(nparts):
        rc = L.hmg_fill_part(handle, kernel, kparams, eps / 10 if eps_aca is None else eps_aca, eps,
                             int(keep_sigma), nthr, part, nparts)
        if rc != 0:
            break
        if progress:
            print(f"[hmgen] n={n}: filled share {part + 1}/{nparts} of {L.hmg_num_blocks(handle)} "
                  f"blocks, {time.perf_counter() - t0:.0f}s", flush=True)
    if rc != 0:
        L.hmg_destroy(handle)
        raise RuntimeError(f"hmg_fill failed ({rc})")
    nb = L.hmg_num_blocks(handle)
    perm = np.empty(n, np.int64)
    L.hmg_get_perm(handle, perm)
    rb, re, cb, ce = (np.empty(nb, np.int64) for _ in range(4))
    adm, tau, sig, rank = (np.empty(nb, np.int32) for _ in range(4))
    L.hmg_get_blocks(handle, rb, re, cb, ce, adm, tau, sig, rank)
    ap, bp, sp = (np.empty(nb, np.uint64) for _ in range(3))
    L.hmg_get_factor_ptrs(handle, ap, bp, sp)
    H = HMatrix(n=n, points=pts, kernel=kernel, kparams=kparams, leaf=leaf, eta=eta, eps=eps,
                keep_sigma=bool(keep_sigma), perm=perm, rb=rb, re=re, cb=cb, ce=ce, adm=adm,
                rank=rank, a_ptr=ap, b_ptr=bp, s_ptr=sp, handle=handle.value)
    H.build_seconds = time.perf_counter() - t0
    return H


def round_to(x: np.ndarray, dt: int) -> np.ndarray:
    """Generator-side RNE rounding of FP64 values to a storage format."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    out = np.empty_like(x)
    lib().hmg_round(x, x.shape[0], dt, out)
    return out


def truncate(U: np.ndarray, V: np.ndarray, eps: float):
    """Algorithm 1 (QR + SVD truncation) on U (m x r), V (n x r): returns
    W (m x k), S (k), X (n x k) with U V^T ~ W diag(S) X^T."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    m, r = U.shape
    n = V.shape[0]
    W = np.zeros(m * r)
    X = np.zeros(n * r)
    S = np.zeros(r)
    k = lib().hmg_truncate(np.ascontiguousarray(U.T).reshape(-1),
                           np.ascontiguousarray(V.T).reshape(-1), m, n, r, eps, W, X, S)
    return W[: m * k].reshape(k, m).T, S[:k].copy(), X[: n * k].reshape(k, n).T


def dtype_bytes(dt: int) -> int:
    return DT_BYTES[dt]


def frob(x) -> float:
    return math.sqrt(float(np.sum(np.square(x))))
