"""Python binding of libhm (include/hm.h): argument marshalling only.

Every function has the name of the C entry point it calls; all arithmetic
runs in the library's HIP kernels.  PyTorch is used by callers for device
memory and streams; this module only passes raw pointers.  If libhm.so is
missing or fails to load, every call raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HM_LIBRARY selects another build of the same library (the sanitized host
# build of the CPU tests); the default is the in-tree libhm.so
LIB_PATH = os.environ.get("HM_LIBRARY") or os.path.join(HERE, "libhm.so")

HM_OK, HM_EINVAL, HM_EPARTITION, HM_ESHAPE, HM_EDTYPE = 0, -1, -2, -3, -4
HM_ENOMEM, HM_EDEVICE, HM_EBUSY, HM_ESTATE, HM_ETIMEOUT = -5, -6, -7, -8, -9
HM_F64, HM_F32, HM_F16, HM_BF16 = 0, 1, 2, 3
HM_DFL32, HM_DFL40, HM_DFL48, HM_DFL16, HM_DFL24 = 4, 5, 6, 7, 8
HM_AFLP16, HM_AFLP24, HM_AFLP32, HM_AFLP40, HM_AFLP48 = 9, 10, 11, 12, 13
HM_BFL24, HM_BFL40, HM_BFL48 = 14, 15, 16
HM_NUM_DTYPES = 17
HM_NOALLOC_SCRATCH_BYTES = 64 << 20      # fixed workspace of hm_mvm_noalloc (include/hm.h)
HM_DENSE, HM_LOWRANK = 0, 1

HM_ERANK = -10
STATUS_NAMES = {0: "HM_OK", -1: "HM_EINVAL", -2: "HM_EPARTITION", -3: "HM_ESHAPE",
                -4: "HM_EDTYPE", -5: "HM_ENOMEM", -6: "HM_EDEVICE", -7: "HM_EBUSY",
                -8: "HM_ESTATE", -9: "HM_ETIMEOUT", -10: "HM_ERANK"}

# hm_block_desc as a numpy structured dtype (same layout as the C struct).
BLOCK_DTYPE = np.dtype([("row_begin", "<i8"), ("row_end", "<i8"), ("col_begin", "<i8"),
                        ("col_end", "<i8"), ("kind", "<i4"), ("rank", "<i4"),
                        ("ngroups", "<i4"), ("group_cols", "<i4", (4,)),
                        ("group_dtype", "<i4", (4,)), ("has_sigma", "<i4")], align=True)


class PlanOpts(C.Structure):
    _fields_ = [("acc_dtype", C.c_int32), ("vec_dtype", C.c_int32), ("max_nrhs", C.c_int32),
                ("tune", C.c_int32), ("tune_cache", C.c_char_p), ("chunk_rows", C.c_int32),
                ("tile_groups", C.c_int32), ("tile_mix", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("store_bytes", C.c_size_t), ("work_bytes_per_rhs", C.c_size_t),
                ("alg_bytes", C.c_double), ("alg_flops", C.c_double),
                ("overhead_bytes", C.c_double), ("n_dense", C.c_int64),
                ("n_lowrank", C.c_int64), ("n_row_panels", C.c_int64),
                ("n_col_tiles", C.c_int64), ("n_partials", C.c_int64), ("n_t", C.c_int64),
                ("bytes_by_dtype", C.c_size_t * HM_NUM_DTYPES)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "bytes_by_dtype"}
        d["bytes_by_dtype"] = list(self.bytes_by_dtype)
        return d


class HMError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# (name, restype, argtypes) of every entry point declared in include/hm.h
_vp, _i32, _i64, _sz, _dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
_P = C.POINTER
PROTOTYPES = {
    "hm_build_plan": (_i32, [_i64, _i64, _vp, _i64, _P(PlanOpts), _P(_vp)]),
    "hm_plan_info": (_i32, [_vp, _P(PlanInfo)]),
    "hm_plan_destroy": (None, [_vp]),
    "hm_plan_locate": (_i32, [_vp, _i64, _i32, _i64, _i64, _P(_sz), _P(_i32), _P(_sz)]),
    "hm_upload": (_i32, [_vp, _vp, _vp, _vp, _vp, _sz, _vp, _P(_vp)]),
    "hm_matrix_destroy": (None, [_vp]),
    "hm_pack_host": (_i32, [_vp, _vp, _vp, _vp, _vp, _sz]),
    "hm_mvm": (_i32, [_vp, _dbl, _vp, _vp, _vp, _sz, _vp]),
    "hm_mvm_noalloc": (_i32, [_vp, _dbl, _vp, _vp, _vp]),
    "hm_mvm_batch": (_i32, [_vp, _i32, _dbl, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
    "hm_graph_create": (_i32, [_vp, _i32, _dbl, _vp, _i64, _vp, _i64, _vp, _sz, _P(_vp)]),
    "hm_graph_launch": (_i32, [_vp, _vp]),
    "hm_graph_destroy": (None, [_vp]),
    "hm_profile_begin": (_i32, [_vp, _i32]),
    "hm_profile_end": (_i32, [_vp, _P(_dbl), _P(_i64)]),
    "hm_matrix_set_launch": (_i32, [_vp, C.c_char_p]),
    "hm_matrix_get_launch": (_i32, [_vp, C.c_char_p, _sz]),
    "hm_matrix_tune_key": (_i32, [_vp, C.c_char_p, _sz]),
    "hm_stream_read": (_i32, [_vp, _sz, _vp, _vp]),
    "hm_permute": (_i32, [_vp, _i64, _i32, _i32, _i32, _vp, _i64, _vp, _i64, _vp]),
    "hm_server_create": (_i32, [_P(_vp), _i32, _vp, _sz, _P(_vp), _i32, _P(_vp)]),
    "hm_submit": (_i32, [_vp, _i32, _i32, _vp, _i64, _vp, _i64, _P(C.c_uint64)]),
    "hm_poll": (_i32, [_vp, C.c_uint64, _P(_i32), _P(_i32)]),
    "hm_wait": (_i32, [_vp, C.c_uint64, _i64, _P(_i32)]),
    "hm_server_stats": (_i32, [_vp, _P(_dbl), _P(_dbl), _P(_dbl)]),
    "hm_server_destroy": (None, [_vp]),
    "hm_last_error": (C.c_char_p, []),
    # include/hm_construct.h
    "hm_construct_layout": (_i32, [_vp, _i64, _P(_i64), _P(_i64)]),
    "hm_construct_rank_limit": (_i32, [_P(_i32)]),
    "hm_construct": (_i32, [_vp, _i64, _vp, _i64, _vp, _sz, _vp, _vp, _sz, _vp, _sz, _vp, _vp]),
    "hm_construct_pack": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    # include/hm_lu.h
    "hm_lu_create": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _P(_vp)]),
    "hm_lu_factor": (_i32, [_vp, C.c_double, _i32, _vp]),
    "hm_lu_solve": (_i32, [_vp, _vp, _i64, _i64, _vp]),
    "hm_lu_leaf": (_i32, [_vp, _i64, _P(_i32), _vp, _sz, _vp, _sz]),
    "hm_lu_stats_get": (_i32, [_vp, _vp]),
    "hm_lu_profile": (_i32, [_vp, _i32]),
    "hm_lu_destroy": (None, [_vp]),
}

_lib = None


def lib():
    """Load libhm.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run paper_2308_10960_amd.build.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, func: str):
    if st != HM_OK:
        raise HMError(st, func, lib().hm_last_error().decode())


def _ptr(v) -> int | None:
    """Device/host address of a torch tensor, numpy array, or int."""
    if v is None:
        return None
    if isinstance(v, int):
        return v
    if hasattr(v, "data_ptr"):
        return v.data_ptr()
    if isinstance(v, np.ndarray):
        return v.ctypes.data
    raise TypeError(type(v))


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ------------------------------------------------------------------ entry points

def make_blocks(rb, re, cb, ce, kind, rank, ngroups, group_cols, group_dtype, has_sigma):
    """hm_block_desc array from per-block arrays (no arithmetic)."""
    n = len(rb)
    d = np.zeros(n, BLOCK_DTYPE)
    d["row_begin"], d["row_end"], d["col_begin"], d["col_end"] = rb, re, cb, ce
    d["kind"], d["rank"], d["ngroups"] = kind, rank, ngroups
    d["group_cols"], d["group_dtype"] = group_cols, group_dtype
    d["has_sigma"] = has_sigma
    return d


def hm_build_plan(n_rows: int, n_cols: int, blocks: np.ndarray, acc_dtype: int = HM_F64,
                  max_nrhs: int = 1, tune_cache: str | None = None, chunk_rows: int = 0,
                  tile_groups: int = 0, tile_mix: int = 0) -> int:
    """chunk_rows, tile_groups, tile_mix: the column-tile shape (0: tune cache or built-in)."""
    blocks = np.ascontiguousarray(blocks, dtype=BLOCK_DTYPE)
    opts = PlanOpts(acc_dtype, acc_dtype, max_nrhs, 1 if tune_cache else 0,
                    tune_cache.encode() if tune_cache else None, chunk_rows, tile_groups, tile_mix)
    out = C.c_void_p()
    _check(lib().hm_build_plan(n_rows, n_cols, blocks.ctypes.data, blocks.shape[0],
                               C.byref(opts), C.byref(out)), "hm_build_plan")
    return out.value


def hm_plan_info(plan: int) -> dict:
    info = PlanInfo()
    _check(lib().hm_plan_info(plan, C.byref(info)), "hm_plan_info")
    return info.as_dict()


def hm_plan_destroy(plan: int) -> None:
    lib().hm_plan_destroy(plan)


def hm_plan_locate(plan: int, block: int, which: int, i: int, j: int, lo: bool = False):
    """(byte offset, dtype) of a stored factor entry; with lo=True also the
    offset of its low bytes (DFL40 / DFL48; 0 for the other formats)."""
    off, dt, lo_off = C.c_size_t(), C.c_int32(), C.c_size_t()
    _check(lib().hm_plan_locate(plan, block, which, i, j, C.byref(off), C.byref(dt), C.byref(lo_off)),
           "hm_plan_locate")
    return (off.value, dt.value, lo_off.value) if lo else (off.value, dt.value)


def hm_upload(plan: int, a_ptrs: np.ndarray, b_ptrs: np.ndarray, s_ptrs: np.ndarray | None,
              d_store, store_bytes: int, stream=None) -> int:
    a_ptrs = np.ascontiguousarray(a_ptrs, dtype=np.uint64)
    b_ptrs = np.ascontiguousarray(b_ptrs, dtype=np.uint64)
    sp = None if s_ptrs is None else np.ascontiguousarray(s_ptrs, dtype=np.uint64)
    out = C.c_void_p()
    _check(lib().hm_upload(plan, a_ptrs.ctypes.data, b_ptrs.ctypes.data,
                           None if sp is None else sp.ctypes.data, _ptr(d_store), store_bytes,
                           _stream(stream), C.byref(out)), "hm_upload")
    return out.value


def hm_pack_host(plan: int, a_ptrs: np.ndarray, b_ptrs: np.ndarray, s_ptrs, h_buf: np.ndarray):
    a_ptrs = np.ascontiguousarray(a_ptrs, dtype=np.uint64)
    b_ptrs = np.ascontiguousarray(b_ptrs, dtype=np.uint64)
    sp = None if s_ptrs is None else np.ascontiguousarray(s_ptrs, dtype=np.uint64)
    _check(lib().hm_pack_host(plan, a_ptrs.ctypes.data, b_ptrs.ctypes.data,
                              None if sp is None else sp.ctypes.data, h_buf.ctypes.data,
                              h_buf.nbytes), "hm_pack_host")


def hm_matrix_destroy(mat: int) -> None:
    lib().hm_matrix_destroy(mat)


def hm_mvm(mat: int, alpha: float, d_x, d_y, d_work, work_bytes: int, stream=None) -> None:
    _check(lib().hm_mvm(mat, alpha, _ptr(d_x), _ptr(d_y), _ptr(d_work), work_bytes,
                        _stream(stream)), "hm_mvm")


def hm_mvm_noalloc(mat: int, alpha: float, d_x, d_y, stream=None) -> None:
    """hm_mvm with the library's fixed device workspace (no allocation)."""
    _check(lib().hm_mvm_noalloc(mat, alpha, _ptr(d_x), _ptr(d_y), _stream(stream)), "hm_mvm_noalloc")


def hm_mvm_batch(mat: int, nrhs: int, alpha: float, d_X, ldx: int, d_Y, ldy: int, d_work,
                 work_bytes: int, stream=None) -> None:
    _check(lib().hm_mvm_batch(mat, nrhs, alpha, _ptr(d_X), ldx, _ptr(d_Y), ldy, _ptr(d_work),
                              work_bytes, _stream(stream)), "hm_mvm_batch")


def hm_graph_create(mat: int, nrhs: int, alpha: float, d_X, ldx: int, d_Y, ldy: int, d_work,
                    work_bytes: int) -> int:
    g = C.c_void_p()
    _check(lib().hm_graph_create(mat, nrhs, alpha, _ptr(d_X), ldx, _ptr(d_Y), ldy, _ptr(d_work),
                                 work_bytes, C.byref(g)), "hm_graph_create")
    return g.value


def hm_graph_launch(graph: int, stream=None) -> None:
    _check(lib().hm_graph_launch(graph, _stream(stream)), "hm_graph_launch")


def hm_graph_destroy(graph: int) -> None:
    lib().hm_graph_destroy(graph)


def hm_profile_begin(mat: int, max_calls: int) -> None:
    _check(lib().hm_profile_begin(mat, max_calls), "hm_profile_begin")


def hm_profile_end(mat: int):
    """Returns ([ms_col, ms_reduce, ms_row] summed over calls, calls)."""
    ms = (C.c_double * 3)()
    calls = C.c_int64()
    _check(lib().hm_profile_end(mat, ms, C.byref(calls)), "hm_profile_end")
    return list(ms), calls.value


def hm_matrix_set_launch(mat: int, params: str) -> None:
    _check(lib().hm_matrix_set_launch(mat, params.encode()), "hm_matrix_set_launch")


def hm_matrix_get_launch(mat: int) -> str:
    buf = C.create_string_buffer(128)
    _check(lib().hm_matrix_get_launch(mat, buf, 128), "hm_matrix_get_launch")
    return buf.value.decode()


def hm_matrix_tune_key(mat: int) -> str:
    buf = C.create_string_buffer(128)
    _check(lib().hm_matrix_tune_key(mat, buf, 128), "hm_matrix_tune_key")
    return buf.value.decode()


def hm_permute(d_perm, n: int, dtype: int, direction: int, nvec: int, d_in, ld_in: int, d_out, ld_out: int,
               stream=None) -> None:
    _check(lib().hm_permute(_ptr(d_perm), n, dtype, direction, nvec, _ptr(d_in), ld_in, _ptr(d_out), ld_out,
                            _stream(stream)), "hm_permute")


def hm_stream_read(d_buf, nbytes: int, d_out, stream=None) -> None:
    _check(lib().hm_stream_read(_ptr(d_buf), nbytes, _ptr(d_out), _stream(stream)),
           "hm_stream_read")


def hm_server_create(mats, d_arena, arena_bytes: int, streams) -> int:
    m = (C.c_void_p * len(mats))(*mats)
    s = (C.c_void_p * len(streams))(*[_stream(x) for x in streams])
    out = C.c_void_p()
    _check(lib().hm_server_create(m, len(mats), _ptr(d_arena), arena_bytes, s, len(streams),
                                  C.byref(out)), "hm_server_create")
    return out.value


def hm_submit(server: int, mat: int, nrhs: int, h_X, ldx: int, h_Y, ldy: int) -> int:
    t = C.c_uint64()
    _check(lib().hm_submit(server, mat, nrhs, _ptr(h_X), ldx, _ptr(h_Y), ldy, C.byref(t)),
           "hm_submit")
    return t.value


def hm_poll(server: int, ticket: int):
    done, res = C.c_int32(), C.c_int32()
    _check(lib().hm_poll(server, ticket, C.byref(done), C.byref(res)), "hm_poll")
    return bool(done.value), res.value


def hm_wait(server: int, ticket: int, timeout_us: int) -> int:
    """Returns the request's status; raises HMError(HM_ETIMEOUT) on timeout."""
    res = C.c_int32()
    _check(lib().hm_wait(server, ticket, timeout_us, C.byref(res)), "hm_wait")
    return res.value


def hm_server_stats(server: int):
    p50, p99, mps = C.c_double(), C.c_double(), C.c_double()
    _check(lib().hm_server_stats(server, C.byref(p50), C.byref(p99), C.byref(mps)),
           "hm_server_stats")
    return p50.value, p99.value, mps.value


def hm_server_destroy(server: int) -> None:
    lib().hm_server_destroy(server)


# ------------------------------------------------------------ construction

HM_KERNEL_LAPLACE, HM_KERNEL_EXP = 0, 1
HM_CONSTRUCT_MAX_RANK = 128

# hm_cblock as a numpy structured dtype (same layout as the C struct).
CBLOCK_DTYPE = np.dtype([("rb", "<i8"), ("cb", "<i8"), ("m", "<i4"), ("n", "<i4"), ("adm", "<i4"),
                         ("cap", "<i4"), ("out", "<i8"), ("scr", "<i8")], align=True)


class ConstructOpts(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("keep_sigma", C.c_int32), ("params", C.c_double * 2),
                ("eps_aca", C.c_double), ("eps", C.c_double)]


def hm_construct_layout(blocks: np.ndarray):
    """Sets cap (where 0), out and scr in place; returns (out doubles, scratch doubles)."""
    assert blocks.dtype == CBLOCK_DTYPE and blocks.flags.c_contiguous
    o, sc = C.c_int64(), C.c_int64()
    _check(lib().hm_construct_layout(blocks.ctypes.data, blocks.shape[0], C.byref(o), C.byref(sc)),
           "hm_construct_layout")
    return o.value, sc.value


def hm_construct_rank_limit() -> int:
    r = C.c_int32()
    _check(lib().hm_construct_rank_limit(C.byref(r)), "hm_construct_rank_limit")
    return r.value


def hm_construct(d_points, n_points: int, blocks: np.ndarray, d_desc, desc_bytes: int, kernel: int, params,
                 eps_aca: float, eps: float, keep_sigma: bool, d_out, out_bytes: int, d_scr, scr_bytes: int,
                 d_rank, stream=None) -> None:
    assert blocks.dtype == CBLOCK_DTYPE and blocks.flags.c_contiguous
    p = (C.c_double * 2)(*[float(v) for v in params[:2]])
    opts = ConstructOpts(kernel, int(keep_sigma), p, eps_aca, eps)
    _check(lib().hm_construct(_ptr(d_points), n_points, blocks.ctypes.data, blocks.shape[0], _ptr(d_desc),
                              desc_bytes, C.byref(opts), _ptr(d_out), out_bytes, _ptr(d_scr), scr_bytes,
                              _ptr(d_rank), _stream(stream)), "hm_construct")


# ------------------------------------------------------------ H-LU

HM_LU_MAX_RANK, HM_LU_MAX_LEAF = 256, 64


class LuTree(C.Structure):
    _fields_ = [("n_clusters", C.c_int64), ("begin", C.c_void_p), ("end", C.c_void_p),
                ("son0", C.c_void_p), ("son1", C.c_void_p)]


class LuStats(C.Structure):
    _fields_ = [("kernels", C.c_int64), ("truncations", C.c_int64), ("max_rank", C.c_int32),
                ("reserved", C.c_int32), ("factor_doubles", C.c_double), ("stored_bytes", C.c_double),
                ("arena_peak", C.c_size_t), ("trunc_ms", C.c_double), ("trunc_flops", C.c_double),
                ("timed_truncations", C.c_int64)]


def hm_lu_create(begin, end, son0, son1, tau, sigma, kind, rank, a_ptrs, b_ptrs, arena_bytes: int) -> int:
    """Host arrays (numpy); a_ptrs / b_ptrs: uint64 host addresses of each leaf's factors."""
    arrs = [np.ascontiguousarray(begin, np.int64), np.ascontiguousarray(end, np.int64),
            np.ascontiguousarray(son0, np.int32), np.ascontiguousarray(son1, np.int32)]
    tree = LuTree(arrs[0].shape[0], *[a.ctypes.data for a in arrs])
    leaf = [np.ascontiguousarray(v, np.int32) for v in (tau, sigma, kind, rank)]
    ap = np.ascontiguousarray(a_ptrs, np.uint64)
    bp = np.ascontiguousarray(b_ptrs, np.uint64)
    out = C.c_void_p()
    _check(lib().hm_lu_create(C.byref(tree), leaf[0].shape[0], *[v.ctypes.data for v in leaf], ap.ctypes.data,
                              bp.ctypes.data, arena_bytes, C.byref(out)), "hm_lu_create")
    return out.value


def hm_lu_factor(F: int, eps: float, dtype: int = HM_F64, stream=None) -> None:
    _check(lib().hm_lu_factor(F, eps, dtype, _stream(stream)), "hm_lu_factor")


def hm_lu_solve(F: int, d_x, ld: int, nrhs: int, stream=None) -> None:
    _check(lib().hm_lu_solve(F, _ptr(d_x), ld, nrhs, _stream(stream)), "hm_lu_solve")


def hm_lu_leaf(F: int, i: int, m: int, n: int, dense: bool):
    """Leaf i of the factors: the dense block, or (U, V) of the low-rank one."""
    k = C.c_int32()
    if dense:
        a = np.empty(m * n)
        _check(lib().hm_lu_leaf(F, i, C.byref(k), a.ctypes.data, a.size, None, 0), "hm_lu_leaf")
        return a.reshape(n, m).T
    st = lib().hm_lu_leaf(F, i, C.byref(k), None, 0, None, 0)
    if st not in (HM_OK, HM_ENOMEM):
        _check(st, "hm_lu_leaf")
    r = k.value
    a, b = np.empty(max(m * r, 1)), np.empty(max(n * r, 1))
    _check(lib().hm_lu_leaf(F, i, C.byref(k), a.ctypes.data, a.size, b.ctypes.data, b.size), "hm_lu_leaf")
    return a[:m * r].reshape(r, m).T, b[:n * r].reshape(r, n).T


def hm_lu_stats_get(F: int) -> dict:
    st = LuStats()
    _check(lib().hm_lu_stats_get(F, C.byref(st)), "hm_lu_stats_get")
    return {k: getattr(st, k) for k, _ in LuStats._fields_ if k != "reserved"}


def hm_lu_profile(F: int, on: bool) -> None:
    _check(lib().hm_lu_profile(F, int(on)), "hm_lu_profile")


def hm_lu_destroy(F: int) -> None:
    lib().hm_lu_destroy(F)


def hm_last_error() -> str:
    return lib().hm_last_error().decode()
