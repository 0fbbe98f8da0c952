"""Oracle: plain FP64 H-matrix-vector product plus decoding of stored formats.

TEST INFRASTRUCTURE ONLY.  The product definition follows Sec. 2.1
(Definitions "Block Tree", "H-Matrix") and Eq. (1); see hm_oracle.c.

Format rounding (for the mixed-precision "decoded" oracle) follows the
IEEE-754 binary formats of Table 1 with round-to-nearest-even applied once,
directly from FP64:
  FP32 and FP16 use numpy's own conversions (correctly rounded from double);
  BF16 (1-8-7, Table 1) is rounded here from its definition;
  DFL (Sec. 3.2: FP64's sign and 11 exponent bits, the mantissa cut to make
  a whole number of bytes) is rounded here from its definition;
  AFLP (Sec. 3.2: per data block, values scaled and shifted by 1, only the
  exponent bits the block's range needs, the mantissa filling the bytes)
  is rounded here from its definition, one data block per call;
  BFL (Sec. 3.2: FP32's sign and 8 exponent bits, the mantissa filling
  whole bytes) is rounded here from its definition.
Parity pins for every function live in tests/test_oracle_*.py.
"""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
# all-cores timing variant (bitwise equal to the plain loop; see hm_oracle_omp.c)
_SRC_OMP = os.path.join(_HERE, "hm_oracle_omp.c")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lib_omp = None

F64, F32, F16, BF16 = 0, 1, 2, 3
DFL32, DFL40, DFL48, DFL16, DFL24 = 4, 5, 6, 7, 8
DFL_BYTES = {DFL32: 4, DFL40: 5, DFL48: 6, DFL16: 2, DFL24: 3}
AFLP16, AFLP24, AFLP32, AFLP40, AFLP48 = 9, 10, 11, 12, 13
AFLP_BYTES = {AFLP16: 2, AFLP24: 3, AFLP32: 4, AFLP40: 5, AFLP48: 6}
BFL24, BFL40, BFL48 = 14, 15, 16
BFL_BYTES = {BFL24: 3, BFL40: 5, BFL48: 6}

# Table 1: unit roundoff u = 2^-(m+1) for m explicit mantissa bits.
UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "tf32": 2.0 ** -11,
                 "bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp8": 2.0 ** -4}

# (exponent bits, explicit mantissa bits) per format, Table 1.
FORMAT_BITS = {"fp64": (11, 52), "fp32": (8, 23), "tf32": (8, 10), "bf16": (8, 7),
               "fp16": (5, 10), "fp8": (4, 3)}


def _limits(e: int, m: int):
    bias = 2 ** (e - 1) - 1
    emax = bias
    emin = 1 - bias
    fmax = (2.0 - 2.0 ** -m) * 2.0 ** emax
    tiny = 2.0 ** (emin - m)          # smallest subnormal
    return fmax, tiny


FORMAT_LIMITS = {k: _limits(*v) for k, v in FORMAT_BITS.items()}


def dynamic_range(fmt: str) -> float:
    """log10(largest finite / smallest positive subnormal) (Table 2)."""
    fmax, tiny = FORMAT_LIMITS[fmt]
    return math.log10(fmax) - math.log10(tiny)


# ------------------------------------------------------------------ rounding

def round_f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_f16(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def round_bf16(x) -> np.ndarray:
    """RNE of FP64 values to BF16 (8 exponent bits, 7 explicit mantissa bits).

    Written from the format definition: the kept significand has 8 bits, the
    smallest normal exponent is -126, subnormals are spaced 2^-133, values
    that round beyond the largest finite value become infinite.
    """
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    fin = np.isfinite(x) & (x != 0)
    xf = x[fin]
    _, e = np.frexp(xf)                          # |x| = f 2^e, f in [0.5, 1)
    lsb = np.maximum(e - 1, -126) - 7            # exponent of the last kept bit
    q = np.rint(np.ldexp(xf, -lsb))              # rint: ties to even
    r = np.ldexp(q, lsb)
    fmax = FORMAT_LIMITS["bf16"][0]
    r = np.where(np.abs(r) > fmax, np.copysign(np.inf, xf), r)
    out[fin] = r
    return out


def round_dfl(x, nbytes: int) -> np.ndarray:
    """RNE of FP64 values to the DFL format of nbytes bytes (Sec. 3.2).

    Written from the format definition: sign and the 11 exponent bits of
    FP64, m = 8 nbytes - 12 explicit mantissa bits, so the kept significand
    has m + 1 bits, the smallest normal exponent is -1022 as in FP64 and
    subnormals are spaced 2^(-1022 - m); values that round beyond FP64's
    largest finite exponent become infinite.  nbytes = 8 is FP64 itself.
    """
    m = 8 * nbytes - 12
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    fin = np.isfinite(x) & (x != 0)
    xf = x[fin]
    _, e = np.frexp(xf)                          # |x| = f 2^e, f in [0.5, 1)
    lsb = np.maximum(e - 1, -1022) - m           # exponent of the last kept bit
    q = np.rint(np.ldexp(xf, -lsb))              # rint: ties to even
    with np.errstate(over="ignore"):
        r = np.ldexp(q, lsb)                     # inf beyond the largest finite value
    out[fin] = r
    return out


def round_bfl(x, nbytes: int) -> np.ndarray:
    """RNE of FP64 values to the BFL format of nbytes bytes (Sec. 3.2).

    Written from the format definition: sign, FP32's 8 exponent bits (bias
    127) and m = 8 nbytes - 9 explicit mantissa bits; 2 and 4 bytes are
    BF16 and FP32.  Reading: magnitudes that round below the smallest normal
    value 2^-126 become zero (no subnormals), and values that round beyond
    the largest finite value raise ValueError (no infinities).
    """
    m = 8 * nbytes - 9
    x = np.asarray(x, dtype=np.float64)
    if not np.all(np.isfinite(x)):
        raise ValueError("BFL: values must be finite")
    out = np.zeros_like(x)
    nz = x != 0
    xf = x[nz]
    _, e = np.frexp(xf)                          # |x| = f 2^e, f in [0.5, 1)
    lsb = e - 1 - m                              # exponent of the last kept bit
    r = np.ldexp(np.rint(np.ldexp(xf, -lsb)), lsb)
    if np.any(np.abs(r) >= 2.0 ** 128):
        raise ValueError("BFL: value beyond the largest finite value")
    out[nz] = np.where(np.abs(r) < 2.0 ** -126, 0.0, r)
    return out


def _rne_bits(d: np.ndarray, m: int) -> np.ndarray:
    """RNE of positive normal FP64 values to m explicit mantissa bits."""
    _, e = np.frexp(d)                           # d = f 2^e, f in [0.5, 1)
    lsb = e - 1 - m
    return np.ldexp(np.rint(np.ldexp(d, -lsb)), lsb)


def aflp_params(x, nbytes: int):
    """(k, e, m) of one AFLP data block of nbytes-byte values (Sec. 3.2).

    The block's nonzero magnitudes are scaled by 2^-k (2^k the power of two
    at or below the smallest of them) and shifted by 1, so they lie in
    [2, 2R + 1) with R = largest / smallest.  The exponent field holds the
    binary exponent j >= 1 of such a value; j = 0, the binade [1, 2), is
    the code of zero.  e is the fewest bits whose 2^e exponents hold every
    rounded value of the block, and m = 8 nbytes - 1 - e explicit mantissa
    bits fill the bytes.  A block without nonzeros gives
    (0, 0, 8 nbytes - 1).  Raises ValueError for values that are not finite
    or a range that needs more than 10 exponent bits.
    """
    x = np.asarray(x, dtype=np.float64)
    if not np.all(np.isfinite(x)):
        raise ValueError("AFLP: values must be finite")
    a = np.abs(x[x != 0])
    if a.size == 0:
        return 0, 0, 8 * nbytes - 1
    k = int(np.frexp(a.min())[1]) - 1            # 2^k <= min < 2^(k+1)
    with np.errstate(over="ignore"):
        dmax = np.ldexp(a.max(), -k) + 1.0
    if not np.isfinite(dmax):
        raise ValueError("AFLP: dynamic range too large")
    top = int(np.frexp(dmax)[1]) - 1             # exponent of the largest shifted value (>= 1)
    e = top.bit_length()                         # buckets 0 .. top need e bits
    while True:
        m = 8 * nbytes - 1 - e
        if e > 10 or m < 1:
            raise ValueError(f"AFLP: a range of 2^{top} does not fit {nbytes} bytes")
        top_r = int(np.frexp(_rne_bits(np.array([dmax]), m)[0])[1]) - 1
        if top_r < 2 ** e:                       # rounding up may open the next bucket
            return k, e, m
        e += 1


def round_aflp(x, nbytes: int) -> np.ndarray:
    """AFLP rounding of one data block x (any shape) to nbytes-byte values
    (Sec. 3.2): d = |v| 2^-k + 1 rounded to nearest even with m explicit
    mantissa bits (k, m from aflp_params), stored value sign(v) (d - 1) 2^k;
    zeros stay zero."""
    x = np.asarray(x, dtype=np.float64)
    k, e, m = aflp_params(x, nbytes)
    out = np.zeros_like(x)
    nz = x != 0
    d = np.ldexp(np.abs(x[nz]), -k) + 1.0
    out[nz] = np.copysign(np.ldexp(_rne_bits(d, m) - 1.0, k), x[nz])
    return out


def round_to(x, dt: int) -> np.ndarray:
    """x rounded to storage format dt (for AFLP, x is one data block)."""
    if dt == F64:
        return np.asarray(x, dtype=np.float64)
    if dt in DFL_BYTES:
        return round_dfl(x, DFL_BYTES[dt])
    if dt in AFLP_BYTES:
        return round_aflp(x, AFLP_BYTES[dt])
    if dt in BFL_BYTES:
        return round_bfl(x, BFL_BYTES[dt])
    if dt == F32:
        return round_f32(x)
    if dt == F16:
        return round_f16(x)
    if dt == BF16:
        return round_bf16(x)
    raise ValueError(dt)


# ------------------------------------------------------------------ C oracle

def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC]
    cmd_omp = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-fopenmp", "-o", _LIB_OMP + ".tmp",
               _SRC_OMP]
    for c, out in ((cmd, _LIB), (cmd_omp, _LIB_OMP)):
        if verbose:
            print(" ".join(c), flush=True)
        subprocess.run(c, check=True)
        os.replace(out + ".tmp", out)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.oracle_hmvm.argtypes = [C.c_int64, C.c_int64, C.c_int64, i64p, i64p, i64p, i64p,
                                  i32p, i32p, u64p, u64p, u64p, C.c_double, f64p, f64p]
        L.oracle_hmvm.restype = C.c_int
        L.oracle_hmvm_multi.argtypes = [C.c_int64, C.c_int64, C.c_int64, i64p, i64p, i64p,
                                        i64p, i32p, i32p, u64p, u64p, u64p, C.c_double,
                                        C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.c_int64]
        L.oracle_hmvm_multi.restype = C.c_int
        _lib = L
    return _lib


def blocks_in_rows(H, rows) -> np.ndarray:
    """Indices (ascending) of the leaves whose row cluster contains one of
    ``rows``: by the definition of the H-matrix (a sum over the leaves of
    the block partition, Sec. 2.1), y at those rows is the sum over these
    leaves alone."""
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    first = np.searchsorted(rows, np.asarray(H.rb, dtype=np.int64), side="left")
    return np.nonzero((first < rows.shape[0]) &
                      (rows[np.minimum(first, rows.shape[0] - 1)] < np.asarray(H.re)))[0]


def _table(H, factors=None, blocks=None):
    """Block table for the C routines; ``blocks`` restricts it to those
    leaf indices (then ``factors``, if given, lists only those leaves)."""
    i64 = lambda v: np.ascontiguousarray(v, dtype=np.int64)
    i32 = lambda v: np.ascontiguousarray(v, dtype=np.int32)
    sel = slice(None) if blocks is None else np.asarray(blocks, dtype=np.int64)
    adm = np.asarray(H.adm)[sel]
    kind = i32(adm != 0)
    rank = i32(np.where(adm != 0, np.asarray(H.rank)[sel], 0))
    rb, re, cb, ce = (i64(np.asarray(v)[sel]) for v in (H.rb, H.re, H.cb, H.ce))
    if factors is None:
        ap, bp, sp = (np.ascontiguousarray(np.asarray(p)[sel], dtype=np.uint64)
                      for p in (H.a_ptr, H.b_ptr, H.s_ptr))
        keep = None
    else:
        keep = factors
        ap = np.array([f[0].ctypes.data if f[0] is not None and f[0].size else 0 for f in factors], np.uint64)
        bp = np.array([f[1].ctypes.data if f[1] is not None and f[1].size else 0 for f in factors], np.uint64)
        sp = np.array([f[2].ctypes.data if f[2] is not None and f[2].size else 0 for f in factors], np.uint64)
    return (rb, re, cb, ce, kind, rank, ap, bp, sp, keep)


def hmvm(H, x, y=None, alpha: float = 1.0, factors=None, n_rows=None, n_cols=None,
         blocks=None) -> np.ndarray:
    """y + alpha * A_H x in FP64 (returns a new array; y defaults to zero).

    ``H`` is any object with block-table arrays rb, re, cb, ce, adm, rank and
    per-block factor pointers a_ptr, b_ptr, s_ptr (FP64, column-major); or
    ``factors`` gives per-block (a, b, s) FP64 arrays (Fortran order) instead.
    ``blocks`` (e.g. from blocks_in_rows) sums over those leaves only: exact
    at the rows they cover, partial elsewhere.
    """
    L = _load()
    n_rows = H.n if n_rows is None else n_rows
    n_cols = H.n if n_cols is None else n_cols
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(n_rows) if y is None else np.array(y, dtype=np.float64, copy=True)
    rb, re, cb, ce, kind, rank, ap, bp, sp, keep = _table(H, factors, blocks)
    rc = L.oracle_hmvm(n_rows, n_cols, rb.shape[0], rb, re, cb, ce, kind, rank, ap, bp, sp,
                       float(alpha), x, out)
    if rc != 0:
        raise RuntimeError(f"oracle_hmvm failed ({rc})")
    del keep
    return out


def _load_omp():
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP):
            build()
        L = C.CDLL(_LIB_OMP)
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.oracle_hmvm_omp.argtypes = [C.c_int64, C.c_int64, C.c_int64, i64p, i64p, i64p, i64p,
                                      i32p, i32p, u64p, u64p, u64p, C.c_double, f64p, f64p,
                                      C.c_int32, C.c_int64]
        L.oracle_hmvm_omp.restype = C.c_int
        _lib_omp = L
    return _lib_omp


def hmvm_omp(H, x, y=None, alpha: float = 1.0, factors=None, nthreads: int = 0,
             rows_per_task: int = 64):
    """hmvm on all cores (OpenMP over ranges of rows, t_b per block first):
    bitwise the result of hmvm for any thread count.  A timing variant, not
    a second oracle.  Returns (y, threads used)."""
    L = _load_omp()
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(H.n) if y is None else np.array(y, dtype=np.float64, copy=True)
    rb, re, cb, ce, kind, rank, ap, bp, sp, keep = _table(H, factors)
    used = L.oracle_hmvm_omp(H.n, H.n, rb.shape[0], rb, re, cb, ce, kind, rank, ap, bp, sp,
                             float(alpha), x, out, int(nthreads), int(rows_per_task))
    if used < 1:
        raise RuntimeError(f"oracle_hmvm_omp failed ({used})")
    del keep
    return out, int(used)


def hmvm_multi(H, X, Y=None, alpha: float = 1.0, factors=None, blocks=None) -> np.ndarray:
    """Column-by-column product for X (n x r, any layout); ``blocks`` as in
    hmvm."""
    L = _load()
    X = np.asfortranarray(X, dtype=np.float64)
    n, r = X.shape
    out = np.zeros((H.n, r), order="F") if Y is None else np.array(Y, dtype=np.float64, order="F", copy=True)
    rb, re, cb, ce, kind, rank, ap, bp, sp, keep = _table(H, factors, blocks)
    rc = L.oracle_hmvm_multi(H.n, n, rb.shape[0], rb, re, cb, ce, kind, rank, ap, bp, sp,
                             float(alpha), r, X.ctypes.data, n, out.ctypes.data, H.n)
    if rc != 0:
        raise RuntimeError(f"oracle_hmvm_multi failed ({rc})")
    del keep
    return out


def _fview(ptr: int, rows: int, cols: int) -> np.ndarray:
    if ptr == 0 or rows * cols == 0:
        return np.zeros((rows, cols), order="F")
    buf = (C.c_double * (rows * cols)).from_address(int(ptr))
    return np.ctypeslib.as_array(buf).reshape(cols, rows).T


def decoded_factors(H, sigma_dtype: int = F32, blocks=None):
    """Per-block FP64 copies of the factors after rounding to their storage
    formats (groups of columns per Sec. 3.3; one format per dense block).
    Singular values are rounded to ``sigma_dtype``.  Returns a list of
    (a, b, s) Fortran-ordered FP64 arrays usable as ``factors=`` (for the
    leaves ``blocks`` only, if given, in that order)."""
    out = []
    for i in (range(H.rb.shape[0]) if blocks is None else blocks):
        m = int(H.re[i] - H.rb[i])
        nb = int(H.ce[i] - H.cb[i])
        dts = H.group_dtype[i]
        if not H.adm[i]:
            D = _fview(H.a_ptr[i], m, nb)
            out.append((np.asfortranarray(round_to(D, int(dts[0]))), None, None))
            continue
        k = int(H.rank[i])
        W = _fview(H.a_ptr[i], m, k)
        X = _fview(H.b_ptr[i], nb, k)
        Wd = np.empty((m, k), order="F")
        Xd = np.empty((nb, k), order="F")
        c0 = 0
        for g in range(int(H.ngroups[i])):
            kc = int(H.group_cols[i][g])
            dt = int(dts[g])
            Wd[:, c0:c0 + kc] = round_to(W[:, c0:c0 + kc], dt)
            Xd[:, c0:c0 + kc] = round_to(X[:, c0:c0 + kc], dt)
            c0 += kc
        s = None
        if H.keep_sigma and k:
            s = np.ascontiguousarray(round_to(_fview(H.s_ptr[i], k, 1)[:, 0], sigma_dtype))
        out.append((Wd, Xd, s))
    return out
