"""Named workloads (synthetic stand-ins for the paper's model problems, Sec. 5.1).

sphere-laplace: Fibonacci-lattice points on the unit sphere, kernel
  1/(4 pi |x-y|) with diagonal 1/(4 pi h), h = mean nearest-neighbour distance
  (stand-in for the Laplace single-layer BEM matrix).
cube-exp: uniform random points in the unit cube (seed 0), kernel
  exp(-|x-y|/0.1) with 1e-3 added on the diagonal; this is the Matern
  covariance of Sec. 5.1 at nu = 1/2, length 0.1 (stand-in for the paper's
  nu = 1/3 problem).
All use a binary geometric-bisection cluster tree with leaf size 64 and
standard admissibility with eta = 2.
"""

from __future__ import annotations

import time

from .geometry import fibonacci_sphere, cube_points
from .hmatrix import build_hmatrix, dfl_format, bfl_format, KERNEL_LAPLACE, KERNEL_EXP, DT_F64, DT_F32

PRESETS = {
    # small parity case
    "sphere4k": dict(geometry="sphere", n=4096, kernel="laplace", eps=1e-6, dtype="f64"),
    # throughput point: n = 2^18, eps = 1e-6, plain FP64
    "sphere256k": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-6, dtype="f64"),
    # high-accuracy FP64 point: n = 2^18, eps = 1e-8
    "sphere256k_e8": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-8, dtype="f64"),
    # mixed-precision storage, FP32 accumulation
    "sphere256k_mixed": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-6, dtype="mixed"),
    # batched multi-RHS: n = 2^20 cube, FP32 factors, 32 right-hand sides
    "cube1m": dict(geometry="cube", n=1048576, kernel="exp", eps=1e-6, dtype="f32", nrhs=32),
    # mixed-precision storage at eps = 1e-8 with FP64 accumulation: dense
    # (near-field) blocks and y in FP64, low-rank column groups in
    # FP32 / FP16 / BF16 within the stated 1e-6 result tolerance, s in FP64
    "sphere256k_e8_mixed": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-8, dtype="mixed64"),
    "sphere4k_e8_mixed": dict(geometry="sphere", n=4096, kernel="laplace", eps=1e-8, dtype="mixed64"),
    # small mixed case for parity
    "sphere4k_mixed": dict(geometry="sphere", n=4096, kernel="laplace", eps=1e-6, dtype="mixed"),
    "cube4k": dict(geometry="cube", n=4096, kernel="exp", eps=1e-6, dtype="f32"),
    # byte-aligned truncated FP64 storage (DFL, Sec. 3.2), FP64 accumulation:
    # eps = 1e-6 -> DFL32, eps = 1e-8 -> DFL40
    "sphere256k_dfl": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-6, dtype="dfl"),
    "sphere256k_e8_dfl": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-8, dtype="dfl"),
    "sphere4k_dfl": dict(geometry="sphere", n=4096, kernel="laplace", eps=1e-6, dtype="dfl"),
    # adaptive per-column precision over the DFL formats (APLR, Sec. 3.3),
    # FP64 accumulation, every block within eps / 2 of its own norm
    "sphere256k_aplr": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-6, dtype="aplr"),
    "sphere256k_e8_aplr": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-8, dtype="aplr"),
    "sphere4k_aplr": dict(geometry="sphere", n=4096, kernel="laplace", eps=1e-8, dtype="aplr"),
    # adaptive-exponent byte-aligned storage (AFLP, Sec. 3.2) per block,
    # FP64 accumulation: the fewest bytes keeping m_eps mantissa bits
    "sphere256k_aflp": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-6, dtype="aflp"),
    "sphere256k_e8_aflp": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-8, dtype="aflp"),
    "sphere4k_aflp": dict(geometry="sphere", n=4096, kernel="laplace", eps=1e-6, dtype="aflp"),
    # FP32's exponent with the mantissa filling whole bytes (BFL, Sec. 3.2),
    # FP64 accumulation: eps = 1e-8 -> BFL40 (eps = 1e-6 gives FP32 itself)
    "sphere256k_e8_bfl": dict(geometry="sphere", n=262144, kernel="laplace", eps=1e-8, dtype="bfl"),
    "sphere4k_bfl": dict(geometry="sphere", n=4096, kernel="laplace", eps=1e-8, dtype="bfl"),
}

SEED_POINTS, SEED_X, SEED_RHS, SEED_REQUESTS = 0, 1, 2, 3
MIXED_TOL = 1e-6


def preset(name: str) -> dict:
    return dict(PRESETS[name])


def make_points(geometry: str, n: int):
    if geometry == "sphere":
        return fibonacci_sphere(n)
    if geometry == "cube":
        return cube_points(n, SEED_POINTS)
    raise ValueError(geometry)


def build_preset(name: str, *, n: int | None = None, eps: float | None = None,
                 dtype: str | None = None, nthreads: int | None = None, leaf: int = 64,
                 eta: float = 2.0, filler=None):
    """Build a preset's H-matrix; n / eps / dtype override the preset.
    ``filler``: a callable that fills the leaves of the tree-only H-matrix
    (e.g. on the GPU) instead of the host construction."""
    p = preset(name)
    n = p["n"] if n is None else n
    eps = p["eps"] if eps is None else eps
    dtype = p["dtype"] if dtype is None else dtype
    pts = make_points(p["geometry"], n)
    kern = KERNEL_LAPLACE if p["kernel"] == "laplace" else KERNEL_EXP
    mixed = dtype in ("mixed", "mixed64")
    t0 = time.perf_counter()
    H = build_hmatrix(pts, kern, leaf=leaf, eta=eta, eps=eps, keep_sigma=mixed or dtype == "aplr",
                      nthreads=nthreads, fill=filler is None)
    if filler is not None:
        H.fill_stats = filler(H)
        H.build_seconds = time.perf_counter() - t0
    bad = 0
    if dtype == "mixed":
        bad = H.select_precision(MIXED_TOL / 2)
    elif dtype == "mixed64":
        bad = H.select_precision(MIXED_TOL / 2, dense_f64=True, sigma_f64=True)
    elif dtype == "aplr":
        bad = H.select_precision_dfl(eps / 2)
    elif dtype == "dfl":
        H.set_uniform_dtype(dfl_format(eps))
    elif dtype == "aflp":
        H.select_aflp(eps)
    elif dtype == "bfl":
        H.set_uniform_dtype(bfl_format(eps))
    else:
        H.set_uniform_dtype(DT_F64 if dtype == "f64" else DT_F32)
    if bad:
        raise RuntimeError(f"{name} (n={n}, eps={eps}, {dtype}): {bad} blocks cannot be stored "
                           "within their share of the error budget")
    H.dtype_mode = dtype
    H.preset = name
    return H
