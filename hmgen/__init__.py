"""Seeded synthetic H-matrix construction (input generator).

Builds the operand of the H-matrix-vector product from a point cloud and a
kernel function: cluster tree and block tree (Sec. 2.1, Definitions "Cluster
Tree", "Block Tree", "H-Matrix"), dense near-field leaves, and low-rank
far-field leaves by ACA followed by the QR+SVD truncation of Algorithm 1
(Sec. 2.2) at the fixed accuracy of Eq. (1).  It also chooses per-block
storage formats for the mixed-precision form (Sec. 3.3).

This package holds none of the matrix-vector product arithmetic.  It feeds
both the GPU library (through its C-ABI) and the CPU oracle, which do not
share code with each other.
"""

from .geometry import fibonacci_sphere, cube_points, mean_nn_distance
from .hmatrix import (HMatrix, build_hmatrix, DT_F64, DT_F32, DT_F16, DT_BF16, DT_DFL32, DT_DFL40,
                      DT_DFL48, dfl_mantissa_bits, dfl_format, bfl_format)
from .presets import PRESETS, preset, build_preset
from .vectors import uniform_vector, gaussian_block

__all__ = [
    "fibonacci_sphere", "cube_points", "mean_nn_distance",
    "HMatrix", "build_hmatrix", "DT_F64", "DT_F32", "DT_F16", "DT_BF16", "DT_DFL32", "DT_DFL40",
    "DT_DFL48", "dfl_mantissa_bits", "dfl_format", "bfl_format",
    "PRESETS", "preset", "build_preset", "uniform_vector", "gaussian_block",
]
