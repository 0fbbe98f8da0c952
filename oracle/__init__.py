"""CPU oracle for the H-matrix-vector product (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this package.  It shares no code with the GPU library
and never calls it.
"""

from .oracle import (build, hmvm, hmvm_omp, hmvm_multi, blocks_in_rows, decoded_factors, round_f32, round_f16, F64, F32, F16, BF16,
                     round_bf16, round_to, UNIT_ROUNDOFF, FORMAT_LIMITS, dynamic_range, DFL32, DFL40, DFL48,
                     DFL16, DFL24, DFL_BYTES, round_dfl, AFLP16, AFLP24, AFLP32, AFLP40,
                     AFLP48, AFLP_BYTES, aflp_params, round_aflp, BFL24, BFL40, BFL48, BFL_BYTES,
                     round_bfl)

__all__ = ["F64", "F32", "F16", "BF16", "build", "hmvm", "hmvm_omp", "hmvm_multi", "blocks_in_rows", "decoded_factors", "round_f32", "round_f16",
           "round_bf16", "round_to", "UNIT_ROUNDOFF", "FORMAT_LIMITS", "dynamic_range", "DFL32", "DFL40", "DFL48",
           "DFL16", "DFL24", "DFL_BYTES", "round_dfl", "AFLP16", "AFLP24", "AFLP32", "AFLP40",
           "AFLP48", "AFLP_BYTES", "aflp_params", "round_aflp", "BFL24", "BFL40", "BFL48",
           "BFL_BYTES", "round_bfl"]
