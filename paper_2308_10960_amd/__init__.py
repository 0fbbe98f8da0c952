"""MI355X-native H-matrix-vector product (HIP kernels behind a C-ABI).

``hm`` is the ctypes binding of include/hm.h (same entry-point names);
``matrix.DeviceHMatrix`` wraps a plan, its device store and workspace in
torch-allocated device memory.
"""

from . import hm
from .matrix import DeviceHMatrix, blocks_from_table, batch_slots

__all__ = ["hm", "DeviceHMatrix", "blocks_from_table", "batch_slots"]
