"""MI355X-native hot path of the decoupled solidification / macro-segregation
scheme (arXiv 2303.10783): HIP kernels behind the C ABI of include/sol.h,
with a thin ctypes binding."""
from .binding import (Batch, Case, SolError, TorchDevice, load,  # noqa: F401
                      sol_footprint_bytes)
