"""MI355X-native q-LSKUM flux residual and pseudo-time update.

The solver is the HIP library libqlskum.so behind the C ABI of
include/qlskum.h; `paper_2108_07031_amd.qlskum` is its thin ctypes binding.
"""
__all__ = ["qlskum"]
