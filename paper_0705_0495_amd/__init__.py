"""MI355X-native PIC-MCC hot path for the capacitively coupled rf discharge
in oxygen (electrons, O-, O2+) of Bronold et al., "Radio-frequency
discharges in Oxygen. Part 1: Modeling".

The computation lives in libpic.so (HIP kernels for gfx950 behind the C ABI of
include/pic.h); this package is its Python binding.
"""
from .binding import Discharge, PicError, autotune_batch, lib, step_batch, step_batch_static  # noqa: F401

__all__ = ["Discharge", "PicError", "autotune_batch", "lib", "step_batch", "step_batch_static"]
