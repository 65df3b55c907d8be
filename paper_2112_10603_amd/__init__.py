"""MI355X-native view interpolation (VINet forward pass) — Python binding.

The compute path is ``lib/libffv.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/ffv.h``); :mod:`.ffv` marshals torch device tensors into it.
"""
from .ffv import FfvError, Net, debug_fault, lap_loss, lib, op_conv, stitch_cluster  # noqa: F401
