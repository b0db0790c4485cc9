"""Measured dense matrix-core peak of the current GPU (binding of hfx_mfma_peak)."""
from __future__ import annotations

import ctypes

from . import _abi as A

KINDS = {"fp64": 0, "fp32": 1, "bf16": 2}
DATASHEET_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6}  # MI355X dense, 2 FLOPs per multiply-add


def mfma_peak(kind: str = "fp64"):
    """(TFLOP/s, shader clock MHz) of one MFMA kind measured on the current device, on torch's
    current stream."""
    import torch
    tf, mhz = ctypes.c_double(0.0), ctypes.c_double(0.0)
    stream = torch.cuda.current_stream().cuda_stream
    A.check(A.lib().hfx_mfma_peak(KINDS[kind], ctypes.c_void_p(stream), ctypes.byref(tf), ctypes.byref(mhz)))
    return tf.value, mhz.value
