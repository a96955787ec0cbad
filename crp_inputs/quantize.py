"""Storage rounding of field grids to 16-bit formats, as values on the host.

The device upload rounds each FP32 value to nearest even into FP16 or BF16;
these functions produce the same dequantized values in FP32, so that a
reference run can use exactly the grid the device stores.
"""
import numpy as np


def round_to_f16(values32: np.ndarray) -> np.ndarray:
    """FP32 -> FP16 (round to nearest even) -> FP32."""
    v = np.asarray(values32, dtype=np.float32)
    return v.astype(np.float16).astype(np.float32)


def round_to_bf16(values32: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 (round to nearest even on the 16 dropped bits) -> FP32."""
    v = np.ascontiguousarray(values32, dtype=np.float32)
    b = v.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).reshape(v.shape)
