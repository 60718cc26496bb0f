"""Emulation of reduced-precision storage (round to nearest, ties to even).

Used to predict the error of applying a BRAS operator whose element inverses
are stored in FP32 or BF16 (parity unpinned: these are extensions the paper
does not discuss; they state errors against the float64 operator).
"""
import numpy as np


def round_fp32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(a):
    """float64 -> float32 (RNE) -> bfloat16 (RNE on the top 16 bits) -> float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
