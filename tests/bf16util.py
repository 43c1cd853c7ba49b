"""Round-to-nearest-even FP32 -> BF16 on the host (test helper).

The result is returned as float32 holding the BF16 value.  Pinned against
torch's bfloat16 conversion in test_bf16_rounding.py."""

import numpy as np


def bf16_rne(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    u = np.where(finite, r, u)
    return u.astype(np.uint32).view(np.float32).reshape(np.shape(x))
