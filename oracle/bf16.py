"""BF16 numerical-semantics model of the fine operator (oracle).

Test infrastructure only.

Follows Sec. 3.5 (BF16 numerical semantics): the element input tile is rounded
to BF16, the element matrix is exact in BF16 (s*K_e is an integer matrix with
entries of magnitude <= 88), products accumulate in FP32 and E_e is applied in
FP32.  The model rounds u to BF16 (round to nearest even) and evaluates the rest
exactly in FP64; an FP32-accumulating device result differs from it only by
FP32 summation rounding.
"""
import numpy as np

from . import mesh


def round_bf16(x):
    """Round FP64 values to the nearest BF16 value (ties to even), via FP32."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    b = (b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def apply_K_bf16_model(dims, E, u, fixed, nu=0.3):
    """M K M bf16(u): the exact value of the BF16-input fine operator."""
    ub = round_bf16(np.where(np.asarray(fixed, dtype=bool), 0.0, u))
    return mesh.apply_K_elementwise(dims, E, ub, nu, fixed)
