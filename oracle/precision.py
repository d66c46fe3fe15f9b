"""Storage rounding of an operator, for parity of the low-precision forms.  Test infrastructure.

A complex64 operator stores each element as (float32(re), float32(im)), rounded to
nearest.  A bf16-pair operator stores (bf16(re), bf16(im)), each obtained by rounding
to float32 and then to bfloat16 with round-to-nearest-even (the upper 16 bits of the
float32 pattern after adding 0x7FFF plus the lowest kept bit).  Applying the FP64
definition to the rounded operator isolates the arithmetic of a low-precision product
from the rounding of its storage.
"""
import numpy as np

ROUNDED_KEYS = ("U", "V", "S", "D", "SX", "SY")


def to_f32(a: np.ndarray) -> np.ndarray:
    return a.astype(np.complex64).astype(np.complex128)


def _bf16(x: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def to_bf16_pair(a: np.ndarray) -> np.ndarray:
    return _bf16(a.real) + 1j * _bf16(a.imag)


def round_operator(op, storage: str) -> dict:
    """A copy of the operator mapping with U, V, S, D and the coupling factors SX, SY (when
    present) rounded to the storage format."""
    f = {"c64": to_f32, "bf16pair": to_bf16_pair}[storage]
    out = dict(op)
    for k in ROUNDED_KEYS:
        if op.get(k) is not None:
            out[k] = f(np.asarray(op[k]))
    return out
