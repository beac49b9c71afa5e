"""Bitwise comparison of float64 bound arrays, the bar of the parity tests:
+0 and -0 count as different values, as in the hashes of the stored
expectations (tests/golden)."""
import numpy as np


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.int64)


def same_bits(a, b) -> bool:
    a, b = _bits(a), _bits(b)
    return a.shape == b.shape and bool(np.array_equal(a, b))


def differing(a, b):
    """Indices where two equally shaped arrays differ bitwise."""
    return np.nonzero(_bits(a) != _bits(b))[0]
