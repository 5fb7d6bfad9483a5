"""Helpers for the GPU tests: move seeded column stores to the device and run
the library through its C ABI binding."""
import numpy as np

import synth


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def colstore32(A, lda=None):
    """dense m x n float64 -> float32 column store (n, lda) (numpy)."""
    return synth.to_colstore(A, lda=lda, dtype=np.float32)


def stored_dense(cs, m):
    """float32 column store -> the m x n float64 values it holds."""
    return synth.from_colstore(cs, m)


def f64cs(A):
    """dense m x n -> float64 column store with ld = m (oracle input)."""
    return synth.to_colstore(A, lda=A.shape[0], dtype=np.float64)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)
