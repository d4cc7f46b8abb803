"""Batched inner products in FP64 (paper Sec. 7, simultaneous inner products).

<a, b>_k = sum over sites and components of conj(a[..., k]) * b[..., k], one
value per RHS column k, conjugate-linear in the first argument.  Inputs of
lower precision are converted to FP64 before any multiplication.
"""

from __future__ import annotations

import numpy as np


def dot(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per-column inner products of two fields (..., N) -> complex128 (N,)."""
    a = np.asarray(a).astype(np.complex128)
    b = np.asarray(b).astype(np.complex128)
    N = a.shape[-1]
    return np.einsum("in,in->n", a.reshape(-1, N).conj(), b.reshape(-1, N))


def norm2(a: np.ndarray) -> np.ndarray:
    """Per-column squared 2-norms (N,)."""
    a = np.asarray(a).astype(np.complex128)
    N = a.shape[-1]
    a = a.reshape(-1, N)
    return np.einsum("in,in->n", a.real, a.real) + np.einsum("in,in->n", a.imag, a.imag)
