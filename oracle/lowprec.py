"""Emulation of the BF16/FP16 operand rounding of the matrix-core coarse
stencil (paper Sec. 6 coarse operator; the paper runs single precision, the
reduced-precision coarse level is this implementation's choice and is
checked here against exact FP64 arithmetic on the rounded operands).

Rounding rule: a value is first rounded to FP32, then to BF16 or FP16 with
round-to-nearest, ties to even.  FP16 vector operands are first multiplied by
2^-E per right-hand side, with max_k max(|Re x|, |Im x|) = m 2^E, m in
[0.5, 1) (1 for an all-zero column); powers of two make that scaling exact.
The BF16 rounding is written on the FP32 bit pattern; FP16 uses numpy's
float16 conversion, which rounds to nearest even.
"""

from __future__ import annotations

import numpy as np

from .mg import coarse_apply, prolong, restrict


def round_bf16(x) -> np.ndarray:
    """Round real values to BF16 (via FP32), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    r = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f16(x) -> np.ndarray:
    """Round real values to FP16 (via FP32), returned as float64."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def _round_complex(z, fmt):
    fn = round_bf16 if fmt == "bf16" else round_f16
    z = np.asarray(z)
    return fn(z.real) + 1j * fn(z.imag)


def column_scale(e: np.ndarray) -> np.ndarray:
    """Per-RHS power of two 2^-E for FP16 operands, e of shape (..., N)."""
    N = e.shape[-1]
    f = np.asarray(e, dtype=np.complex64).reshape(-1, N)
    mx = np.maximum(np.abs(f.real), np.abs(f.imag)).max(axis=0).astype(np.float32)
    _, E = np.frexp(mx)
    return np.where(mx > 0, np.ldexp(1.0, -E), 1.0)


def coarse_apply_lowprec(B, e, dims, fmt: str) -> np.ndarray:
    """D_c e with blocks and vectors rounded as above, products and sums exact
    (FP64).  B (Vc, 9, Nb, Nb) any precision, e (Vc, Nb, N) FP32 values."""
    assert fmt in ("bf16", "f16")
    Bq = _round_complex(np.asarray(B, dtype=np.complex128).astype(np.complex64), fmt)
    e32 = np.asarray(e, dtype=np.complex64)
    if fmt == "f16":
        sc = column_scale(e32)
        eq = _round_complex((e32 * sc.astype(np.float32)).astype(np.complex64), fmt)
        return coarse_apply(Bq, eq, dims) / sc
    return coarse_apply(Bq, _round_complex(e32, fmt), dims)


def restrict_lowprec(basis, f, dims, block) -> np.ndarray:
    """P^dag f (Sec. 5 project) with the basis and the fine field rounded to
    BF16 as above (basis via its FP32 copy), products and sums exact (FP64):
    what matrix-core BF16 operands with exact products compute, up to the
    order of the FP32 accumulation."""
    bq = _round_complex(np.asarray(basis, dtype=np.complex128).astype(np.complex64), "bf16")
    fq = _round_complex(np.asarray(f, dtype=np.complex64), "bf16")
    return restrict(bq, fq, dims, block)


def prolong_lowprec(basis, y, dims, block) -> np.ndarray:
    """P y (Sec. 5 promote) with basis and coarse field rounded to BF16, exact sums."""
    bq = _round_complex(np.asarray(basis, dtype=np.complex128).astype(np.complex64), "bf16")
    yq = _round_complex(np.asarray(y, dtype=np.complex64), "bf16")
    return prolong(bq, yq, dims, block)
