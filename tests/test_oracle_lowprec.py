"""Pins of the BF16/FP16 rounding emulation against hand-worked bit patterns
and against torch's own float32 -> bfloat16 conversion (an independent
implementation of round-to-nearest-even)."""

import numpy as np
import torch

import oracle as O
import synth


def test_bf16_hand_cases():
    u = 2.0 ** -8  # half an ulp of bf16 at 1.0 (bf16 keeps 8 significant bits)
    cases = {
        1.0: 1.0,
        1.0 + u: 1.0,  # tie -> even (mantissa 0)
        1.0 + 3 * u: 1.0 + 4 * u,  # tie -> even (mantissa 2)
        1.0 + 1.5 * u: 1.0 + 2 * u,  # above the tie -> up
        -(1.0 + 1.5 * u): -(1.0 + 2 * u),
        3.0: 3.0,
        0.0: 0.0,
    }
    for x, want in cases.items():
        assert O.round_bf16(np.array([x]))[0] == want, x


def test_bf16_matches_torch():
    x = synth.rng(3).standard_normal(100000).astype(np.float32) * 10.0 ** synth.rng(4).integers(-20, 20, 100000)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.round_bf16(x), want)


def test_f16_hand_cases():
    u = 2.0 ** -11  # half an ulp of fp16 at 1.0
    assert O.round_f16(np.array([1.0 + u]))[0] == 1.0
    assert O.round_f16(np.array([1.0 + 3 * u]))[0] == 1.0 + 4 * u
    assert O.round_f16(np.array([65504.0]))[0] == 65504.0


def test_column_scale_powers_of_two():
    e = np.zeros((3, 2, 4), dtype=np.complex64)
    e[0, 0, 0] = 0.75 + 0.1j     # max 0.75 = 0.75 * 2^0 -> E = 0 -> scale 1
    e[1, 1, 1] = 3.0 - 7.9j      # max 7.9 = 0.9875 * 2^3 -> scale 1/8
    e[2, 0, 2] = 1.0             # max 1 = 0.5 * 2^1 -> scale 1/2
    sc = O.column_scale(e)       # column 3 all zero -> 1
    np.testing.assert_array_equal(sc, [1.0, 0.125, 0.5, 1.0])


def test_lowprec_apply_close_to_exact():
    """Rounded operands change a random stencil apply by about the unit
    roundoff of the format (2^-8 for bf16, 2^-11 for fp16)."""
    dims = (2, 2, 2, 2)
    B = synth.gaussian_blocks(16, 8, 1)
    e = synth.coarse_source(16, 8, 5, 2, np.complex64)
    exact = O.coarse_apply(B, e, dims)
    for fmt, u in (("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)):
        got = O.coarse_apply_lowprec(B, e, dims, fmt)
        rel = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        assert u / 20 < rel < 2 * u, (fmt, rel)


def test_lowprec_intergrid_exact_on_representable_and_close_otherwise():
    """BF16 restrict/prolong emulation: with operands already exactly
    representable in BF16 it equals the plain restrict/prolong; with generic
    operands it moves the result by about the BF16 unit roundoff 2^-8, and
    P^dag P = 1 holds to that accuracy."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    V = synth.volume(dims)
    basis = O.block_orthonormalise(synth.gaussian_vectors(V, 4, 12, 3), dims, block)
    f = synth.spinor_source(dims, 3, 4, np.complex64)
    bq = O.round_bf16(basis.real) + 1j * O.round_bf16(basis.imag)
    fq = O.round_bf16(f.real) + 1j * O.round_bf16(f.imag)
    np.testing.assert_array_equal(O.restrict_lowprec(bq, fq, dims, block), O.restrict(bq, fq, dims, block))
    y = synth.coarse_source(16, 8, 3, 5, np.complex64)
    yq = O.round_bf16(y.real) + 1j * O.round_bf16(y.imag)
    np.testing.assert_array_equal(O.prolong_lowprec(bq, yq, dims, block), O.prolong(bq, yq, dims, block))
    u = 2.0 ** -8
    for got, exact in ((O.restrict_lowprec(basis, f, dims, block), O.restrict(basis, f, dims, block)),
                       (O.prolong_lowprec(basis, y, dims, block), O.prolong(basis, y, dims, block))):
        rel = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        assert u / 20 < rel < 2 * u, rel
    back = O.restrict_lowprec(basis, O.prolong(basis, y, dims, block), dims, block)
    assert np.linalg.norm(back - y) / np.linalg.norm(y) < 2 * u


def _self_only(b, e, fmt):
    """Stencil on a one-site lattice (all nine directions act on the site
    itself) with only the self block nonzero: the result is round(b) round(e)."""
    b = np.atleast_2d(np.asarray(b, dtype=np.complex128))
    B = np.zeros((1, 9) + b.shape, dtype=np.complex128)
    B[0, 0] = b
    ev = np.asarray(e, dtype=np.complex64).reshape(1, b.shape[1], -1)
    return O.coarse_apply_lowprec(B, ev, (1, 1, 1, 1), fmt)


def test_coarse_lowprec_hand_cases():
    """Worked by hand from the rounding rule (blocks via FP32, then to the
    format with ties to even; both operands rounded; FP16 vectors scaled per
    right-hand side by a power of two first)."""
    # FP64 block 1 + 2^-8 + 2^-30: FP32 drops 2^-30 (below half an FP32 ulp),
    # which leaves the BF16 tie 1 + 2^-8 -> even -> 1.  Rounding FP64 straight
    # to BF16 would give 1 + 2^-7.
    assert _self_only(1 + 2.0**-8 + 2.0**-30, 1.0, "bf16")[0, 0, 0] == 1.0
    # the same double-rounding case for FP16 (ulp 2^-10 at 1)
    assert _self_only(1 + 2.0**-11 + 2.0**-30, 1.0, "f16")[0, 0, 0] == 1.0
    # both operands 1 + 3 2^-9 = 1 + 0.75 BF16 ulp -> 1 + 2^-7 each:
    # (1 + 2^-7)^2 = 1 + 2^-6 + 2^-14 (rounding one operand only gives another value)
    v = 1 + 3 * 2.0**-9
    assert _self_only(v, v, "bf16")[0, 0, 0] == 1 + 2.0**-6 + 2.0**-14
    # imaginary parts are rounded the same way: (i v) v -> i (1 + 2^-7)^2
    assert _self_only(1j * v, v, "bf16")[0, 0, 0] == 1j * (1 + 2.0**-6 + 2.0**-14)
    # FP16 range: 1e6 does not fit FP16, but scaled by 2^-20 it is
    # 0.11110100001|001... in binary, which rounds down to 1953 2^-11, so the
    # apply returns 1953 2^-11 2^20 = 999936
    assert _self_only(1.0, 1e6, "f16")[0, 0, 0] == 999936.0
    # the scale is one per right-hand side: next to 1e6 in the same column a
    # component 1e-3 scales to ~9.5e-10, below the smallest FP16 subnormal
    # (2^-24), and drops out; in the column whose maximum is 1 (scale 2^-1)
    # it survives: 1e-3 2^-1 = 1.024 2^-11 rounds to 1049 2^-21, so the apply
    # returns 1049 2^-20
    b2 = np.eye(2)
    got = _self_only(b2, np.array([[1e6, 1e-3], [1e-3, 1.0]]), "f16")
    assert got[0, 1, 0] == 0.0
    assert got[0, 0, 1] == 1049 * 2.0**-20


def _representable(g, shape, bits):
    """Complex values k 2^-4 with |k| < 2^bits: exact in BF16 (bits <= 8) or FP16."""
    k = g.integers(-(2**bits) + 1, 2**bits, size=shape + (2,)).astype(np.float64)
    return (k[..., 0] + 1j * k[..., 1]) * 2.0**-4


def test_coarse_lowprec_exact_on_representable():
    """Operands that are already BF16 (FP16, after the per-RHS power of two)
    values pass the rounding unchanged, so the emulation must equal the
    plain FP64 stencil bit for bit (the products and sums of these small
    dyadic values are exact in FP64)."""
    dims = (2, 3, 1, 2)
    V = 12
    g = synth.rng(11)
    for fmt, bits in (("bf16", 8), ("f16", 11)):
        B = _representable(g, (V, 9, 4, 4), bits)
        e = _representable(g, (V, 4, 3), bits).astype(np.complex64)
        e[:, :, 1] *= 2.0**9  # a column whose FP16 scale is far from 1
        np.testing.assert_array_equal(O.coarse_apply_lowprec(B, e, dims, fmt), O.coarse_apply(B, e, dims))


def test_coarse_lowprec_matches_torch_rounding():
    """Generic operands: the emulation equals the plain stencil on operands
    rounded by torch's own float32 -> bfloat16 / float16 conversions (an
    independent round-to-nearest-even), blocks via FP32, FP16 vectors after
    the per-column power of two (pinned by hand above)."""
    dims = (2, 2, 3, 2)
    V = 24
    B = synth.gaussian_blocks(V, 6, 21)
    e = synth.coarse_source(V, 6, 4, 22, np.complex64)

    def tr(z, dt):
        z = np.asarray(z, dtype=np.complex64)
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dt).to(torch.float64).numpy()
        return f(z.real) + 1j * f(z.imag)

    want = O.coarse_apply(tr(B, torch.bfloat16), tr(e, torch.bfloat16), dims)
    np.testing.assert_array_equal(O.coarse_apply_lowprec(B, e, dims, "bf16"), want)
    sc = O.column_scale(e)
    want = O.coarse_apply(tr(B, torch.float16), tr(e * sc.astype(np.float32), torch.float16), dims) / sc
    np.testing.assert_array_equal(O.coarse_apply_lowprec(B, e, dims, "f16"), want)
