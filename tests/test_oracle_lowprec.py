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
