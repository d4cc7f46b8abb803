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
