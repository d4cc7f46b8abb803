"""Pins of the batched inner products: per-column agreement with numpy's vdot
on FP64-converted inputs, conjugate-linearity, norm = dot(a, a)."""

import numpy as np

import oracle as O
import synth


def test_dot_matches_vdot_per_column():
    a = synth.spinor_source((2, 2, 2, 4), 5, 1)
    b = synth.spinor_source((2, 2, 2, 4), 5, 9)
    d = O.dot(a, b)
    for k in range(5):
        assert abs(d[k] - np.vdot(a[:, :, k], b[:, :, k])) <= 1e-12 * abs(d[k])


def test_dot_fp32_inputs_converted_before_products():
    a = synth.spinor_source((2, 2, 2, 2), 3, 1).astype(np.complex64)
    b = synth.spinor_source((2, 2, 2, 2), 3, 2).astype(np.complex64)
    d = O.dot(a, b)
    for k in range(3):
        ref = np.vdot(a[:, :, k].astype(np.complex128), b[:, :, k].astype(np.complex128))
        assert abs(d[k] - ref) <= 1e-13 * abs(ref)


def test_dot_conjugate_linear_and_norm():
    a = synth.spinor_source((2, 2, 2, 2), 2, 3)
    b = synth.spinor_source((2, 2, 2, 2), 2, 4)
    c = 0.3 - 1.7j
    np.testing.assert_allclose(O.dot(c * a, b), np.conj(c) * O.dot(a, b), rtol=1e-13)
    np.testing.assert_allclose(O.dot(a, c * b), c * O.dot(a, b), rtol=1e-13)
    np.testing.assert_allclose(O.norm2(a), O.dot(a, a).real, rtol=1e-13)
    np.testing.assert_allclose(O.dot(a, a).imag, 0, atol=1e-12)
