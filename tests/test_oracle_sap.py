"""Pins of the SAP oracle (oracle/sap.py) against what the definition fixes:
the block operator is the dense operator with every coupling between two
different blocks removed (brute force from the independent sparse assembly),
it keeps a vector inside its block, it inherits gamma_5-hermiticity, and a
colour half-cycle with (nearly) exact block solves leaves no residual on the
blocks it solved."""

import numpy as np
import pytest

import oracle as O
from oracle import sap as S
import synth

KAPPA, CSW = 0.13, 1.0
DIMS, BLOCK = (4, 4, 4, 4), (2, 2, 2, 2)


@pytest.fixture(scope="module")
def op():
    U = synth.gauge_haar(DIMS, 71)
    A = O.clover_packed(U, DIMS, CSW, KAPPA)
    return U, A


def test_block_colour_is_a_two_colouring():
    c = S.block_colour(DIMS, BLOCK)
    agg = O.aggregate_index(DIMS, BLOCK)
    s = np.arange(synth.volume(DIMS))
    X = np.stack([s % 4, (s // 4) % 4, (s // 16) % 4, s // 64], axis=1)
    for mu in range(4):
        nb = ((X + np.eye(4, dtype=int)[mu]) % 4) @ np.array([1, 4, 16, 64])
        cross = agg != agg[nb]
        assert np.all(c[cross] != c[nb][cross])  # neighbouring blocks differ in colour
        assert np.all(c[~cross] == c[nb][~cross])
    assert np.sum(c == 0) == np.sum(c == 1)
    with pytest.raises(ValueError):
        S.block_colour((6, 4, 4, 4), BLOCK)  # three blocks along x: no two-colouring


def test_block_operator_equals_dense_with_cross_block_couplings_removed(op):
    U, A = op
    D = O.dwc_sparse(U, A, KAPPA, DIMS).toarray()
    agg = np.repeat(O.aggregate_index(DIMS, BLOCK), 12)
    Dblk = np.where(agg[:, None] == agg[None, :], D, 0.0)
    psi = synth.spinor_source(DIMS, 3, 5)
    V = synth.volume(DIMS)
    want = (Dblk @ psi.reshape(V * 12, 3)).reshape(V, 12, 3)
    got = S.dwc_blocks(U, A, KAPPA, psi, DIMS, BLOCK)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    # and the dropped part is exactly the cross-block hops of D
    rest = ((D - Dblk) @ psi.reshape(V * 12, 3)).reshape(V, 12, 3)
    assert np.max(np.abs(got + rest - O.dwc(U, A, KAPPA, psi, DIMS))) < 1e-13


def test_block_operator_keeps_a_block_and_is_gamma5_hermitian(op):
    U, A = op
    agg = O.aggregate_index(DIMS, BLOCK)
    psi = synth.spinor_source(DIMS, 2, 7)
    psi[agg != 5] = 0.0
    out = S.dwc_blocks(U, A, KAPPA, psi, DIMS, BLOCK)
    assert np.all(out[agg != 5] == 0.0) and np.linalg.norm(out) > 0
    phi = synth.spinor_source(DIMS, 2, 8)
    chi = synth.spinor_source(DIMS, 2, 9)
    g5 = np.repeat([1.0, 1.0, -1.0, -1.0], 3)[None, :, None]
    lhs = np.einsum("sck,sck->k", phi.conj(), S.dwc_blocks(U, A, KAPPA, chi, DIMS, BLOCK))
    rhs = np.einsum("sck,sck->k", (g5 * S.dwc_blocks(U, A, KAPPA, g5 * phi, DIMS, BLOCK)).conj(), chi)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))


def test_exact_block_solves_clear_the_residual_of_the_last_colour(op):
    """With the block systems solved to convergence (many MR steps on small
    blocks), the colour-1 half of a cycle leaves b - D x = 0 on every
    colour-1 block, and a cycle reduces the residual."""
    U, A = op
    b = synth.spinor_source(DIMS, 2, 11)
    x = S.sap_cycles(U, A, KAPPA, b, np.zeros_like(b), DIMS, BLOCK, 1, 300)
    r = b - O.dwc(U, A, KAPPA, x, DIMS)
    c = S.block_colour(DIMS, BLOCK)
    assert np.linalg.norm(r[c == 1]) < 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(r) < 0.5 * np.linalg.norm(b)


def test_mr_step_length_per_block_and_column(op):
    """One MR step from zero on a colour: e = alpha_B r|_B with alpha_B the
    block's <q, r> / ||q||^2, computed here block by block with np.vdot."""
    U, A = op
    b = synth.spinor_source(DIMS, 2, 13)
    x = S.sap_cycles(U, A, KAPPA, b, np.zeros_like(b), DIMS, BLOCK, 1, 1)
    agg = O.aggregate_index(DIMS, BLOCK)
    c = S.block_colour(DIMS, BLOCK)
    rho = np.where((c == 0)[:, None, None], b, 0.0)
    q = np.where((c == 0)[:, None, None], S.dwc_blocks(U, A, KAPPA, rho, DIMS, BLOCK), 0.0)
    x0 = np.zeros_like(b)
    for B in np.unique(agg[c == 0]):
        m = agg == B
        for k in range(2):
            a = np.vdot(q[m][:, :, k], rho[m][:, :, k]) / np.vdot(q[m][:, :, k], q[m][:, :, k]).real
            x0[m, :, k] = a * rho[m][:, :, k]
    # the first colour's blocks are x0 exactly; the second colour was solved on b - D x0
    assert np.max(np.abs(x[c == 0] - x0[c == 0])) < 1e-14
