"""The pins must be able to fail: plant plausible mistakes in the oracle (on the
CPU, through monkeypatching) and check that at least one pin catches each."""

import numpy as np
import pytest

import oracle.mg as M
import oracle.wilson as W
from tests import test_oracle_fine as TF
from tests import test_oracle_mg as TM


def test_flipped_hop_projectors_caught(monkeypatch):
    """(1 + gamma) forward / (1 - gamma) backward keeps the spectrum but not D(p)."""
    real = W.gamma_matrices

    def flipped():
        g = real().copy()
        g[:4] *= -1
        return g

    monkeypatch.setattr(W, "gamma_matrices", flipped)
    with pytest.raises(AssertionError):
        TF.test_free_field_plane_wave((2, 4, 2, 4))


def test_dropped_time_boundary_phase_caught(monkeypatch):
    real = W._shift
    monkeypatch.setattr(W, "_shift", lambda f, mu, step, t_bc=1.0: real(f, mu, step, 1.0))
    with pytest.raises(AssertionError):
        TF.test_free_field_spectrum_closed_form((2, 4, 2, 4), -1.0)


def test_clover_normalisation_caught(monkeypatch):
    real = W.field_strength
    monkeypatch.setattr(W, "field_strength", lambda U, dims: {k: 2 * v for k, v in real(U, dims).items()})
    with pytest.raises(AssertionError):
        TF.test_clover_constant_abelian_field()


def test_clover_leaf_orientation_caught(monkeypatch):
    """A reversed leaf (Q -> Q^dag for the first leaf) is still gauge covariant."""
    real = W.plaquette_leaves

    def bad(U, dims, mu, nu):
        Q = real(U, dims, mu, nu)
        Um = W._lat(U[:, mu], dims)
        Un = W._lat(U[:, nu], dims)
        L1 = W._flat(Um @ W._shift(Un, mu, 1) @ W._dag(W._shift(Um, nu, 1)) @ W._dag(Un))
        return Q - L1 + W._dag(L1)

    monkeypatch.setattr(W, "plaquette_leaves", bad)
    with pytest.raises(AssertionError):
        TF.test_clover_constant_abelian_field()


def test_backward_link_not_daggered_caught(monkeypatch):
    real_einsum = np.einsum

    def einsum(spec, *ops, **kw):
        if spec == "vba,vsbn->vsan":  # U^dag psi in the backward hop
            return real_einsum("vab,vsbn->vsan", ops[0], *ops[1:], **kw)
        return real_einsum(spec, *ops, **kw)

    monkeypatch.setattr(W.np, "einsum", einsum)
    with pytest.raises(AssertionError):
        TF.test_gauge_covariance((2, 4, 2, 4))


def test_swapped_coarse_directions_caught(monkeypatch):
    """Swapping the +t and -t blocks is invisible at coarse extent 2 (A+t = A-t),
    so the lattice used has coarse extent 3 in t."""
    dirs = list(M.DIRS)
    dirs[7], dirs[8] = dirs[8], dirs[7]
    monkeypatch.setattr(M, "DIRS", dirs)
    with pytest.raises(AssertionError):
        TM.test_galerkin_fine_vs_dense((2, 4, 2, 6), (1, 2, 2, 2), 2)


def test_restrict_without_conjugate_caught(monkeypatch):
    real_einsum = np.einsum

    def einsum(spec, *ops, **kw):
        if spec == "vic,vcn->vin":
            return real_einsum(spec, np.conj(ops[0]), *ops[1:], **kw)
        return real_einsum(spec, *ops, **kw)

    monkeypatch.setattr(M.np, "einsum", einsum)
    with pytest.raises(AssertionError):
        TM.test_restrict_prolong_explicit_loops()
