"""Pins of the oracle's reference solve: the sparse operator is assembled
from the definition independently of the stencil apply and must agree with
it; the solution must satisfy the system; the smallest singular value of the
free operator has a closed form in momentum space."""

import numpy as np
import pytest

import oracle as O
import synth

KAPPA = 0.13


@pytest.mark.parametrize("dims,t_bc", [((2, 4, 2, 6), -1.0), ((4, 2, 2, 2), 1.0), ((2, 2, 4, 4), -1.0)])
def test_sparse_matches_stencil(dims, t_bc):
    U = synth.gauge_haar(dims, 3)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    psi = synth.spinor_source(dims, 3, 9)
    D = O.dwc_sparse(U, A, KAPPA, dims, t_bc)
    got = (D @ psi.reshape(-1, 3)).reshape(psi.shape)
    np.testing.assert_allclose(got, O.dwc(U, A, KAPPA, psi, dims, t_bc), atol=1e-13)


def test_solve_ref_residual():
    dims = (4, 4, 2, 6)
    U = synth.gauge_haar(dims, 4)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    b = synth.spinor_source(dims, 2, 1)
    x = O.solve_ref(U, A, KAPPA, b, dims)
    assert np.all(O.true_residual(U, A, KAPPA, x, b, dims) < 1e-12)


@pytest.mark.parametrize("t_bc", [-1.0, 1.0])
def test_sigma_min_free_field_closed_form(t_bc):
    """Unit links: D(p) = a + i sum_mu b_mu gamma_mu is normal with singular
    values sqrt(a^2 + |b|^2), a = 1 - 2k sum cos p, b = 2k sin p."""
    dims = (2, 4, 2, 4)
    U = synth.gauge_unit(dims)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    Lx, Ly, Lz, Lt = dims
    best = np.inf
    for nx in range(Lx):
        for ny in range(Ly):
            for nz in range(Lz):
                for nt in range(Lt):
                    p = np.array([2 * np.pi * nx / Lx, 2 * np.pi * ny / Ly, 2 * np.pi * nz / Lz,
                                  (2 * nt + (1 if t_bc < 0 else 0)) * np.pi / Lt])
                    a = 1 - 2 * KAPPA * np.cos(p).sum()
                    b2 = (2 * KAPPA) ** 2 * (np.sin(p) ** 2).sum()
                    best = min(best, np.sqrt(a * a + b2))
    got = O.sigma_min(U, A, KAPPA, dims, t_bc=t_bc, mass_form=False)
    assert abs(got - best) < 1e-7 * best
    # the mass form divides by 2 kappa
    np.testing.assert_allclose(O.sigma_min(U, A, KAPPA, dims, t_bc=t_bc), best / (2 * KAPPA), rtol=1e-7)
