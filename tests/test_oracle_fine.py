"""Pins of the fine-level oracle (Wilson hop + clover) against what the physics fixes.

Every check here is independent of the oracle's own formulas: closed forms in
momentum space, exact symmetries (gamma5-hermiticity, gauge covariance), a
constant abelian field whose clover term is known by hand, and structural
identities of the clover blocks.  Lattices are small and non-cubic so that a
transposed axis or a wrong neighbour index cannot hide.
"""

import numpy as np
import pytest

import oracle as O
import synth

KAPPA = 0.13

# Chiral-basis gamma matrices typed out entry by entry (the test does not
# take them from the oracle).
_i = 1j
G1 = np.array([[0, 0, 0, -_i], [0, 0, -_i, 0], [0, _i, 0, 0], [_i, 0, 0, 0]])
G2 = np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]])
G3 = np.array([[0, 0, -_i, 0], [0, 0, 0, _i], [_i, 0, 0, 0], [0, -_i, 0, 0]])
G4 = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]])
G5 = np.diag([1, 1, -1, -1])
GAM = [G1, G2, G3, G4]
GAMMA5_12 = np.kron(G5, np.eye(3))


def _coords(dims):
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    return np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)


def _dense(U, A, kappa, dims, t_bc=-1.0):
    V = synth.volume(dims)
    I = np.eye(V * 12).reshape(V * 12, V, 12).transpose(1, 2, 0)
    return O.dwc(U, A, kappa, I, dims, t_bc).reshape(V * 12, V * 12)


def _momenta(dims, t_bc):
    Lx, Ly, Lz, Lt = dims
    ps = []
    for nx in range(Lx):
        for ny in range(Ly):
            for nz in range(Lz):
                for nt in range(Lt):
                    pt = (2 * nt + (1 if t_bc < 0 else 0)) * np.pi / Lt
                    ps.append(np.array([2 * np.pi * nx / Lx, 2 * np.pi * ny / Ly, 2 * np.pi * nz / Lz, pt]))
    return ps


def _multiset_close(a, b, tol):
    a = np.sort_complex(np.round(a, 9))
    b = np.sort_complex(np.round(b, 9))
    return np.max(np.abs(a - b)) < tol


def test_gamma_basis_matches_typed_matrices():
    g = O.gamma_matrices()
    for k in range(4):
        np.testing.assert_array_equal(g[k], GAM[k])
    np.testing.assert_array_equal(g[4], G5)
    for m in range(4):
        for n in range(4):
            ac = GAM[m] @ GAM[n] + GAM[n] @ GAM[m]
            np.testing.assert_allclose(ac, 2 * np.eye(4) * (m == n), atol=0)


@pytest.mark.parametrize("dims,t_bc", [((2, 4, 2, 4), -1.0), ((4, 2, 2, 2), 1.0)])
def test_free_field_spectrum_closed_form(dims, t_bc):
    """Unit links: the spectrum is {1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p)}, 6-fold."""
    U = synth.gauge_unit(dims)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    ev = np.linalg.eigvals(_dense(U, A, KAPPA, dims, t_bc))
    exp = []
    for p in _momenta(dims, t_bc):
        re = 1 - 2 * KAPPA * np.cos(p).sum()
        im = 2 * KAPPA * np.sqrt((np.sin(p) ** 2).sum())
        exp += [re + 1j * im] * 6 + [re - 1j * im] * 6
    assert _multiset_close(ev, np.array(exp), 1e-12)


@pytest.mark.parametrize("dims", [(2, 4, 2, 4), (4, 2, 6, 2)])
def test_free_field_plane_wave(dims):
    """psi = exp(i p.x) chi is mapped to D(p) psi with
    D(p) = 1 - 2k sum cos p_mu + 2ik sum gamma_mu sin p_mu (antiperiodic t)."""
    U = synth.gauge_unit(dims)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    X = _coords(dims)
    g = synth.rng(11)
    for p in _momenta(dims, -1.0)[:: max(1, len(_momenta(dims, -1.0)) // 7)]:
        chi = synth.gaussian_complex(g, (4, 3))
        phase = np.exp(1j * (X @ p))
        psi = (phase[:, None, None] * chi[None]).reshape(-1, 12, 1)
        Dp = (1 - 2 * KAPPA * np.cos(p).sum()) * np.eye(4) + 2j * KAPPA * sum(
            GAM[m] * np.sin(p[m]) for m in range(4)
        )
        want = (phase[:, None, None] * (Dp @ chi)[None]).reshape(-1, 12, 1)
        got = O.dwc(U, A, KAPPA, psi, dims)
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_mass_form_plane_wave():
    """D_m = D/(2k): on the free field D_m(p) = (4 + m0) - sum cos p + i sum gamma sin p."""
    dims = (2, 2, 4, 4)
    m0 = -0.37
    kappa = 1.0 / (2 * (4 + m0))
    U = synth.gauge_unit(dims)
    A = O.clover_packed(U, dims, 1.0, kappa)
    X = _coords(dims)
    p = _momenta(dims, -1.0)[5]
    chi = synth.gaussian_complex(synth.rng(3), (4, 3))
    phase = np.exp(1j * (X @ p))
    psi = (phase[:, None, None] * chi[None]).reshape(-1, 12, 1)
    Dp = (4 + m0 - np.cos(p).sum()) * np.eye(4) + 1j * sum(GAM[m] * np.sin(p[m]) for m in range(4))
    want = (phase[:, None, None] * (Dp @ chi)[None]).reshape(-1, 12, 1)
    np.testing.assert_allclose(O.dwc_mass(U, A, kappa, psi, dims), want, atol=1e-13)


def test_pure_gauge_equals_free_field():
    """U_mu(x) = L(x) L(x+mu)^dag: plaquettes are 1, the clover term vanishes and
    the spectrum equals the free one."""
    dims = (2, 4, 2, 4)
    Lam = synth.gauge_transform_field(dims, 5)
    U = O.gauge_transform(synth.gauge_unit(dims), Lam, dims)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    Afree = O.clover_packed(synth.gauge_unit(dims), dims, 1.0, KAPPA)
    np.testing.assert_allclose(A, Afree, atol=1e-14)
    ev = np.linalg.eigvals(_dense(U, A, KAPPA, dims))
    ev0 = np.linalg.eigvals(_dense(synth.gauge_unit(dims), Afree, KAPPA, dims))
    assert _multiset_close(ev, ev0, 1e-11)


@pytest.mark.parametrize("dims", [(2, 4, 2, 4), (4, 2, 4, 6)])
def test_gamma5_hermiticity(dims):
    """<phi, D psi> = <g5 D g5 phi, psi> on Haar links with the clover term."""
    U = synth.gauge_haar(dims, 1)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    phi = synth.spinor_source(dims, 3, 100)
    psi = synth.spinor_source(dims, 3, 200)
    g5 = lambda f: np.einsum("ij,vjn->vin", GAMMA5_12, f)
    lhs = np.einsum("vin,vin->n", phi.conj(), O.dwc(U, A, KAPPA, psi, dims))
    rhs = np.einsum("vin,vin->n", g5(O.dwc(U, A, KAPPA, g5(phi), dims)).conj(), psi)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(lhs))


@pytest.mark.parametrize("dims", [(2, 4, 2, 4), (4, 2, 6, 2)])
def test_gauge_covariance(dims):
    """D[U^L](L psi) = L (D[U] psi), with U^L_mu(x) = L(x) U_mu(x) L(x+mu)^dag."""
    U = synth.gauge_haar(dims, 2)
    Lam = synth.gauge_transform_field(dims, 3)
    UL = O.gauge_transform(U, Lam, dims)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    AL = O.clover_packed(UL, dims, 1.0, KAPPA)
    psi = synth.spinor_source(dims, 2, 7)
    lhs = O.dwc(UL, AL, KAPPA, O.spinor_gauge_transform(psi, Lam), dims)
    rhs = O.spinor_gauge_transform(O.dwc(U, A, KAPPA, psi, dims), Lam)
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_clover_structure_two_routes():
    """A_chi Hermitian, tr(A_chi - 1) = 0, chiral blocks decouple (C commutes with
    gamma5), and the gamma-product route agrees with the Pauli-block route."""
    dims = (2, 4, 2, 4)
    U = synth.gauge_haar(dims, 4)
    Ad = O.clover_dense(U, dims, 1.0, KAPPA)
    np.testing.assert_allclose(Ad, np.conj(np.swapaxes(Ad, 1, 2)), atol=1e-15)
    np.testing.assert_allclose(Ad[:, :6, 6:], 0, atol=1e-15)
    np.testing.assert_allclose(Ad[:, 6:, :6], 0, atol=1e-15)
    np.testing.assert_allclose(Ad @ GAMMA5_12, GAMMA5_12 @ Ad, atol=1e-15)
    tr = np.trace(Ad[:, :6, :6] - np.eye(6), axis1=1, axis2=2)
    np.testing.assert_allclose(tr, 0, atol=1e-14)
    A1 = O.clover_packed(U, dims, 1.0, KAPPA)
    A2 = O.clover_packed_direct(U, dims, 1.0, KAPPA)
    np.testing.assert_allclose(A1, A2, atol=1e-14)
    # a random field is not trivially zero
    assert np.abs(A1[:, :, 6:]).max() > 1e-2


def test_clover_constant_abelian_field():
    """U_x(x) = diag(e^{i phi y}, e^{-i phi y}, 1), other links 1, phi = 2 pi / Ly.
    Every x-y plaquette equals diag(e^{-i phi}, e^{i phi}, 1), so
    F_xy = diag(-i sin phi, i sin phi, 0); with sigma_xy = diag(-1, 1, -1, 1)
    in the chiral basis, A = 1 + c kappa sin(phi) diag(-1,1,-1,1) (x) diag(1,-1,0)."""
    dims = (2, 6, 2, 4)
    csw, kappa = 1.3, 0.11
    Ly = dims[1]
    phi = 2 * np.pi / Ly
    X = _coords(dims)
    U = synth.gauge_unit(dims)
    y = X[:, 1]
    U[:, 0, 0, 0] = np.exp(1j * phi * y)
    U[:, 0, 1, 1] = np.exp(-1j * phi * y)
    Ad = O.clover_dense(U, dims, csw, kappa)
    want = np.eye(12) + csw * kappa * np.sin(phi) * np.kron(np.diag([-1, 1, -1, 1]), np.diag([1, -1, 0]))
    np.testing.assert_allclose(Ad, np.broadcast_to(want, Ad.shape), atol=1e-14)


def test_special_cases():
    """kappa = 0 gives D = A; c_sw = 0 gives A = 1 (pure Wilson)."""
    dims = (2, 2, 4, 2)
    U = synth.gauge_haar(dims, 9)
    psi = synth.spinor_source(dims, 2, 1)
    A = O.clover_packed(U, dims, 1.0, 0.13)
    np.testing.assert_allclose(O.dwc(U, A, 0.0, psi, dims), O.clover_apply(A, psi), atol=0)
    A0 = O.clover_packed(U, dims, 0.0, 0.13)
    np.testing.assert_allclose(O.clover_apply(A0, psi), psi, atol=0)


def test_mrhs_equals_columns():
    """Applying D to N columns at once equals applying it column by column."""
    dims = (2, 4, 2, 4)
    U = synth.gauge_haar(dims, 1)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    psi = synth.spinor_source(dims, 4, 50)
    full = O.dwc(U, A, KAPPA, psi, dims)
    for k in range(4):
        col = O.dwc(U, A, KAPPA, synth.spinor_source(dims, 1, 50 + k), dims)
        np.testing.assert_allclose(full[:, :, k:k + 1], col, atol=1e-15)


def test_pack_roundtrip_and_layout():
    M = synth.gaussian_complex(synth.rng(1), (5, 6, 6))
    M = M + np.conj(np.swapaxes(M, 1, 2))
    p = O.pack_hermitian6(M)
    assert p.shape == (5, 36)
    np.testing.assert_allclose(O.unpack_hermitian6(p), M, atol=0)
    # entry order: 6 diagonal reals, then (1,0), (2,0), (2,1), ...
    assert p[0, 6] == M[0, 1, 0].real and p[0, 7] == M[0, 1, 0].imag
    assert p[0, 10] == M[0, 2, 1].real and p[0, 35] == M[0, 5, 4].imag


def test_dwc_sites_matches_whole_lattice():
    """The per-site evaluation used for large-lattice sampling equals the full apply."""
    dims = (4, 2, 6, 4)
    U = synth.gauge_haar(dims, 1)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    psi = synth.spinor_source(dims, 3, 4)
    full = O.dwc(U, A, KAPPA, psi, dims)
    sites = np.array([0, 1, 5, 17, 47, 95, 96, 191])
    np.testing.assert_allclose(O.dwc_sites(U, A, KAPPA, psi, dims, sites), full[sites], atol=1e-14)
