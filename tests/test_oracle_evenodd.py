"""Pins of the even-odd oracle (checkerboard layout, M_eooe, M_ooee and its
inverse, the Schur complement) against what the physics and the algebra fix:
hand-worked layout entries, the free-field plane-wave closed form of the hop
on each checkerboard, gauge covariance on Haar links, B B^-1 = 1 for the
clover blocks, and the Schur system checked against an independent sparse
solve of the full operator."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle import evenodd as EO
import synth

KAPPA = 0.13

# chiral-basis gamma matrices typed out (not taken from the oracle)
_i = 1j
G1 = np.array([[0, 0, 0, -_i], [0, 0, -_i, 0], [0, _i, 0, 0], [_i, 0, 0, 0]])
G2 = np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]])
G3 = np.array([[0, 0, -_i, 0], [0, 0, 0, _i], [_i, 0, 0, 0], [0, -_i, 0, 0]])
G4 = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]])
GAM = [G1, G2, G3, G4]


def test_checkerboard_layout_by_hand():
    dims = (4, 2, 2, 2)
    # s = 0 is (0,0,0,0), even; s = 1 is (1,0,0,0), odd; s = 4 is (0,1,0,0), odd; s = 5 is (1,1,0,0), even
    e, o = EO.cb_sites(dims, 0), EO.cb_sites(dims, 1)
    assert e[0] == 0 and o[0] == 1 and e[2] == 5 and o[2] == 4
    assert sorted(np.concatenate([e, o]).tolist()) == list(range(synth.volume(dims)))
    f = synth.spinor_source(dims, 3, 5)
    np.testing.assert_array_equal(EO.from_cb(EO.to_cb(f, dims, 0), EO.to_cb(f, dims, 1), dims), f)
    with pytest.raises(ValueError):
        EO.cb_sites((3, 2, 2, 2), 0)


@pytest.mark.parametrize("out_parity", [0, 1])
def test_hop_eo_free_plane_wave(out_parity):
    """U = 1: a plane wave with momenta 2 pi n / L (antiperiodic in t: (2n + 1) pi / Lt)
    has H psi = e^{ipx} [2 sum cos p - 2i sum gamma_mu sin p] chi, and every hop joins
    opposite parities, so H_{p,1-p} psi_{1-p} is that closed form on parity p."""
    dims = (4, 2, 2, 6)
    Lx, Ly, Lz, Lt = dims
    p = np.array([2 * np.pi * 1 / Lx, 2 * np.pi * 1 / Ly, 0.0, (2 * 1 + 1) * np.pi / Lt])
    s = np.arange(synth.volume(dims))
    X = np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)
    ph = np.exp(1j * X @ p)
    chi = synth.gaussian_complex(synth.rng(3), (4, 3))
    psi = (ph[:, None, None] * chi[None]).reshape(-1, 12, 1)
    K = 2 * np.cos(p).sum() * np.eye(4) - 2j * sum(GAM[m] * np.sin(p[m]) for m in range(4))
    Hpsi = (ph[:, None, None] * (K @ chi)[None]).reshape(-1, 12, 1)
    got = EO.hop_eo(synth.gauge_unit(dims), EO.to_cb(psi, dims, 1 - out_parity), dims, out_parity, t_bc=-1.0)
    np.testing.assert_allclose(got, EO.to_cb(Hpsi, dims, out_parity), atol=1e-12)


@pytest.mark.parametrize("out_parity", [0, 1])
def test_hop_eo_gauge_covariance(out_parity):
    """H_pq[U^L](L psi) = L (H_pq[U] psi) with U^L_mu(x) = L(x) U_mu(x) L(x + mu)^dag."""
    dims = (4, 4, 2, 4)
    U = synth.gauge_haar(dims, 11)
    Lam = synth.gauge_transform_field(dims, 12)
    psi = synth.spinor_source(dims, 2, 13)
    q = 1 - out_parity
    lhs = EO.hop_eo(O.gauge_transform(U, Lam, dims), EO.to_cb(O.spinor_gauge_transform(psi, Lam), dims, q),
                    dims, out_parity)
    # L (H_pq psi): rotate the result site by site with L at the parity-p sites
    h = EO.hop_eo(U, EO.to_cb(psi, dims, q), dims, out_parity)
    rhs = O.spinor_gauge_transform(h, Lam[EO.cb_sites(dims, out_parity)])
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_clover_inverse_is_the_inverse():
    dims = (2, 2, 2, 4)
    U = synth.gauge_haar(dims, 21)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    M = O.unpack_hermitian6(A)
    Mi = O.unpack_hermitian6(EO.clover_inverse(A))
    np.testing.assert_allclose(M @ Mi, np.broadcast_to(np.eye(6), M.shape), atol=1e-13)
    np.testing.assert_allclose(Mi, np.conj(np.swapaxes(Mi, -1, -2)), atol=1e-15)
    # by hand: the inverse of 2 * identity
    two = np.zeros(36)
    two[:6] = 2.0
    np.testing.assert_allclose(EO.clover_inverse(two), np.r_[np.full(6, 0.5), np.zeros(30)], atol=1e-16)


def test_clover_cb_is_the_sites_block():
    dims = (2, 2, 2, 2)
    U = synth.gauge_haar(dims, 22)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    psi = synth.spinor_source(dims, 2, 23)
    for p in (0, 1):
        got = EO.clover_cb(A, EO.to_cb(psi, dims, p), dims, p)
        M = O.unpack_hermitian6(A)
        for i, s in enumerate(EO.cb_sites(dims, p)):
            want = np.concatenate([M[s, 0] @ psi[s, :6], M[s, 1] @ psi[s, 6:]])
            np.testing.assert_allclose(got[i], want, atol=1e-14)


def test_schur_system_against_full_solve():
    """4^4 Haar links, c_sw = 1: x from a sparse LU solve of the full D x = b satisfies
    Dhat x_e = b_e + kappa H_eo A_o^-1 b_o and x_o = A_o^-1 (b_o + kappa H_oe x_e)."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_haar(dims, 31)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    b = synth.spinor_source(dims, 1, 32)
    D = O.dwc_sparse(U, A, KAPPA, dims).tocsc()
    x = spla.spsolve(D, b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(O.dwc(U, A, KAPPA, x, dims) - b) < 1e-10 * np.linalg.norm(b)
    x_e, x_o = EO.to_cb(x, dims, 0), EO.to_cb(x, dims, 1)
    lhs = EO.schur_ee(U, A, KAPPA, x_e, dims)
    rhs = EO.schur_rhs(U, A, KAPPA, b, dims)
    assert np.linalg.norm(lhs - rhs) < 1e-11 * np.linalg.norm(rhs)
    Ai = EO.clover_inverse(A)
    x_o2 = EO.clover_cb(Ai, EO.to_cb(b, dims, 1) + KAPPA * EO.hop_eo(U, x_e, dims, 1), dims, 1)
    assert np.linalg.norm(x_o2 - x_o) < 1e-11 * np.linalg.norm(x_o)


def test_coarse_schur_against_dense_solve():
    """Gaussian 9-point stencil (+4 I on the self blocks) on a 4x2x2x2 coarse lattice,
    Nb = 8: x from a dense solve of D_c x = b satisfies the coarse Schur system."""
    cdims, nb = (4, 2, 2, 2), 8
    Vc = synth.volume(cdims)
    B = synth.gaussian_blocks(Vc, nb, 41)
    I = np.eye(Vc * nb).reshape(Vc * nb, Vc, nb).transpose(1, 2, 0)
    D = O.coarse_apply(B, I, cdims).reshape(Vc * nb, Vc * nb)
    b = synth.coarse_source(Vc, nb, 2, 42)
    x = np.linalg.solve(D, b.reshape(Vc * nb, 2)).reshape(b.shape)
    x_e = EO.to_cb(x, cdims, 0)
    lhs = EO.coarse_schur_ee(B, x_e, cdims)
    rhs = EO.coarse_schur_rhs(B, b, cdims)
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(rhs)
    Sinv = EO.coarse_self_inverse(B)
    x_o = EO.coarse_self_cb(Sinv, EO.to_cb(b, cdims, 1) - EO.coarse_hop_eo(B, x_e, cdims, 1), cdims, 1)
    assert np.linalg.norm(x_o - EO.to_cb(x, cdims, 1)) < 1e-12 * np.linalg.norm(x_o)


def test_coarse_hop_eo_by_hand():
    """One nonzero hop block: B_{+x} at site 0 of a 4x2x2x2 lattice couples e(site 1)
    into the output at site 0 (parity 0 <- parity 1); every other entry stays zero."""
    cdims, nb = (4, 2, 2, 2), 3
    Vc = synth.volume(cdims)
    B = np.zeros((Vc, 9, nb, nb), dtype=np.complex128)
    M = synth.gaussian_complex(synth.rng(5), (nb, nb))
    B[0, 1] = M  # direction +x at site 0
    B[:, 0] = np.eye(nb)  # self blocks do not enter the hop
    e = synth.coarse_source(Vc, nb, 1, 6)
    got = EO.coarse_hop_eo(B, EO.to_cb(e, cdims, 1), cdims, 0)
    want = np.zeros_like(got)
    i0 = int(np.where(EO.cb_sites(cdims, 0) == 0)[0][0])
    want[i0] = M @ e[1]
    np.testing.assert_allclose(got, want, atol=1e-14)
