"""Pins of the multigrid oracle: Galerkin coarse operator against dense brute
force, intergrid algebra, QR uniqueness of the block orthonormalisation,
coarse gamma5-hermiticity, and explicit-loop brute force for the stencil and
the restriction on tiny lattices."""

import numpy as np
import pytest

import oracle as O
import synth

KAPPA = 0.13


def _dense_fine(U, A, dims):
    V = synth.volume(dims)
    I = np.eye(V * 12).reshape(V * 12, V, 12).transpose(1, 2, 0)
    return O.dwc(U, A, KAPPA, I, dims).reshape(V * 12, V * 12)


def _dense_prolong(W, dims, block):
    Vc = synth.volume(O.coarse_dims(dims, block))
    nb = 2 * W.shape[1]
    I = np.eye(Vc * nb).reshape(Vc * nb, Vc, nb).transpose(1, 2, 0)
    return O.prolong(W, I, dims, block).reshape(W.shape[0] * W.shape[2], Vc * nb)


def _dense_coarse(B, cdims):
    Vc, _, nb, _ = B.shape
    I = np.eye(Vc * nb).reshape(Vc * nb, Vc, nb).transpose(1, 2, 0)
    return O.coarse_apply(B, I, cdims).reshape(Vc * nb, Vc * nb)


def _coords(dims):
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    return np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)


@pytest.mark.parametrize(
    "dims,block,nv",
    [
        ((4, 2, 2, 4), (2, 2, 1, 2), 3),  # coarse extents (2, 1, 2, 2): aliasing and self-wrap
        ((2, 4, 2, 6), (1, 2, 2, 2), 2),  # block extent 1 in x, coarse extent 3 in t
    ],
)
def test_galerkin_fine_vs_dense(dims, block, nv):
    U = synth.gauge_haar(dims, 1)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    W = O.block_orthonormalise(synth.gaussian_vectors(synth.volume(dims), nv, 12, 7), dims, block)
    B = O.galerkin_fine(U, A, KAPPA, W, dims, block)
    P = _dense_prolong(W, dims, block)
    want = P.conj().T @ _dense_fine(U, A, dims) @ P
    got = _dense_coarse(B, O.coarse_dims(dims, block))
    np.testing.assert_allclose(got, want, atol=1e-13)


@pytest.mark.slow
def test_galerkin_4444_to_2222():
    """The 4^4 -> 2^4 brute-force case (3072 x 3072 dense fine operator)."""
    dims, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 2
    U = synth.gauge_haar(dims, 12)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    W = O.block_orthonormalise(synth.gaussian_vectors(256, nv, 12, 13), dims, block)
    B = O.galerkin_fine(U, A, KAPPA, W, dims, block)
    P = _dense_prolong(W, dims, block)
    want = P.conj().T @ _dense_fine(U, A, dims) @ P
    np.testing.assert_allclose(_dense_coarse(B, (2, 2, 2, 2)), want, atol=1e-13)


def test_galerkin_coarse_vs_dense():
    """Second coarsening: P2^dag D_c P2 for a Gaussian stencil on a 4x2x2x4 level."""
    cdims, block2, nv2, nb = (4, 2, 2, 4), (2, 1, 2, 2), 2, 6
    Vc = synth.volume(cdims)
    B = synth.gaussian_blocks(Vc, nb, 3)
    W2 = O.block_orthonormalise(synth.gaussian_vectors(Vc, nv2, nb, 4), cdims, block2)
    B2 = O.galerkin_coarse(B, W2, cdims, block2)
    P2 = _dense_prolong(W2, cdims, block2)
    want = P2.conj().T @ _dense_coarse(B, cdims) @ P2
    np.testing.assert_allclose(_dense_coarse(B2, O.coarse_dims(cdims, block2)), want, atol=1e-12)


def test_coarse_apply_explicit_loops():
    """Stencil apply against a loop over sites with explicit neighbour indices."""
    cdims = (3, 2, 1, 4)
    Vc, nb = synth.volume(cdims), 4
    B = synth.gaussian_blocks(Vc, nb, 5)
    e = synth.coarse_source(Vc, nb, 2, 6)
    X = _coords(cdims)
    want = np.zeros_like(e)
    for A in range(Vc):
        want[A] += B[A, 0] @ e[A]
        for mu in range(4):
            for sgn, d in ((+1, 1 + 2 * mu), (-1, 2 + 2 * mu)):
                y = X[A].copy()
                y[mu] = (y[mu] + sgn) % cdims[mu]
                nbr = y[0] + cdims[0] * (y[1] + cdims[1] * (y[2] + cdims[2] * y[3]))
                want[A] += B[A, d] @ e[nbr]
    np.testing.assert_allclose(O.coarse_apply(B, e, cdims), want, atol=1e-13)


def test_restrict_prolong_explicit_loops():
    dims, block, nv = (4, 2, 2, 2), (2, 1, 2, 2), 2
    V = synth.volume(dims)
    W = synth.gaussian_vectors(V, nv, 12, 1)
    f = synth.spinor_source(dims, 2, 2)
    cd = O.coarse_dims(dims, block)
    X = _coords(dims)
    y = np.zeros((synth.volume(cd), 2 * nv, 2), dtype=complex)
    for s in range(V):
        c = X[s] // np.array(block)
        A = c[0] + cd[0] * (c[1] + cd[1] * (c[2] + cd[2] * c[3]))
        for chi in range(2):
            for i in range(nv):
                for comp in range(6 * chi, 6 * chi + 6):
                    y[A, chi * nv + i] += np.conj(W[s, i, comp]) * f[s, comp]
    np.testing.assert_allclose(O.restrict(W, f, dims, block), y, atol=1e-13)
    # prolong is the adjoint of restrict: <P e, f> = <e, R f>
    e = synth.coarse_source(synth.volume(cd), 2 * nv, 2, 3)
    lhs = O.dot(O.prolong(W, e, dims, block), f)
    rhs = O.dot(e, O.restrict(W, f, dims, block))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_intergrid_algebra():
    """R P = 1 on orthonormalised bases, P R is a projector."""
    dims, block, nv = (4, 2, 4, 2), (2, 2, 2, 2), 3
    W = O.block_orthonormalise(synth.gaussian_vectors(synth.volume(dims), nv, 12, 8), dims, block)
    P = _dense_prolong(W, dims, block)
    np.testing.assert_allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-14)
    PR = P @ P.conj().T
    np.testing.assert_allclose(PR @ PR, PR, atol=1e-14)


def test_block_orthonormalise_is_the_qr_factor():
    """Q^dag Q = 1 and Q^dag W upper triangular with positive real diagonal, per
    (aggregate, chirality): the conditions that fix the thin-QR Q uniquely."""
    dims, block, nv = (4, 2, 2, 2), (2, 2, 1, 2), 4
    V = synth.volume(dims)
    Wraw = synth.gaussian_vectors(V, nv, 12, 9)
    Q = O.block_orthonormalise(Wraw, dims, block)
    agg = O.aggregate_index(dims, block)
    for A in range(agg.max() + 1):
        sites = np.where(agg == A)[0]
        for chi in range(2):
            cs = slice(6 * chi, 6 * chi + 6)
            Wm = np.transpose(Wraw[sites][:, :, cs], (0, 2, 1)).reshape(-1, nv)
            Qm = np.transpose(Q[sites][:, :, cs], (0, 2, 1)).reshape(-1, nv)
            np.testing.assert_allclose(Qm.conj().T @ Qm, np.eye(nv), atol=1e-14)
            R = Qm.conj().T @ Wm
            np.testing.assert_allclose(np.tril(R, -1), 0, atol=1e-13)
            d = np.diag(R)
            assert np.all(d.real > 0)
            np.testing.assert_allclose(d.imag, 0, atol=1e-13)
            np.testing.assert_allclose(Qm @ R, Wm, atol=1e-13)


def test_block_normalise():
    dims, block = (4, 2, 2, 2), (2, 2, 2, 2)
    f = synth.spinor_source(dims, 3, 4)
    agg = O.aggregate_index(dims, block)
    f[agg == 1, 6:, 2] = 0  # one zero (aggregate, chirality, RHS) block
    g, norms = O.block_normalise(f, dims, block)
    for A in range(agg.max() + 1):
        for chi in range(2):
            blk = g[agg == A][:, 6 * chi:6 * chi + 6]
            n = np.sqrt(np.sum(np.abs(blk) ** 2, axis=(0, 1)))
            if A == 1 and chi == 1:
                assert n[2] == 0 and norms[A, chi, 2] == 0
                n = n[:2]
            np.testing.assert_allclose(n, 1.0, atol=1e-14)
    assert np.all(np.isfinite(g))


def test_coarse_gamma5_hermiticity():
    """gamma5 P = P Gamma5 implies B_{-mu}(A+mu) = G5 B_{+mu}(A)^dag G5 and a
    Gamma5-Hermitian self block, G5 = diag(+1_{n_v}, -1_{n_v})."""
    dims, block, nv = (4, 4, 2, 4), (2, 2, 2, 2), 2
    U = synth.gauge_haar(dims, 21)
    A = O.clover_packed(U, dims, 1.0, KAPPA)
    W = O.block_orthonormalise(synth.gaussian_vectors(synth.volume(dims), nv, 12, 22), dims, block)
    B = O.galerkin_fine(U, A, KAPPA, W, dims, block)
    cd = O.coarse_dims(dims, block)
    G5 = np.diag([1.0] * nv + [-1.0] * nv)
    X = _coords(cd)
    for Ac in range(synth.volume(cd)):
        np.testing.assert_allclose(G5 @ B[Ac, 0].conj().T @ G5, B[Ac, 0], atol=1e-14)
        for mu in range(4):
            y = X[Ac].copy()
            y[mu] = (y[mu] + 1) % cd[mu]
            An = y[0] + cd[0] * (y[1] + cd[1] * (y[2] + cd[2] * y[3]))
            np.testing.assert_allclose(
                B[An, 2 + 2 * mu], G5 @ B[Ac, 1 + 2 * mu].conj().T @ G5, atol=1e-14
            )


def test_block_orthonormalise_flags_rank_deficiency():
    import pytest

    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    v = synth.gaussian_vectors(synth.volume(dims), 4, 12, 5)
    v[:, 3] = v[:, 1]
    with pytest.raises(np.linalg.LinAlgError):
        O.block_orthonormalise(v, dims, block)
