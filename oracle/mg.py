"""Aggregation multigrid pieces in FP64 (paper Sec. 5 intergrid operators and
Sec. 6 coarse-level operator).

Definitions (standard aggregation MG; the paper gives the sizes, not the
formulas).  A level holds fields f of shape (V, ncomp, N).  Aggregates are
blocks b = (bx, by, bz, bt) of sites; aggregate index
A = X + Cx*(Y + Cy*(Z + Cz*T)) with X = x // bx etc.  The two chiralities of
a level are the first and second halves of its components (spinor components
0..5 and 6..11 on the fine level).  Given n_v basis vectors v_i (V, n_v, ncomp),
the prolongator P maps a coarse field with Nb = 2 n_v components per
aggregate, index chi*n_v + i, to

    (P y)(x)_c = sum_i v_i(x)_c y(A(x), chi(c)*n_v + i),

the restriction is R = P^dag, and the coarse operator is the Galerkin
product D_c = P^dag D P, stored as a 9-point stencil of dense Nb x Nb blocks
B_d(A), d in (self, +x, -x, +y, -y, +z, -z, +t, -t):

    (D_c e)(A) = sum_d B_d(A) e(A + d).

B_{+mu}(A) collects only the couplings through fine hops that cross the +mu
face of A, so when a coarse extent is 2 (A + mu == A - mu) the two blocks
stay distinct, and when it is 1 both act on A itself.
"""

from __future__ import annotations

import numpy as np

from .conventions import DIRS, dir_index
from .wilson import clover_apply, hop_dir


def coarse_dims(dims, block):
    for L, b in zip(dims, block):
        if L % b:
            raise ValueError(f"block {block} does not divide lattice {dims}")
    return tuple(L // b for L, b in zip(dims, block))


def aggregate_index(dims, block) -> np.ndarray:
    """Aggregate A(x) of every site x, shape (V,)."""
    Lx, Ly, Lz, Lt = dims
    Cx, Cy, Cz, Ct = coarse_dims(dims, block)
    s = np.arange(Lx * Ly * Lz * Lt)
    x, y, z, t = s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)
    X, Y, Z, T = x // block[0], y // block[1], z // block[2], t // block[3]
    return X + Cx * (Y + Cy * (Z + Cz * T))


def _agg_sites(dims, block):
    """Sites of each aggregate, shape (Vc, sites_per_aggregate), in site order."""
    agg = aggregate_index(dims, block)
    order = np.argsort(agg, kind="stable")
    nper = int(np.prod(block))
    return order.reshape(-1, nper)


def block_orthonormalise(vecs: np.ndarray, dims, block) -> np.ndarray:
    """Orthonormalise n_v vectors per (aggregate, chirality).

    For every aggregate A and chirality chi, the restrictions w_i = P_chi v_i|_A
    (i = 1..n_v, in order) are replaced by the Q factor of their thin QR
    decomposition W = Q R with real positive diag(R); that Q is unique, so any
    Gram-Schmidt ordering reproduces it up to rounding.  Raises LinAlgError when
    some |R_ii| <= 1e-10 |w_i| (a numerically rank-deficient block).
    """
    V, n_v, ncomp = vecs.shape
    h = ncomp // 2
    sites = _agg_sites(dims, block)
    out = np.empty_like(vecs, dtype=np.complex128)
    for chi in range(2):
        cs = slice(chi * h, (chi + 1) * h)
        # W[A] : (sites*h, n_v)
        W = vecs[sites][:, :, :, cs]  # (Vc, nper, n_v, h)
        W = np.transpose(W, (0, 1, 3, 2)).reshape(sites.shape[0], -1, n_v)
        Q, R = np.linalg.qr(W)
        d = np.diagonal(R, axis1=-2, axis2=-1)
        # rank deficiency: |R_ii| (the part of w_i not spanned by w_0..w_{i-1})
        # below 1e-10 |w_i|
        if np.any(np.abs(d) <= 1e-10 * np.linalg.norm(W, axis=1)):
            raise np.linalg.LinAlgError("rank-deficient aggregate")
        Q = Q * (d / np.abs(d))[:, None, :]
        Q = Q.reshape(sites.shape[0], sites.shape[1], h, n_v).transpose(0, 1, 3, 2)
        tmp = np.empty((V, n_v, h), dtype=np.complex128)
        tmp[sites.reshape(-1)] = Q.reshape(-1, n_v, h)
        out[:, :, cs] = tmp
    return out


def restrict(basis: np.ndarray, f: np.ndarray, dims, block) -> np.ndarray:
    """y = P^dag f (paper Sec. 5, project): y(A, chi*n_v + i) = sum_{x in A, c in chi}
    conj(v_i(x)_c) f(x)_c.  basis (V, n_v, ncomp), f (V, ncomp, N) -> (Vc, 2 n_v, N)."""
    V, n_v, ncomp = basis.shape
    h = ncomp // 2
    agg = aggregate_index(dims, block)
    Vc = int(agg.max()) + 1
    N = f.shape[-1]
    y = np.zeros((Vc, 2 * n_v, N), dtype=np.complex128)
    for chi in range(2):
        cs = slice(chi * h, (chi + 1) * h)
        per_site = np.einsum("vic,vcn->vin", basis[:, :, cs].conj(), f[:, cs])
        part = np.zeros((Vc, n_v, N), dtype=np.complex128)
        np.add.at(part, agg, per_site)
        y[:, chi * n_v:(chi + 1) * n_v] = part
    return y


def prolong(basis: np.ndarray, y: np.ndarray, dims, block) -> np.ndarray:
    """f = P y (paper Sec. 5, promote): f(x)_c = sum_i v_i(x)_c y(A(x), chi(c)*n_v + i)."""
    V, n_v, ncomp = basis.shape
    h = ncomp // 2
    agg = aggregate_index(dims, block)
    N = y.shape[-1]
    f = np.zeros((V, ncomp, N), dtype=np.complex128)
    for chi in range(2):
        cs = slice(chi * h, (chi + 1) * h)
        yc = y[agg, chi * n_v:(chi + 1) * n_v]  # (V, n_v, N)
        f[:, cs] = np.einsum("vic,vin->vcn", basis[:, :, cs], yc)
    return f


def block_normalise(f: np.ndarray, dims, block):
    """Divide every (RHS, aggregate, chirality) block of f by its 2-norm; a zero
    block stays zero.  Lower-precision inputs are widened to FP64 before the
    norms are formed.  Returns (normalised field, norms (Vc, 2, N))."""
    V, ncomp, N = f.shape
    h = ncomp // 2
    f = np.asarray(f).astype(np.complex128)  # widen before squaring, as for inner products
    agg = aggregate_index(dims, block)
    Vc = int(agg.max()) + 1
    out = np.empty_like(f, dtype=np.complex128)
    norms = np.zeros((Vc, 2, N))
    for chi in range(2):
        cs = slice(chi * h, (chi + 1) * h)
        sq = np.sum(np.abs(f[:, cs]) ** 2, axis=1)  # (V, N)
        tot = np.zeros((Vc, N))
        np.add.at(tot, agg, sq)
        nrm = np.sqrt(tot)
        norms[:, chi] = nrm
        scale = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 0.0)
        out[:, cs] = f[:, cs] * scale[agg][:, None, :]
    return out, norms


def _galerkin(apply_dir, basis, dims, block):
    """Blocks B_d(A) = sum_{x in A} W(x)^dag (D_d W)(x) for every direction d, by
    applying the direction-resolved operator D_d to every chirality-projected
    basis column and restricting the result."""
    V, n_v, ncomp = basis.shape
    h = ncomp // 2
    nb = 2 * n_v
    # columns: W_{chi, j} = P_chi v_j as fields (V, ncomp), stacked as N = nb RHS
    cols = np.zeros((V, ncomp, nb), dtype=np.complex128)
    for chi in range(2):
        cs = slice(chi * h, (chi + 1) * h)
        cols[:, cs, chi * n_v:(chi + 1) * n_v] = np.transpose(basis[:, :, cs], (0, 2, 1))
    Vc = int(np.prod(coarse_dims(dims, block)))
    B = np.zeros((Vc, 9, nb, nb), dtype=np.complex128)
    for d, (sign, mu) in enumerate(DIRS):
        B[:, d] = restrict(basis, apply_dir(sign, mu, cols), dims, block)
    return B


def galerkin_fine(U, Apacked, kappa, basis, dims, block, t_bc=-1.0) -> np.ndarray:
    """Coarse stencil blocks (Vc, 9, Nb, Nb) of P^dag D P for the fine kappa-form D."""

    def apply_dir(sign, mu, f):
        if sign == 0:
            return clover_apply(Apacked, f) - kappa * hop_dir(U, f, dims, t_bc, 0, -1, block)
        return -kappa * hop_dir(U, f, dims, t_bc, sign, mu, block)

    return _galerkin(apply_dir, basis, dims, block)


def coarse_apply_dir(B, e, dims, sign, mu, block=None):
    """Direction-resolved coarse stencil on a lattice of extent dims.

    With block=None the full direction term B_d(A) e(A + d) is returned.  With
    a block (used when this level is coarsened again), sign=0 returns the self
    block plus every hop that stays inside the aggregate of the next level,
    and sign=+-1 only the hops that cross that aggregate's +-mu face.
    """
    from .wilson import _flat, _lat, _shift

    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    s = np.arange(V)
    coord = [s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)]

    def term(sg, m):
        d = dir_index(sg, m)
        if sg == 0:
            src = e
        else:
            src = _flat(_shift(_lat(e, dims), m, sg))
        return np.einsum("vij,vjn->vin", B[:, d], src)

    if block is None:
        return term(sign, mu)
    out = np.zeros(e.shape, dtype=np.complex128)
    if sign == 0:
        out += term(0, -1)
        for m in range(4):
            fwd_face = coord[m] % block[m] == block[m] - 1
            bwd_face = coord[m] % block[m] == 0
            out += term(+1, m) * (~fwd_face)[:, None, None]
            out += term(-1, m) * (~bwd_face)[:, None, None]
    elif sign > 0:
        face = coord[mu] % block[mu] == block[mu] - 1
        out += term(+1, mu) * face[:, None, None]
    else:
        face = coord[mu] % block[mu] == 0
        out += term(-1, mu) * face[:, None, None]
    return out


def coarse_apply(B: np.ndarray, e: np.ndarray, dims) -> np.ndarray:
    """(D_c e)(A) = sum_d B_d(A) e(A + d), periodic, no boundary phase (paper Sec. 6).
    B (Vc, 9, Nb, Nb), e (Vc, Nb, N)."""
    e = np.asarray(e, dtype=np.complex128)
    out = np.zeros(e.shape, dtype=np.complex128)
    for sign, mu in DIRS:
        out += coarse_apply_dir(B, e, dims, sign, mu)
    return out


def galerkin_coarse(B, basis, dims, block) -> np.ndarray:
    """Blocks of the next coarser level, P^dag D_c P, for a stencil operator B on
    a lattice of extent dims blocked by block."""

    def apply_dir(sign, mu, f):
        return coarse_apply_dir(B, f, dims, sign, mu, block)

    return _galerkin(apply_dir, basis, dims, block)
