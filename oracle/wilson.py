"""Fine-level Wilson-clover operator in FP64 (paper Sec. 4: hopping term D_hop
and clover term M_ooee on the fine level).

Definitions (standard; the paper prints none):

  Hopping term (Wilson parameter r = 1)
      (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                          + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]
  with links periodic and the fermion field antiperiodic in time when
  t_bc = -1: a hop that wraps around the t boundary (either way) is
  multiplied by t_bc.

  Clover field strength from the four plaquette leaves in the mu-nu plane
  around x,   F_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / 8.

  kappa-normalised operator
      D = 1 - kappa H + C,  C(x) = i c_sw kappa sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x),
  and the mass-normalised D_m = D / (2 kappa), kappa = 1 / (2 (4 + m0)).

Array layout: psi (V, 12, N), U (V, 4, 3, 3), site s = x + Lx*(y + Ly*(z + Lz*t)).
"""

from __future__ import annotations

import numpy as np

from .conventions import chiral_sigma_blocks, gamma_matrices, sigma_munu

# lattice axis of direction mu once a (V, ...) array is viewed as (Lt, Lz, Ly, Lx, ...)
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def _lat(f: np.ndarray, dims) -> np.ndarray:
    Lx, Ly, Lz, Lt = dims
    return f.reshape((Lt, Lz, Ly, Lx) + f.shape[1:])


def _flat(f: np.ndarray) -> np.ndarray:
    return f.reshape((-1,) + f.shape[4:])


def _shift(f_lat: np.ndarray, mu: int, step: int, t_bc: float = 1.0) -> np.ndarray:
    """g(x) = f(x + step*mu) on the lattice view, with the t-boundary factor applied
    to values that wrapped around in the time direction."""
    g = np.roll(f_lat, -step, axis=_AXIS[mu])
    if mu == 3 and t_bc != 1.0:
        g = g.copy()
        if step > 0:
            g[-step:] *= t_bc
        else:
            g[:(-step)] *= t_bc
    return g


def _dag(M: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(M, -1, -2))


def _spin_colour(psi: np.ndarray) -> np.ndarray:
    """(V, 12, N) -> (V, 4, 3, N)."""
    return psi.reshape(psi.shape[0], 4, 3, psi.shape[-1])


def _hop_terms(U, psi, dims, t_bc, mask_fwd=None, mask_bwd=None):
    """Sum of hopping contributions, optionally masked per direction.

    mask_fwd[mu] / mask_bwd[mu] are boolean site masks (V,) that keep the
    forward / backward hop into site x; None keeps all sites.
    """
    g = gamma_matrices()
    I4 = np.eye(4)
    U = np.asarray(U, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    ps = _spin_colour(psi)
    out = np.zeros_like(ps)
    for mu in range(4):
        Umu = U[:, mu]
        # forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
        fwd = _flat(_shift(_lat(ps, dims), mu, +1, t_bc))
        t = np.einsum("vab,vsbn->vsan", Umu, fwd)
        t = np.einsum("st,vtan->vsan", I4 - g[mu], t)
        if mask_fwd is not None:
            t = t * mask_fwd[mu][:, None, None, None]
        out += t
        # backward: (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
        w = np.einsum("vba,vsbn->vsan", Umu.conj(), ps)
        bwd = _flat(_shift(_lat(w, dims), mu, -1, t_bc))
        t = np.einsum("st,vtan->vsan", I4 + g[mu], bwd)
        if mask_bwd is not None:
            t = t * mask_bwd[mu][:, None, None, None]
        out += t
    return out.reshape(psi.shape)


def hop(U: np.ndarray, psi: np.ndarray, dims, t_bc: float = -1.0) -> np.ndarray:
    """H psi for psi of shape (V, 12, N) (paper Sec. 4, D_hop)."""
    return _hop_terms(U, psi, dims, t_bc)


def hop_dir(U, psi, dims, t_bc, sign: int, mu: int, block) -> np.ndarray:
    """Direction-resolved hop used by the Galerkin construction.

    sign=+1: only the forward hops into x whose source x+mu lies in the next
    aggregate along +mu (x_mu % b_mu == b_mu - 1); sign=-1: only backward hops
    whose source lies in the previous aggregate (x_mu % b_mu == 0); sign=0:
    all hops that stay inside x's aggregate.
    """
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    s = np.arange(V)
    coord = [s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)]
    on_fwd_face = [coord[m] % block[m] == block[m] - 1 for m in range(4)]
    on_bwd_face = [coord[m] % block[m] == 0 for m in range(4)]
    zero = np.zeros(V, dtype=bool)
    if sign == 0:
        mf = [~on_fwd_face[m] for m in range(4)]
        mb = [~on_bwd_face[m] for m in range(4)]
    elif sign > 0:
        mf = [on_fwd_face[m] if m == mu else zero for m in range(4)]
        mb = [zero] * 4
    else:
        mf = [zero] * 4
        mb = [on_bwd_face[m] if m == mu else zero for m in range(4)]
    return _hop_terms(U, psi, dims, t_bc, mf, mb)


def plaquette_leaves(U: np.ndarray, dims, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x): sum of the four mu-nu plaquettes that start and end at x,
    all traversed in the same (mu then nu) sense.  Shape (V, 3, 3)."""
    Um = _lat(U[:, mu], dims)
    Un = _lat(U[:, nu], dims)
    s = _shift
    L1 = Um @ s(Un, mu, +1) @ _dag(s(Um, nu, +1)) @ _dag(Un)
    L2 = Un @ _dag(s(s(Um, mu, -1), nu, +1)) @ _dag(s(Un, mu, -1)) @ s(Um, mu, -1)
    L3 = _dag(s(Um, mu, -1)) @ _dag(s(s(Un, mu, -1), nu, -1)) @ s(s(Um, mu, -1), nu, -1) @ s(Un, nu, -1)
    L4 = _dag(s(Un, nu, -1)) @ s(Um, nu, -1) @ s(s(Un, mu, +1), nu, -1) @ _dag(Um)
    return _flat(L1 + L2 + L3 + L4)


def field_strength(U: np.ndarray, dims) -> dict:
    """F_{mu nu}(x) = (Q - Q^dag)/8 for mu < nu; anti-Hermitian, no trace removed."""
    F = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Q = plaquette_leaves(U, dims, mu, nu)
            F[(mu, nu)] = (Q - _dag(Q)) / 8.0
    return F


def clover_dense(U, dims, csw: float, kappa: float) -> np.ndarray:
    """A(x) = 1 + i c_sw kappa sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x) as (V, 12, 12).

    Route (i): full 4x4 sigma matrices built from gamma products, Kronecker
    product with the colour matrix, index 3*spin + colour.
    """
    F = field_strength(U, dims)
    V = U.shape[0]
    A = np.zeros((V, 12, 12), dtype=np.complex128)
    for (mu, nu), Fm in F.items():
        s = sigma_munu(mu, nu)
        A += np.einsum("st,vab->vsatb", s, Fm).reshape(V, 12, 12)
    A *= 1j * csw * kappa
    A += np.eye(12)
    return A


def pack_hermitian6(M: np.ndarray) -> np.ndarray:
    """Pack Hermitian 6x6 matrices (..., 6, 6) into 36 reals: the 6 real diagonal
    entries, then the 15 strictly-lower entries in row-major order as (re, im)."""
    out = np.empty(M.shape[:-2] + (36,), dtype=np.float64)
    for i in range(6):
        out[..., i] = M[..., i, i].real
    k = 6
    for i in range(6):
        for j in range(i):
            out[..., k] = M[..., i, j].real
            out[..., k + 1] = M[..., i, j].imag
            k += 2
    return out


def unpack_hermitian6(p: np.ndarray) -> np.ndarray:
    M = np.zeros(p.shape[:-1] + (6, 6), dtype=np.complex128)
    for i in range(6):
        M[..., i, i] = p[..., i]
    k = 6
    for i in range(6):
        for j in range(i):
            z = p[..., k] + 1j * p[..., k + 1]
            M[..., i, j] = z
            M[..., j, i] = np.conj(z)
            k += 2
    return M


def clover_packed(U, dims, csw, kappa) -> np.ndarray:
    """Packed chiral blocks (V, 2, 36) sliced out of the dense route (i)."""
    A = clover_dense(U, dims, csw, kappa)
    return np.stack([pack_hermitian6(A[:, :6, :6]), pack_hermitian6(A[:, 6:, 6:])], axis=1)


def clover_packed_direct(U, dims, csw, kappa) -> np.ndarray:
    """Packed chiral blocks (V, 2, 36), route (ii): each 6x6 block is assembled
    from the explicit 2x2 chiral pieces of sigma_{mu nu} (Pauli algebra), with
    no 4x4 gamma matrix involved."""
    F = field_strength(U, dims)
    V = U.shape[0]
    blocks = [np.zeros((V, 6, 6), dtype=np.complex128) for _ in range(2)]
    for (mu, nu), Fm in F.items():
        bp, bm = chiral_sigma_blocks(mu, nu)
        for chi, b in enumerate((bp, bm)):
            blocks[chi] += np.einsum("st,vab->vsatb", b, Fm).reshape(V, 6, 6)
    out = []
    for chi in range(2):
        Ab = 1j * csw * kappa * blocks[chi] + np.eye(6)
        out.append(pack_hermitian6(Ab))
    return np.stack(out, axis=1)


def clover_apply(Apacked: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """A psi with A given as packed chiral blocks (V, 2, 36); psi (V, 12, N)."""
    M = unpack_hermitian6(np.asarray(Apacked, dtype=np.float64))  # (V, 2, 6, 6)
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    out[:, :6] = np.einsum("vij,vjn->vin", M[:, 0], psi[:, :6])
    out[:, 6:] = np.einsum("vij,vjn->vin", M[:, 1], psi[:, 6:])
    return out


def dwc(U, Apacked, kappa, psi, dims, t_bc=-1.0) -> np.ndarray:
    """D psi = A psi - kappa H psi, with A = 1 + C (paper Sec. 4, D_hop plus M_ooee)."""
    return clover_apply(Apacked, psi) - kappa * hop(U, psi, dims, t_bc)


def dwc_mass(U, Apacked, kappa, psi, dims, t_bc=-1.0) -> np.ndarray:
    """Mass-normalised D_m psi = D psi / (2 kappa)."""
    return dwc(U, Apacked, kappa, psi, dims, t_bc) / (2.0 * kappa)


def gauge_transform(U: np.ndarray, Lam: np.ndarray, dims) -> np.ndarray:
    """U^Lambda_mu(x) = Lambda(x) U_mu(x) Lambda(x + mu)^dag (links periodic)."""
    out = np.empty_like(U)
    Ll = _lat(Lam, dims)
    for mu in range(4):
        Lp = _flat(_shift(Ll, mu, +1))
        out[:, mu] = Lam @ U[:, mu] @ _dag(Lp)
    return out


def spinor_gauge_transform(psi: np.ndarray, Lam: np.ndarray) -> np.ndarray:
    """(Lambda psi)(x): colour rotation of every spin component."""
    ps = _spin_colour(psi)
    return np.einsum("vab,vsbn->vsan", Lam, ps).reshape(psi.shape)


def dwc_sites(U, Apacked, kappa, psi, dims, sites, t_bc=-1.0) -> np.ndarray:
    """(D psi)(x) at the listed sites only, shape (len(sites), 12, N).

    Same definition as dwc(), evaluated by gathering the eight neighbours of
    each requested site explicitly; used to check outputs of lattices too
    large for a whole-lattice FP64 apply.
    """
    Lx, Ly, Lz, Lt = dims
    L = np.array(dims)
    stride = np.array([1, Lx, Lx * Ly, Lx * Ly * Lz])
    sites = np.asarray(sites)
    X = np.stack([sites % Lx, (sites // Lx) % Ly, (sites // (Lx * Ly)) % Lz, sites // (Lx * Ly * Lz)], axis=1)
    g = gamma_matrices()
    I4 = np.eye(4)
    N = psi.shape[-1]
    acc = np.zeros((len(sites), 4, 3, N), dtype=np.complex128)
    for mu in range(4):
        for sgn in (+1, -1):
            Y = X.copy()
            Y[:, mu] = (Y[:, mu] + sgn) % L[mu]
            nb = Y @ stride
            wrapped = (X[:, mu] == L[mu] - 1) if sgn > 0 else (X[:, mu] == 0)
            ph = np.where(wrapped & (mu == 3), t_bc, 1.0)
            p = np.asarray(psi[nb], dtype=np.complex128).reshape(len(sites), 4, 3, N)
            if sgn > 0:
                link = np.asarray(U[sites, mu], dtype=np.complex128)
                proj = I4 - g[mu]
            else:
                link = np.conj(np.swapaxes(np.asarray(U[nb, mu], dtype=np.complex128), -1, -2))
                proj = I4 + g[mu]
            t = np.einsum("vab,vsbn->vsan", link, p)
            acc += ph[:, None, None, None] * np.einsum("st,vtan->vsan", proj, t)
    A_here = np.asarray(Apacked[sites], dtype=np.float64)
    here = np.asarray(psi[sites], dtype=np.complex128)
    return clover_apply(A_here, here) - kappa * acc.reshape(len(sites), 12, N)
