"""Even-odd (checkerboard) pieces of the fine operator in FP64 (paper Sec. 4:
M_eooe, the hopping term between the two checkerboarded lattices, and
M_ooee, the clover term on one checkerboard), the inverse of the clover
term, and the Schur complement they form.

TEST INFRASTRUCTURE: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module (see the package
docstring).

Definitions (standard; the paper names the operators but prints no formula):

  parity p(x) = (x + y + z + t) mod 2.  With all extents even, every hop
  joins sites of opposite parity, so with fields split as (psi_e, psi_o)

      D = [[ A_e        , -kappa H_eo ],
           [ -kappa H_oe, A_o         ]],

  where H_pq = (H restricted to output parity p and input parity q) is
  M_eooe and A_p (the clover blocks on parity p) is M_ooee.  Eliminating the
  odd sites gives the Schur complement on the even sites

      Dhat psi_e = A_e psi_e - kappa^2 H_eo A_o^-1 H_oe psi_e,

  and D x = b is equivalent to Dhat x_e = b_e + kappa H_eo A_o^-1 b_o,
  x_o = A_o^-1 (b_o + kappa H_oe x_e).

Checkerboard layout: with Lx even the sites s = 2i and s = 2i + 1 have
opposite parity; a field on parity p is stored as (V/2, 12, N) whose entry i
is the one of those two sites that has parity p.
"""

from __future__ import annotations

import numpy as np

from .wilson import hop, pack_hermitian6, unpack_hermitian6, clover_apply


def parity(dims) -> np.ndarray:
    """p(x) = (x + y + z + t) mod 2 for every site s (lexicographic, x fastest)."""
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    x, y, z, t = s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)
    return (x + y + z + t) % 2


def cb_sites(dims, p: int) -> np.ndarray:
    """Full-lattice site of every checkerboard index i on parity p."""
    if dims[0] % 2:
        raise ValueError("the checkerboard layout needs an even x extent")
    par = parity(dims)
    pair = np.arange(par.size // 2)
    first = 2 * pair
    return np.where(par[first] == p, first, first + 1)


def to_cb(f: np.ndarray, dims, p: int) -> np.ndarray:
    """Full-lattice field (V, ...) -> its parity-p part (V/2, ...)."""
    return np.asarray(f)[cb_sites(dims, p)]


def from_cb(fe: np.ndarray, fo: np.ndarray, dims) -> np.ndarray:
    """Even and odd parts -> the full-lattice field."""
    out = np.empty((2 * fe.shape[0],) + fe.shape[1:], dtype=np.result_type(fe, fo))
    out[cb_sites(dims, 0)] = fe
    out[cb_sites(dims, 1)] = fo
    return out


def hop_eo(U, psi_cb, dims, out_parity: int, t_bc: float = -1.0) -> np.ndarray:
    """M_eooe: H_{p,1-p} psi for psi given on parity 1 - p, result on parity p.
    The definition written out: place psi on its sites of the full lattice
    (zeros elsewhere), apply the full hopping term, keep the parity-p sites."""
    V = int(np.prod(dims))
    psi_cb = np.asarray(psi_cb, dtype=np.complex128)
    full = np.zeros((V,) + psi_cb.shape[1:], dtype=np.complex128)
    full[cb_sites(dims, 1 - out_parity)] = psi_cb
    return hop(U, full, dims, t_bc)[cb_sites(dims, out_parity)]


def clover_cb(Apacked, psi_cb, dims, p: int) -> np.ndarray:
    """M_ooee: the clover blocks of the parity-p sites applied to psi on parity p."""
    return clover_apply(np.asarray(Apacked)[cb_sites(dims, p)], psi_cb)


def clover_inverse(Apacked) -> np.ndarray:
    """Packed inverses (..., 2, 36) of the Hermitian 6x6 chiral blocks, by
    numpy's dense inverse of each block."""
    M = unpack_hermitian6(np.asarray(Apacked, dtype=np.float64))
    return pack_hermitian6(np.linalg.inv(M))


def schur_ee(U, Apacked, kappa: float, psi_e, dims, t_bc: float = -1.0) -> np.ndarray:
    """Dhat psi_e = A_e psi_e - kappa^2 H_eo A_o^-1 H_oe psi_e on the even sites."""
    Ainv = clover_inverse(Apacked)
    h_o = hop_eo(U, psi_e, dims, 1, t_bc)
    g_o = clover_cb(Ainv, h_o, dims, 1)
    return clover_cb(Apacked, psi_e, dims, 0) - kappa**2 * hop_eo(U, g_o, dims, 0, t_bc)


def schur_rhs(U, Apacked, kappa: float, b, dims, t_bc: float = -1.0) -> np.ndarray:
    """b_e + kappa H_eo A_o^-1 b_o: the even-site right-hand side of the Schur system."""
    Ainv = clover_inverse(Apacked)
    b_o = to_cb(b, dims, 1)
    return to_cb(b, dims, 0) + kappa * hop_eo(U, clover_cb(Ainv, b_o, dims, 1), dims, 0, t_bc)


# ---- coarse level (paper Sec. 6: the coarse-level M_eooe) ------------------------------
# With all coarse extents even the 9-point stencil splits the same way,
#     D_c = [[ S_e , H_eo ],
#            [ H_oe, S_o  ]],
# S the self blocks B_self of one parity and H the eight hop directions; the
# Schur complement on the even sites is S_e - H_eo S_o^-1 H_oe, and D_c x = b
# is equivalent to (S_e - H_eo S_o^-1 H_oe) x_e = b_e - H_eo S_o^-1 b_o,
# x_o = S_o^-1 (b_o - H_oe x_e).


def coarse_hop_eo(B, e_cb, dims, out_parity: int) -> np.ndarray:
    """The eight hop directions of the coarse stencil B (Vc, 9, Nb, Nb) from parity
    1 - p to parity p: place e on its sites, apply the stencil without its self
    blocks, keep the parity-p sites."""
    from .mg import coarse_apply

    Bh = np.array(B, dtype=np.complex128, copy=True)
    Bh[:, 0] = 0.0
    V = int(np.prod(dims))
    e_cb = np.asarray(e_cb, dtype=np.complex128)
    full = np.zeros((V,) + e_cb.shape[1:], dtype=np.complex128)
    full[cb_sites(dims, 1 - out_parity)] = e_cb
    return coarse_apply(Bh, full, dims)[cb_sites(dims, out_parity)]


def coarse_self_inverse(B) -> np.ndarray:
    """Inverses (Vc, Nb, Nb) of the self blocks B[:, 0], by numpy's dense inverse."""
    return np.linalg.inv(np.asarray(B, dtype=np.complex128)[:, 0])


def coarse_self_cb(S, e_cb, dims, p: int) -> np.ndarray:
    """Per-site blocks S (Vc, Nb, Nb) of the parity-p sites applied to e on parity p."""
    return np.einsum("vij,vjn->vin", np.asarray(S)[cb_sites(dims, p)], np.asarray(e_cb, dtype=np.complex128))


def coarse_schur_ee(B, e_e, dims) -> np.ndarray:
    """(S_e - H_eo S_o^-1 H_oe) e_e on the even coarse sites."""
    B = np.asarray(B, dtype=np.complex128)
    Sinv = coarse_self_inverse(B)
    g = coarse_self_cb(Sinv, coarse_hop_eo(B, e_e, dims, 1), dims, 1)
    return coarse_self_cb(B[:, 0], e_e, dims, 0) - coarse_hop_eo(B, g, dims, 0)


def coarse_schur_rhs(B, b, dims) -> np.ndarray:
    """b_e - H_eo S_o^-1 b_o."""
    B = np.asarray(B, dtype=np.complex128)
    g = coarse_self_cb(coarse_self_inverse(B), to_cb(b, dims, 1), dims, 1)
    return to_cb(b, dims, 0) - coarse_hop_eo(B, g, dims, 0)
