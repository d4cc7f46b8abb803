"""Conventions the oracle fixes where the paper is silent.

The paper does not print its Dirac operator (Sec. 2 and Sec. 4 only name the
hopping and clover terms), so the standard lattice definitions are adopted:

* Euclidean, Hermitian gamma matrices in the chiral basis,
  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3),
  gamma_4 = [[0, 1], [1, 0]], gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).
  In this basis sigma_{mu nu} commutes with gamma_5 and is block diagonal, so
  the clover term splits into two 6x6 chiral blocks.
* sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu].
* Direction index mu = 0..3 is x, y, z, t (gamma_{mu+1} belongs to mu).
* Coarse-stencil direction order d = (self, +x, -x, +y, -y, +z, -z, +t, -t).
"""

from __future__ import annotations

import numpy as np

PAULI = np.array(
    [
        [[0, 1], [1, 0]],
        [[0, -1j], [1j, 0]],
        [[1, 0], [0, -1]],
    ],
    dtype=np.complex128,
)

# (sign, mu) for the nine coarse-stencil directions; sign 0 marks the self term.
DIRS = [(0, -1), (+1, 0), (-1, 0), (+1, 1), (-1, 1), (+1, 2), (-1, 2), (+1, 3), (-1, 3)]


def dir_index(sign: int, mu: int) -> int:
    """Position of direction (sign, mu) in DIRS."""
    if sign == 0:
        return 0
    return 1 + 2 * mu + (0 if sign > 0 else 1)


def gamma_matrices() -> np.ndarray:
    """Array g[0..4] = gamma_1, gamma_2, gamma_3, gamma_4, gamma_5 (4x4, chiral basis)."""
    Z = np.zeros((2, 2), dtype=np.complex128)
    I2 = np.eye(2, dtype=np.complex128)
    g = np.zeros((5, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k] = np.block([[Z, -1j * PAULI[k]], [1j * PAULI[k], Z]])
    g[3] = np.block([[Z, I2], [I2, Z]])
    g[4] = g[0] @ g[1] @ g[2] @ g[3]
    return g


def sigma_munu(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] as a 4x4 matrix."""
    g = gamma_matrices()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def chiral_sigma_blocks(mu: int, nu: int):
    """The two 2x2 diagonal blocks (chirality +, -) of sigma_{mu nu}, mu < nu.

    Written directly from the Pauli algebra rather than from the 4x4 gamma
    products (this is the second, independent route to the clover term):
    for spatial j < k, gamma_j gamma_k = diag(s_j s_k, s_j s_k), hence
    sigma_{jk} = -eps_{jkl} s_l on both chiralities; for k < 4,
    [gamma_k, gamma_4] = diag(-2i s_k, 2i s_k), hence sigma_{k4} = diag(s_k, -s_k).
    """
    assert 0 <= mu < nu <= 3
    if nu == 3:
        s = PAULI[mu]
        return s.copy(), -s
    l = 3 - mu - nu  # the remaining spatial index
    eps = 1.0 if (mu, nu, l) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1.0
    b = -eps * PAULI[l]
    return b.copy(), b.copy()
