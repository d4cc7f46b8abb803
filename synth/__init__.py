"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and nothing else: gauge links, sources and
basis vectors for the Wilson-clover MRHS workloads.  It holds none of the
operator arithmetic (no hopping term, clover term, restriction or Galerkin
product), so the CPU oracle and the HIP path can both take their inputs from
here without sharing any code of the method.

Layouts (site index s = x + Lx*(y + Ly*(z + Lz*t))):
  gauge   : complex array (V, 4, 3, 3)        U_mu(x)[a, b], mu = 0..3 = x, y, z, t
  spinor  : complex array (V, 12, N)          component = 3*spin + colour, RHS last
  vectors : complex array (V, n_v, ncomp)     basis / null-vector candidates

All generators use numpy's PCG64 so that a seed fixes the values on any
machine.  Every call returns complex128 unless a dtype is given; callers
round to FP32 themselves.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "rng",
    "gaussian_complex",
    "haar_su3",
    "smooth_su3",
    "gauge_haar",
    "gauge_smooth",
    "gauge_unit",
    "gauge_transform_field",
    "spinor_source",
    "coarse_source",
    "gaussian_vectors",
    "gaussian_blocks",
]


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_complex(g: np.random.Generator, shape, dtype=np.complex128) -> np.ndarray:
    """Real and imaginary parts independently N(0, 1)."""
    fdt = np.float32 if np.dtype(dtype) == np.complex64 else np.float64
    re = g.standard_normal(shape, dtype=fdt)
    im = g.standard_normal(shape, dtype=fdt)
    out = np.empty(shape, dtype=dtype)
    out.real = re
    out.imag = im
    return out


def haar_su3(g: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(3) matrices.

    QR of a complex Gaussian matrix with entries (N(0,1) + i N(0,1))/sqrt(2);
    the columns of Q are rephased by R_ii/|R_ii| (Mezzadri's fix, which makes Q
    Haar on U(3)), then Q is divided by the principal cube root of det Q.
    Left multiplication by SU(3) commutes with both steps, so the result is
    Haar on SU(3).
    """
    G = gaussian_complex(g, (n, 3, 3)) / np.sqrt(2.0)
    Q, R = np.linalg.qr(G)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q = Q / (det ** (1.0 / 3.0))[:, None, None]
    return Q


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return lam


def smooth_su3(g: np.random.Generator, n: int, eps: float = 0.3) -> np.ndarray:
    """n matrices U = exp(i*eps*H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0, 1).

    H is Hermitian and traceless, so U is exactly unitary with det U = 1; the
    exponential is taken through the eigendecomposition of H.
    """
    h = g.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, _gell_mann()) / 2.0
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("nij,nj,nkj->nik", v, ph, v.conj())


def gauge_haar(dims, seed: int) -> np.ndarray:
    V = volume(dims)
    return haar_su3(rng(seed), V * 4).reshape(V, 4, 3, 3)


def gauge_smooth(dims, seed: int, eps: float = 0.3) -> np.ndarray:
    V = volume(dims)
    return smooth_su3(rng(seed), V * 4, eps).reshape(V, 4, 3, 3)


def gauge_unit(dims) -> np.ndarray:
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gauge_transform_field(dims, seed: int) -> np.ndarray:
    """A Haar-random SU(3) matrix Lambda(x) per site, shape (V, 3, 3)."""
    return haar_su3(rng(seed), volume(dims))


def spinor_source(dims, nrhs: int, seed_base: int, dtype=np.complex128) -> np.ndarray:
    """Gaussian spinors (V, 12, nrhs); column k is drawn from seed seed_base + k."""
    V = volume(dims)
    out = np.empty((V, 12, nrhs), dtype=dtype)
    for k in range(nrhs):
        out[:, :, k] = gaussian_complex(rng(seed_base + k), (V, 12), dtype)
    return out


def coarse_source(nsites: int, ncomp: int, nrhs: int, seed_base: int, dtype=np.complex128) -> np.ndarray:
    """Gaussian coarse fields (nsites, ncomp, nrhs); column k from seed seed_base + k."""
    out = np.empty((nsites, ncomp, nrhs), dtype=dtype)
    for k in range(nrhs):
        out[:, :, k] = gaussian_complex(rng(seed_base + k), (nsites, ncomp), dtype)
    return out


def gaussian_vectors(nsites: int, n_v: int, ncomp: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Gaussian basis candidates (nsites, n_v, ncomp)."""
    return gaussian_complex(rng(seed), (nsites, n_v, ncomp), dtype)


def gaussian_blocks(nsites: int, nb: int, seed: int, shift: float = 4.0) -> np.ndarray:
    """Stencil blocks (nsites, 9, nb, nb), Gaussian entries, +shift*I on the self block (index 0)."""
    B = gaussian_complex(rng(seed), (nsites, 9, nb, nb))
    B[:, 0] += shift * np.eye(nb)
    return B
