"""Reference solves and residuals in FP64 (paper Sec. 8: the quantity the
multigrid-preconditioned FGMRES drives down is the residual of the fine
Wilson-clover system; the oracle solves that system directly).

The fine operator is assembled as a scipy sparse matrix straight from its
definition, block by block (12 x 12 per coupled site pair):

  diagonal block at x             A(x) = diag(A_+(x), A_-(x))
  block (x, x + mu)              -kappa (1 - gamma_mu) (x) U_mu(x)          [times t_bc across the t boundary]
  block (x, x - mu)              -kappa (1 + gamma_mu) (x) U_mu(x - mu)^dag [times t_bc across the t boundary]

with row/column index 12 s + 3 spin + colour.  Couplings that land on the same
site pair are summed (lattice extent 2 or 1).  The system is solved by
scipy's restarted GMRES to a relative residual of 1e-13 per column (a sparse
LU of a 4-d lattice operator fills in far too much beyond a few hundred
sites).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .conventions import gamma_matrices
from .wilson import dwc, unpack_hermitian6


def dwc_sparse(U, Apacked, kappa, dims, t_bc=-1.0):
    """D = A - kappa H as a (12V x 12V) CSR matrix."""
    Lx, Ly, Lz, Lt = dims
    L = np.array(dims)
    V = Lx * Ly * Lz * Lt
    s = np.arange(V)
    X = np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)
    stride = np.array([1, Lx, Lx * Ly, Lx * Ly * Lz])
    g = gamma_matrices()
    I4 = np.eye(4)
    rows, cols, vals = [], [], []
    ii, jj = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")

    def add(src_sites, dst_sites, blocks):
        rows.append((12 * dst_sites[:, None, None] + ii[None]).ravel())
        cols.append((12 * src_sites[:, None, None] + jj[None]).ravel())
        vals.append(blocks.reshape(-1))

    M = unpack_hermitian6(np.asarray(Apacked, dtype=np.float64))
    diag = np.zeros((V, 12, 12), dtype=np.complex128)
    diag[:, :6, :6] = M[:, 0]
    diag[:, 6:, 6:] = M[:, 1]
    add(s, s, diag)
    U = np.asarray(U, dtype=np.complex128)
    for mu in range(4):
        for sgn in (+1, -1):
            Y = X.copy()
            Y[:, mu] = (Y[:, mu] + sgn) % L[mu]
            nb = Y @ stride
            wrapped = (X[:, mu] == L[mu] - 1) if sgn > 0 else (X[:, mu] == 0)
            ph = np.where(wrapped & (mu == 3), t_bc, 1.0)
            if sgn > 0:
                link = U[s, mu]
                proj = I4 - g[mu]
            else:
                link = np.conj(np.swapaxes(U[nb, mu], -1, -2))
                proj = I4 + g[mu]
            blk = -kappa * ph[:, None, None] * np.einsum("st,vab->vsatb", proj, link).reshape(V, 12, 12)
            add(nb, s, blk)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(12 * V, 12 * V))


def solve_ref(U, Apacked, kappa, b, dims, t_bc=-1.0, rtol=1e-13):
    """x with D x = b for every column of b (V, 12, N), by restarted GMRES."""
    D = dwc_sparse(U, Apacked, kappa, dims, t_bc)
    V, _, N = b.shape
    rhs = np.asarray(b, dtype=np.complex128).reshape(V * 12, N)
    x = np.empty_like(rhs)
    for k in range(N):
        xk, info = spla.gmres(D, rhs[:, k], rtol=rtol, atol=0.0, restart=100, maxiter=200)
        if info != 0:
            raise RuntimeError(f"reference GMRES did not converge for column {k} (info {info})")
        x[:, k] = xk
    return x.reshape(V, 12, N)


def true_residual(U, Apacked, kappa, x, b, dims, t_bc=-1.0):
    """||b_k - D x_k|| / ||b_k|| per column, FP64."""
    r = np.asarray(b, dtype=np.complex128) - dwc(U, Apacked, kappa, x, dims, t_bc)
    N = r.shape[-1]
    return np.linalg.norm(r.reshape(-1, N), axis=0) / np.linalg.norm(np.asarray(b).reshape(-1, N), axis=0)


def sigma_min(U, Apacked, kappa, dims, t_bc=-1.0, mass_form=True, inner_rtol=1e-12, tol=1e-8):
    """Smallest singular value of D (or of D_m = D / (2 kappa) with mass_form),
    as 1 / sqrt(largest eigenvalue of D^-1 D^-dag), by Lanczos on that
    Hermitian operator; each application solves with D^dag and D by GMRES."""
    D = dwc_sparse(U, Apacked, kappa, dims, t_bc)
    DH = D.conj().T.tocsr()
    n = D.shape[0]

    def mv(v):
        w, i1 = spla.gmres(DH, np.asarray(v, dtype=np.complex128).ravel(), rtol=inner_rtol, atol=0.0, restart=100,
                           maxiter=500)
        z, i2 = spla.gmres(D, w, rtol=inner_rtol, atol=0.0, restart=100, maxiter=500)
        if i1 or i2:
            raise RuntimeError("inner GMRES of sigma_min did not converge")
        return z

    op = spla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    lam = spla.eigsh(op, k=1, which="LM", return_eigenvectors=False, tol=tol, ncv=16)[0]
    s = 1.0 / np.sqrt(lam)
    return s / (2.0 * kappa) if mass_form else s
