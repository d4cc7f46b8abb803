"""Schwarz alternating procedure (SAP) for the fine operator, FP64.

TEST INFRASTRUCTURE: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module (see the package
docstring).

The paper's outlook (Sec. 9) names Schwarz-type (SAP) smoothing as a next
step for the multigrid; the method is the standard multiplicative Schwarz
iteration on a two-coloured block decomposition (Luescher's SAP), written out
here from its definition:

  blocks     the aggregates of extent b = (bx, by, bz, bt) of the lattice,
             block coordinates (X, Y, Z, T) = (x // bx, ...); block colour
             c(B) = (X + Y + Z + T) mod 2, a proper two-colouring when every
             L_mu / b_mu is even (neighbouring blocks differ in colour).
  D_B        D restricted to block B with Dirichlet boundaries: the clover
             term and every hop whose source and target both lie in B; hops
             that cross the block boundary (including the periodic wrap) are
             dropped.  D_blk = sum_B D_B is block diagonal.
  SAP cycle  for c = 0, 1:  r = b - D x;  on every block B of colour c,
             e_B ~ D_B^-1 r|_B by `mr_iters` minimal-residual steps from zero,
             alpha = <q, rho>_B / ||q||^2_B per (block, right-hand side) with
             q = D_B rho (sums over the block's sites and components);
             x += sum_{B of colour c} e_B.
"""

from __future__ import annotations

import numpy as np

from .mg import aggregate_index, coarse_dims
from .wilson import clover_apply, hop_dir


def block_colour(dims, block) -> np.ndarray:
    """Colour (X + Y + Z + T) mod 2 of the block of every site, shape (V,)."""
    C = coarse_dims(dims, block)
    if any(c % 2 for c in C):
        raise ValueError(f"SAP needs an even number of blocks per direction, got {C}")
    a = aggregate_index(dims, block)
    X, Y, Z, T = a % C[0], (a // C[0]) % C[1], (a // (C[0] * C[1])) % C[2], a // (C[0] * C[1] * C[2])
    return (X + Y + Z + T) % 2


def dwc_blocks(U, Apacked, kappa, psi, dims, block, t_bc=-1.0) -> np.ndarray:
    """D_blk psi: the clover term and the hops inside each block (Dirichlet)."""
    return clover_apply(Apacked, psi) - kappa * hop_dir(U, psi, dims, t_bc, 0, 0, block)


def block_sums(a, dims, block) -> np.ndarray:
    """Sum over the sites and components of every block, per column: (nblocks, N)."""
    agg = aggregate_index(dims, block)
    nb = int(agg.max()) + 1
    per_site = np.asarray(a).sum(axis=1)  # (V, N)
    out = np.zeros((nb,) + per_site.shape[1:], dtype=per_site.dtype)
    np.add.at(out, agg, per_site)
    return out


def sap_cycles(U, Apacked, kappa, b, x, dims, block, ncycles: int, mr_iters: int, t_bc=-1.0) -> np.ndarray:
    """x after `ncycles` SAP cycles on D x = b from the given x (FP64)."""
    from .wilson import dwc

    b = np.asarray(b, dtype=np.complex128)
    x = np.array(x, dtype=np.complex128, copy=True)
    colour = block_colour(dims, block)
    agg = aggregate_index(dims, block)
    for _ in range(ncycles):
        for c in (0, 1):
            on = (colour == c)[:, None, None]
            rho = np.where(on, b - dwc(U, Apacked, kappa, x, dims, t_bc), 0.0)
            e = np.zeros_like(rho)
            for _ in range(mr_iters):
                q = np.where(on, dwc_blocks(U, Apacked, kappa, rho, dims, block, t_bc), 0.0)
                num = block_sums(np.conj(q) * rho, dims, block)
                den = block_sums(np.abs(q) ** 2, dims, block).real
                alpha = np.divide(num, den, out=np.zeros_like(num), where=den > 0)[agg][:, None, :]
                e = e + alpha * rho
                rho = rho - alpha * q
            x = x + e
    return x
