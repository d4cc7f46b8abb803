"""Plain FP64 CPU oracle for the MRHS Wilson-clover multigrid hot path.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never calls it and
shares no code with it; the two meet only at the seeded inputs in ``synth``.

The paper (Richtmann, Meyer, Wettig, "MRHS multigrid solver for Wilson-clover
fermions", LATTICE2022) names the operators it accelerates -- the fine
hopping and clover terms (Sec. 4), the intergrid project/promote operators
(Sec. 5), the coarse-level hopping term (Sec. 6), batched inner products
(Sec. 7) and the FGMRES + multigrid solve (Sec. 8) -- but prints no formula.
Every formula here is the textbook definition written out in numpy, under
the conventions stated in ``conventions`` (gamma basis, hop sign, clover
normalisation, boundary phase); each function cites the section it serves.

Arrays use the library layout: site s = x + Lx*(y + Ly*(z + Lz*t)),
spinor component 3*spin + colour, RHS index last.
"""

from .conventions import (  # noqa: F401
    gamma_matrices,
    sigma_munu,
    chiral_sigma_blocks,
    DIRS,
    dir_index,
)
from .wilson import (  # noqa: F401
    hop,
    hop_dir,
    field_strength,
    clover_dense,
    clover_packed,
    clover_packed_direct,
    pack_hermitian6,
    unpack_hermitian6,
    clover_apply,
    dwc,
    dwc_mass,
    dwc_sites,
    gauge_transform,
    spinor_gauge_transform,
)
from .mg import (  # noqa: F401
    coarse_dims,
    aggregate_index,
    block_orthonormalise,
    restrict,
    prolong,
    block_normalise,
    galerkin_fine,
    galerkin_coarse,
    coarse_apply,
    coarse_apply_dir,
)
from .blas import dot, norm2  # noqa: F401
from .lowprec import round_bf16, round_f16, column_scale, coarse_apply_lowprec, restrict_lowprec, prolong_lowprec  # noqa: F401
from .solve import dwc_sparse, solve_ref, true_residual, sigma_min  # noqa: F401
