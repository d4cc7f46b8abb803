"""GPU parity of the even-odd pieces (M_eooe, M_ooee and its inverse, the Schur
complement) against the FP64 oracle, and against the full-lattice kernels.

Tolerances as for the full operator: 1e-12 relative L2 in FP64, 1e-6 in FP32.
The checkerboard hop must also equal the full-lattice hop of a field that is
zero on the output parity, bit for bit in FP32 (same per-site arithmetic).
"""

import numpy as np
import pytest

import oracle as O
from oracle import evenodd as EO
import synth

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.13, 1.0


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def lat(gpu_lib):
    dims = (4, 6, 4, 8)  # non-cubic, all extents even
    U = synth.gauge_haar(dims, 4001)
    A = O.clover_packed(U, dims, CSW, KAPPA)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, KAPPA)
    return dims, U, A, ctx


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("nrhs", [1, 5, 24, 64])
@pytest.mark.parametrize("p", [0, 1])
def test_hop_eo(lat, dt, nrhs, p):
    import torch

    dims, U, A, ctx = lat
    psi = EO.to_cb(synth.spinor_source(dims, nrhs, 50, dt), dims, 1 - p)
    out = torch.empty(psi.shape, dtype=torch.complex128 if dt == np.complex128 else torch.complex64, device="cuda")
    ctx.hop_eo(out, dev(psi), p)
    tol = 1e-12 if dt == np.complex128 else 1e-6
    assert rel(out.cpu().numpy(), EO.hop_eo(U, psi, dims, p)) < tol


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("p", [0, 1])
def test_clover_eo(lat, dt, inverse, p):
    import torch

    dims, U, A, ctx = lat
    psi = EO.to_cb(synth.spinor_source(dims, 6, 60, dt), dims, p)
    out = torch.empty(psi.shape, dtype=torch.complex128 if dt == np.complex128 else torch.complex64, device="cuda")
    ctx.clover_eo(out, dev(psi), p, inverse=inverse)
    blocks = EO.clover_inverse(A) if inverse else A
    tol = 1e-12 if dt == np.complex128 else 1e-6
    assert rel(out.cpu().numpy(), EO.clover_cb(blocks, psi, dims, p)) < tol


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("nrhs", [1, 3, 64])
def test_schur(lat, dt, nrhs):
    import torch

    dims, U, A, ctx = lat
    psi = EO.to_cb(synth.spinor_source(dims, nrhs, 70, dt), dims, 0)
    out = torch.empty(psi.shape, dtype=torch.complex128 if dt == np.complex128 else torch.complex64, device="cuda")
    ctx.schur(out, dev(psi))
    tol = 1e-12 if dt == np.complex128 else 1e-6
    assert rel(out.cpu().numpy(), EO.schur_ee(U, A, KAPPA, psi, dims)) < tol


def _full_vs_eo(gpu_lib, dims, seed, nrhs):
    """FP32: hop_eo of an odd field equals the full-lattice hop of the field placed on
    the odd sites (zero on the even ones), read on the even sites, bit for bit."""
    import torch

    U = synth.gauge_haar(dims, seed)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, KAPPA)
    f = synth.spinor_source(dims, nrhs, seed + 1, np.complex64)
    f_odd = EO.to_cb(f, dims, 1)
    full = EO.from_cb(np.zeros_like(f_odd), f_odd, dims)
    h = torch.empty(full.shape, dtype=torch.complex64, device="cuda")
    ctx.hop(h, dev(full))
    he = torch.empty(f_odd.shape, dtype=torch.complex64, device="cuda")
    ctx.hop_eo(he, dev(f_odd), 0)
    np.testing.assert_array_equal(he.cpu().numpy(), EO.to_cb(h.cpu().numpy(), dims, 0))


def test_hop_eo_equals_full_hop(gpu_lib):
    _full_vs_eo(gpu_lib, (4, 6, 4, 8), 4101, 6)


def test_hop_eo_equals_full_hop_24(gpu_lib):
    """The 24^4 benchmark lattice at Nrhs = 24, the size the benchmark times."""
    _full_vs_eo(gpu_lib, (24, 24, 24, 24), 4201, 24)


def test_odd_extent_rejected(gpu_lib):
    import torch

    dims = (4, 4, 4, 3)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(synth.gauge_unit(dims))
    V2 = synth.volume(dims) // 2
    a = torch.zeros((V2, 12, 2), dtype=torch.complex64, device="cuda")
    b = torch.zeros_like(a)
    with pytest.raises(gpu_lib.MrhsError, match="SHAPE"):
        ctx.hop_eo(b, a, 0)


def test_singular_clover_rejected(gpu_lib):
    import torch

    dims = (2, 2, 2, 2)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(synth.gauge_unit(dims))
    A = np.zeros((synth.volume(dims), 2, 36))
    A[:, :, :6] = 1.0
    A[3, 1, 2] = 0.0  # one block with a zero row and column
    ctx.set_clover(A, KAPPA)
    a = torch.ones((8, 12, 2), dtype=torch.complex64, device="cuda")
    b = torch.zeros_like(a)
    ctx.clover_eo(b, a, 0)  # the blocks themselves are fine
    with pytest.raises(gpu_lib.MrhsError, match="STATE"):
        ctx.clover_eo(b, a, 1, inverse=True)


# ---- coarse level ---------------------------------------------------------------------

def _coarse(gpu_lib, cdims, seed, shift=4.0):
    """A hierarchy whose level 1 is cdims with Nb = 32 and Gaussian blocks (+shift I
    on the self blocks; 12 keeps every self block's condition number near 10 or below,
    so the rounding of its inverse to FP32 / BF16 stays within the usual tolerances)."""
    ctx = gpu_lib.Context(tuple(2 * c for c in cdims), t_bc=-1)
    ctx.set_gauge(synth.gauge_unit(tuple(2 * c for c in cdims)))
    ctx.build_clover(CSW, KAPPA)
    mg = gpu_lib.Multigrid(ctx, [(2, 2, 2, 2)], [16])
    B = synth.gaussian_blocks(synth.volume(cdims), 32, seed, shift=shift)
    mg.set_blocks(1, B)
    return ctx, mg, B


@pytest.mark.parametrize("cdims", [(4, 6, 2, 4), (6, 6, 6, 6)])
@pytest.mark.parametrize("nrhs", [1, 12, 33])
@pytest.mark.parametrize("p", [0, 1])
def test_coarse_hop_eo(gpu_lib, cdims, nrhs, p):
    import torch

    ctx, mg, B = _coarse(gpu_lib, cdims, 5000 + nrhs)
    Vh = synth.volume(cdims) // 2
    e = EO.to_cb(synth.coarse_source(synth.volume(cdims), 32, nrhs, 5100, np.complex64), cdims, 1 - p)
    want = EO.coarse_hop_eo(B, e, cdims, p)
    for prec, tol in (("f32", 1e-6), ("bf16", 2e-2), ("f16", 2e-2)):
        out = torch.empty((Vh, 32, nrhs), dtype=torch.complex64, device="cuda")
        mg.coarse_hop_eo(1, out, dev(e), p, prec=prec)
        Bp = B.astype(np.complex64) if prec == "f32" else B
        w = EO.coarse_hop_eo(Bp, e, cdims, p) if prec == "f32" else want
        assert rel(out.cpu().numpy(), w) < tol, prec


@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("p", [0, 1])
def test_coarse_self_eo(gpu_lib, inverse, p):
    import torch

    cdims, nrhs = (4, 6, 2, 4), 24
    ctx, mg, B = _coarse(gpu_lib, cdims, 5200, shift=12.0)
    Vh = synth.volume(cdims) // 2
    e = EO.to_cb(synth.coarse_source(synth.volume(cdims), 32, nrhs, 5300, np.complex64), cdims, p)
    S = EO.coarse_self_inverse(B) if inverse else B[:, 0]
    want = EO.coarse_self_cb(S, e, cdims, p)
    for prec, tol in (("f32", 1e-6), ("bf16", 2e-2), ("f16", 2e-2)):
        out = torch.empty((Vh, 32, nrhs), dtype=torch.complex64, device="cuda")
        mg.coarse_self_eo(1, out, dev(e), p, inverse=inverse, prec=prec)
        assert rel(out.cpu().numpy(), want) < tol, prec


def test_coarse_schur_composed(gpu_lib):
    """S_e x - H_eo S_o^-1 H_oe x from the three GPU calls (FP32) against the oracle."""
    import torch

    cdims, nrhs = (6, 6, 6, 6), 12
    ctx, mg, B = _coarse(gpu_lib, cdims, 5400, shift=12.0)
    Vh = synth.volume(cdims) // 2
    x = EO.to_cb(synth.coarse_source(synth.volume(cdims), 32, nrhs, 5500, np.complex64), cdims, 0)
    t1 = torch.empty((Vh, 32, nrhs), dtype=torch.complex64, device="cuda")
    t2 = torch.empty_like(t1)
    t3 = torch.empty_like(t1)
    t4 = torch.empty_like(t1)
    xd = dev(x)
    mg.coarse_hop_eo(1, t1, xd, 1)
    mg.coarse_self_eo(1, t2, t1, 1, inverse=True)
    mg.coarse_hop_eo(1, t3, t2, 0)
    mg.coarse_self_eo(1, t4, xd, 0)
    got = (t4 - t3).cpu().numpy()
    assert rel(got, EO.coarse_schur_ee(B, x, cdims)) < 1e-5


def test_coarse_eo_odd_extent_rejected(gpu_lib):
    import torch

    cdims = (3, 3, 3, 3)
    ctx, mg, B = _coarse(gpu_lib, cdims, 5600)
    a = torch.zeros((40, 32, 2), dtype=torch.complex64, device="cuda")
    b = torch.zeros_like(a)
    with pytest.raises((gpu_lib.MrhsError, ValueError)):
        mg.coarse_hop_eo(1, b, a, 0)


# t-walk shapes of the checkerboard hop on the 4x6x4x8 lattice: spatial block
# (Bx, By, Bz) of at least 16 sites, Ts output sites per run (Ts | Lt / 2 = 4),
# RHS per thread (0: the default for the parity of nrhs)
WALKS = [((4, 2, 2, 1), 0), ((2, 6, 2, 2), 1), ((4, 6, 4, 4), 0), ((2, 2, 4, 4), 2), ((4, 3, 2, 2), 1)]


@pytest.mark.parametrize("walk,R", WALKS)
@pytest.mark.parametrize("nrhs", [1, 6, 13, 24])
def test_hop_eo_walk_bitwise(lat, walk, R, nrhs):
    """The t-walk checkerboard hop gives the tiled kernel's fields bit for bit
    (both output parities, and the two fused Schur launches), whatever the
    block, run length and RHS per thread; the walks wrap through the
    antiperiodic t boundary.  The tiled kernel is pinned to the oracle above."""
    import torch

    dims, U, A, ctx = lat
    if R == 2 and nrhs % 2:
        pytest.skip("two RHS per thread need an even nrhs")
    ctx.set_eo_walk(nrhs, None)
    outs = {}
    for p in (0, 1):
        psi = dev(EO.to_cb(synth.spinor_source(dims, nrhs, 70 + p, np.complex64), dims, 1 - p))
        o = torch.empty_like(psi)
        ctx.hop_eo(o, psi, p)
        outs[p] = (psi, o.clone())
    chi = dev(EO.to_cb(synth.spinor_source(dims, nrhs, 80, np.complex64), dims, 0))
    s0 = torch.empty_like(chi)
    ctx.schur(s0, chi)
    ctx.set_eo_walk(nrhs, walk, R)
    on, r, tile, _, _ = ctx.get_eo_walk(nrhs)
    assert on and tuple(tile) == walk and r == R
    for p in (0, 1):
        psi, o0 = outs[p]
        o = torch.empty_like(psi)
        ctx.hop_eo(o, psi, p)
        assert torch.equal(o, o0), p
    s1 = torch.empty_like(chi)
    ctx.schur(s1, chi)
    assert torch.equal(s1, s0)
    ctx.set_eo_walk(nrhs, None)


def test_eo_walk_rejects_bad_shapes(lat, gpu_lib):
    dims, U, A, ctx = lat
    for tile, R in [((4, 4, 4, 1), 0), ((2, 2, 2, 1), 0), ((4, 6, 4, 3), 0), ((4, 6, 4, 1), 2), ((4, 6, 4, 1), 3)]:
        n = 5 if R == 2 else 6
        with pytest.raises(gpu_lib.MrhsError, match="INVALID_ARG"):
            ctx.set_eo_walk(n, tile, R)  # block not dividing 6, < 16 sites, Ts not dividing 4, R = 2 at odd nrhs, R = 3


def test_tune_chooses_a_checkerboard_kernel(gpu_lib):
    """mrhs_tune times the checkerboard hop on a lattice with even extents and
    keeps a valid choice, tiled or walk, with both times recorded."""
    dims = (8, 8, 8, 8)
    U = synth.gauge_haar(dims, 4002)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, KAPPA)
    ctx.tune([4, 7])
    for n in (4, 7):
        on, r, tile, us, ut = ctx.get_eo_walk(n)
        assert ut > 0 and us > 0 and us <= ut * 1.0001
        if on:
            assert all(d % b == 0 for d, b in zip(dims[:3], tile[:3])) and (dims[3] // 2) % tile[3] == 0
    ctx.close()
