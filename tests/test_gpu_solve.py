"""GPU multigrid-preconditioned FGMRES against the FP64 oracle.

What is pinned: every solution's true residual ||b - D x|| / ||b||, recomputed
by the oracle on the host in FP64, is at most 1e-10 (the solver's target);
on 8^4 the solution also matches the oracle's own GMRES solution to within
the condition-number bound cond(D) * 1e-10 (cond(D) of these Haar-link
operators is below 10, checked loosely as 1e-8).  Iteration counts, the
setup and the smoother are not unique and are not compared.
"""

import os

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.13, 1.0


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def build(mrhs, dims, U, blocks, n_v, seed=100, setup_iters=2, smooth_steps=6):
    ctx = mrhs.Context(dims, t_bc=-1)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, KAPPA)
    mg = mrhs.Multigrid(ctx, blocks, n_v)
    for l in range(len(blocks)):
        mg.set_basis(l, synth.gaussian_vectors(mg.volume[l], n_v[l], mg.ncomp[l], seed + l))
    mg.setup(setup_iters, smooth_steps)
    return ctx, mg


@pytest.fixture(scope="module")
def small(gpu_lib):
    dims = (8, 8, 8, 8)
    U = synth.gauge_haar(dims, 808)
    A = O.clover_packed(U, dims, CSW, KAPPA)
    ctx, mg = build(gpu_lib, dims, U, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    return dims, U, A, ctx, mg


@pytest.mark.parametrize("coarse", ["bf16", "f16", "f32"])
@pytest.mark.parametrize("nrhs", [1, 12])
def test_solve_8444_three_level(small, coarse, nrhs):
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, nrhs, 9000)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), tol=1e-10, restart=8, max_iters=400, nu_pre=0, nu_post=4, coarsest_iters=16,
                  coarse_prec=coarse)
    assert all(st["converged"]) and max(st["rel_resid"]) <= 1e-10
    xs = x.cpu().numpy()
    assert np.all(O.true_residual(U, A, KAPPA, xs, b, dims) <= 1e-10)
    if nrhs == 1 and coarse == "bf16":
        xr = O.solve_ref(U, A, KAPPA, b, dims)
        assert np.linalg.norm(xs - xr) / np.linalg.norm(xr) < 1e-8


def test_graph_replay_is_bitwise_equal(small):
    import torch

    dims, U, A, ctx, mg = small
    b = dev(synth.spinor_source(dims, 6, 123))
    x1 = torch.zeros_like(b)
    x2 = torch.zeros_like(b)
    s1 = mg.solve(x1, b, use_graph=True, coarse_prec="bf16")
    s2 = mg.solve(x2, b, use_graph=False, coarse_prec="bf16")
    assert s1["iters"] == s2["iters"]
    assert torch.equal(x1, x2)


def test_mrhs_matches_srhs_solutions(small):
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, 8, 321)
    xb = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    mg.solve(xb, dev(b), coarse_prec="bf16")
    for k in (0, 7):
        xk = torch.zeros((b.shape[0], 12, 1), dtype=torch.complex128, device="cuda")
        mg.solve(xk, dev(b[:, :, k:k + 1]), coarse_prec="bf16")
        d = np.linalg.norm(xk.cpu().numpy()[:, :, 0] - xb.cpu().numpy()[:, :, k])
        assert d / np.linalg.norm(xk.cpu().numpy()) < 1e-9


def test_unpreconditioned_and_warm_restart(small, gpu_lib):
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, 3, 55)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), max_iters=2, check=False)
    assert st["status"] == 7 and not all(st["converged"])  # MRHS_ERR_NOT_CONVERGED, stats filled
    assert st["iters"] == 2
    st = mg.solve(x, dev(b), precondition=False, restart=15, max_iters=2000)  # resumes from the partial x
    assert all(st["converged"])
    assert np.all(O.true_residual(U, A, KAPPA, x.cpu().numpy(), b, dims) <= 1e-10)


def test_plane_wave_eigenvector_one_step(gpu_lib):
    """On unit links a plane wave times an eigenvector of D(p) is an exact
    eigenvector of D: unpreconditioned GMRES ends after one step, up to the
    FP32 rounding of the stored direction (relative residual ~1e-8)."""
    import torch

    dims = (4, 4, 4, 4)
    U = synth.gauge_unit(dims)
    ctx, mg = build(gpu_lib, dims, U, [(2, 2, 2, 2)], [4], setup_iters=0)
    s = np.arange(synth.volume(dims))
    X = np.stack([s % 4, (s // 4) % 4, (s // 16) % 4, s // 64], axis=1)
    p = np.array([2 * np.pi / 4, 0.0, 2 * np.pi * 2 / 4, 3 * np.pi / 4])
    g = O.gamma_matrices()
    Dp = (1 - 2 * KAPPA * np.cos(p).sum()) * np.eye(4) + 2j * KAPPA * sum(g[m] * np.sin(p[m]) for m in range(4))
    w, vecs = np.linalg.eig(Dp)
    chi = np.kron(vecs[:, 0], np.array([1.0, 0.5j, -0.25]))
    b = (np.exp(1j * (X @ p))[:, None] * chi[None, :]).reshape(-1, 12, 1)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), tol=1e-6, precondition=False, restart=4, max_iters=10)
    assert st["iters"] == 1 and st["converged"][0] and st["rel_resid"][0] < 1e-6


def test_solve_16_four_config_shapes(gpu_lib):
    """16^4 smooth links (U = exp(0.3 i H)), three levels 16^4 -> 4^4 -> 2^4,
    BF16 coarse levels, 12 right-hand sides; true residual by the oracle."""
    import torch

    dims = (16, 16, 16, 16)
    U = synth.gauge_smooth(dims, 16)
    A = O.clover_packed(U, dims, CSW, KAPPA)
    ctx, mg = build(gpu_lib, dims, U, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    b = synth.spinor_source(dims, 12, 777)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), coarse_prec="bf16", max_iters=600)
    assert all(st["converged"])
    assert np.all(O.true_residual(U, A, KAPPA, x.cpu().numpy(), b, dims) <= 1e-10)


def test_adaptive_setup_keeps_basis_orthonormal_and_solves(gpu_lib):
    """Setup with adaptive passes (inverse iteration v <- K v through the
    hierarchy's own V-cycle): every (aggregate, chirality) block of the level-0 basis stays
    orthonormal to FP64 rounding, the level-1 operator is the oracle's
    Galerkin product P^dag D P of that basis, and the preconditioned solve
    reaches the true residual."""
    import torch

    dims = (8, 8, 8, 8)
    U = synth.gauge_smooth(dims, 31)
    kappa = 0.134
    A = O.clover_packed(U, dims, CSW, kappa)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, kappa)
    mg = gpu_lib.Multigrid(ctx, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    for l in range(2):
        mg.set_basis(l, synth.gaussian_vectors(mg.volume[l], 16, mg.ncomp[l], 900 + l))
    mg.setup(2, 10, 2, nu_post=4, coarsest_iters=32, coarse_prec="f32")
    W = mg.get_basis(0)  # (V, n_v, 12)
    agg = O.aggregate_index(dims, (4, 4, 4, 4))
    for a in range(mg.volume[1]):
        blk = W[agg == a]  # (256, 16, 12)
        for chi in range(2):
            Q = blk[:, :, 6 * chi:6 * chi + 6].transpose(0, 2, 1).reshape(-1, 16)
            assert np.max(np.abs(Q.conj().T @ Q - np.eye(16))) < 1e-12
    B1 = O.galerkin_fine(U, A, kappa, W, dims, (4, 4, 4, 4))
    got = mg.get_blocks(1)
    assert np.linalg.norm(got - B1) / np.linalg.norm(B1) < 1e-12
    b = synth.spinor_source(dims, 4, 1234)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), tol=1e-10, restart=8, max_iters=300, nu_post=4, coarsest_iters=32, coarse_prec="bf16")
    assert all(st["converged"])
    assert np.all(O.true_residual(U, A, kappa, x.cpu().numpy(), b, dims) <= 1e-10)


@pytest.mark.parametrize("eta", [0.0, 0.01, 1.0])
def test_reorth_threshold_any_value_converges(small, eta):
    """The second Gram-Schmidt pass (never, on large cancellation, always) does
    not change what is computed: every setting reaches the true residual."""
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, 3, 4321)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), reorth_eta=eta, coarse_prec="bf16")
    assert all(st["converged"])
    if eta == 0.0:
        assert st["reorth"] == 0
    if eta == 1.0:
        assert st["reorth"] == st["iters"]
    assert np.all(O.true_residual(U, A, KAPPA, x.cpu().numpy(), b, dims) <= 1e-10)


def test_reorth_threshold_out_of_range(small, gpu_lib):
    import torch

    dims, U, A, ctx, mg = small
    b = dev(synth.spinor_source(dims, 1, 1))
    x = torch.zeros_like(b)
    with pytest.raises(gpu_lib.MrhsError, match="INVALID_ARG"):
        mg.solve(x, b, reorth_eta=1.5)


@pytest.mark.parametrize("nrhs", [1, 12, 64])
def test_solve_even_odd_smoother(small, nrhs):
    """Fine smoothing on the even-odd Schur complement: same 1e-10 true residual,
    up to the largest batch (64 RHS)."""
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, nrhs, 9100)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), tol=1e-10, restart=8, max_iters=400, nu_pre=1, nu_post=3, coarsest_iters=16,
                  coarse_prec="bf16", fine_eo=True)
    assert all(st["converged"]) and max(st["rel_resid"]) <= 1e-10
    assert np.all(O.true_residual(U, A, KAPPA, x.cpu().numpy(), b, dims) <= 1e-10)


def test_even_odd_smoother_graph_replay_is_bitwise_equal(small):
    import torch

    dims, U, A, ctx, mg = small
    b = dev(synth.spinor_source(dims, 4, 9200))
    x1 = torch.zeros_like(b)
    x2 = torch.zeros_like(b)
    s1 = mg.solve(x1, b, use_graph=True, coarse_prec="bf16", fine_eo=True)
    s2 = mg.solve(x2, b, use_graph=False, coarse_prec="bf16", fine_eo=True)
    assert s1["iters"] == s2["iters"]
    assert torch.equal(x1, x2)


def _eo_smoother_ref(U, A, kappa, b, dims, nu):
    """nu minimal-residual steps from zero on the even-odd Schur system
    Dhat e_e = b_e + kappa H_eo A_o^-1 b_o, step alpha_k = <q_k, rho_k> /
    ||q_k||^2 per right-hand side with q = Dhat rho, then the odd sites
    e_o = A_o^-1 (b_o + kappa H_oe e_e); FP64 throughout, from the oracle's
    even-odd pieces."""
    from oracle import evenodd as E

    b = np.asarray(b, dtype=np.complex128)
    rho = E.schur_rhs(U, A, kappa, b, dims)
    ee = np.zeros_like(rho)
    for _ in range(nu):
        q = E.schur_ee(U, A, kappa, rho, dims)
        N = q.shape[-1]
        num = np.einsum("sck,sck->k", q.conj(), rho)
        den = np.einsum("sck,sck->k", q.conj(), q).real
        alpha = (num / den).reshape(1, 1, N)
        ee = ee + alpha * rho
        rho = rho - alpha * q
    Ainv = E.clover_inverse(A)
    eo = E.clover_cb(Ainv, E.to_cb(b, dims, 1) + kappa * E.hop_eo(U, ee, dims, 1), dims, 1)
    return E.from_cb(ee, eo, dims)


@pytest.mark.parametrize("dims,block,nv,nrhs", [
    ((8, 8, 8, 8), (4, 4, 4, 4), 16, 1),
    ((8, 8, 8, 8), (4, 4, 4, 4), 16, 5),
    ((8, 8, 8, 8), (4, 4, 4, 4), 16, 12),
    ((8, 8, 8, 8), (4, 4, 4, 4), 16, 24),
    ((8, 8, 8, 8), (4, 4, 4, 4), 16, 64),
    ((4, 6, 4, 6), (2, 2, 2, 2), 4, 12),
    ((4, 6, 4, 6), (2, 2, 2, 2), 4, 3),
])
@pytest.mark.parametrize("walk", [False, True])
def test_even_odd_smoother_alone(gpu_lib, dims, block, nv, nrhs, walk):
    """The fine even-odd smoother by itself: with two levels, no pre-smoothing
    and no coarsest-level steps the coarse correction is exactly zero, so the
    V-cycle returns nu_post = 3 even-odd MR steps applied to v.  Its step
    lengths come from the per-workgroup sums in the checkerboard hop's
    epilogue; any slip in their column mapping (Nrhs not dividing 256, one
    RHS per thread, a ragged last workgroup on the 4x6x4x6 lattice) changes
    alpha and fails the comparison with the FP64 reference at the FP32 bar.
    With `walk` the checkerboard hops run as the t-walk kernel, whose sums are
    grouped per walk workgroup (a partial workgroup at the end of each block's
    threads on 4x6x4x6)."""
    import torch

    U = synth.gauge_haar(dims, 4242)
    A = O.clover_packed(U, dims, CSW, KAPPA)
    ctx, mg = build(gpu_lib, dims, U, [block], [nv], setup_iters=1, smooth_steps=4)
    if walk:
        ctx.set_eo_walk(nrhs, (4, 4, 2, 2) if dims[0] == 8 else (2, 2, 4, 3))
    v = synth.spinor_source(dims, nrhs, 9300, np.complex64)
    z = torch.empty(v.shape, dtype=torch.complex64, device="cuda")
    mg.precondition(z, dev(v), nu_pre=0, nu_post=3, coarsest_iters=0, coarse_prec="bf16", fine_eo=True)
    want = _eo_smoother_ref(U, A, KAPPA, v, dims, 3)
    got = z.cpu().numpy()
    for k in range(nrhs):
        err = np.linalg.norm(got[:, :, k] - want[:, :, k]) / np.linalg.norm(want[:, :, k])
        assert err < 1e-5, (k, err)
    mg.close()
    ctx.close()


@pytest.mark.timeout(1200)
def test_solve_24x24x24x128_bench_settings(gpu_lib, capsys, tmp_path):
    """The solve workload the benchmark times (24^3 x 128 smooth links at the
    tuned bare mass, three levels, BF16 coarse levels and intergrid, even-odd
    fine smoother, graph-replayed V-cycle, the benchmark's set-up and V-cycle
    parameters, coarse even-odd smoother on the 6^3 x 32 level, its outer
    Krylov basis precision, and its first two right-hand sides): every column's true
    residual, recomputed by the FP64 oracle on the host, is at most 1e-10."""
    import json
    import shutil
    import time

    import torch

    import bench

    t0 = time.time()

    def say(msg):
        with capsys.disabled():
            print(f"  [24^3x128 solve {time.time() - t0:5.0f} s] {msg}", flush=True)

    dims = bench.SOLVE_DIMS
    mass = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "smooth_links_mass.json")))
    kappa = mass["kappa"]
    say("generating links")
    U = synth.gauge_smooth(dims, 5)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, kappa)
    cache = tmp_path / "fine.txt"
    shutil.copyfile(bench.TUNE_CACHE, cache)
    ctx.tune([2, 16], str(cache))
    mg = gpu_lib.Multigrid(ctx, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    for l in range(2):
        mg.set_basis(l, synth.gaussian_vectors(mg.volume[l], 16, mg.ncomp[l], 600 + l))
    say("set-up")
    mg.setup(**bench.SOLVE_SETUP, coarse_prec="bf16", **bench.SOLVE_VC)
    b = synth.spinor_source(dims, 2, 4000)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    say("solve")
    st = mg.solve(x, dev(b), tol=1e-10, restart=bench.SOLVE_RESTART, max_iters=bench.SOLVE_MAXIT,
                  coarse_prec="bf16", use_graph=True, fine_eo=bench.SOLVE_MRHS_FINE_EO,
                  coarse_eo=bench.SOLVE_MRHS_COARSE_EO,
                  krylov_prec=gpu_lib.F32 if bench.SOLVE_KRYLOV_F32 else gpu_lib.F64, **bench.SOLVE_VC)
    assert all(st["converged"])
    xs = x.cpu().numpy()
    mg.close()
    ctx.close()
    del x
    torch.cuda.empty_cache()
    say(f"{st['iters']} outer steps; oracle clover and residual")
    A = O.clover_packed(U, dims, CSW, kappa)
    res = O.true_residual(U, A, kappa, xs, b, dims)
    say(f"oracle true residual {res}")
    assert np.all(res <= 1e-10), res


def test_graph_recaptured_after_kappa_change(gpu_lib):
    """A captured V-cycle holds kappa by value: after the clover term is rebuilt
    with another kappa (same hierarchy, no new set-up) the graph-replayed solve
    must still equal the eager one bit for bit and solve the new operator."""
    import torch

    dims = (8, 8, 8, 8)
    U = synth.gauge_haar(dims, 818)
    ctx, mg = build(gpu_lib, dims, U, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    b = synth.spinor_source(dims, 3, 9400)
    x0 = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    mg.solve(x0, dev(b), use_graph=True, coarse_prec="bf16", fine_eo=True)
    kappa2 = 0.125
    ctx.build_clover(CSW, kappa2)
    x1 = torch.zeros_like(x0)
    x2 = torch.zeros_like(x0)
    s1 = mg.solve(x1, dev(b), use_graph=True, coarse_prec="bf16", fine_eo=True)
    s2 = mg.solve(x2, dev(b), use_graph=False, coarse_prec="bf16", fine_eo=True)
    assert s1["iters"] == s2["iters"]
    assert torch.equal(x1, x2)
    A2 = O.clover_packed(U, dims, CSW, kappa2)
    assert np.all(O.true_residual(U, A2, kappa2, x1.cpu().numpy(), b, dims) <= 1e-10)
    mg.close()
    ctx.close()


def _coarse_eo_smoother_ref(B, r, dims, nu):
    """nu MR steps from zero on the coarse Schur system
    (S_e - H_eo S_o^-1 H_oe) e_e = r_e - H_eo S_o^-1 r_o, then
    e_o = S_o^-1 (r_o - H_oe e_e); FP64, from the oracle's coarse even-odd
    pieces."""
    from oracle import evenodd as E

    B = np.asarray(B, dtype=np.complex128)
    rho = E.coarse_schur_rhs(B, r, dims)
    ee = np.zeros_like(rho)
    for _ in range(nu):
        q = E.coarse_schur_ee(B, rho, dims)
        num = np.einsum("sck,sck->k", q.conj(), rho)
        den = np.einsum("sck,sck->k", q.conj(), q).real
        a = (num / den)[None, None, :]
        ee = ee + a * rho
        rho = rho - a * q
    Si = E.coarse_self_inverse(B)
    eo = E.coarse_self_cb(Si, E.to_cb(r, dims, 1) - E.coarse_hop_eo(B, ee, dims, 1), dims, 1)
    return E.from_cb(ee, eo, dims)


@pytest.mark.parametrize("nrhs", [1, 12, 40])
def test_coarse_even_odd_smoother_alone(gpu_lib, nrhs):
    """The coarse even-odd smoother by itself: three levels 8^4 -> 4^4 -> 2^4,
    no pre- or fine post-smoothing and no coarsest-level steps, so the V-cycle
    returns P (3 even-odd MR steps on level 1)(R v).  Against the FP64 oracle's
    coarse Schur pieces on the oracle's own Galerkin blocks and basis; the
    device runs the level in BF16 (restrict, prolong and stencil), hence the
    2e-2 bar."""
    import torch

    dims, blk = (8, 8, 8, 8), (2, 2, 2, 2)
    U = synth.gauge_haar(dims, 5151)
    A = O.clover_packed(U, dims, CSW, KAPPA)
    ctx = gpu_lib.Context(dims, t_bc=-1)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, KAPPA)
    mg = gpu_lib.Multigrid(ctx, [blk, blk], [16, 16])
    v0 = synth.gaussian_vectors(synth.volume(dims), 16, 12, 61)
    mg.set_basis(0, v0)
    mg.block_orthonormalise(0)
    mg.build_coarse(1)
    mg.set_basis(1, synth.gaussian_vectors(mg.volume[1], 16, 32, 62))
    mg.block_orthonormalise(1)
    mg.build_coarse(2)
    W0 = O.block_orthonormalise(v0, dims, blk)
    B1 = O.galerkin_fine(U, A, KAPPA, W0, dims, blk)
    v = synth.spinor_source(dims, nrhs, 9500, np.complex64)
    z = torch.empty(v.shape, dtype=torch.complex64, device="cuda")
    mg.precondition(z, dev(v), nu_pre=0, nu_post=0, coarsest_iters=0, coarse_prec="bf16", coarse_eo=True)
    got = z.cpu().numpy()
    # nu_post applies to every level above the coarsest; with nu_post = 0 the
    # level-1 smoother does nothing, so use the two-call difference below
    assert np.all(got == 0)
    mg.precondition(z, dev(v), nu_pre=0, nu_post=3, coarsest_iters=0, coarse_prec="bf16", coarse_eo=True, fine_eo=True)
    x1 = _coarse_eo_smoother_ref(B1, O.restrict(W0, v, dims, blk), mg.dims[1], 3)
    # the fine level then smooths P x1 with three even-odd MR steps on the residual
    want = O.prolong(W0, x1, dims, blk) + _eo_smoother_ref(U, A, KAPPA, v - O.dwc(U, A, KAPPA, O.prolong(W0, x1, dims, blk),
                                                                                     dims), dims, 3)
    err = np.linalg.norm(z.cpu().numpy() - want) / np.linalg.norm(want)
    assert err < 2e-2, err
    mg.close()
    ctx.close()


@pytest.mark.parametrize("nrhs", [1, 12])
def test_solve_coarse_even_odd_smoother(gpu_lib, nrhs):
    """Solves with the coarse even-odd smoother on level 1 (16^4 smooth links,
    three levels 16^4 -> 4^4 -> 2^4, BF16 coarse levels, fine even-odd
    smoother): every column reaches the 1e-10 true residual recomputed by the
    oracle; graph replay equals the eager V-cycles bit for bit."""
    import torch

    dims = (16, 16, 16, 16)
    U = synth.gauge_smooth(dims, 16)
    A = O.clover_packed(U, dims, CSW, KAPPA)
    ctx, mg = build(gpu_lib, dims, U, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    b = synth.spinor_source(dims, nrhs, 778)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    kw = dict(tol=1e-10, max_iters=600, nu_post=4, coarsest_iters=32, coarse_prec="bf16", fine_eo=True, coarse_eo=True)
    st = mg.solve(x, dev(b), use_graph=True, **kw)
    assert all(st["converged"])
    assert np.all(O.true_residual(U, A, KAPPA, x.cpu().numpy(), b, dims) <= 1e-10)
    x2 = torch.zeros_like(x)
    st2 = mg.solve(x2, dev(b), use_graph=False, **kw)
    assert st2["iters"] == st["iters"] and torch.equal(x, x2)
    mg.close()
    ctx.close()


@pytest.mark.parametrize("dims,block,nrhs,cycles,iters", [
    ((8, 8, 8, 8), (2, 2, 2, 2), 1, 1, 4),
    ((8, 8, 8, 8), (2, 2, 2, 2), 12, 2, 3),
    ((8, 8, 8, 8), (4, 4, 4, 4), 5, 1, 4),
    ((4, 8, 4, 8), (2, 2, 2, 2), 24, 1, 2),
])
def test_sap_smoother_alone(gpu_lib, dims, block, nrhs, cycles, iters):
    """The Schwarz smoother by itself: two levels, no coarse-grid correction
    (coarsest_iters = 0), so the V-cycle returns `cycles` SAP cycles from zero
    on D z = v.  Against the FP64 oracle (oracle.sap), per column, at the FP32
    bar; several block sizes, cycles and MR steps per block, Nrhs not dividing
    256."""
    import torch

    from oracle import sap as S

    U = synth.gauge_haar(dims, 6161)
    A = O.clover_packed(U, dims, CSW, KAPPA)
    ctx, mg = build(gpu_lib, dims, U, [block], [4], setup_iters=1, smooth_steps=2)
    v = synth.spinor_source(dims, nrhs, 9600, np.complex64)
    z = torch.empty(v.shape, dtype=torch.complex64, device="cuda")
    mg.precondition(z, dev(v), nu_pre=0, nu_post=cycles, coarsest_iters=0, coarse_prec="f32", fine_sap=True,
                    sap_iters=iters)
    want = S.sap_cycles(U, A, KAPPA, v, np.zeros_like(v, dtype=np.complex128), dims, block, cycles, iters)
    got = z.cpu().numpy()
    for k in range(nrhs):
        err = np.linalg.norm(got[:, :, k] - want[:, :, k]) / np.linalg.norm(want[:, :, k])
        assert err < 1e-5, (k, err)
    mg.close()
    ctx.close()


def test_sap_rejects_odd_block_counts_and_eo_together(gpu_lib):
    import torch

    dims = (6, 4, 4, 4)
    U = synth.gauge_haar(dims, 1)
    ctx, mg = build(gpu_lib, dims, U, [(2, 2, 2, 2)], [4], setup_iters=0)
    v = dev(synth.spinor_source(dims, 1, 1, np.complex64))
    z = torch.empty_like(v)
    with pytest.raises(gpu_lib.MrhsError, match="SHAPE"):  # three blocks along x
        mg.precondition(z, v, fine_sap=True)
    with pytest.raises(gpu_lib.MrhsError, match="INVALID_ARG"):
        mg.precondition(z, v, fine_sap=True, fine_eo=True)
    mg.close()
    ctx.close()


@pytest.mark.parametrize("nrhs", [1, 12])
def test_solve_sap_smoother(small, nrhs):
    """Solves with SAP smoothing on the fine level (8^4, three levels, BF16
    coarse levels): the 1e-10 true residual recomputed by the oracle."""
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, nrhs, 9700)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), tol=1e-10, restart=8, max_iters=400, nu_pre=0, nu_post=1, coarsest_iters=16,
                  coarse_prec="bf16", fine_sap=True, sap_iters=4)
    assert all(st["converged"])
    assert np.all(O.true_residual(U, A, KAPPA, x.cpu().numpy(), b, dims) <= 1e-10)


@pytest.mark.parametrize("nrhs", [1, 12])
def test_solve_fp32_krylov_basis(small, gpu_lib, nrhs):
    """Krylov basis stored in FP32 between FP64 restarts: the same FP64
    true-residual target, checked by the oracle, in about as many steps as
    the FP64 basis, and the graph-replayed V-cycle (which then reads each
    FP32 basis vector in place) gives the graph-free run's solution bit for
    bit."""
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, nrhs, 9100)
    x64 = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    s64 = mg.solve(x64, dev(b), coarse_prec="bf16", fine_eo=1)
    x32 = torch.zeros_like(x64)
    s32 = mg.solve(x32, dev(b), coarse_prec="bf16", fine_eo=1, krylov_prec=gpu_lib.F32)
    assert all(s32["converged"]) and max(s32["rel_resid"]) <= 1e-10
    assert np.all(O.true_residual(U, A, KAPPA, x32.cpu().numpy(), b, dims) <= 1e-10)
    assert s32["iters"] <= s64["iters"] + 3, (s32["iters"], s64["iters"])
    x_ng = torch.zeros_like(x64)
    s_ng = mg.solve(x_ng, dev(b), coarse_prec="bf16", fine_eo=1, krylov_prec=gpu_lib.F32, use_graph=False)
    assert s_ng["iters"] == s32["iters"] and torch.equal(x_ng, x32)
    # and the FP64 basis still solves after the FP32 one (buffers re-sized back)
    x64b = torch.zeros_like(x64)
    s64b = mg.solve(x64b, dev(b), coarse_prec="bf16", fine_eo=1)
    assert s64b["iters"] == s64["iters"] and torch.equal(x64b, x64)


def test_unpreconditioned_fp32_krylov_and_bad_precision(small, gpu_lib):
    """Plain restarted GMRES with an FP32 basis still reaches the FP64 target
    through its FP64 restarts; a basis precision other than FP64 or FP32 is
    refused."""
    import torch

    dims, U, A, ctx, mg = small
    b = synth.spinor_source(dims, 3, 56)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st = mg.solve(x, dev(b), precondition=False, restart=15, max_iters=2000, krylov_prec=gpu_lib.F32)
    assert all(st["converged"]) and st["cycles"] >= 2
    assert np.all(O.true_residual(U, A, KAPPA, x.cpu().numpy(), b, dims) <= 1e-10)
    with pytest.raises(gpu_lib.MrhsError, match="UNSUPPORTED"):
        mg.solve(torch.zeros_like(x), dev(b), krylov_prec=gpu_lib.BF16)


def test_vcycle_same_with_walk_and_fused_residual(small, tmp_path):
    """With the fine kernel tuned to the t-walk, the V-cycle's fine-level
    residual r = b - D x runs as one fused launch; with the tiled kernel it
    is the operator and a subtraction.  Both compute the same FP32 values,
    so the preconditioned vectors agree bit for bit (full-lattice and
    even-odd smoothers)."""
    import torch

    dims, U, A, ctx, mg = small
    n = 6
    v = dev(synth.spinor_source(dims, n, 9400, np.complex64))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    from test_gpu_fine import _hip_runtime_version

    def run(tile, curve, fine_eo):
        cache = tmp_path / f"c{curve}.txt"
        cache.write_text(f"{arch} {_hip_runtime_version()} {' '.join(map(str, dims))} {n} 2 "
                         f"{' '.join(map(str, tile))} {curve} 0 0 1 0 1.0\n")
        ctx.tune([n], str(cache))
        assert bool(ctx.get_tuning(n)[2] & 128) == (curve == 2)
        z = torch.empty_like(v)
        mg.precondition(z, v, nu_pre=1, nu_post=2, coarsest_iters=8, coarse_prec="bf16", fine_eo=fine_eo)
        return z
    for fine_eo in (False, True):
        z_walk = run((4, 4, 2, 2), 2, fine_eo)
        z_tiled = run((2, 2, 2, 2), 0, fine_eo)
        assert torch.equal(z_tiled, z_walk), fine_eo


def test_solve_same_with_f64_walk(small):
    """The outer solver's FP64 residuals run the tiled FP64 kernel or the FP64
    t-walk; the two give the same bits, so the whole solve does too."""
    import torch

    dims, U, A, ctx, mg = small
    n = 4
    b = dev(synth.spinor_source(dims, n, 9500))
    out = []
    for tile in (None, (4, 4, 4, 4), (8, 2, 4, 2)):
        ctx.set_f64_walk(n, tile, 1 if tile else 0)
        x = torch.zeros_like(b)
        st = mg.solve(x, b, use_graph=False, coarse_prec="bf16", restart=6)
        assert all(st["converged"])
        out.append((st["iters"], x))
    ctx.set_f64_walk(n, None)
    for iters, x in out[1:]:
        assert iters == out[0][0]
        assert torch.equal(x, out[0][1])
