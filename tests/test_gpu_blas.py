"""GPU parity of the batched level-1 operations (simultaneous inner products)
against the FP64 oracle.

The GPU widens FP32 inputs to FP64 before multiplying, as the oracle does, so
the two differ only in the order of the FP64 sums.  Summing n terms in any
order is off by at most about log2(n) * 1.1e-16 * sum|term| for a tree and
n * 1.1e-16 * sum|term| for a running sum; the check allows 1e-12 * sum|term|
per column, which covers both orders up to n ~ 1e4 sequential (the GPU's
partials are short sequential runs joined by a tree).
"""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _abs_sum(a, b):
    """sum_s |a_s| |b_s| per column: the scale of the rounding error of a dot."""
    n = a.shape[-1]
    return np.einsum("in,in->n", np.abs(a.reshape(-1, n).astype(np.complex128)),
                     np.abs(b.reshape(-1, n).astype(np.complex128)))


def _check_dot(got, a, b, want):
    assert np.all(np.abs(got - want) <= 1e-12 * _abs_sum(a, b)), np.max(np.abs(got - want) / _abs_sum(a, b))


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context((4, 4, 4, 4), t_bc=-1)
    yield c
    c.close()


SHAPES = [(1, 1, 1), (7, 3, 5), (4096, 12, 1), (1296, 32, 24), (333, 12, 64), (81, 32, 13), (10000, 12, 48)]


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
@pytest.mark.parametrize("shape", SHAPES)
def test_dot_norm_vs_oracle(ctx, shape, dt):
    import torch

    ns, nc, n = shape
    a = synth.coarse_source(ns, nc, n, 10, dt)
    b = synth.coarse_source(ns, nc, n, 500, dt)
    ta, tb = _dev(torch, a), _dev(torch, b)
    got = ctx.dot(ta, tb)
    _check_dot(got, a, b, O.dot(a, b))
    got_n = ctx.norm2(ta)
    np.testing.assert_allclose(got_n, O.norm2(a), rtol=1e-12, atol=0)
    # device output stays on the device and matches the host path bit for bit
    od = torch.empty(n, dtype=torch.complex128, device="cuda")
    ctx.dot(ta, tb, out=od)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(od.cpu().numpy(), got)


def test_dot_deterministic_and_column_independent(ctx):
    import torch

    a = synth.coarse_source(5000, 12, 24, 1, np.complex64)
    b = synth.coarse_source(5000, 12, 24, 2, np.complex64)
    ta, tb = _dev(torch, a), _dev(torch, b)
    r1 = ctx.dot(ta, tb)
    r2 = ctx.dot(ta, tb)
    np.testing.assert_array_equal(r1, r2)
    # norm of a is the real dot <a, a>
    np.testing.assert_allclose(ctx.norm2(ta), ctx.dot(ta, ta).real, rtol=1e-14)


@pytest.mark.parametrize("n", [12, 7])  # FP32 at even n: the column-pair kernel; odd n: one column per thread
@pytest.mark.parametrize("m", [1, 3, 9, 16])
@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_multi_dot(ctx, m, dt, n):
    import torch

    ns, nc = 2000, 12
    w = synth.coarse_source(ns, nc, n, 9, dt)
    vs = [synth.coarse_source(ns, nc, n, 100 + 50 * j, dt) for j in range(m)]
    got = ctx.multi_dot([_dev(torch, v) for v in vs], _dev(torch, w))
    for j, v in enumerate(vs):
        _check_dot(got[j], v, w, O.dot(v, w))


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_axpy(ctx, dt):
    import torch

    ns, nc, n = 777, 12, 6
    x = synth.coarse_source(ns, nc, n, 3, dt)
    y = synth.coarse_source(ns, nc, n, 4, dt)
    alpha = synth.gaussian_complex(synth.rng(5), (n,))
    ty = _dev(torch, y)
    ctx.axpy(ty, alpha, _dev(torch, x))
    want = y.astype(np.complex128) + alpha[None, None, :] * x.astype(np.complex128)
    tol = 1e-6 if dt == np.complex64 else 1e-15
    got = ty.cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < tol


def test_blas_rejects_bad_args(ctx, gpu_lib):
    import torch

    a = torch.zeros((4, 12, 65), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpu_lib.MrhsError, match="SHAPE"):
        ctx.norm2(a)
    v = torch.zeros((4, 12, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpu_lib.MrhsError, match="SHAPE"):
        ctx.multi_dot([v] * 17, v)


def test_dot_full_size(ctx):
    """24^4 fine fields, 12 components, Nrhs = 24, FP32 inputs, FP64 sums."""
    import torch

    dims = (24, 24, 24, 24)
    a = synth.spinor_source(dims, 24, 7000, np.complex64)
    b = synth.spinor_source(dims, 24, 8000, np.complex64)
    got = ctx.dot(_dev(torch, a), _dev(torch, b))
    _check_dot(got, a, b, O.dot(a, b))
    got = ctx.norm2(_dev(torch, a))
    np.testing.assert_allclose(got, O.norm2(a), rtol=1e-12, atol=0)
