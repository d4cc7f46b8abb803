"""The allocation-free multi-dot (mrhs_multi_dot_noalloc) against the
allocating one (mrhs_multi_dot), through the C-ABI: same kernels, so the
results must agree bit for bit, on two calls in a row (the second on a
smaller input, so stale partials of the first would show) and for host and
device destinations; both also match the FP64 oracle's inner products."""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _fields(torch, dims, m, n, seed, dt):
    vs = [torch.from_numpy(synth.spinor_source(dims, n, seed + 10 * j, dt)).cuda() for j in range(m)]
    w = torch.from_numpy(synth.spinor_source(dims, n, seed + 999, dt)).cuda()
    return vs, w


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_noalloc_multi_dot_matches_allocating_one(gpu_lib, dt):
    import torch

    ctx = gpu_lib.Context((8, 8, 8, 8), t_bc=-1)
    for dims, m, n, seed in (((8, 8, 8, 8), 16, 24, 100), ((8, 8, 8, 8), 3, 5, 200)):
        vs, w = _fields(torch, dims, m, n, seed, dt)
        want = ctx.multi_dot(vs, w)
        got = ctx.multi_dot(vs, w, noalloc=True)
        np.testing.assert_array_equal(got, want)
        dev = torch.empty((m, n), dtype=torch.complex128, device="cuda")
        ctx.multi_dot(vs, w, out=dev, noalloc=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(dev.cpu().numpy(), want)
        ref = np.array([O.dot(v.cpu().numpy(), w.cpu().numpy()) for v in vs])
        scale = np.array([np.einsum("sck,sck->k", np.abs(v.cpu().numpy()), np.abs(w.cpu().numpy())) for v in vs])
        assert np.all(np.abs(got - ref) <= 1e-12 * scale)
    ctx.close()


def test_noalloc_multi_dot_rejects_bad_sizes(gpu_lib):
    import torch

    ctx = gpu_lib.Context((4, 4, 4, 4), t_bc=-1)
    vs, w = _fields(torch, (4, 4, 4, 4), 17, 2, 300, np.complex64)
    with pytest.raises(gpu_lib.MrhsError, match="SHAPE"):
        ctx.multi_dot(vs, w, noalloc=True)
    ctx.close()
