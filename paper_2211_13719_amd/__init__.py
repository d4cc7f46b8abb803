"""MI355X MRHS Wilson-clover multigrid hot path: thin Python binding over libmrhs.

Every operation runs in the HIP library (``libmrhs.so``, built in-tree for
gfx950); this module only marshals arguments.  PyTorch provides device
memory and the stream: fields are CUDA/HIP tensors of dtype complex64 (FP32)
or complex128 (FP64) laid out [site][component][rhs], exactly the C layout.

    ctx = Context((24, 24, 24, 24), t_bc=-1)
    ctx.set_gauge(U)                  # (V, 4, 3, 3) complex, host or device
    ctx.build_clover(csw=1.0, kappa=0.13)
    ctx.dwc(out, psi)                 # out = (A - kappa H) psi, psi (V, 12, N)
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import BF16, F16, F32, F64, MrhsError  # noqa: F401

lib = _lib.lib

__all__ = ["Context", "Multigrid", "MrhsError", "F64", "F32", "BF16", "F16", "lib"]


def _torch():
    import torch

    return torch


def _prec_of(t) -> int:
    torch = _torch()
    if t.dtype in (torch.complex128, torch.float64):
        return F64
    if t.dtype in (torch.complex64, torch.float32):
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr_of(a):
    """(pointer, prec, on_device) of a numpy array or a torch tensor (contiguous)."""
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        if a.dtype in (np.complex128, np.float64):
            p = F64
        elif a.dtype in (np.complex64, np.float32):
            p = F32
        else:
            raise TypeError(f"unsupported dtype {a.dtype}")
        return a.ctypes.data, p, 0
    if not a.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return a.data_ptr(), _prec_of(a), int(a.is_cuda)


class Context:
    """One lattice on one GPU; wraps an ``mrhs_ctx``."""

    def __init__(self, dims, t_bc: int = -1, device: int = 0, stream=None):
        torch = _torch()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = C.c_void_p()
        d = (C.c_int32 * 4)(*self.dims)
        st = lib.mrhs_create(C.byref(h), d, int(t_bc), int(device), C.c_void_p(stream.cuda_stream))
        if st != 0:
            raise MrhsError(st, lib.mrhs_last_error(None).decode())
        self._h = h

    # -- plumbing -------------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            raise MrhsError(st, lib.mrhs_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.mrhs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def synchronize(self):
        self._check(lib.mrhs_synchronize(self._h))

    def set_stream(self, stream):
        self._stream = stream
        self._check(lib.mrhs_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    # -- gauge and clover ---------------------------------------------------------
    def set_gauge(self, U):
        if tuple(U.shape) != (self.V, 4, 3, 3):
            raise ValueError(f"gauge shape {tuple(U.shape)} != {(self.V, 4, 3, 3)}")
        p, prec, dev = _ptr_of(U)
        self._check(lib.mrhs_set_gauge(self._h, C.c_void_p(p), prec, dev))

    def build_clover(self, csw: float, kappa: float):
        self._check(lib.mrhs_build_clover(self._h, float(csw), float(kappa)))
        self.kappa = float(kappa)

    def set_clover(self, A, kappa: float):
        if tuple(A.shape) != (self.V, 2, 36):
            raise ValueError(f"clover shape {tuple(A.shape)} != {(self.V, 2, 36)}")
        p, prec, dev = _ptr_of(A)
        self._check(lib.mrhs_set_clover(self._h, C.c_void_p(p), prec, dev, float(kappa)))
        self.kappa = float(kappa)

    def get_clover(self, prec: int = F64) -> np.ndarray:
        out = np.empty((self.V, 2, 36), dtype=np.float64 if prec == F64 else np.float32)
        self._check(lib.mrhs_get_clover(self._h, C.c_void_p(out.ctypes.data), prec, 0))
        return out

    # -- fine operator ---------------------------------------------------------------
    def _fine(self, fn, out, inp):
        if inp.dim() != 3 or inp.shape[0] != self.V or inp.shape[1] != 12:
            raise ValueError(f"field shape {tuple(inp.shape)} is not (V={self.V}, 12, N)")
        if out.shape != inp.shape or out.dtype != inp.dtype:
            raise ValueError("out must match in (shape and dtype)")
        if not (inp.is_cuda and out.is_cuda):
            raise ValueError("fields must be device tensors")
        pi, prec, _ = _ptr_of(inp)
        po, _, _ = _ptr_of(out)
        self._check(fn(self._h, C.c_void_p(po), C.c_void_p(pi), int(inp.shape[2]), prec))
        return out

    def dwc(self, out, inp):
        """out = (A - kappa H) inp."""
        return self._fine(lib.mrhs_dwc_apply, out, inp)

    def hop(self, out, inp):
        """out = H inp."""
        return self._fine(lib.mrhs_hop_apply, out, inp)

    def clover(self, out, inp):
        """out = A inp."""
        return self._fine(lib.mrhs_clover_apply, out, inp)

    # -- even-odd (checkerboard) pieces ----------------------------------------------------
    def _half(self, out, inp):
        if inp.dim() != 3 or inp.shape[0] != self.V // 2 or inp.shape[1] != 12:
            raise ValueError(f"checkerboard field shape {tuple(inp.shape)} is not (V/2={self.V // 2}, 12, N)")
        if out.shape != inp.shape or out.dtype != inp.dtype:
            raise ValueError("out must match in (shape and dtype)")
        if not (inp.is_cuda and out.is_cuda):
            raise ValueError("fields must be device tensors")
        pi, prec, _ = _ptr_of(inp)
        po, _, _ = _ptr_of(out)
        return C.c_void_p(po), C.c_void_p(pi), int(inp.shape[2]), prec

    def hop_eo(self, out, inp, out_parity: int):
        """M_eooe: out (parity out_parity) = H inp (the other parity); fields (V/2, 12, N)."""
        po, pi, n, prec = self._half(out, inp)
        self._check(lib.mrhs_hop_eo_apply(self._h, po, pi, n, int(out_parity), prec))
        return out

    def clover_eo(self, out, inp, parity: int, inverse: bool = False):
        """M_ooee on one parity: out = A_p inp, or A_p^-1 inp with inverse=True."""
        po, pi, n, prec = self._half(out, inp)
        self._check(lib.mrhs_clover_eo_apply(self._h, po, pi, n, int(parity), int(bool(inverse)), prec))
        return out

    def schur(self, out, inp):
        """out = (A_e - kappa^2 H_eo A_o^-1 H_oe) inp on the even sites."""
        po, pi, n, prec = self._half(out, inp)
        self._check(lib.mrhs_schur_apply(self._h, po, pi, n, prec))
        return out

    # -- autotuning ------------------------------------------------------------------------
    def tune(self, nrhs_list, cache_path=None):
        """Pick the fastest FP32 fine-kernel launch configuration for each nrhs."""
        arr = (C.c_int32 * len(nrhs_list))(*[int(n) for n in nrhs_list])
        path = cache_path.encode() if cache_path else None
        self._check(lib.mrhs_tune(self._h, arr, len(nrhs_list), path))

    def get_tuning(self, nrhs: int):
        """(rhs_per_thread, tile, curve, microseconds) in use for nrhs (zeros when untuned)."""
        r = C.c_int32()
        t = (C.c_int32 * 4)()
        cv = C.c_int32()
        us = C.c_float()
        self._check(lib.mrhs_get_tuning(self._h, int(nrhs), C.byref(r), t, C.byref(cv), C.byref(us)))
        return int(r.value), tuple(t), int(cv.value), float(us.value)

    # -- batched level-1 operations ---------------------------------------------------
    @staticmethod
    def _field_shape(t):
        if t.dim() != 3:
            raise ValueError(f"field must be (nsites, ncomp, nrhs), got {tuple(t.shape)}")
        if not t.is_cuda:
            raise ValueError("fields must be device tensors")
        return int(t.shape[0]), int(t.shape[1]), int(t.shape[2])

    def dot(self, a, b, out=None):
        """Per-column <a_k, b_k> (complex128, FP64 sums).  With ``out`` (a device
        complex128 tensor of nrhs entries) the call stays asynchronous."""
        ns, nc, n = self._field_shape(a)
        if b.shape != a.shape or b.dtype != a.dtype:
            raise ValueError("a and b must match")
        pa, prec, _ = _ptr_of(a)
        pb, _, _ = _ptr_of(b)
        if out is not None:
            self._check(lib.mrhs_dot(self._h, C.c_void_p(out.data_ptr()), C.c_void_p(pa), C.c_void_p(pb), ns, nc, n,
                                     prec, 1))
            return out
        res = np.empty(n, dtype=np.complex128)
        self._check(lib.mrhs_dot(self._h, C.c_void_p(res.ctypes.data), C.c_void_p(pa), C.c_void_p(pb), ns, nc, n,
                                 prec, 0))
        return res

    def norm2(self, a, out=None):
        """Per-column ||a_k||^2 (float64)."""
        ns, nc, n = self._field_shape(a)
        pa, prec, _ = _ptr_of(a)
        if out is not None:
            self._check(lib.mrhs_norm2(self._h, C.c_void_p(out.data_ptr()), C.c_void_p(pa), ns, nc, n, prec, 1))
            return out
        res = np.empty(n, dtype=np.float64)
        self._check(lib.mrhs_norm2(self._h, C.c_void_p(res.ctypes.data), C.c_void_p(pa), ns, nc, n, prec, 0))
        return res

    def set_eo_walk(self, nrhs: int, tile=None, rhs_per_thread: int = 0):
        """Checkerboard hop kernel for nrhs: tile (Bx, By, Bz, Ts) = t-walk, None = tiled."""
        t = None if tile is None else (C.c_int32 * 4)(*[int(v) for v in tile])
        self._check(lib.mrhs_set_eo_walk(self._h, int(nrhs), t, int(rhs_per_thread)))

    def get_eo_walk(self, nrhs: int):
        """(on, rhs_per_thread, tile, us, us_tiled) of the checkerboard hop for nrhs."""
        on, r = C.c_int32(), C.c_int32()
        t = (C.c_int32 * 4)()
        us, ut = C.c_float(), C.c_float()
        self._check(lib.mrhs_get_eo_walk(self._h, int(nrhs), C.byref(on), C.byref(r), t, C.byref(us), C.byref(ut)))
        return bool(on.value), r.value, tuple(t), float(us.value), float(ut.value)

    def set_f64_walk(self, nrhs: int, tile=None, variant: int = 0):
        """FP64 operator kernel for nrhs: tile (Bx, By, Bz, Ts) = t-walk, None = tiled;
        variant bit 0 non-temporal stores, bit 1 two-workgroup register budget."""
        t = None if tile is None else (C.c_int32 * 4)(*[int(v) for v in tile])
        self._check(lib.mrhs_set_f64_walk(self._h, int(nrhs), t, int(variant)))

    def get_f64_walk(self, nrhs: int):
        """(on, tile, variant, us, us_tiled) of the FP64 operator for nrhs."""
        on, v = C.c_int32(), C.c_int32()
        t = (C.c_int32 * 4)()
        us, ut = C.c_float(), C.c_float()
        self._check(lib.mrhs_get_f64_walk(self._h, int(nrhs), C.byref(on), t, C.byref(v), C.byref(us), C.byref(ut)))
        return bool(on.value), tuple(t), v.value, float(us.value), float(ut.value)

    def read_probe(self, buf, sweeps: int, grid: int, depth: int = 8) -> float:
        """Milliseconds for `sweeps` grid-stride reads of the device tensor buf,
        `depth` independent 16-byte loads in flight per thread."""
        ms = C.c_float()
        self._check(lib.mrhs_read_probe(self._h, C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                        int(sweeps), int(grid), int(depth), C.byref(ms)))
        return float(ms.value)

    def multi_dot(self, vs, w, out=None, noalloc=False):
        """(m, nrhs) complex128 array of <v_j,k, w_k>; into the device tensor
        `out` (complex128, (m, nrhs)) when given.  noalloc selects the entry
        point that allocates nothing (fixed device scratch array)."""
        ns, nc, n = self._field_shape(w)
        m = len(vs)
        ptrs = (C.c_void_p * m)()
        for j, v in enumerate(vs):
            if v.shape != w.shape or v.dtype != w.dtype or not v.is_contiguous():
                raise ValueError("every v_j must match w")
            ptrs[j] = v.data_ptr()
        pw, prec, _ = _ptr_of(w)
        fn = lib.mrhs_multi_dot_noalloc if noalloc else lib.mrhs_multi_dot
        if out is not None:
            if tuple(out.shape) != (m, n) or not out.is_cuda or not out.is_contiguous() or \
                    out.dtype != _torch().complex128:
                raise ValueError(f"out must be a contiguous complex128 device tensor of shape {(m, n)}")
            self._check(fn(self._h, C.c_void_p(out.data_ptr()), ptrs, m, C.c_void_p(pw), ns, nc, n, prec, 1))
            return out
        res = np.empty((m, n), dtype=np.complex128)
        self._check(fn(self._h, C.c_void_p(res.ctypes.data), ptrs, m, C.c_void_p(pw), ns, nc, n, prec, 0))
        return res

    def axpy(self, y, alpha, x):
        """y_k += alpha_k x_k in place; alpha is a length-nrhs complex sequence."""
        ns, nc, n = self._field_shape(y)
        if x.shape != y.shape or x.dtype != y.dtype:
            raise ValueError("x and y must match")
        al = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha, dtype=np.complex128), (n,)))
        py, prec, _ = _ptr_of(y)
        px, _, _ = _ptr_of(x)
        self._check(lib.mrhs_axpy(self._h, C.c_void_p(py), C.c_void_p(al.ctypes.data), C.c_void_p(px), ns, nc, n,
                                  prec, 0))
        return y


_PREC_NAMES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}


class Multigrid:
    """Aggregation hierarchy on a Context's lattice; wraps an ``mrhs_mg``.

    blocks[l] is the aggregate extent of coarsening step l and n_v[l] its
    number of basis vectors; level l + 1 has 2 n_v[l] components per site.
    """

    def __init__(self, ctx: Context, blocks, n_v):
        self.ctx = ctx
        nlev = len(blocks) + 1
        if len(n_v) != len(blocks):
            raise ValueError("need one n_v per coarsening step")
        p = _lib.MgParams()
        p.nlevels = nlev
        for l, b in enumerate(blocks):
            for m in range(4):
                p.block[l][m] = int(b[m])
            p.n_v[l] = int(n_v[l])
        h = C.c_void_p()
        ctx._check(lib.mrhs_mg_create(ctx.handle, C.byref(p), C.byref(h)))
        self._h = h
        self.nlevels = nlev
        self.n_v = [int(v) for v in n_v]
        self.dims, self.ncomp = [], []
        for l in range(nlev):
            d = (C.c_int32 * 4)()
            nc = C.c_int32()
            ctx._check(lib.mrhs_mg_level_info(h, l, d, C.byref(nc)))
            self.dims.append(tuple(d))
            self.ncomp.append(int(nc.value))
        self.volume = [int(np.prod(d)) for d in self.dims]

    def close(self):
        if getattr(self, "_h", None):
            lib.mrhs_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _check(self, st):
        self.ctx._check(st)

    # -- basis --------------------------------------------------------------------------
    def set_basis(self, level: int, vecs):
        want = (self.volume[level], self.n_v[level], self.ncomp[level])
        if tuple(vecs.shape) != want:
            raise ValueError(f"basis shape {tuple(vecs.shape)} != {want}")
        p, prec, dev = _ptr_of(vecs)
        self._check(lib.mrhs_mg_set_basis(self._h, level, C.c_void_p(p), prec, dev))

    def get_basis(self, level: int) -> np.ndarray:
        out = np.empty((self.volume[level], self.n_v[level], self.ncomp[level]), dtype=np.complex128)
        self._check(lib.mrhs_mg_get_basis(self._h, level, C.c_void_p(out.ctypes.data), F64, 0))
        return out

    def block_orthonormalise(self, level: int):
        self._check(lib.mrhs_mg_block_orthonormalise(self._h, level))

    # -- intergrid ----------------------------------------------------------------------
    def _pair(self, a, b, la, lb):
        for t, l in ((a, la), (b, lb)):
            if t.dim() != 3 or t.shape[0] != self.volume[l] or t.shape[1] != self.ncomp[l]:
                raise ValueError(f"field {tuple(t.shape)} is not (V={self.volume[l]}, {self.ncomp[l]}, N) on level {l}")
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("fields must be contiguous device tensors")
        if a.shape[2] != b.shape[2] or a.dtype != b.dtype:
            raise ValueError("fields must share nrhs and dtype")
        return int(a.shape[2]), _prec_of(a)

    def _ig_prec(self, prec, field_prec):
        if prec is None:
            return field_prec
        if field_prec != F32:
            raise ValueError("matrix-core intergrid operators take FP32 fields")
        return _PREC_NAMES[prec]

    def restrict(self, level: int, coarse, fine, prec=None):
        """coarse = P^dag fine; prec "bf16" runs on the matrix cores (FP32 fields)."""
        n, p = self._pair(coarse, fine, level + 1, level)
        p = self._ig_prec(prec, p)
        self._check(lib.mrhs_restrict(self._h, level, C.c_void_p(coarse.data_ptr()), C.c_void_p(fine.data_ptr()), n,
                                      p))
        return coarse

    def prolong(self, level: int, fine, coarse, prec=None):
        """fine = P coarse; prec "bf16" runs on the matrix cores (FP32 fields)."""
        n, p = self._pair(fine, coarse, level, level + 1)
        p = self._ig_prec(prec, p)
        self._check(lib.mrhs_prolong(self._h, level, C.c_void_p(fine.data_ptr()), C.c_void_p(coarse.data_ptr()), n,
                                     p))
        return fine

    def block_normalise(self, level: int, fields, norms=None):
        n, prec = self._pair(fields, fields, level, level)
        pn = C.c_void_p(norms.data_ptr()) if norms is not None else None
        self._check(lib.mrhs_block_normalise(self._h, level, C.c_void_p(fields.data_ptr()), n, prec, pn))
        return fields

    # -- coarse operator ------------------------------------------------------------------
    def set_blocks(self, level: int, blocks):
        nb = self.ncomp[level]
        want = (self.volume[level], 9, nb, nb)
        if tuple(blocks.shape) != want:
            raise ValueError(f"block shape {tuple(blocks.shape)} != {want}")
        p, prec, dev = _ptr_of(blocks)
        self._check(lib.mrhs_coarse_set_blocks(self._h, level, C.c_void_p(p), prec, dev))

    def get_blocks(self, level: int) -> np.ndarray:
        nb = self.ncomp[level]
        out = np.empty((self.volume[level], 9, nb, nb), dtype=np.complex128)
        self._check(lib.mrhs_coarse_get_blocks(self._h, level, C.c_void_p(out.ctypes.data), F64, 0))
        return out

    def build_coarse(self, level: int):
        self._check(lib.mrhs_mg_build_coarse(self._h, level))

    def coarse_apply(self, level: int, out, inp, prec=None):
        """out = D_c inp on coarse level ``level``; prec is "f64", "f32", "bf16" or "f16"
        (default: the fields' own precision)."""
        n, fprec = self._pair(out, inp, level, level)
        p = fprec if prec is None else _PREC_NAMES[prec]
        self._check(lib.mrhs_coarse_apply(self._h, level, C.c_void_p(out.data_ptr()), C.c_void_p(inp.data_ptr()), n,
                                          p))
        return out

    def tune(self, nrhs_list):
        """Time the FP32 coarse stencil kernels (matrix cores vs vector ALU) per level and nrhs."""
        arr = (C.c_int32 * len(nrhs_list))(*[int(n) for n in nrhs_list])
        self._check(lib.mrhs_mg_tune(self._h, arr, len(nrhs_list)))

    def get_tuning(self, level: int, nrhs: int) -> str:
        """"valu" or "mfma": the FP32 stencil kernel level uses for nrhs."""
        v = C.c_int32()
        self._check(lib.mrhs_mg_get_tuning(self._h, int(level), int(nrhs), C.byref(v), None))
        return "valu" if v.value else "mfma"

    def set_lowp_cfg(self, level: int, nrhs: int, cfg: int):
        """Launch shape of the BF16/FP16 stencil on level for nrhs, by hand (0..3)."""
        self._check(lib.mrhs_mg_set_lowp_cfg(self._h, int(level), int(nrhs), int(cfg)))

    def coarse_mr_solve(self, level: int, x, b, iters: int, prec="bf16"):
        """x ~ D_c^-1 b by `iters` MR steps from zero on coarse level `level`
        (complex64 fields (V_level, Nb, N))."""
        n, fprec = self._pair(x, b, level, level)
        if fprec != F32:
            raise TypeError("coarse MR works on complex64 fields")
        self._check(lib.mrhs_coarse_mr_solve(self._h, int(level), C.c_void_p(x.data_ptr()), C.c_void_p(b.data_ptr()),
                                             n, int(iters), _PREC_NAMES[prec]))
        return x

    def get_lowp_tuning(self, level: int, nrhs: int) -> dict:
        """Launch shape of the BF16/FP16 stencil on level for nrhs."""
        v, c = C.c_int32(), C.c_int32()
        self._check(lib.mrhs_mg_get_tuning(self._h, int(level), int(nrhs), C.byref(v), C.byref(c)))
        return {"waves_per_site": 8 if c.value & 1 else 4, "rhs_per_workgroup": 64 if c.value & 2 else 32,
                "cfg": int(c.value)}

    def _half_pair(self, a, b, level):
        for t in (a, b):
            if t.dim() != 3 or t.shape[0] != self.volume[level] // 2 or t.shape[1] != self.ncomp[level]:
                raise ValueError(f"field {tuple(t.shape)} is not (V/2={self.volume[level] // 2}, "
                                 f"{self.ncomp[level]}, N) on level {level}")
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("fields must be contiguous device tensors")
        if a.shape[2] != b.shape[2] or a.dtype != b.dtype:
            raise ValueError("fields must share nrhs and dtype")
        if _prec_of(a) != F32:
            raise ValueError("the even-odd stencil calls take FP32 fields")
        return int(a.shape[2])

    def coarse_hop_eo(self, level: int, out, inp, out_parity: int, prec="f32"):
        """Coarse M_eooe: the eight hop directions of D_c from parity 1 - out_parity to
        out_parity; checkerboard fields (V/2, Nb, N) in FP32, arithmetic prec."""
        n = self._half_pair(out, inp, level)
        self._check(lib.mrhs_coarse_hop_eo_apply(self._h, level, C.c_void_p(out.data_ptr()),
                                                 C.c_void_p(inp.data_ptr()), n, int(out_parity),
                                                 _PREC_NAMES[prec]))
        return out

    def coarse_self_eo(self, level: int, out, inp, parity: int, inverse: bool = False, prec="f32"):
        """Self blocks (or their inverses) of the parity-p coarse sites applied to inp."""
        n = self._half_pair(out, inp, level)
        self._check(lib.mrhs_coarse_self_eo_apply(self._h, level, C.c_void_p(out.data_ptr()),
                                                  C.c_void_p(inp.data_ptr()), n, int(parity), int(bool(inverse)),
                                                  _PREC_NAMES[prec]))
        return out

    # -- solver ---------------------------------------------------------------------------
    @staticmethod
    def _vc(nu_pre=0, nu_post=4, coarsest_iters=16, coarse_prec="bf16", fine_eo=False, coarse_eo=False,
            fine_sap=False, sap_iters=4):
        v = _lib.VcycleParams()
        v.nu_pre, v.nu_post, v.coarsest_iters = int(nu_pre), int(nu_post), int(coarsest_iters)
        v.coarse_prec = _PREC_NAMES[coarse_prec]
        v.fine_eo = int(bool(fine_eo))
        v.coarse_eo = int(bool(coarse_eo))
        v.fine_sap = int(bool(fine_sap))
        v.sap_iters = int(sap_iters)
        return v

    def setup(self, setup_iters: int = 3, smooth_steps: int = 8, adapt_iters: int = 0, **vc):
        """Refine the basis vectors already set on every step (smoothing of D x = 0),
        block-orthonormalise them and build all coarse operators; then adapt_iters
        passes of inverse iteration v <- K v with K the hierarchy's own V-cycle (vc options)."""
        p = _lib.SetupParams()
        p.setup_iters, p.smooth_steps, p.adapt_iters = int(setup_iters), int(smooth_steps), int(adapt_iters)
        p.vc = self._vc(**vc)
        self._check(lib.mrhs_mg_setup(self._h, C.byref(p)))

    def precondition(self, z, v, **vc):
        """z = V-cycle(v) for FP32 fine fields (V, 12, N)."""
        n, prec = self._pair(z, v, 0, 0)
        if prec != F32:
            raise TypeError("the V-cycle works on complex64 fields")
        p = self._vc(**vc)
        self._check(lib.mrhs_mg_precondition(self._h, C.c_void_p(z.data_ptr()), C.c_void_p(v.data_ptr()), n,
                                             C.byref(p)))
        return z

    def solve(self, x, b, tol=1e-10, restart=8, max_iters=500, precondition=True, use_graph=True, timers=False,
              check=True, reorth_eta=0.01, krylov_prec=F64, **vc):
        """Solve D x_k = b_k (complex128 fields (V, 12, N); x holds the initial guess).
        krylov_prec F32 stores the outer Krylov basis in FP32 (FP64 restarts).
        Returns a dict of statistics; raises MrhsError unless converged when check is set."""
        n, prec = self._pair(x, b, 0, 0)
        if prec != F64:
            raise TypeError("x and b must be complex128")
        p = _lib.SolveParams()
        p.tol, p.restart, p.max_iters = float(tol), int(restart), int(max_iters)
        p.precondition, p.use_graph, p.timers = int(bool(precondition)), int(bool(use_graph)), int(bool(timers))
        p.vc = self._vc(**vc)
        p.reorth_eta = float(reorth_eta)
        p.krylov_prec = int(krylov_prec)
        st = _lib.SolveStats()
        status = lib.mrhs_mg_solve(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(b.data_ptr()), n, C.byref(p),
                                   C.byref(st))
        out = {
            "nrhs": st.nrhs,
            "iters": st.iters,
            "cycles": st.cycles,
            "reorth": st.reorth,
            "converged": [bool(st.converged[k]) for k in range(n)],
            "rel_resid": [float(st.rel_resid[k]) for k in range(n)],
            "seconds_total": st.seconds_total,
            "seconds_precond": st.seconds_precond,
            "seconds_phase": dict(zip(("fine", "restrict", "prolong", "coarse"), list(st.seconds_phase))),
            "status": status,
        }
        if check and status != 0:
            self._check(status)
        return out
