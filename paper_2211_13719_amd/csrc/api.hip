// C-ABI entry points of libmrhs: context handling, argument validation and
// dispatch to the kernel launchers.  Every entry point validates on the host
// before launching anything and converts failures to an mrhs_status with a
// message in the context.
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <new>

#include "internal.h"

namespace {
thread_local std::string g_create_error;

const char* prec_name(mrhs_prec p) {
  switch (p) {
    case MRHS_F64:
      return "f64";
    case MRHS_F32:
      return "f32";
    case MRHS_BF16:
      return "bf16";
    case MRHS_F16:
      return "f16";
  }
  return "?";
}
}  // namespace

namespace mrhs {

mrhs_status fail(mrhs_ctx ctx, mrhs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_create_error = buf;
  return st;
}

mrhs_status hip_fail(mrhs_ctx ctx, hipError_t e, const char* what) {
  const mrhs_status st = (e == hipErrorOutOfMemory) ? MRHS_ERR_OOM : MRHS_ERR_HIP;
  return fail(ctx, st, "%s failed: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

mrhs_status ensure(mrhs_ctx ctx, Buffer& b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return MRHS_OK;
  release(b);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, MRHS_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  b.p = p;
  b.bytes = bytes;
  return MRHS_OK;
}

void release(Buffer& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

}  // namespace mrhs

using namespace mrhs;

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

mrhs_status check_field_args(mrhs_ctx ctx, const void* out, const void* in, int32_t nrhs, mrhs_prec prec,
                             size_t elems_per_rhs_site, int64_t nsites) {
  if (!out || !in) return fail(ctx, MRHS_ERR_INVALID_ARG, "null field pointer");
  if (!aligned16(out) || !aligned16(in)) return fail(ctx, MRHS_ERR_INVALID_ARG, "field pointers must be 16-byte aligned");
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  if (prec != MRHS_F32 && prec != MRHS_F64)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "precision %s not supported for this call", prec_name(prec));
  const size_t csize = (prec == MRHS_F64) ? 16 : 8;
  const size_t bytes = (size_t)nsites * elems_per_rhs_site * nrhs * csize;
  const char* a = static_cast<const char*>(in);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return fail(ctx, MRHS_ERR_INVALID_ARG, "in and out overlap");
  return MRHS_OK;
}

mrhs_status fine_apply(mrhs_ctx ctx, int mode, void* out, const void* in, int32_t nrhs, mrhs_prec prec) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_field_args(ctx, out, in, nrhs, prec, 12, ctx->g.V);
  if (st != MRHS_OK) return st;
  if (mode != 2 && !ctx->have_gauge) return fail(ctx, MRHS_ERR_STATE, "gauge field not set");
  if (mode != 1 && !ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "clover term not set");
  DeviceGuard dg(ctx->device);
  hipError_t e;
  if (prec == MRHS_F32)
    e = launch_fine_f32(ctx->g, ctx->t_bc, mode, (float)ctx->kappa, ctx->U32.p, ctx->A32.p, in, out, nrhs,
                        ctx->stream, &ctx->fine_cfg[nrhs]);
  else
    e = launch_fine_f64(ctx->g, ctx->t_bc, mode, ctx->kappa, ctx->U64.p, ctx->A64.p, in, out, nrhs, ctx->stream,
                        &ctx->f64_walk[nrhs]);
  if (e != hipSuccess) return hip_fail(ctx, e, "fine operator launch");
  return MRHS_OK;
}

// Copy n doubles or floats (given prec) from a host or device pointer into
// the FP64 and FP32 library buffers.
mrhs_status import_real_array(mrhs_ctx ctx, const void* src, mrhs_prec prec, int on_device, size_t n,
                              Buffer& b64, Buffer& b32) {
  mrhs_status st = ensure(ctx, b64, n * 8);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, b32, n * 4);
  if (st != MRHS_OK) return st;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (prec == MRHS_F64) {
    MRHS_HIP(ctx, hipMemcpyAsync(b64.p, src, n * 8, kind, ctx->stream));
    MRHS_HIP(ctx, launch_convert_f64_to_f32(static_cast<const double*>(b64.p), static_cast<float*>(b32.p), n,
                                            ctx->stream));
  } else {
    MRHS_HIP(ctx, hipMemcpyAsync(b32.p, src, n * 4, kind, ctx->stream));
    MRHS_HIP(ctx, launch_convert_f32_to_f64(static_cast<const float*>(b32.p), static_cast<double*>(b64.p), n,
                                            ctx->stream));
  }
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MRHS_OK;
}

}  // namespace

namespace mrhs {

// Checkerboard tables (see fine.hip): built on first use; every extent must
// be even, so that each hop joins the two parities and s = 2i, 2i + 1 always
// hold one site of each.
mrhs_status ensure_eo_tables(mrhs_ctx ctx) {
  if (ctx->eo_tab[0].p && ctx->eo_tab[1].p && ctx->eo_order[0].p && ctx->eo_order[1].p) return MRHS_OK;
  const Geom& g = ctx->g;
  for (int m = 0; m < 4; ++m)
    if (g.L[m] % 2)
      return fail(ctx, MRHS_ERR_SHAPE, "the even-odd operators need even extents (L[%d] = %d)", m, g.L[m]);
  const int nhalf = g.V / 2;
  for (int p = 0; p < 2; ++p) {
    std::vector<int> t((size_t)nhalf * 16, 0);
    for (int i = 0; i < nhalf; ++i) {
      int c[4], r = 2 * i;
      for (int m = 0; m < 4; ++m) {
        c[m] = r % g.L[m];
        r /= g.L[m];
      }
      const int s = 2 * i + (((c[0] + c[1] + c[2] + c[3]) & 1) == p ? 0 : 1);
      if (s != 2 * i) c[0] += 1;
      int* e = &t[(size_t)i * 16];
      for (int m = 0; m < 4; ++m) {
        const int up = c[m] == g.L[m] - 1 ? -(g.L[m] - 1) : 1;
        const int dn = c[m] == 0 ? g.L[m] - 1 : -1;
        const int sf = s + up * g.stride[m], sb = s + dn * g.stride[m];
        e[2 * m] = sf / 2;  // checkerboard index of a neighbour (other parity)
        e[2 * m + 1] = sb / 2;
        e[9 + m] = sb;  // lattice site of the backward neighbour
      }
      e[8] = s;
    }
    mrhs_status st = ensure(ctx, ctx->eo_tab[p], t.size() * 4);
    if (st != MRHS_OK) return st;
    MRHS_HIP(ctx, hipMemcpy(ctx->eo_tab[p].p, t.data(), t.size() * 4, hipMemcpyHostToDevice));
  }
  // traversal: the full kernel's default tiled order, keeping the sites of
  // each parity (as checkerboard indices s / 2)
  std::vector<int> full((size_t)g.V);
  MRHS_HIP(ctx, hipMemcpy(full.data(), g.order, full.size() * 4, hipMemcpyDeviceToHost));
  for (int p = 0; p < 2; ++p) {
    std::vector<int> ord;
    ord.reserve(nhalf);
    for (int s : full) {
      int c[4], r = s;
      for (int m = 0; m < 4; ++m) {
        c[m] = r % g.L[m];
        r /= g.L[m];
      }
      if (((c[0] + c[1] + c[2] + c[3]) & 1) == p) ord.push_back(s / 2);
    }
    if ((int)ord.size() != nhalf) return fail(ctx, MRHS_ERR_SHAPE, "checkerboard traversal is incomplete");
    mrhs_status st = ensure(ctx, ctx->eo_order[p], ord.size() * 4);
    if (st != MRHS_OK) return st;
    MRHS_HIP(ctx, hipMemcpy(ctx->eo_order[p].p, ord.data(), ord.size() * 4, hipMemcpyHostToDevice));
  }
  return MRHS_OK;
}

mrhs_status ensure_clover_inverse(mrhs_ctx ctx) {
  if (ctx->have_clover_inv) return MRHS_OK;
  const size_t n = (size_t)ctx->g.V * 2 * 36;
  mrhs_status st = ensure(ctx, ctx->Ainv64, n * 8);
  if (st == MRHS_OK) st = ensure(ctx, ctx->Ainv32, n * 4);
  Buffer flag;
  if (st == MRHS_OK) st = ensure(ctx, flag, sizeof(int));
  if (st != MRHS_OK) return st;
  int h = 0;
  hipError_t e = hipMemsetAsync(flag.p, 0, sizeof(int), ctx->stream);
  if (e == hipSuccess)
    e = launch_clover_invert((long)ctx->g.V * 2, ctx->A64.p, ctx->Ainv64.p, ctx->Ainv32.p, static_cast<int*>(flag.p),
                             ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  release(flag);
  if (e != hipSuccess) return hip_fail(ctx, e, "clover inversion");
  if (h) return fail(ctx, MRHS_ERR_STATE, "a clover block is singular");
  ctx->have_clover_inv = true;
  return MRHS_OK;
}

// Site traversal of the fine kernels.  Sites are grouped in tiles of extent
// T; tiles are visited t-row by t-row (the tile index along t outermost, so
// that with Lt / T_t = 8 each XCD, which takes a contiguous eighth of the
// traversal, works on its own slab of time slices), and within a t-row
// either lexicographically (curve 0) or along a Morton curve in (x, y, z)
// (curve 1), which keeps tiles that are neighbours in y and z close in time.
// Sites inside a tile are lexicographic.
const int* fine_order_table(mrhs_ctx ctx, const int T[4], int curve) {
  std::array<int, 5> key{T[0], T[1], T[2], T[3], curve};
  for (auto& o : ctx->orders)
    if (o.first == key) return static_cast<const int*>(o.second.p);
  const Geom& g = ctx->g;
  for (int m = 0; m < 4; ++m)
    if (T[m] < 1 || g.L[m] % T[m]) return nullptr;
  const int n0 = g.L[0] / T[0], n1 = g.L[1] / T[1], n2 = g.L[2] / T[2], n3 = g.L[3] / T[3];
  // order of the tiles inside one t-row
  std::vector<std::array<int, 3>> row;
  for (int bz = 0; bz < n2; ++bz)
    for (int by = 0; by < n1; ++by)
      for (int bx = 0; bx < n0; ++bx) row.push_back({bx, by, bz});
  if (curve == 1) {
    auto morton = [](const std::array<int, 3>& c) {
      unsigned long long k = 0;
      for (int bit = 0; bit < 10; ++bit)
        for (int d = 0; d < 3; ++d) k |= (unsigned long long)((c[d] >> bit) & 1) << (3 * bit + d);
      return k;
    };
    std::stable_sort(row.begin(), row.end(),
                     [&](const std::array<int, 3>& a, const std::array<int, 3>& b) { return morton(a) < morton(b); });
  }
  std::vector<int> ord;
  ord.reserve((size_t)g.V);
  for (int bt = 0; bt < n3; ++bt)
    for (const auto& c : row)
      for (int lt = 0; lt < T[3]; ++lt)
        for (int lz = 0; lz < T[2]; ++lz)
          for (int ly = 0; ly < T[1]; ++ly)
            for (int lx = 0; lx < T[0]; ++lx) {
              const int x = c[0] * T[0] + lx, y = c[1] * T[1] + ly, z = c[2] * T[2] + lz, t = bt * T[3] + lt;
              ord.push_back(x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t)));
            }
  Buffer b;
  if (ensure(ctx, b, ord.size() * 4) != MRHS_OK) return nullptr;
  if (hipMemcpy(b.p, ord.data(), ord.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    release(b);
    return nullptr;
  }
  ctx->orders.push_back({key, b});
  return static_cast<const int*>(b.p);
}

}  // namespace mrhs

extern "C" {

mrhs_status mrhs_create(mrhs_ctx* out, const int32_t dims[4], int32_t t_bc, int32_t device, void* stream) {
  g_create_error.clear();
  if (!out || !dims) return fail(nullptr, MRHS_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (t_bc != 1 && t_bc != -1) return fail(nullptr, MRHS_ERR_INVALID_ARG, "t_bc must be +1 or -1, got %d", t_bc);
  int64_t V = 1;
  for (int m = 0; m < 4; ++m) {
    if (dims[m] < 2) return fail(nullptr, MRHS_ERR_SHAPE, "lattice extent %d in direction %d is below 2", dims[m], m);
    V *= dims[m];
  }
  if (V * 64 >= (int64_t(1) << 31)) return fail(nullptr, MRHS_ERR_SHAPE, "lattice volume %lld too large", (long long)V);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, MRHS_ERR_INVALID_ARG, "device %d not available (%d devices)", device, ndev);
  mrhs_ctx ctx = new (std::nothrow) mrhs_ctx_s();
  if (!ctx) return fail(nullptr, MRHS_ERR_OOM, "host allocation failed");
  for (int m = 0; m < 4; ++m) ctx->g.L[m] = dims[m];
  ctx->g.V = (int)V;
  ctx->g.stride[0] = 1;
  ctx->g.stride[1] = dims[0];
  ctx->g.stride[2] = dims[0] * dims[1];
  ctx->g.stride[3] = dims[0] * dims[1] * dims[2];
  set_tile(ctx->g);
  ctx->t_bc = t_bc;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  {
    DeviceGuard dg(device);
    // neighbour table: per site (+x, -x, +y, -y), (+z, -z, +t, -t)
    std::vector<int> nb((size_t)V * 8);
    for (int s = 0; s < (int)V; ++s) {
      int c[4], r = s;
      for (int m = 0; m < 4; ++m) {
        c[m] = r % dims[m];
        r /= dims[m];
      }
      for (int m = 0; m < 4; ++m) {
        const int up = c[m] == dims[m] - 1 ? -(dims[m] - 1) : 1;
        const int dn = c[m] == 0 ? dims[m] - 1 : -1;
        nb[(size_t)s * 8 + 2 * m] = s + up * ctx->g.stride[m];
        nb[(size_t)s * 8 + 2 * m + 1] = s + dn * ctx->g.stride[m];
      }
    }
    mrhs_status st = ensure(ctx, ctx->nbr, nb.size() * 4);
    hipError_t e = st == MRHS_OK ? hipMemcpy(ctx->nbr.p, nb.data(), nb.size() * 4, hipMemcpyHostToDevice) : hipSuccess;
    ctx->g.nbr = static_cast<const int4*>(ctx->nbr.p);
    ctx->g.order = st == MRHS_OK && e == hipSuccess ? fine_order_table(ctx, ctx->g.T) : nullptr;
    if (st != MRHS_OK || e != hipSuccess || !ctx->g.order) {
      g_create_error = "building the index tables failed";
      release(ctx->nbr);
      for (auto& o : ctx->orders) release(o.second);
      delete ctx;
      return MRHS_ERR_OOM;
    }
    // device address of the fixed scratch array of the allocation-free calls
    e = noalloc_scratch_init(device, nullptr);
    if (e != hipSuccess) {
      g_create_error = std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e);
      release(ctx->nbr);
      for (auto& o : ctx->orders) release(o.second);
      delete ctx;
      return MRHS_ERR_HIP;
    }
  }
  *out = ctx;
  return MRHS_OK;
}

void mrhs_destroy(mrhs_ctx ctx) {
  if (!ctx) return;
  DeviceGuard dg(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  release(ctx->U64);
  release(ctx->U32);
  release(ctx->A64);
  release(ctx->A32);
  release(ctx->work);
  release(ctx->scal);
  release(ctx->nbr);
  for (auto& o : ctx->orders) release(o.second);
  for (int p = 0; p < 2; ++p) {
    release(ctx->eo_tab[p]);
    release(ctx->eo_order[p]);
  }
  release(ctx->Ainv64);
  release(ctx->Ainv32);
  release(ctx->eo_work);
  delete ctx;
}

const char* mrhs_last_error(mrhs_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

mrhs_status mrhs_set_stream(mrhs_ctx ctx, void* stream) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  ctx->stream = static_cast<hipStream_t>(stream);
  return MRHS_OK;
}

mrhs_status mrhs_synchronize(mrhs_ctx ctx) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  DeviceGuard dg(ctx->device);
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_set_gauge(mrhs_ctx ctx, const void* U, mrhs_prec prec, int32_t on_device) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (!U) return fail(ctx, MRHS_ERR_INVALID_ARG, "null gauge pointer");
  if (prec != MRHS_F64 && prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "gauge precision %s not supported", prec_name(prec));
  DeviceGuard dg(ctx->device);
  const size_t n = (size_t)ctx->g.V * 4 * 9 * 2;
  mrhs_status st = import_real_array(ctx, U, prec, on_device, n, ctx->U64, ctx->U32);
  if (st != MRHS_OK) return st;
  // The fermion boundary factor multiplies every hop through the t-links of
  // the last time slice (forward from t = Lt-1, backward into t = 0), so it
  // is folded into those links once.  Plaquettes cross that slice an even
  // number of times, so the clover term built from these links is unchanged.
  MRHS_HIP(ctx, launch_fold_boundary_phase(ctx->g, ctx->t_bc, ctx->U64.p, ctx->U32.p, ctx->stream));
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->have_gauge = true;
  ctx->have_clover = false;  // a clover term built from old links is stale
  ctx->have_clover_inv = false;
  ++ctx->op_gen;
  return MRHS_OK;
}

mrhs_status mrhs_build_clover(mrhs_ctx ctx, double csw, double kappa) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (!ctx->have_gauge) return fail(ctx, MRHS_ERR_STATE, "gauge field not set");
  DeviceGuard dg(ctx->device);
  const size_t n = (size_t)ctx->g.V * 2 * 36;
  mrhs_status st = ensure(ctx, ctx->A64, n * 8);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, ctx->A32, n * 4);
  if (st != MRHS_OK) return st;
  Buffer F;
  st = ensure(ctx, F, (size_t)ctx->g.V * 6 * 9 * 16);
  if (st != MRHS_OK) return st;
  hipError_t e = launch_clover_build(ctx->g, csw, kappa, ctx->U64.p, F.p, ctx->A64.p, ctx->A32.p, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  release(F);
  if (e != hipSuccess) return hip_fail(ctx, e, "clover build");
  ctx->kappa = kappa;
  ctx->have_clover = true;
  ctx->have_clover_inv = false;
  ++ctx->op_gen;
  return MRHS_OK;
}

mrhs_status mrhs_set_clover(mrhs_ctx ctx, const void* A, mrhs_prec prec, int32_t on_device, double kappa) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (!A) return fail(ctx, MRHS_ERR_INVALID_ARG, "null clover pointer");
  if (prec != MRHS_F64 && prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "clover precision %s not supported", prec_name(prec));
  DeviceGuard dg(ctx->device);
  const size_t n = (size_t)ctx->g.V * 2 * 36;
  mrhs_status st = import_real_array(ctx, A, prec, on_device, n, ctx->A64, ctx->A32);
  if (st != MRHS_OK) return st;
  ctx->kappa = kappa;
  ctx->have_clover = true;
  ctx->have_clover_inv = false;
  ++ctx->op_gen;
  return MRHS_OK;
}

mrhs_status mrhs_get_clover(mrhs_ctx ctx, void* A, mrhs_prec prec, int32_t on_device) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (!A) return fail(ctx, MRHS_ERR_INVALID_ARG, "null clover pointer");
  if (!ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "clover term not set");
  if (prec != MRHS_F64 && prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "clover precision %s not supported", prec_name(prec));
  DeviceGuard dg(ctx->device);
  const size_t n = (size_t)ctx->g.V * 2 * 36;
  const Buffer& b = (prec == MRHS_F64) ? ctx->A64 : ctx->A32;
  const size_t bytes = n * (prec == MRHS_F64 ? 8 : 4);
  MRHS_HIP(ctx, hipMemcpyAsync(A, b.p, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               ctx->stream));
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_dwc_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec) {
  return fine_apply(ctx, 0, out, in, nrhs, prec);
}

mrhs_status mrhs_hop_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec) {
  return fine_apply(ctx, 1, out, in, nrhs, prec);
}

mrhs_status mrhs_clover_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec) {
  return fine_apply(ctx, 2, out, in, nrhs, prec);
}

mrhs_status mrhs_hop_eo_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, int32_t out_parity,
                              mrhs_prec prec) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (out_parity != 0 && out_parity != 1) return fail(ctx, MRHS_ERR_INVALID_ARG, "parity must be 0 or 1");
  mrhs_status st = check_field_args(ctx, out, in, nrhs, prec, 12, ctx->g.V / 2);
  if (st != MRHS_OK) return st;
  if (!ctx->have_gauge) return fail(ctx, MRHS_ERR_STATE, "gauge field not set");
  DeviceGuard dg(ctx->device);
  st = ensure_eo_tables(ctx);
  if (st != MRHS_OK) return st;
  const int p64 = prec == MRHS_F64;
  MRHS_HIP(ctx, launch_hop_eo(p64, ctx->g.V / 2, static_cast<const int4*>(ctx->eo_tab[out_parity].p),
                              static_cast<const int*>(ctx->eo_order[out_parity].p), p64 ? ctx->U64.p : ctx->U32.p,
                              in, out, nrhs, ctx->stream, 0, nullptr, nullptr, 0.0, &ctx->g, out_parity,
                              &ctx->eo_walk[nrhs]));
  return MRHS_OK;
}

mrhs_status mrhs_set_eo_walk(mrhs_ctx ctx, int32_t nrhs, const int32_t* tile, int32_t rhs_per_thread) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  EoWalk w;
  if (tile) {
    if (!eo_walk_fits(ctx->g, tile, nrhs, rhs_per_thread))
      return fail(ctx, MRHS_ERR_INVALID_ARG, "checkerboard walk %dx%dx%d x %d (R = %d) does not fit the lattice",
                  tile[0], tile[1], tile[2], tile[3], rhs_per_thread);
    w.on = 1;
    w.R = rhs_per_thread;
    for (int m = 0; m < 3; ++m) w.B[m] = tile[m];
    w.Ts = tile[3];
  }
  ctx->eo_walk[nrhs] = w;
  ctx->op_gen++;  // captured V-cycles hold the launch shape
  return MRHS_OK;
}

mrhs_status mrhs_get_eo_walk(mrhs_ctx ctx, int32_t nrhs, int32_t* on, int32_t* rhs_per_thread, int32_t tile[4],
                             float* us, float* us_tiled) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  const EoWalk& w = ctx->eo_walk[nrhs];
  if (on) *on = w.on;
  if (rhs_per_thread) *rhs_per_thread = w.R;
  if (tile) {
    for (int m = 0; m < 3; ++m) tile[m] = w.B[m];
    tile[3] = w.Ts;
  }
  if (us) *us = w.us;
  if (us_tiled) *us_tiled = w.us_tiled;
  return MRHS_OK;
}

mrhs_status mrhs_set_f64_walk(mrhs_ctx ctx, int32_t nrhs, const int32_t* tile, int32_t variant) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  F64Walk w;
  if (tile) {
    if (!f64_walk_fits(ctx->g, tile, nrhs))
      return fail(ctx, MRHS_ERR_INVALID_ARG, "FP64 walk %dx%dx%d x %d does not fit the lattice", tile[0], tile[1],
                  tile[2], tile[3]);
    w.on = 1;
    for (int m = 0; m < 3; ++m) w.B[m] = tile[m];
    w.Ts = tile[3];
    w.nt = variant & 1;
    w.occ = (variant & 2) ? 2 : 0;
  }
  ctx->f64_walk[nrhs] = w;
  ctx->op_gen++;  // captured solver graphs hold the launch shape
  return MRHS_OK;
}

mrhs_status mrhs_get_f64_walk(mrhs_ctx ctx, int32_t nrhs, int32_t* on, int32_t tile[4], int32_t* variant,
                              float* us, float* us_tiled) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  const F64Walk& w = ctx->f64_walk[nrhs];
  if (on) *on = w.on;
  if (tile) {
    for (int m = 0; m < 3; ++m) tile[m] = w.B[m];
    tile[3] = w.Ts;
  }
  if (variant) *variant = w.nt + (w.occ == 2 ? 2 : 0);
  if (us) *us = w.us;
  if (us_tiled) *us_tiled = w.us_tiled;
  return MRHS_OK;
}

mrhs_status mrhs_clover_eo_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, int32_t parity,
                                 int32_t inverse, mrhs_prec prec) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (parity != 0 && parity != 1) return fail(ctx, MRHS_ERR_INVALID_ARG, "parity must be 0 or 1");
  mrhs_status st = check_field_args(ctx, out, in, nrhs, prec, 12, ctx->g.V / 2);
  if (st != MRHS_OK) return st;
  if (!ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "clover term not set");
  DeviceGuard dg(ctx->device);
  st = ensure_eo_tables(ctx);
  if (st == MRHS_OK && inverse) st = ensure_clover_inverse(ctx);
  if (st != MRHS_OK) return st;
  const int p64 = prec == MRHS_F64;
  const void* A = inverse ? (p64 ? ctx->Ainv64.p : ctx->Ainv32.p) : (p64 ? ctx->A64.p : ctx->A32.p);
  MRHS_HIP(ctx, launch_clover_eo(p64, ctx->g.V / 2, static_cast<const int4*>(ctx->eo_tab[parity].p), A, in,
                                 nullptr, 0.0, out, nrhs, ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_schur_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_field_args(ctx, out, in, nrhs, prec, 12, ctx->g.V / 2);
  if (st != MRHS_OK) return st;
  if (!ctx->have_gauge || !ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "fine operator not set");
  DeviceGuard dg(ctx->device);
  st = ensure_eo_tables(ctx);
  if (st == MRHS_OK) st = ensure_clover_inverse(ctx);
  const int p64 = prec == MRHS_F64;
  const size_t half = (size_t)(ctx->g.V / 2) * 12 * nrhs * (p64 ? 16 : 8);
  if (st == MRHS_OK) st = ensure(ctx, ctx->eo_work, half);
  if (st != MRHS_OK) return st;
  void* t2 = ctx->eo_work.p;
  const int nh = ctx->g.V / 2;
  const auto* te = static_cast<const int4*>(ctx->eo_tab[0].p);
  const auto* to = static_cast<const int4*>(ctx->eo_tab[1].p);
  const void* U = p64 ? ctx->U64.p : ctx->U32.p;
  // t2 = A_o^-1 (H_oe in), out = A_e in - kappa^2 (H_eo t2): two fused launches
  const auto* oe = static_cast<const int*>(ctx->eo_order[0].p);
  const auto* oo = static_cast<const int*>(ctx->eo_order[1].p);
  MRHS_HIP(ctx, launch_hop_eo(p64, nh, to, oo, U, in, t2, nrhs, ctx->stream, 1, p64 ? ctx->Ainv64.p : ctx->Ainv32.p,
                              nullptr, 0.0, &ctx->g, 1, &ctx->eo_walk[nrhs]));
  MRHS_HIP(ctx, launch_hop_eo(p64, nh, te, oe, U, t2, out, nrhs, ctx->stream, 2, p64 ? ctx->A64.p : ctx->A32.p, in,
                              -ctx->kappa * ctx->kappa, &ctx->g, 0, &ctx->eo_walk[nrhs]));
  return MRHS_OK;
}

}  // extern "C"

// ---- batched level-1 operations ----------------------------------------------

namespace {

mrhs_status check_blas_shape(mrhs_ctx ctx, int64_t nsites, int32_t ncomp, int32_t nrhs, mrhs_prec prec) {
  if (nsites < 1 || ncomp < 1 || nsites * (int64_t)ncomp > (int64_t(1) << 40))
    return fail(ctx, MRHS_ERR_SHAPE, "bad field shape nsites=%lld ncomp=%d", (long long)nsites, ncomp);
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  if (prec != MRHS_F32 && prec != MRHS_F64)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "precision %s not supported for this call", prec_name(prec));
  return MRHS_OK;
}

// Runs a reduction whose device result has `bytes` bytes: into `out` directly
// if it is device memory, else into the context's scalar buffer and back.
template <typename F>
mrhs_status reduce_to(mrhs_ctx ctx, double* out, int out_on_device, size_t bytes, size_t scratch, F&& launch) {
  mrhs_status st = ensure(ctx, ctx->work, scratch);
  if (st != MRHS_OK) return st;
  void* dst = out;
  if (!out_on_device) {
    st = ensure(ctx, ctx->scal, bytes);
    if (st != MRHS_OK) return st;
    dst = ctx->scal.p;
  }
  hipError_t e = launch(dst, ctx->work.p);
  if (e != hipSuccess) return hip_fail(ctx, e, "reduction launch");
  if (!out_on_device) {
    MRHS_HIP(ctx, hipMemcpyAsync(out, ctx->scal.p, bytes, hipMemcpyDeviceToHost, ctx->stream));
    MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return MRHS_OK;
}

}  // namespace

extern "C" {

mrhs_status mrhs_dot(mrhs_ctx ctx, double* out, const void* a, const void* b, int64_t nsites, int32_t ncomp,
                     int32_t nrhs, mrhs_prec prec, int32_t out_on_device) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_blas_shape(ctx, nsites, ncomp, nrhs, prec);
  if (st != MRHS_OK) return st;
  if (!out || !a || !b) return fail(ctx, MRHS_ERR_INVALID_ARG, "null pointer");
  if (!aligned16(a) || !aligned16(b)) return fail(ctx, MRHS_ERR_INVALID_ARG, "field pointers must be 16-byte aligned");
  DeviceGuard dg(ctx->device);
  const long rows = (long)nsites * ncomp;
  return reduce_to(ctx, out, out_on_device, (size_t)nrhs * 16, blas_scratch_bytes(nrhs, 1), [&](void* dst, void* w) {
    return launch_dot(prec == MRHS_F64, 0, a, b, rows, nrhs, dst, w, ctx->stream);
  });
}

mrhs_status mrhs_norm2(mrhs_ctx ctx, double* out, const void* a, int64_t nsites, int32_t ncomp, int32_t nrhs,
                       mrhs_prec prec, int32_t out_on_device) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_blas_shape(ctx, nsites, ncomp, nrhs, prec);
  if (st != MRHS_OK) return st;
  if (!out || !a) return fail(ctx, MRHS_ERR_INVALID_ARG, "null pointer");
  if (!aligned16(a)) return fail(ctx, MRHS_ERR_INVALID_ARG, "field pointers must be 16-byte aligned");
  DeviceGuard dg(ctx->device);
  const long rows = (long)nsites * ncomp;
  return reduce_to(ctx, out, out_on_device, (size_t)nrhs * 8, blas_scratch_bytes(nrhs, 1), [&](void* dst, void* w) {
    return launch_dot(prec == MRHS_F64, 1, a, a, rows, nrhs, dst, w, ctx->stream);
  });
}

mrhs_status mrhs_multi_dot(mrhs_ctx ctx, double* out, const void* const* v, int32_t m, const void* w,
                           int64_t nsites, int32_t ncomp, int32_t nrhs, mrhs_prec prec, int32_t out_on_device) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_blas_shape(ctx, nsites, ncomp, nrhs, prec);
  if (st != MRHS_OK) return st;
  if (m < 1 || m > kMaxMultiDot) return fail(ctx, MRHS_ERR_SHAPE, "m = %d outside [1, %d]", m, kMaxMultiDot);
  if (!out || !v || !w) return fail(ctx, MRHS_ERR_INVALID_ARG, "null pointer");
  if (!aligned16(w)) return fail(ctx, MRHS_ERR_INVALID_ARG, "field pointers must be 16-byte aligned");
  for (int j = 0; j < m; ++j)
    if (!v[j] || !aligned16(v[j])) return fail(ctx, MRHS_ERR_INVALID_ARG, "v[%d] null or misaligned", j);
  DeviceGuard dg(ctx->device);
  const long rows = (long)nsites * ncomp;
  return reduce_to(ctx, out, out_on_device, (size_t)m * nrhs * 16, blas_scratch_bytes(nrhs, m),
                   [&](void* dst, void* wk) {
                     return launch_multi_dot(prec == MRHS_F64, v, m, w, rows, nrhs, dst, wk, ctx->stream);
                   });
}

mrhs_status mrhs_axpy(mrhs_ctx ctx, void* y, const double* alpha, const void* x, int64_t nsites, int32_t ncomp,
                      int32_t nrhs, mrhs_prec prec, int32_t alpha_on_device) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_blas_shape(ctx, nsites, ncomp, nrhs, prec);
  if (st != MRHS_OK) return st;
  if (!y || !alpha || !x) return fail(ctx, MRHS_ERR_INVALID_ARG, "null pointer");
  st = check_field_args(ctx, y, x, nrhs, prec, (size_t)ncomp, nsites);
  if (st != MRHS_OK) return st;
  DeviceGuard dg(ctx->device);
  const void* al = alpha;
  if (!alpha_on_device) {
    st = ensure(ctx, ctx->scal, (size_t)nrhs * 16);
    if (st != MRHS_OK) return st;
    MRHS_HIP(ctx, hipMemcpyAsync(ctx->scal.p, alpha, (size_t)nrhs * 16, hipMemcpyHostToDevice, ctx->stream));
    al = ctx->scal.p;
  }
  hipError_t e = launch_axpy(prec == MRHS_F64, y, al, x, (long)nsites * ncomp, nrhs, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "axpy launch");
  if (!alpha_on_device) MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));  // alpha's host memory may be reused
  return MRHS_OK;
}

}  // extern "C"
