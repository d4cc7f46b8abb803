// C-ABI of the multigrid hierarchy: basis vectors and their block
// orthonormalisation, restriction / prolongation / block normalisation
// (paper Sec. 5), coarse stencil blocks by Galerkin projection and the coarse
// operator apply (paper Sec. 6).
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "mg_internal.h"

using namespace mrhs;

namespace {

const char* prec_str(mrhs_prec p) {
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

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

Geom make_geom(const int L[4]) {
  Geom g{};
  for (int m = 0; m < 4; ++m) g.L[m] = L[m];
  g.V = L[0] * L[1] * L[2] * L[3];
  g.stride[0] = 1;
  g.stride[1] = L[0];
  g.stride[2] = L[0] * L[1];
  g.stride[3] = L[0] * L[1] * L[2];
  set_tile(g);
  return g;
}

mrhs_status check_level(mrhs_mg mg, int level, int lo, int hi) {
  if (level < lo || level > hi || level >= mg->nlevels)
    return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "level %d outside [%d, %d] for a %d-level hierarchy", level, lo,
                std::min(hi, mg->nlevels - 1), mg->nlevels);
  return MRHS_OK;
}

mrhs_status check_fields(mrhs_ctx ctx, const void* a, const void* b, int nrhs) {
  if (!a || !b) return fail(ctx, MRHS_ERR_INVALID_ARG, "null field pointer");
  if (!aligned16(a) || !aligned16(b)) return fail(ctx, MRHS_ERR_INVALID_ARG, "field pointers must be 16-byte aligned");
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  return MRHS_OK;
}

}  // namespace

namespace mrhs {

// Rebuilds every derived copy of a level's stencil blocks from the FP64 master.
mrhs_status refresh_blocks(mrhs_mg mg, int level) {
  mrhs_ctx ctx = mg->ctx;
  LevelData& L = mg->lv[level];
  const long n = (long)L.g.V * 9;
  const size_t e = (size_t)n * L.ncomp * L.ncomp;
  mrhs_status st = ensure(ctx, L.BT32, e * 8);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, L.BT64, e * 16);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, launch_block_transpose(L.B64.p, 1, L.BT32.p, 0, n, L.ncomp, ctx->stream));
  MRHS_HIP(ctx, launch_block_transpose(L.B64.p, 1, L.BT64.p, 1, n, L.ncomp, ctx->stream));
  st = pack_blocks_mfma(mg, level);
  if (st != MRHS_OK) return st;
  L.have_blocks = true;
  L.have_sinv = false;
  return MRHS_OK;
}

hipError_t coarse_apply_f32(mrhs_mg mg, int level, const void* in, void* out, int n, hipStream_t s) {
  LevelData& L = mg->lv[level];
  if (mfma_supported(L.ncomp) && !L.f32_valu[n])
    return launch_coarse_mfma_f32(L.g, L.ncomp, n, L.Bf32p.p, in, out, s);
  return launch_coarse_valu(0, L.g, L.ncomp, n, L.BT32.p, in, out, DirFilter{}, s);
}

// Inverted self blocks of a level and their three MFMA packs (synchronises).
mrhs_status ensure_self_inverse(mrhs_mg mg, int level) {
  mrhs_ctx ctx = mg->ctx;
  LevelData& L = mg->lv[level];
  if (L.have_sinv) return MRHS_OK;
  const long V = L.g.V;
  const size_t blk = (size_t)L.ncomp * L.ncomp;
  mrhs_status st = ensure(ctx, L.Sinv64, V * blk * 16);
  if (st == MRHS_OK) st = ensure(ctx, L.SinvF32p, V * blk * 8);
  if (st == MRHS_OK) st = ensure(ctx, L.SinvBf16, V * blk * 4);
  if (st == MRHS_OK) st = ensure(ctx, L.SinvF16, V * blk * 4);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, hipMemsetAsync(mg->flag, 0, sizeof(int), ctx->stream));
  MRHS_HIP(ctx, launch_self_invert(V, L.B64.p, L.Sinv64.p, mg->flag, ctx->stream));
  int h = 0;
  MRHS_HIP(ctx, hipMemcpyAsync(&h, mg->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h) return fail(ctx, MRHS_ERR_STATE, "a self block of level %d is singular", level);
  MRHS_HIP(ctx, launch_pack_block_list(0, L.Sinv64.p, L.SinvF32p.p, V, ctx->stream));
  MRHS_HIP(ctx, launch_pack_block_list(1, L.Sinv64.p, L.SinvBf16.p, V, ctx->stream));
  MRHS_HIP(ctx, launch_pack_block_list(2, L.Sinv64.p, L.SinvF16.p, V, ctx->stream));
  L.have_sinv = true;
  return MRHS_OK;
}

mrhs_status ensure_colscale(mrhs_mg mg) {
  if (mg->colscale.p) return MRHS_OK;
  mrhs_status st = ensure(mg->ctx, mg->colscale, 2 * MRHS_MAX_NRHS * sizeof(float));
  if (st != MRHS_OK) return st;
  MRHS_HIP(mg->ctx, hipMemset(mg->colscale.p, 0, 2 * MRHS_MAX_NRHS * sizeof(float)));
  return MRHS_OK;
}

// Refreshes the FP32 copy of a level's basis from the FP64 master.
mrhs_status refresh_basis32(mrhs_mg mg, int level) {
  mrhs_ctx ctx = mg->ctx;
  LevelData& L = mg->lv[level];
  const size_t n = (size_t)L.g.V * L.ncomp * L.nv;
  mrhs_status st = ensure(ctx, L.basis32, n * 8);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, launch_convert_f64_to_f32(static_cast<const double*>(L.basis64.p), static_cast<float*>(L.basis32.p),
                                          2 * n, ctx->stream));
  L.bf16_ok = false;
  return MRHS_OK;
}

mrhs_status ensure_basis_bf16(mrhs_mg mg, int from) {
  mrhs_ctx ctx = mg->ctx;
  bool packed = false;
  for (int l = std::max(from, 0); l + 1 < mg->nlevels; ++l) {
    LevelData& L = mg->lv[l];
    if (L.bf16_ok || !L.have_basis || !intergrid_mfma_supported(L.agg, L.ncomp / 2, L.nv)) continue;
    const long n = (long)L.g.V * L.ncomp * L.nv;
    mrhs_status st = ensure(ctx, L.Wbf16, (size_t)n * 4);
    if (st != MRHS_OK) return st;
    MRHS_HIP(ctx, launch_pack_basis_bf16(L.basis32.p, L.Wbf16.p, n, ctx->stream));
    L.bf16_ok = true;
    packed = true;
  }
  if (packed) MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MRHS_OK;
}

}  // namespace mrhs

extern "C" {

mrhs_status mrhs_mg_create(mrhs_ctx ctx, const mrhs_mg_params* p, mrhs_mg* out) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (!p || !out) return fail(ctx, MRHS_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (p->nlevels < 2 || p->nlevels > MRHS_MAX_LEVELS)
    return fail(ctx, MRHS_ERR_SHAPE, "nlevels = %d outside [2, %d]", p->nlevels, MRHS_MAX_LEVELS);
  int L[4];
  for (int m = 0; m < 4; ++m) L[m] = ctx->g.L[m];
  int ncomp = 12;
  mrhs_mg mg = new (std::nothrow) mrhs_mg_s();
  if (!mg) return fail(ctx, MRHS_ERR_OOM, "host allocation failed");
  mg->ctx = ctx;
  mg->nlevels = p->nlevels;
  for (int l = 0; l < p->nlevels; ++l) {
    LevelData& lv = mg->lv[l];
    lv.g = make_geom(L);
    lv.ncomp = ncomp;
    if (l == p->nlevels - 1) break;
    const int nv = p->n_v[l];
    if (!intergrid_supported(nv, ncomp / 2)) {
      delete mg;
      return fail(ctx, MRHS_ERR_UNSUPPORTED, "n_v = %d with %d components per chirality is not supported "
                  "(n_v in {4, 8, 16}; components per chirality in {4, 6, 8, 16})", nv, ncomp / 2);
    }
    lv.nv = nv;
    AggGeom& a = lv.agg;
    for (int m = 0; m < 4; ++m) {
      const int b = p->block[l][m];
      if (b < 1 || L[m] % b) {
        delete mg;
        return fail(ctx, MRHS_ERR_SHAPE, "block extent %d does not divide lattice extent %d (level %d, dir %d)", b, L[m],
                    l, m);
      }
      a.L[m] = L[m];
      a.b[m] = b;
      a.C[m] = L[m] / b;
    }
    a.V = lv.g.V;
    a.Vc = a.C[0] * a.C[1] * a.C[2] * a.C[3];
    for (int m = 0; m < 4; ++m) L[m] = a.C[m];
    ncomp = 2 * nv;
  }
  DevGuard dg(ctx->device);
  if (hipMalloc(&mg->flag, sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    delete mg;
    return fail(ctx, MRHS_ERR_OOM, "hipMalloc of a flag failed");
  }
  *out = mg;
  return MRHS_OK;
}

void mrhs_mg_destroy(mrhs_mg mg) {
  if (!mg) return;
  DevGuard dg(mg->ctx->device);
  (void)hipStreamSynchronize(mg->ctx->stream);
  for (auto& L : mg->lv) {
    Buffer* bufs[] = {&L.basis64, &L.basis32, &L.Wbf16, &L.B64,      &L.BT32,     &L.BT64,   &L.Bbf16,
                      &L.Bf16,    &L.Bf32p,   &L.Sinv64, &L.SinvF32p, &L.SinvBf16, &L.SinvF16};
    for (Buffer* b : bufs) release(*b);
  }
  release(mg->tmpA);
  release(mg->tmpB);
  release(mg->tmpC);
  release(mg->colscale);
  if (mg->flag) (void)hipFree(mg->flag);
  mg_solver_release(mg);
  delete mg;
}

mrhs_status mrhs_mg_level_info(mrhs_mg mg, int32_t level, int32_t dims[4], int32_t* ncomp) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_level(mg, level, 0, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  if (dims)
    for (int m = 0; m < 4; ++m) dims[m] = mg->lv[level].g.L[m];
  if (ncomp) *ncomp = mg->lv[level].ncomp;
  return MRHS_OK;
}

mrhs_status mrhs_mg_set_basis(mrhs_mg mg, int32_t level, const void* vecs, mrhs_prec prec, int32_t on_device) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 0, mg->nlevels - 2);
  if (st != MRHS_OK) return st;
  if (!vecs) return fail(ctx, MRHS_ERR_INVALID_ARG, "null basis pointer");
  if (prec != MRHS_F64 && prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "basis precision %s not supported", prec_str(prec));
  DevGuard dg(ctx->device);
  LevelData& L = mg->lv[level];
  const size_t n = (size_t)L.g.V * L.nv * L.ncomp;
  const size_t csz = prec == MRHS_F64 ? 16 : 8;
  st = ensure(ctx, L.basis64, n * 16);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, mg->tmpA, n * csz);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, hipMemcpyAsync(mg->tmpA.p, vecs, n * csz, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               ctx->stream));
  MRHS_HIP(ctx, launch_basis_convert(mg->tmpA.p, prec == MRHS_F64, L.basis64.p, 1, L.g.V, L.nv, L.ncomp, 1, ctx->stream));
  st = refresh_basis32(mg, level);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  L.have_basis = true;
  // coarse levels built from an older basis are stale
  for (int l = level + 1; l < mg->nlevels; ++l) mg->lv[l].have_blocks = false;
  ++ctx->op_gen;
  return MRHS_OK;
}

mrhs_status mrhs_mg_get_basis(mrhs_mg mg, int32_t level, void* vecs, mrhs_prec prec, int32_t on_device) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 0, mg->nlevels - 2);
  if (st != MRHS_OK) return st;
  if (!vecs) return fail(ctx, MRHS_ERR_INVALID_ARG, "null basis pointer");
  if (prec != MRHS_F64 && prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "basis precision %s not supported", prec_str(prec));
  LevelData& L = mg->lv[level];
  if (!L.have_basis) return fail(ctx, MRHS_ERR_STATE, "basis of level %d not set", level);
  DevGuard dg(ctx->device);
  const size_t n = (size_t)L.g.V * L.nv * L.ncomp;
  const size_t csz = prec == MRHS_F64 ? 16 : 8;
  st = ensure(ctx, mg->tmpA, n * csz);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, launch_basis_convert(L.basis64.p, 1, mg->tmpA.p, prec == MRHS_F64, L.g.V, L.nv, L.ncomp, 0, ctx->stream));
  MRHS_HIP(ctx, hipMemcpyAsync(vecs, mg->tmpA.p, n * csz, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               ctx->stream));
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_mg_block_orthonormalise(mrhs_mg mg, int32_t level) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 0, mg->nlevels - 2);
  if (st != MRHS_OK) return st;
  LevelData& L = mg->lv[level];
  if (!L.have_basis) return fail(ctx, MRHS_ERR_STATE, "basis of level %d not set", level);
  DevGuard dg(ctx->device);
  MRHS_HIP(ctx, hipMemsetAsync(mg->flag, 0, sizeof(int), ctx->stream));
  MRHS_HIP(ctx, launch_block_gs(L.agg, L.ncomp / 2, L.nv, L.basis64.p, mg->flag, ctx->stream));
  st = refresh_basis32(mg, level);
  if (st != MRHS_OK) return st;
  int flag = 0;
  MRHS_HIP(ctx, hipMemcpyAsync(&flag, mg->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int l = level + 1; l < mg->nlevels; ++l) mg->lv[l].have_blocks = false;
  ++ctx->op_gen;
  if (flag) return fail(ctx, MRHS_ERR_STATE, "basis of level %d is rank-deficient on some aggregate", level);
  return MRHS_OK;
}

mrhs_status mrhs_restrict(mrhs_mg mg, int32_t level, void* coarse, const void* fine, int32_t nrhs, mrhs_prec prec) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 0, mg->nlevels - 2);
  if (st != MRHS_OK) return st;
  st = check_fields(ctx, coarse, fine, nrhs);
  if (st != MRHS_OK) return st;
  LevelData& L = mg->lv[level];
  if (prec == MRHS_BF16 && !intergrid_mfma_supported(L.agg, L.ncomp / 2, L.nv))
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "BF16 restrict needs n_v = 16 and aggregates of a multiple of 16 sites");
  if (prec != MRHS_F64 && prec != MRHS_F32 && prec != MRHS_BF16)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "restrict precision %s not supported", prec_str(prec));
  if (!L.have_basis) return fail(ctx, MRHS_ERR_STATE, "basis of level %d not set", level);
  DevGuard dg(ctx->device);
  if (prec == MRHS_BF16) {
    st = ensure_basis_bf16(mg, level);
    if (st != MRHS_OK) return st;
    MRHS_HIP(ctx, launch_restrict_bf16(L.agg, L.ncomp / 2, nrhs, L.Wbf16.p, fine, coarse, ctx->stream));
    return MRHS_OK;
  }
  MRHS_HIP(ctx, launch_restrict(prec == MRHS_F64, L.agg, L.ncomp / 2, L.nv, nrhs,
                                prec == MRHS_F64 ? L.basis64.p : L.basis32.p, fine, coarse, ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_prolong(mrhs_mg mg, int32_t level, void* fine, const void* coarse, int32_t nrhs, mrhs_prec prec) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 0, mg->nlevels - 2);
  if (st != MRHS_OK) return st;
  st = check_fields(ctx, fine, coarse, nrhs);
  if (st != MRHS_OK) return st;
  LevelData& L = mg->lv[level];
  if (prec == MRHS_BF16 && !intergrid_mfma_supported(L.agg, L.ncomp / 2, L.nv))
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "BF16 prolong needs n_v = 16 and aggregates of a multiple of 16 sites");
  if (prec != MRHS_F64 && prec != MRHS_F32 && prec != MRHS_BF16)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "prolong precision %s not supported", prec_str(prec));
  if (!L.have_basis) return fail(ctx, MRHS_ERR_STATE, "basis of level %d not set", level);
  DevGuard dg(ctx->device);
  if (prec == MRHS_BF16) {
    st = ensure_basis_bf16(mg, level);
    if (st != MRHS_OK) return st;
    MRHS_HIP(ctx, launch_prolong_bf16(L.agg, L.ncomp / 2, nrhs, L.Wbf16.p, coarse, fine, ctx->stream));
    return MRHS_OK;
  }
  MRHS_HIP(ctx, launch_prolong(prec == MRHS_F64, L.agg, L.ncomp / 2, L.nv, nrhs,
                               prec == MRHS_F64 ? L.basis64.p : L.basis32.p, coarse, fine, ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_block_normalise(mrhs_mg mg, int32_t level, void* fields, int32_t nrhs, mrhs_prec prec,
                                 double* norms) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 0, mg->nlevels - 2);
  if (st != MRHS_OK) return st;
  st = check_fields(ctx, fields, fields, nrhs);
  if (st != MRHS_OK) return st;
  if (prec != MRHS_F64 && prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "block-normalise precision %s not supported", prec_str(prec));
  LevelData& L = mg->lv[level];
  DevGuard dg(ctx->device);
  MRHS_HIP(ctx, launch_block_normalise(prec == MRHS_F64, L.agg, L.ncomp / 2, nrhs, fields, norms, ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_coarse_set_blocks(mrhs_mg mg, int32_t level, const void* blocks, mrhs_prec prec, int32_t on_device) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 1, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  if (!blocks) return fail(ctx, MRHS_ERR_INVALID_ARG, "null block pointer");
  if (prec != MRHS_F64 && prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "block precision %s not supported", prec_str(prec));
  DevGuard dg(ctx->device);
  LevelData& L = mg->lv[level];
  const size_t n = (size_t)L.g.V * 9 * L.ncomp * L.ncomp;
  st = ensure(ctx, L.B64, n * 16);
  if (st != MRHS_OK) return st;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (prec == MRHS_F64) {
    MRHS_HIP(ctx, hipMemcpyAsync(L.B64.p, blocks, n * 16, kind, ctx->stream));
  } else {
    st = ensure(ctx, mg->tmpA, n * 8);
    if (st != MRHS_OK) return st;
    MRHS_HIP(ctx, hipMemcpyAsync(mg->tmpA.p, blocks, n * 8, kind, ctx->stream));
    MRHS_HIP(ctx, launch_convert_f32_to_f64(static_cast<const float*>(mg->tmpA.p), static_cast<double*>(L.B64.p), 2 * n,
                                            ctx->stream));
  }
  st = refresh_blocks(mg, level);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ++ctx->op_gen;
  return MRHS_OK;
}

mrhs_status mrhs_coarse_get_blocks(mrhs_mg mg, int32_t level, void* blocks, mrhs_prec prec, int32_t on_device) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 1, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  if (!blocks) return fail(ctx, MRHS_ERR_INVALID_ARG, "null block pointer");
  if (prec != MRHS_F64) return fail(ctx, MRHS_ERR_UNSUPPORTED, "blocks are exported in f64 only");
  LevelData& L = mg->lv[level];
  if (!L.have_blocks) return fail(ctx, MRHS_ERR_STATE, "blocks of level %d not set", level);
  DevGuard dg(ctx->device);
  const size_t n = (size_t)L.g.V * 9 * L.ncomp * L.ncomp;
  MRHS_HIP(ctx, hipMemcpyAsync(blocks, L.B64.p, n * 16, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               ctx->stream));
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MRHS_OK;
}

// Galerkin coarse operator of `level` (>= 1) from the operator and basis of level-1:
// B_d(A) = sum_{x in A} W(x)^dag (D_d W)(x), W = chirality-split basis columns,
// D_d the direction-resolved operator.  All in FP64.
mrhs_status mrhs_mg_build_coarse(mrhs_mg mg, int32_t level) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 1, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  LevelData& F = mg->lv[level - 1];
  LevelData& C = mg->lv[level];
  if (!F.have_basis) return fail(ctx, MRHS_ERR_STATE, "basis of level %d not set", level - 1);
  if (level == 1) {
    if (!ctx->have_gauge || !ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "fine operator not set");
  } else if (!F.have_blocks) {
    return fail(ctx, MRHS_ERR_STATE, "blocks of level %d not set", level - 1);
  }
  const int nb = C.ncomp;
  if (nb > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_UNSUPPORTED, "Nb = %d above %d", nb, MRHS_MAX_NRHS);
  DevGuard dg(ctx->device);
  const size_t ncol = (size_t)F.g.V * F.ncomp * nb;  // complex entries of one column field
  st = ensure(ctx, mg->tmpA, ncol * 16);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, mg->tmpB, ncol * 16);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, mg->tmpC, (size_t)C.g.V * nb * nb * 16);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, C.B64, (size_t)C.g.V * 9 * nb * nb * 16);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, launch_basis_columns(1, F.basis64.p, mg->tmpA.p, F.g.V, F.ncomp, F.nv, ctx->stream));
  static const int dsign[9] = {0, 1, -1, 1, -1, 1, -1, 1, -1};
  for (int d = 0; d < 9; ++d) {
    DirFilter f;
    f.sign = dsign[d];
    f.mu = d == 0 ? 0 : (d - 1) / 2;
    for (int m = 0; m < 4; ++m) f.b[m] = F.agg.b[m];
    if (level == 1) {
      MRHS_HIP(ctx, launch_fine_dir_f64(ctx->g, ctx->t_bc, ctx->kappa, ctx->U64.p, ctx->A64.p, mg->tmpA.p, mg->tmpB.p, nb, f,
                                        ctx->stream));
    } else {
      MRHS_HIP(ctx, launch_coarse_valu(1, F.g, F.ncomp, nb, F.BT64.p, mg->tmpA.p, mg->tmpB.p, f, ctx->stream));
    }
    MRHS_HIP(ctx, launch_restrict(1, F.agg, F.ncomp / 2, F.nv, nb, F.basis64.p, mg->tmpB.p, mg->tmpC.p, ctx->stream));
    // scatter [A][i][j] into [A][d][i][j]
    const size_t row = (size_t)nb * nb * 16;
    MRHS_HIP(ctx, hipMemcpy2DAsync(static_cast<char*>(C.B64.p) + d * row, 9 * row, mg->tmpC.p, row, row, C.g.V,
                                   hipMemcpyDeviceToDevice, ctx->stream));
  }
  st = refresh_blocks(mg, level);
  if (st != MRHS_OK) return st;
  for (int l = level + 1; l < mg->nlevels; ++l) mg->lv[l].have_blocks = false;
  MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ++ctx->op_gen;
  return MRHS_OK;
}

mrhs_status mrhs_coarse_apply(mrhs_mg mg, int32_t level, void* out, const void* in, int32_t nrhs, mrhs_prec prec) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 1, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  st = check_fields(ctx, out, in, nrhs);
  if (st != MRHS_OK) return st;
  LevelData& L = mg->lv[level];
  if (!L.have_blocks) return fail(ctx, MRHS_ERR_STATE, "blocks of level %d not set", level);
  const size_t csz = prec == MRHS_F64 ? 16 : 8;
  const size_t bytes = (size_t)L.g.V * L.ncomp * nrhs * csz;
  const char* a = static_cast<const char*>(in);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return fail(ctx, MRHS_ERR_INVALID_ARG, "in and out overlap");
  DevGuard dg(ctx->device);
  hipError_t e;
  switch (prec) {
    case MRHS_F64:
      e = launch_coarse_valu(1, L.g, L.ncomp, nrhs, L.BT64.p, in, out, DirFilter{}, ctx->stream);
      break;
    case MRHS_F32:
      // FP32 matrix cores for Nb = 32 unless mrhs_mg_tune found the
      // vector-ALU kernel faster for this level and nrhs
      e = coarse_apply_f32(mg, level, in, out, nrhs, ctx->stream);
      break;
    case MRHS_BF16:
    case MRHS_F16: {
      if (!mfma_supported(L.ncomp))
        return fail(ctx, MRHS_ERR_UNSUPPORTED, "matrix-core stencil needs Nb = 32, got %d", L.ncomp);
      const float* scale = nullptr;
      if (prec == MRHS_F16) {
        st = ensure_colscale(mg);
        if (st != MRHS_OK) return st;
        float* sc = static_cast<float*>(mg->colscale.p);
        e = launch_column_scale(in, (long)L.g.V * L.ncomp, nrhs, sc + MRHS_MAX_NRHS, sc, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "column scale launch");
        scale = sc;
      }
      e = launch_coarse_mfma(prec == MRHS_F16, L.g, L.ncomp, nrhs, prec == MRHS_F16 ? L.Bf16.p : L.Bbf16.p, in, out,
                             scale, ctx->stream, L.lowp_cfg[nrhs]);
      break;
    }
    default:
      return fail(ctx, MRHS_ERR_UNSUPPORTED, "unknown precision %d", (int)prec);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "coarse stencil launch");
  return MRHS_OK;
}

// Shared checks and launch of the two even-odd coarse calls.
static mrhs_status coarse_eo(mrhs_mg mg, int32_t level, void* out, const void* in, int32_t nrhs, int32_t parity,
                             int eo, int inverse, mrhs_prec prec) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  mrhs_status st = check_level(mg, level, 1, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  st = check_fields(ctx, out, in, nrhs);
  if (st != MRHS_OK) return st;
  if (parity != 0 && parity != 1) return fail(ctx, MRHS_ERR_INVALID_ARG, "parity must be 0 or 1");
  LevelData& L = mg->lv[level];
  if (!L.have_blocks) return fail(ctx, MRHS_ERR_STATE, "blocks of level %d not set", level);
  if (!mfma_supported(L.ncomp))
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "even-odd stencil calls need Nb = 32, got %d", L.ncomp);
  for (int m = 0; m < 4; ++m)
    if (L.g.L[m] % 2)
      return fail(ctx, MRHS_ERR_SHAPE, "even-odd calls need even extents (level %d: L[%d] = %d)", level, m,
                  L.g.L[m]);
  if (prec != MRHS_F32 && prec != MRHS_BF16 && prec != MRHS_F16)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "precision must be f32, bf16 or f16");
  const size_t bytes = (size_t)(L.g.V / 2) * L.ncomp * nrhs * 8;
  const char* a = static_cast<const char*>(in);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return fail(ctx, MRHS_ERR_INVALID_ARG, "in and out overlap");
  DevGuard dg(ctx->device);
  if (inverse) {
    st = ensure_self_inverse(mg, level);
    if (st != MRHS_OK) return st;
  }
  const int pk = prec == MRHS_F32 ? 0 : (prec == MRHS_BF16 ? 1 : 2);
  const void* pack;
  int bstride = 9;
  if (inverse) {
    pack = pk == 0 ? L.SinvF32p.p : (pk == 1 ? L.SinvBf16.p : L.SinvF16.p);
    bstride = 1;
  } else {
    pack = pk == 0 ? L.Bf32p.p : (pk == 1 ? L.Bbf16.p : L.Bf16.p);
  }
  const float* scale = nullptr;
  if (pk == 2) {
    st = ensure_colscale(mg);
    if (st != MRHS_OK) return st;
    float* sc = static_cast<float*>(mg->colscale.p);
    MRHS_HIP(ctx, launch_column_scale(in, (long)(L.g.V / 2) * L.ncomp, nrhs, sc + MRHS_MAX_NRHS, sc, ctx->stream));
    scale = sc;
  }
  MRHS_HIP(ctx, launch_coarse_mfma_eo(pk, eo, parity, L.g, L.ncomp, nrhs, pack, bstride, in, out, scale,
                                      ctx->stream));
  return MRHS_OK;
}

mrhs_status mrhs_mg_tune(mrhs_mg mg, const int32_t* nrhs_list, int32_t count) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  if (!nrhs_list || count < 1 || count > 64) return fail(ctx, MRHS_ERR_INVALID_ARG, "bad nrhs list");
  for (int i = 0; i < count; ++i)
    if (nrhs_list[i] < 1 || nrhs_list[i] > MRHS_MAX_NRHS)
      return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs_list[i], MRHS_MAX_NRHS);
  DevGuard dg(ctx->device);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MRHS_HIP(ctx, hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  for (int l = 1; l < mg->nlevels && e == hipSuccess; ++l) {
    LevelData& L = mg->lv[l];
    if (!L.have_blocks || !mfma_supported(L.ncomp)) continue;
    const int nmax = *std::max_element(nrhs_list, nrhs_list + count);
    const size_t bytes = (size_t)L.g.V * L.ncomp * nmax * 8;
    mrhs_status st = ensure(ctx, mg->tmpA, bytes);
    if (st == MRHS_OK) st = ensure(ctx, mg->tmpB, bytes);
    if (st != MRHS_OK) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return st;
    }
    e = hipMemsetAsync(mg->tmpA.p, 0, bytes, ctx->stream);
    for (int i = 0; i < count && e == hipSuccess; ++i) {
      const int n = nrhs_list[i];
      float best[2] = {0.f, 0.f};
      for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        L.f32_valu[n] = (signed char)k;
        std::vector<float> t;
        for (int rep = 0; rep < 6 && e == hipSuccess; ++rep) {
          e = hipEventRecord(e0, ctx->stream);
          if (e == hipSuccess) e = coarse_apply_f32(mg, l, mg->tmpA.p, mg->tmpB.p, n, ctx->stream);
          if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) t.push_back(ms);  // the first launch is a warm-up
        }
        if (e == hipSuccess) {
          std::sort(t.begin(), t.end());
          best[k] = t[t.size() / 2];
        }
      }
      L.f32_valu[n] = (signed char)(e == hipSuccess && best[1] < best[0]);
      // launch shape of the BF16 / FP16 stencil: four or eight wavefronts per
      // site, one or two 32-column tiles per workgroup, the two as separate
      // or interleaved columns (timed in BF16; the FP16 kernel has the same
      // structure)
      float lbest = 1e30f;
      int lcfg = 0;
      for (int c = 0; c < kLowpCfgs && e == hipSuccess; ++c) {
        if (c >= 2 && n <= 32) continue;  // a second tile would be empty
        if (c >= 4 && (n & 1)) continue;  // column pairs need an even nrhs
        std::vector<float> t;
        for (int rep = 0; rep < 6 && e == hipSuccess; ++rep) {
          e = hipEventRecord(e0, ctx->stream);
          if (e == hipSuccess)
            e = launch_coarse_mfma(0, L.g, L.ncomp, n, L.Bbf16.p, mg->tmpA.p, mg->tmpB.p, nullptr, ctx->stream, c);
          if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) t.push_back(ms);
        }
        if (e == hipSuccess) {
          std::sort(t.begin(), t.end());
          if (t[t.size() / 2] < lbest) {
            lbest = t[t.size() / 2];
            lcfg = c;
          }
        }
      }
      L.lowp_cfg[n] = (signed char)lcfg;
      // launch shape of the fused MR step on small levels (timed on a step
      // that is not the first, i.e. with the on-the-fly update)
      if (L.g.V <= kFusedMrMaxSites && e == hipSuccess) {
        const size_t fb = (size_t)L.g.V * L.ncomp * n * 8;
        Buffer x, r2, p2, part, al;
        mrhs_status s2 = ensure(ctx, x, fb);
        if (s2 == MRHS_OK) s2 = ensure(ctx, r2, fb);
        if (s2 == MRHS_OK) s2 = ensure(ctx, p2, fb);
        if (s2 == MRHS_OK) s2 = ensure(ctx, part, coarse_mr_part_bytes(L.g.V));
        if (s2 == MRHS_OK) s2 = ensure(ctx, al, 2 * MRHS_MAX_NRHS * 16);
        if (s2 == MRHS_OK) {
          e = hipMemsetAsync(x.p, 0, fb, ctx->stream);
          if (e == hipSuccess) e = hipMemsetAsync(al.p, 0, 2 * MRHS_MAX_NRHS * 16, ctx->stream);
          if (e == hipSuccess) e = hipMemsetAsync(p2.p, 0, fb, ctx->stream);
          float mbest = 1e30f;
          int mcfg = 0;
          char* a = static_cast<char*>(al.p);
          for (int c = 0; c < 4 && e == hipSuccess; ++c) {
            if ((c & 2) && n <= 32) continue;
            std::vector<float> t;
            for (int rep = 0; rep < 6 && e == hipSuccess; ++rep) {
              e = hipEventRecord(e0, ctx->stream);
              if (e == hipSuccess)
                e = launch_coarse_mr_step(L.g, L.ncomp, n, L.Bbf16.p, mg->tmpA.p, p2.p, r2.p, mg->tmpB.p, x.p, a,
                                          a + MRHS_MAX_NRHS * 16, part.p, 0, c, ctx->stream);
              if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
              if (e == hipSuccess) e = hipEventSynchronize(e1);
              float ms = 0.f;
              if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
              if (rep > 0) t.push_back(ms);
            }
            if (e == hipSuccess) {
              std::sort(t.begin(), t.end());
              if (t[t.size() / 2] < mbest) {
                mbest = t[t.size() / 2];
                mcfg = c;
              }
            }
          }
          L.mr_cfg[n] = (signed char)mcfg;
        }
        (void)hipStreamSynchronize(ctx->stream);
        release(x);
        release(r2);
        release(p2);
        release(part);
        release(al);
        if (s2 != MRHS_OK) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return s2;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(ctx, e, "coarse tuning");
  mg_solver_release(mg);  // captured V-cycles hold the previous kernel choice
  return MRHS_OK;
}

mrhs_status mrhs_mg_get_tuning(mrhs_mg mg, int32_t level, int32_t nrhs, int32_t* f32_valu, int32_t* lowp_cfg) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_level(mg, level, 1, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS)
    return fail(mg->ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  if (!f32_valu) return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "null output");
  const LevelData& L = mg->lv[level];
  *f32_valu = (!mfma_supported(L.ncomp) || L.f32_valu[nrhs]) ? 1 : 0;
  if (lowp_cfg) *lowp_cfg = L.lowp_cfg[nrhs];
  return MRHS_OK;
}

mrhs_status mrhs_mg_set_lowp_cfg(mrhs_mg mg, int32_t level, int32_t nrhs, int32_t cfg) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_status st = check_level(mg, level, 1, MRHS_MAX_LEVELS - 1);
  if (st != MRHS_OK) return st;
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS)
    return fail(mg->ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  if (cfg < 0 || cfg >= kLowpCfgs)
    return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "launch shape %d outside [0, %d]", cfg, kLowpCfgs - 1);
  mg->lv[level].lowp_cfg[nrhs] = (signed char)cfg;
  mg->lv[level].mr_cfg[nrhs] = (signed char)(cfg >= 4 ? cfg - 2 : cfg);  // the MR step has no pair form
  ++mg->ctx->op_gen;  // captured V-cycles hold the previous shape
  return MRHS_OK;
}

mrhs_status mrhs_coarse_hop_eo_apply(mrhs_mg mg, int32_t level, void* out, const void* in, int32_t nrhs,
                                     int32_t out_parity, mrhs_prec prec) {
  return coarse_eo(mg, level, out, in, nrhs, out_parity, 1, 0, prec);
}

mrhs_status mrhs_coarse_self_eo_apply(mrhs_mg mg, int32_t level, void* out, const void* in, int32_t nrhs,
                                      int32_t parity, int32_t inverse, mrhs_prec prec) {
  return coarse_eo(mg, level, out, in, nrhs, parity, 2, inverse ? 1 : 0, prec);
}

}  // extern "C"
