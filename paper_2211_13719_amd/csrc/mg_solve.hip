// Multigrid-preconditioned flexible GMRES on Nrhs right-hand sides at once
// (paper Sec. 8: FGMRES preconditioned by multigrid, applied to many RHS
// simultaneously so that every operator application and every inner product
// serves the whole block).
//
// Outer solver: FGMRES(m) in FP64, one independent Krylov space per
// right-hand side (batched, not block Krylov): per-RHS Hessenberg matrices
// and Givens rotations live on the host, the vectors on the device, and all
// inner products of one Gram-Schmidt step are computed in one pass (classical
// Gram-Schmidt, repeated once when the first pass left less than reorth_eta
// of the vector's squared norm for some RHS).  The preconditioned directions Z are stored in
// FP32; since the same FP32 values enter both D Z and the update x += Z y, the
// Arnoldi relation holds to FP64 rounding and the FP64 true residual can reach
// 1e-10 although the preconditioner works in lower precision.
//
// Preconditioner: a V-cycle over the aggregation hierarchy, all fields FP32.
// On every level above the coarsest: nu_pre minimal-residual (MR) steps, the
// coarse-grid correction x += P V(R r), the residual r = b - D x, nu_post MR
// steps.  On the coarsest level: coarsest_iters MR steps from zero.  The fine
// operator is the FP32 Wilson-clover kernel, coarse operators the stencil in
// the requested arithmetic (FP32, or BF16/FP16 matrix cores with FP32
// accumulation; with BF16 coarse levels the intergrid operators of n_v = 16
// steps run on the BF16 matrix cores as well).  The MR step sizes alpha_k = <D r_k, r_k> / ||D r_k||^2
// are computed and consumed on the device, so one V-cycle is a fixed sequence
// of kernel launches that can be captured once into a HIP graph and replayed.
// With fine_eo the fine-level smoothing passes run their MR steps on the
// even-odd Schur complement A_e - kappa^2 H_eo A_o^-1 H_oe (Sec. 4's M_eooe
// and M_ooee pieces) and reconstruct the odd sites afterwards.
//
// Setup (the paper does not describe one): starting from the caller's basis
// vectors on each level, setup_iters sweeps of MR on the homogeneous system
// D x = 0 (each sweep multiplies the vectors by prod_i (1 - alpha_i D), which
// damps the high modes and keeps the near-null space), a Cholesky-QR of the
// test vectors after every sweep (so that they stay independent), block
// orthonormalisation in FP64 and the Galerkin coarse operator; optionally
// passes of inverse iteration with the hierarchy's own V-cycle.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <vector>

#include "mg_internal.h"

namespace mrhs {

// solver_kernels.hip
size_t solver_scratch_bytes(int nrhs);
hipError_t launch_mr_alpha(const void* p, const void* r, long rows, int nrhs, void* alpha, void* scratch,
                           hipStream_t s);
hipError_t launch_mr_update(void* x, void* r, const void* p, const void* alpha, long rows, int nrhs, hipStream_t s);
hipError_t launch_mr_final(const void* part, int nblk, int nrhs, void* alpha, hipStream_t s);
hipError_t launch_multi_axpy(int x64, void* y, const void* coef, const void* const* xs, int m, double sgn, long rows,
                             int nrhs, hipStream_t s);
hipError_t launch_scale_cols(int prec64, void* y, const void* x, const double* sdev, long rows, int nrhs,
                             hipStream_t s);
hipError_t launch_inv_sqrt(const double* q, double* sdev, int nrhs, double f, hipStream_t s);
hipError_t launch_sub(int prec64, void* out, const void* a, const void* b, long n, hipStream_t s);
hipError_t launch_add_f32(void* y, const void* x, long n, hipStream_t s);
hipError_t launch_axpy_f32(void* y, const void* x, double c, long n, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
size_t col_gram_scratch_bytes();
hipError_t launch_col_gram(const void* v, long rows, int nv, void* scratch, void* g, hipStream_t s);
hipError_t launch_col_transform(void* v, long rows, int nv, const void* T, hipStream_t s);
hipError_t launch_multi_axpy_norm(int prec64, void* y, void* y32, const void* yin, const void* coef, const void* cscale,
                                 const void* const* xs, int m, double sgn, long rows, int nrhs, void* norms,
                                 void* scratch, hipStream_t s);
hipError_t launch_sub_dual(void* out, void* out32, const void* a, const void* b, long n, hipStream_t s);
hipError_t launch_sap_block_mr(const AggGeom& a, int nrhs, int color, void* x, void* rho, const void* q, hipStream_t s);


enum Phase { kFine = 0, kRestrict, kProlong, kCoarse, kPhases };

constexpr int kGraphSlots = kMaxMultiDot;

struct GraphSlot {
  hipGraphExec_t exec = nullptr;
  int n = 0;
  void* out = nullptr;
  const void* in = nullptr;  // the fine-level right-hand side the cycle reads (null: lb[0])
  mrhs_vcycle_params vc{};
  uint64_t gen = 0;  // the context's operator generation at capture
};

struct SolverState {
  hipStream_t stream = nullptr;  // private stream: graphs cannot capture the null stream
  int n = 0;                     // right-hand sides the level buffers hold
  Buffer lb[MRHS_MAX_LEVELS], lx[MRHS_MAX_LEVELS], lr[MRHS_MAX_LEVELS], lp[MRHS_MAX_LEVELS];
  Buffer alpha, part, scl, coef, qn;
  // fused MR steps on small coarse levels: second r and p fields per level
  // (ping-pong), two alpha arrays and the per-(site, column) partial sums
  Buffer lr2[MRHS_MAX_LEVELS], lp2[MRHS_MAX_LEVELS];
  Buffer mralpha, mrpart;
  Buffer gpart, gmat, gT;  // column Gram matrix (setup)
  // even-odd fine smoother: five checkerboard fields of eo_n columns
  Buffer eo, eo_part;
  int eo_n = 0;
  // even-odd coarse smoother: seven checkerboard fields per level of ceo_n columns
  Buffer ceo[MRHS_MAX_LEVELS];
  int ceo_n = 0;
  // outer Krylov: the basis (FP64 or FP32, kprec), the preconditioned
  // directions (FP32), the FP64 work field and, with an FP32 basis, an FP32 one
  int m = 0, on = 0, kprec = -1;
  Buffer V64, Z32, w64, w32;
  // fine-level right-hand side of the V-cycle when it is not lb[0] (an FP32
  // basis vector of the outer solver, read in place)
  const void* b0 = nullptr;
  // captured V-cycles, one per destination slot
  GraphSlot graphs[kGraphSlots];
  // phase timers
  bool timing = false;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
};

void mg_solver_release(mrhs_mg mg) {
  SolverState* st = mg->solver;
  if (!st) return;
  if (st->stream) (void)hipStreamSynchronize(st->stream);
  for (int l = 0; l < MRHS_MAX_LEVELS; ++l) {
    release(st->lb[l]);
    release(st->lx[l]);
    release(st->lr[l]);
    release(st->lp[l]);
    release(st->lr2[l]);
    release(st->lp2[l]);
    release(st->ceo[l]);
  }
  Buffer* b[] = {&st->alpha, &st->part, &st->scl, &st->coef, &st->qn, &st->gpart, &st->gmat, &st->gT,
                 &st->V64, &st->Z32, &st->w64, &st->w32, &st->eo, &st->eo_part, &st->mralpha, &st->mrpart};
  for (Buffer* x : b) release(*x);
  for (auto& gs : st->graphs)
    if (gs.exec) (void)hipGraphExecDestroy(gs.exec);
  for (hipEvent_t e : st->evpool) (void)hipEventDestroy(e);
  if (st->stream) (void)hipStreamDestroy(st->stream);
  delete st;
  mg->solver = nullptr;
}

namespace {

#define SOLVER_HIP(call)                             \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

long level_rows(mrhs_mg mg, int l) { return (long)mg->lv[l].g.V * mg->lv[l].ncomp; }

// Coarse levels small enough for the fused MR step, whose step-length launch
// sums one partial per (site, column) with one workgroup per column (the 3^4
// and 3^3 x 16 levels are 81 and 432 sites).
bool fused_mr_level(mrhs_mg mg, int l) {
  return l >= 1 && mfma_supported(mg->lv[l].ncomp) && mg->lv[l].g.V <= kFusedMrMaxSites;
}

mrhs_status state_of(mrhs_mg mg, SolverState** out) {
  if (!mg->solver) {
    mg->solver = new (std::nothrow) SolverState();
    if (!mg->solver) return fail(mg->ctx, MRHS_ERR_OOM, "host allocation failed");
    hipError_t e = hipStreamCreateWithFlags(&mg->solver->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(mg->ctx, e, "hipStreamCreateWithFlags");
  }
  *out = mg->solver;
  return MRHS_OK;
}

mrhs_status ensure_levels(mrhs_mg mg, SolverState* st, int n) {
  mrhs_ctx ctx = mg->ctx;
  if (n > st->n) {
    for (auto& gs : st->graphs) {
      if (gs.exec) (void)hipGraphExecDestroy(gs.exec);
      gs = GraphSlot{};
    }
    for (int l = 0; l < mg->nlevels; ++l) {
      const size_t bytes = (size_t)level_rows(mg, l) * n * 8;
      Buffer* bs[] = {&st->lb[l], &st->lx[l], &st->lr[l], &st->lp[l], &st->lr2[l], &st->lp2[l]};
      for (Buffer* b : bs) {
        release(*b);
        if ((b == &st->lr2[l] || b == &st->lp2[l]) && !fused_mr_level(mg, l)) continue;
        mrhs_status s = ensure(ctx, *b, bytes);
        if (s != MRHS_OK) return s;
      }
    }
    st->n = n;
  }
  if (!st->mrpart.p) {
    mrhs_status s = ensure(ctx, st->mralpha, 2 * MRHS_MAX_NRHS * 16);
    if (s == MRHS_OK) s = ensure(ctx, st->mrpart, coarse_mr_part_bytes(kFusedMrMaxSites));
    if (s != MRHS_OK) return s;
  }
  mrhs_status s = ensure(ctx, st->alpha, MRHS_MAX_NRHS * 16);
  if (s == MRHS_OK) s = ensure(ctx, st->part, std::max(solver_scratch_bytes(MRHS_MAX_NRHS),
                                                        blas_scratch_bytes(MRHS_MAX_NRHS, kMaxMultiDot)));
  if (s == MRHS_OK) s = ensure(ctx, st->scl, (size_t)kMaxMultiDot * MRHS_MAX_NRHS * 8);
  if (s == MRHS_OK) s = ensure(ctx, st->coef, (size_t)kMaxMultiDot * MRHS_MAX_NRHS * 16);
  if (s == MRHS_OK) s = ensure(ctx, st->qn, MRHS_MAX_NRHS * 8);
  if (s == MRHS_OK) s = ensure_colscale(mg);
  return s;
}

hipEvent_t next_event(SolverState* st) {
  if (st->evused == st->evpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    st->evpool.push_back(e);
  }
  return st->evpool[st->evused++];
}

struct PhaseMark {
  SolverState* st;
  int phase;
  hipEvent_t a = nullptr;
  PhaseMark(SolverState* s, int p) : st(s), phase(p) {
    if (st->timing) {
      a = next_event(st);
      if (a) (void)hipEventRecord(a, st->stream);
    }
  }
  ~PhaseMark() {
    if (st->timing && a) {
      hipEvent_t b = next_event(st);
      if (b) {
        (void)hipEventRecord(b, st->stream);
        st->marks.push_back({phase, {a, b}});
      }
    }
  }
};

// out = D_l in for FP32 fields.
hipError_t apply_level(mrhs_mg mg, int l, void* out, const void* in, int n, mrhs_prec cp, hipStream_t s) {
  mrhs_ctx ctx = mg->ctx;
  if (l == 0)
    return launch_fine_f32(ctx->g, ctx->t_bc, 0, (float)ctx->kappa, ctx->U32.p, ctx->A32.p, in, out, n, s,
                           &ctx->fine_cfg[n]);
  LevelData& L = mg->lv[l];
  if (!mfma_supported(L.ncomp) || cp == MRHS_F32) return coarse_apply_f32(mg, l, in, out, n, s);
  const float* scale = nullptr;
  if (cp == MRHS_F16) {
    float* sc = static_cast<float*>(mg->colscale.p);
    hipError_t e = launch_column_scale(in, level_rows(mg, l), n, sc + MRHS_MAX_NRHS, sc, s);
    if (e != hipSuccess) return e;
    scale = sc;
  }
  return launch_coarse_mfma(cp == MRHS_F16, L.g, L.ncomp, n, cp == MRHS_F16 ? L.Bf16.p : L.Bbf16.p, in, out, scale, s,
                            L.lowp_cfg[n]);
}

// r = b - D_l x (FP32 fields, p a work field): on the fine level one fused
// launch where the tuned kernel allows it, else the operator into p and the
// subtraction (same arithmetic either way).
hipError_t residual_level(mrhs_mg mg, int l, void* r, const void* b, const void* x, void* p, int n, mrhs_prec cp,
                          hipStream_t s) {
  mrhs_ctx ctx = mg->ctx;
  hipError_t e = hipSuccess;
  if (l == 0 && launch_fine_residual_f32(ctx->g, (float)ctx->kappa, ctx->U32.p, ctx->A32.p, x, b, r, n, s,
                                         &ctx->fine_cfg[n], &e))
    return e;
  e = apply_level(mg, l, p, x, n, cp, s);
  if (e == hipSuccess) e = launch_sub(0, r, b, p, level_rows(mg, l) * n, s);
  return e;
}

// nu MR steps on a small coarse level with BF16 operands, two launches each
// (fused stencil, update and per-site inner products; step length), then one
// launch for the last update of x and r.  p and the level's second r / p
// fields are overwritten.
hipError_t mr_steps_fused(mrhs_mg mg, SolverState* st, int l, void* x, void* r, void* p, int n, int nu) {
  if (nu <= 0) return hipSuccess;
  LevelData& L = mg->lv[l];
  void* R[2] = {r, st->lr2[l].p};
  void* P[2] = {p, st->lp2[l].p};
  char* a = static_cast<char*>(st->mralpha.p);
  void* A[2] = {a, a + MRHS_MAX_NRHS * 16};
  for (int i = 0; i < nu; ++i) {
    const int cur = i & 1, prv = (i + 1) & 1;
    hipError_t e = launch_coarse_mr_step(L.g, L.ncomp, n, L.Bbf16.p, i == 0 ? R[0] : R[prv], P[prv], R[cur], P[cur],
                                         x, A[prv], A[cur], st->mrpart.p, i == 0, L.mr_cfg[n], st->stream);
    if (e != hipSuccess) return e;
  }
  const int last = (nu - 1) & 1;
  return launch_mr_finish(x, R[last], P[last], r, A[last], level_rows(mg, l), n, st->stream);
}

// nu MR steps on D_l x = b with x and r = b - D x kept up to date.
hipError_t mr_steps(mrhs_mg mg, SolverState* st, int l, void* x, void* r, void* p, int n, int nu, mrhs_prec cp) {
  if (cp == MRHS_BF16 && fused_mr_level(mg, l) && st->lr2[l].p && st->mrpart.p)
    return mr_steps_fused(mg, st, l, x, r, p, n, nu);
  const long rows = level_rows(mg, l);
  for (int i = 0; i < nu; ++i) {
    hipError_t e = apply_level(mg, l, p, r, n, cp, st->stream);
    if (e == hipSuccess) e = launch_mr_alpha(p, r, rows, n, st->alpha.p, st->part.p, st->stream);
    if (e == hipSuccess) e = launch_mr_update(x, r, p, st->alpha.p, rows, n, st->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Fine-level smoothing on the even-odd Schur complement: with r = b - D x,
//   rhat = r_e + kappa H_eo A_o^-1 r_o,  nu MR steps on Dhat e_e = rhat from 0,
//   e_o = A_o^-1 (r_o + kappa H_oe e_e),  x += e,  and r = b - D x when the
// caller still needs the residual (not after the last smoothing pass).
// Dhat = A_e - kappa^2 H_eo A_o^-1 H_oe.  Checkerboard work fields live in
// st->eo: rho, q, e_e, t_o, t_o2; r and x stay full-lattice fields whose
// parity rows the kernels read or update in place.
hipError_t eo_smooth(mrhs_mg mg, SolverState* st, void* x, void* r, const void* b, void* p, int n, int nu,
                     bool need_r) {
  mrhs_ctx ctx = mg->ctx;
  if (nu <= 0) return hipSuccess;
  const int nh = ctx->g.V / 2;
  const long hrows = (long)nh * 12;
  const size_t hb = (size_t)hrows * n * 8;
  char* w = static_cast<char*>(st->eo.p);
  void *rho = w, *q = w + hb, *ee = w + 2 * hb, *to = w + 3 * hb, *to2 = w + 4 * hb;
  const auto* tabe = static_cast<const int4*>(ctx->eo_tab[0].p);
  const auto* tabo = static_cast<const int4*>(ctx->eo_tab[1].p);
  const auto* orde = static_cast<const int*>(ctx->eo_order[0].p);
  const auto* ordo = static_cast<const int*>(ctx->eo_order[1].p);
  const void* U = ctx->U32.p;
  const void* A = ctx->A32.p;
  const void* Ai = ctx->Ainv32.p;
  const double k = ctx->kappa;
  hipStream_t s = st->stream;
  // rhat = r_e + kappa H_eo (A_o^-1 r_o), reading r's rows in place
  hipError_t e = launch_clover_eo(0, nh, tabo, Ai, r, nullptr, 0.0, to, n, s, true);
  const Geom* g = &ctx->g;
  const EoWalk* ew = &ctx->eo_walk[n];
  if (e == hipSuccess) e = launch_hop_eo(0, nh, tabe, orde, U, to, rho, n, s, 3, nullptr, r, k, g, 0, ew);
  if (e == hipSuccess) e = launch_zero(ee, hb, s);
  for (int i = 0; i < nu && e == hipSuccess; ++i) {
    // q = Dhat rho: to2 = A_o^-1 (H_oe rho), q = A_e rho - kappa^2 (H_eo to2), fused launches;
    // the second also sums <q, rho> and ||q||^2 per workgroup for the step length
    int nblk = 0;
    e = launch_hop_eo(0, nh, tabo, ordo, U, rho, to2, n, s, 1, Ai, nullptr, 0.0, g, 1, ew);
    if (e == hipSuccess)
      e = launch_hop_eo_dot(nh, tabe, orde, U, to2, q, A, rho, -k * k, n, st->eo_part.p, &nblk, s, g, 0, ew);
    if (e == hipSuccess) e = launch_mr_final(st->eo_part.p, nblk, n, st->alpha.p, s);
    if (e == hipSuccess) e = launch_mr_update(ee, rho, q, st->alpha.p, hrows, n, s);
  }
  // x_o += A_o^-1 (r_o + kappa H_oe e_e) in one launch, x_e += e_e
  if (e == hipSuccess) e = launch_hop_eo(0, nh, tabo, ordo, U, ee, x, n, s, 4, Ai, r, k, g, 1, ew);
  if (e == hipSuccess) e = launch_eo_scatter_add(nh, tabe, x, ee, n, s);
  // r = b - D x
  if (need_r && e == hipSuccess) e = residual_level(mg, 0, r, b, x, p, n, MRHS_F32, s);
  return e;
}

// Coarse levels (not the coarsest) where the even-odd smoother applies:
// Nb = 32 and all extents even.
bool coarse_eo_level(mrhs_mg mg, int l) {
  if (l < 1 || l >= mg->nlevels - 1 || !mfma_supported(mg->lv[l].ncomp) || mg->lv[l].g.V / 2 > 65535) return false;
  for (int m = 0; m < 4; ++m)
    if (mg->lv[l].g.L[m] % 2) return false;
  return true;
}

// Smoothing on a coarse level's even-odd Schur complement with BF16
// operands (D_c = [[S_e, H_eo], [H_oe, S_o]], S the self blocks, H the hop
// directions), with r = b - D_c x:
//   t_o = S_o^-1 r_o,  rhat = r_e - H_eo t_o,
//   nu MR steps on Shat e_e = rhat from 0, Shat = S_e - H_eo S_o^-1 H_oe,
//   e_o = S_o^-1 (r_o - H_oe e_e),  x += e,  and r = b - D_c x if needed.
// One MR step: a_o = H_oe rho, t_o = S_o^-1 a_o, q = S_e rho - H_eo t_o (one
// launch), then the step length and the update.
hipError_t coarse_eo_smooth(mrhs_mg mg, SolverState* st, int l, void* x, void* r, const void* b, void* p, int n, int nu,
                            bool need_r) {
  if (nu <= 0) return hipSuccess;
  LevelData& L = mg->lv[l];
  const int nb = L.ncomp;
  const long hrows = (long)(L.g.V / 2) * nb;
  const size_t hb = (size_t)hrows * n * 8;
  char* w = static_cast<char*>(st->ceo[l].p);
  void *re = w, *ro = w + hb, *f2 = w + 2 * hb, *f3 = w + 3 * hb, *rho = w + 4 * hb, *q = w + 5 * hb, *ee = w + 6 * hb;
  hipStream_t s = st->stream;
  const void* B = L.Bbf16.p;
  const void* Si = L.SinvBf16.p;
  hipError_t e = launch_coarse_cb_rows(0, L.g, nb, n, r, re, 0, s);
  if (e == hipSuccess) e = launch_coarse_cb_rows(1, L.g, nb, n, r, ro, 0, s);
  // rhat = r_e - H_eo S_o^-1 r_o
  if (e == hipSuccess) e = launch_coarse_mfma_eo(1, 2, 1, L.g, nb, n, Si, 1, ro, f2, nullptr, s);
  if (e == hipSuccess) e = launch_coarse_mfma_eo(1, 1, 0, L.g, nb, n, B, 9, f2, f3, nullptr, s);
  if (e == hipSuccess) e = launch_sub(0, rho, re, f3, hrows * n, s);
  if (e == hipSuccess) e = launch_zero(ee, hb, s);
  for (int i = 0; i < nu && e == hipSuccess; ++i) {
    e = launch_coarse_mfma_eo(1, 1, 1, L.g, nb, n, B, 9, rho, f2, nullptr, s);
    if (e == hipSuccess) e = launch_coarse_mfma_eo(1, 2, 1, L.g, nb, n, Si, 1, f2, f3, nullptr, s);
    if (e == hipSuccess) e = launch_coarse_schur(0, L.g, nb, n, B, rho, f3, q, s);
    if (e == hipSuccess) e = launch_mr_alpha(q, rho, hrows, n, st->alpha.p, st->part.p, s);
    if (e == hipSuccess) e = launch_mr_update(ee, rho, q, st->alpha.p, hrows, n, s);
  }
  // e_o = S_o^-1 (r_o - H_oe e_e); x += e
  if (e == hipSuccess) e = launch_coarse_mfma_eo(1, 1, 1, L.g, nb, n, B, 9, ee, f2, nullptr, s);
  if (e == hipSuccess) e = launch_sub(0, f3, ro, f2, hrows * n, s);
  if (e == hipSuccess) e = launch_coarse_mfma_eo(1, 2, 1, L.g, nb, n, Si, 1, f3, f2, nullptr, s);
  if (e == hipSuccess) e = launch_coarse_cb_rows(0, L.g, nb, n, ee, x, 1, s);
  if (e == hipSuccess) e = launch_coarse_cb_rows(1, L.g, nb, n, f2, x, 1, s);
  if (need_r && e == hipSuccess) e = apply_level(mg, l, p, x, n, MRHS_BF16, s);
  if (need_r && e == hipSuccess) e = launch_sub(0, r, b, p, level_rows(mg, l) * n, s);
  return e;
}

// Schwarz alternating procedure on the fine level (nu cycles; see the header):
// blocks are the level-0 aggregates.  On entry r = b - D x; the residual of
// each colour's half-cycle is r itself (its rows of that colour serve as the
// block solves' rho), recomputed before the second colour and, if the caller
// needs it, at the end.
hipError_t sap_smooth(mrhs_mg mg, SolverState* st, void* x, void* r, const void* b, void* p, int n, int nu,
                      int iters, bool need_r) {
  mrhs_ctx ctx = mg->ctx;
  const AggGeom& a = mg->lv[0].agg;
  hipStream_t s = st->stream;
  hipError_t e = hipSuccess;
  for (int cyc = 0; cyc < nu && e == hipSuccess; ++cyc) {
    for (int c = 0; c < 2 && e == hipSuccess; ++c) {
      if (cyc > 0 || c > 0) {
        e = residual_level(mg, 0, r, b, x, p, n, MRHS_F32, s);
      }
      DirFilter f;
      f.sign = 0;
      f.color = c;
      for (int m = 0; m < 4; ++m) f.b[m] = a.b[m];
      for (int i = 0; i < iters && e == hipSuccess; ++i) {
        e = launch_fine_dir_f32(ctx->g, (float)ctx->kappa, ctx->U32.p, ctx->A32.p, r, p, n, f, s);
        if (e == hipSuccess) e = launch_sap_block_mr(a, n, c, x, r, p, s);
      }
    }
  }
  if (need_r && e == hipSuccess) e = residual_level(mg, 0, r, b, x, p, n, MRHS_F32, s);
  return e;
}

// The smoothing pass of the V-cycle on level l.
hipError_t smooth(mrhs_mg mg, SolverState* st, int l, void* x, void* r, const void* b, void* p, int n, int nu,
                  const mrhs_vcycle_params& vc, bool need_r) {
  if (l == 0 && vc.fine_sap) return sap_smooth(mg, st, x, r, b, p, n, nu, vc.sap_iters, need_r);
  if (l == 0 && vc.fine_eo) return eo_smooth(mg, st, x, r, b, p, n, nu, need_r);
  if (vc.coarse_eo && vc.coarse_prec == MRHS_BF16 && coarse_eo_level(mg, l) && st->ceo[l].p)
    return coarse_eo_smooth(mg, st, l, x, r, b, p, n, nu, need_r);
  return mr_steps(mg, st, l, x, r, p, n, nu, vc.coarse_prec);
}

// x_l ~ D_l^{-1} b_l (buffers lb[l] -> lx[l]).
hipError_t vcycle(mrhs_mg mg, SolverState* st, int l, int n, const mrhs_vcycle_params& vc, void* xout = nullptr) {
  const long rows = level_rows(mg, l);
  const size_t bytes = (size_t)rows * n * 8;
  const void* b = (l == 0 && st->b0) ? st->b0 : st->lb[l].p;
  void* x = xout ? xout : st->lx[l].p;
  void* r = st->lr[l].p;
  void* p = st->lp[l].p;
  const mrhs_prec cp = vc.coarse_prec;
  const int ph = l == 0 ? kFine : kCoarse;
  hipError_t e;
  // Without pre-smoothing x stays zero until the coarse-grid correction, so
  // the correction is prolongated straight into x and restricted from b.
  const bool coarsest = l == mg->nlevels - 1;
  const bool pre = coarsest || vc.nu_pre > 0;
  if (pre) {
    PhaseMark pm(st, ph);
    e = launch_zero(x, bytes, st->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r, b, bytes, hipMemcpyDeviceToDevice, st->stream);
    if (e != hipSuccess) return e;
    if (coarsest) return mr_steps(mg, st, l, x, r, p, n, vc.coarsest_iters, cp);
    e = smooth(mg, st, l, x, r, b, p, n, vc.nu_pre, vc, true);
    if (e != hipSuccess) return e;
  }
  LevelData& L = mg->lv[l];
  // BF16 coarse levels take the BF16 matrix-core intergrid kernels where they apply
  const bool ig16 = cp == MRHS_BF16 && L.bf16_ok;
  {
    PhaseMark pm(st, kRestrict);
    const void* rin = pre ? r : b;
    e = ig16 ? launch_restrict_bf16(L.agg, L.ncomp / 2, n, L.Wbf16.p, rin, st->lb[l + 1].p, st->stream)
             : launch_restrict(0, L.agg, L.ncomp / 2, L.nv, n, L.basis32.p, rin, st->lb[l + 1].p, st->stream);
    if (e != hipSuccess) return e;
  }
  e = vcycle(mg, st, l + 1, n, vc);
  if (e != hipSuccess) return e;
  {
    PhaseMark pm(st, kProlong);
    void* pout = pre ? p : x;
    e = ig16 ? launch_prolong_bf16(L.agg, L.ncomp / 2, n, L.Wbf16.p, st->lx[l + 1].p, pout, st->stream)
             : launch_prolong(0, L.agg, L.ncomp / 2, L.nv, n, L.basis32.p, st->lx[l + 1].p, pout, st->stream);
    if (e != hipSuccess) return e;
  }
  PhaseMark pm(st, ph);
  e = pre ? launch_add_f32(x, p, rows * n, st->stream) : hipSuccess;
  if (e == hipSuccess) e = residual_level(mg, l, r, b, x, p, n, cp, st->stream);
  if (e == hipSuccess) e = smooth(mg, st, l, x, r, b, p, n, vc.nu_post, vc, false);
  return e;
}

// Runs one V-cycle on st->b0 (lb[0] if null) -> xout (lx[0] if null), from a captured graph
// when asked.  One graph is kept per slot (the outer solver uses slot j for
// its direction Z_j), so the V-cycle writes straight into its destination.
mrhs_status run_vcycle(mrhs_mg mg, SolverState* st, int n, const mrhs_vcycle_params& vc, bool graph,
                       void* xout = nullptr, int slot = 0) {
  mrhs_ctx ctx = mg->ctx;
  if (!graph || st->timing) {
    SOLVER_HIP(vcycle(mg, st, 0, n, vc, xout));
    return MRHS_OK;
  }
  if (slot < 0 || slot >= kGraphSlots) return fail(ctx, MRHS_ERR_INVALID_ARG, "graph slot %d out of range", slot);
  GraphSlot& gs = st->graphs[slot];
  const bool same = gs.exec && gs.n == n && gs.out == xout && gs.vc.nu_pre == vc.nu_pre &&
                    gs.vc.nu_post == vc.nu_post && gs.vc.coarsest_iters == vc.coarsest_iters &&
                    gs.vc.coarse_prec == vc.coarse_prec && gs.vc.fine_eo == vc.fine_eo &&
                    gs.vc.coarse_eo == vc.coarse_eo && gs.vc.fine_sap == vc.fine_sap &&
                    gs.vc.sap_iters == vc.sap_iters && gs.in == st->b0 &&
                    gs.gen == ctx->op_gen;
  if (!same) {
    if (gs.exec) {
      (void)hipGraphExecDestroy(gs.exec);
      gs.exec = nullptr;
    }
    hipGraph_t gr = nullptr;
    SOLVER_HIP(hipStreamBeginCapture(st->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = vcycle(mg, st, 0, n, vc, xout);
    hipError_t e2 = hipStreamEndCapture(st->stream, &gr);
    if (e != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return hip_fail(ctx, e, "V-cycle capture");
    }
    SOLVER_HIP(e2);
    e = hipGraphInstantiate(&gs.exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    SOLVER_HIP(e);
    gs.n = n;
    gs.vc = vc;
    gs.out = xout;
    gs.in = st->b0;
    gs.gen = ctx->op_gen;
  }
  SOLVER_HIP(hipGraphLaunch(gs.exec, st->stream));
  return MRHS_OK;
}

void drop_graphs(SolverState* st) {
  for (auto& gs : st->graphs) {
    if (gs.exec) (void)hipGraphExecDestroy(gs.exec);
    gs = GraphSlot{};
  }
}

mrhs_status check_vc(mrhs_mg mg, const mrhs_vcycle_params* vc) {
  if (!vc) return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "null V-cycle parameters");
  if (vc->nu_pre < 0 || vc->nu_post < 0 || vc->coarsest_iters < 0 || vc->nu_pre + vc->nu_post > 64 ||
      vc->coarsest_iters > 1000)
    return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "V-cycle iteration counts out of range");
  if (vc->coarse_prec != MRHS_F32 && vc->coarse_prec != MRHS_BF16 && vc->coarse_prec != MRHS_F16)
    return fail(mg->ctx, MRHS_ERR_UNSUPPORTED, "coarse precision must be f32, bf16 or f16");
  if (vc->fine_eo != 0 && vc->fine_eo != 1) return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "fine_eo must be 0 or 1");
  if (vc->coarse_eo != 0 && vc->coarse_eo != 1) return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "coarse_eo must be 0 or 1");
  if (vc->fine_sap != 0 && vc->fine_sap != 1) return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "fine_sap must be 0 or 1");
  if (vc->fine_sap) {
    if (vc->fine_eo) return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "fine_sap and fine_eo exclude each other");
    if (vc->sap_iters < 1 || vc->sap_iters > 64)
      return fail(mg->ctx, MRHS_ERR_INVALID_ARG, "sap_iters = %d outside [1, 64]", vc->sap_iters);
    if (mg->nlevels < 2) return fail(mg->ctx, MRHS_ERR_STATE, "SAP blocks are the level-0 aggregates: need two levels");
    for (int m = 0; m < 4; ++m)
      if (mg->lv[0].agg.C[m] % 2)
        return fail(mg->ctx, MRHS_ERR_SHAPE, "SAP needs an even number of blocks per direction (direction %d: %d)", m,
                    mg->lv[0].agg.C[m]);
  }
  return MRHS_OK;
}

// Index tables, inverse clover blocks and checkerboard work fields of the
// even-odd fine smoother (outside any graph capture).
mrhs_status prepare_eo(mrhs_mg mg, SolverState* st, int n, const mrhs_vcycle_params& vc) {
  mrhs_ctx ctx = mg->ctx;
  if (vc.coarse_eo && vc.coarse_prec == MRHS_BF16) {
    // inverse self blocks and checkerboard work fields of every coarse level
    // the even-odd smoother runs on
    const bool grow = n > st->ceo_n;
    if (grow) {
      for (auto& gs : st->graphs) {
        if (gs.exec) (void)hipGraphExecDestroy(gs.exec);
        gs = GraphSlot{};
      }
    }
    for (int l = 1; l < mg->nlevels; ++l) {
      if (!coarse_eo_level(mg, l)) continue;
      mrhs_status s = ensure_self_inverse(mg, l);
      if (s != MRHS_OK) return s;
      if (grow || !st->ceo[l].p) {
        release(st->ceo[l]);
        s = ensure(ctx, st->ceo[l], (size_t)7 * (mg->lv[l].g.V / 2) * mg->lv[l].ncomp * std::max(n, st->ceo_n) * 8);
        if (s != MRHS_OK) return s;
      }
    }
    if (grow) st->ceo_n = n;
  }
  if (!vc.fine_eo) return MRHS_OK;
  mrhs_status s = ensure_eo_tables(ctx);
  if (s == MRHS_OK) s = ensure_clover_inverse(ctx);
  if (s != MRHS_OK) return s;
  if (n > st->eo_n) {
    for (auto& gs : st->graphs) {
      if (gs.exec) (void)hipGraphExecDestroy(gs.exec);
      gs = GraphSlot{};
    }
    release(st->eo);
    release(st->eo_part);
    s = ensure(ctx, st->eo, (size_t)5 * (ctx->g.V / 2) * 12 * n * 8);
    if (s == MRHS_OK) s = ensure(ctx, st->eo_part, hop_eo_dot_scratch_bytes(ctx->g.V / 2, n));
    if (s != MRHS_OK) return s;
    st->eo_n = n;
  }
  return MRHS_OK;
}

mrhs_status check_ready(mrhs_mg mg) {
  mrhs_ctx ctx = mg->ctx;
  if (!ctx->have_gauge || !ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "fine operator not set");
  for (int l = 0; l + 1 < mg->nlevels; ++l)
    if (!mg->lv[l].have_basis) return fail(ctx, MRHS_ERR_STATE, "basis of level %d not set", l);
  for (int l = 1; l < mg->nlevels; ++l)
    if (!mg->lv[l].have_blocks) return fail(ctx, MRHS_ERR_STATE, "coarse operator of level %d not built", l);
  return MRHS_OK;
}

// Orders the private stream after everything already queued on the context stream.
mrhs_status join_ctx_stream(mrhs_mg mg, SolverState* st) {
  mrhs_ctx ctx = mg->ctx;
  hipEvent_t e = next_event(st);
  if (!e) return fail(ctx, MRHS_ERR_HIP, "hipEventCreate failed");
  SOLVER_HIP(hipEventRecord(e, ctx->stream));
  SOLVER_HIP(hipStreamWaitEvent(st->stream, e, 0));
  return MRHS_OK;
}

// Orthonormalises the n <= 16 columns of an FP32 field [rows][n] as a whole
// (Cholesky QR applied twice: Gram matrix in FP64 on the device, Cholesky
// and triangular inverse on the host, v <- v R^-1 on the device), so that
// repeated smoothing or inverse iteration of a set of test vectors is a
// subspace iteration and the set keeps n independent directions.  Falls back
// to normalising each column when the Gram matrix is numerically singular.
mrhs_status orthonormalise_columns(mrhs_mg mg, SolverState* st, void* v, long rows, int n) {
  mrhs_ctx ctx = mg->ctx;
  hipStream_t ss = st->stream;
  mrhs_status s = ensure(ctx, st->gpart, col_gram_scratch_bytes());
  if (s == MRHS_OK) s = ensure(ctx, st->gmat, 256 * sizeof(double2));
  if (s == MRHS_OK) s = ensure(ctx, st->gT, 256 * sizeof(float2));
  if (s != MRHS_OK) return s;
  for (int pass = 0; pass < 2; ++pass) {
    double2 G[256];
    SOLVER_HIP(launch_col_gram(v, rows, n, st->gpart.p, st->gmat.p, ss));
    SOLVER_HIP(hipMemcpyAsync(G, st->gmat.p, sizeof(G), hipMemcpyDeviceToHost, ss));
    SOLVER_HIP(hipStreamSynchronize(ss));
    // G = R^dag R, R upper triangular with real positive diagonal
    std::complex<double> R[16][16] = {}, Ri[16][16] = {};
    auto g = [&](int a, int b) { return std::complex<double>(G[16 * a + b].x, G[16 * a + b].y); };
    bool ok = true;
    for (int j = 0; j < n && ok; ++j) {
      double d = g(j, j).real();
      for (int k = 0; k < j; ++k) d -= std::norm(R[k][j]);
      if (!(d > 1e-20 * g(j, j).real()) || !(d > 0.0)) {
        ok = false;
        break;
      }
      R[j][j] = std::sqrt(d);
      for (int i = j + 1; i < n; ++i) {
        std::complex<double> z = g(j, i);
        for (int k = 0; k < j; ++k) z -= std::conj(R[k][j]) * R[k][i];
        R[j][i] = z / R[j][j];
      }
    }
    if (!ok) {
      SOLVER_HIP(launch_dot(0, 1, v, v, rows, n, st->qn.p, st->part.p, ss));
      SOLVER_HIP(launch_inv_sqrt(static_cast<const double*>(st->qn.p), static_cast<double*>(st->scl.p), n, 1.0, ss));
      SOLVER_HIP(launch_scale_cols(0, v, v, static_cast<const double*>(st->scl.p), rows, n, ss));
      return MRHS_OK;
    }
    for (int i = n - 1; i >= 0; --i) {
      Ri[i][i] = 1.0 / R[i][i];
      for (int j = i + 1; j < n; ++j) {
        std::complex<double> z = 0.0;
        for (int k = i; k < j; ++k) z += Ri[i][k] * R[k][j];
        Ri[i][j] = -z / R[j][j];
      }
    }
    float2 T[256];
    for (int a = 0; a < 16; ++a)
      for (int b = 0; b < 16; ++b)
        T[16 * a + b] = (a < n && b < n) ? make_float2((float)Ri[a][b].real(), (float)Ri[a][b].imag())
                                         : make_float2(0.f, 0.f);
    SOLVER_HIP(hipMemcpyAsync(st->gT.p, T, sizeof(T), hipMemcpyHostToDevice, ss));
    SOLVER_HIP(launch_col_transform(v, rows, n, st->gT.p, ss));
    SOLVER_HIP(hipStreamSynchronize(ss));  // T lives on this stack frame
  }
  return MRHS_OK;
}

// FP64 copy of level l's FP32 basis, block orthonormalisation and the
// Galerkin operator of level l + 1.
mrhs_status rebuild_next(mrhs_mg mg, SolverState* st, int l) {
  mrhs_ctx ctx = mg->ctx;
  LevelData& L = mg->lv[l];
  const size_t cnt = (size_t)L.g.V * L.ncomp * L.nv;
  SOLVER_HIP(launch_convert_f32_to_f64(static_cast<const float*>(L.basis32.p), static_cast<double*>(L.basis64.p),
                                       2 * cnt, st->stream));
  SOLVER_HIP(hipStreamSynchronize(st->stream));
  mrhs_status s = mrhs_mg_block_orthonormalise(mg, l);
  if (s != MRHS_OK) return s;
  return mrhs_mg_build_coarse(mg, l + 1);
}

}  // namespace
}  // namespace mrhs

using namespace mrhs;

extern "C" {

mrhs_status mrhs_mg_precondition(mrhs_mg mg, void* z, const void* v, int32_t nrhs, const mrhs_vcycle_params* vc) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  if (!z || !v || !aligned16(z) || !aligned16(v)) return fail(ctx, MRHS_ERR_INVALID_ARG, "null or misaligned field");
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  mrhs_status s = check_vc(mg, vc);
  if (s == MRHS_OK) s = check_ready(mg);
  if (s != MRHS_OK) return s;
  SolverState* st;
  s = state_of(mg, &st);
  if (s == MRHS_OK) s = ensure_levels(mg, st, nrhs);
  if (s == MRHS_OK) s = prepare_eo(mg, st, nrhs, *vc);
  if (s != MRHS_OK) return s;
  st->timing = false;
  st->evused = 0;
  if (vc->coarse_prec == MRHS_BF16) s = ensure_basis_bf16(mg, 0);
  if (s == MRHS_OK) s = join_ctx_stream(mg, st);
  if (s != MRHS_OK) return s;
  const size_t bytes = (size_t)level_rows(mg, 0) * nrhs * 8;
  SOLVER_HIP(hipMemcpyAsync(st->lb[0].p, v, bytes, hipMemcpyDeviceToDevice, st->stream));
  s = run_vcycle(mg, st, nrhs, *vc, false);
  if (s != MRHS_OK) return s;
  SOLVER_HIP(hipMemcpyAsync(z, st->lx[0].p, bytes, hipMemcpyDeviceToDevice, st->stream));
  SOLVER_HIP(hipStreamSynchronize(st->stream));
  return MRHS_OK;
}

mrhs_status mrhs_coarse_mr_solve(mrhs_mg mg, int32_t level, void* x, const void* b, int32_t nrhs, int32_t iters,
                                 mrhs_prec prec) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  if (level < 1 || level >= mg->nlevels)
    return fail(ctx, MRHS_ERR_INVALID_ARG, "level %d outside [1, %d]", level, mg->nlevels - 1);
  if (!x || !b || !aligned16(x) || !aligned16(b)) return fail(ctx, MRHS_ERR_INVALID_ARG, "null or misaligned field");
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  if (iters < 0 || iters > 100000) return fail(ctx, MRHS_ERR_INVALID_ARG, "iters = %d outside [0, 100000]", iters);
  if (prec != MRHS_F32 && prec != MRHS_BF16 && prec != MRHS_F16)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "coarse MR precision must be f32, bf16 or f16");
  LevelData& L = mg->lv[level];
  if (!L.have_blocks) return fail(ctx, MRHS_ERR_STATE, "blocks of level %d not set", level);
  if (prec != MRHS_F32 && !mfma_supported(L.ncomp))
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "matrix-core stencil needs Nb = 32, got %d", L.ncomp);
  const size_t bytes = (size_t)level_rows(mg, level) * nrhs * 8;
  {
    const char* xa = static_cast<const char*>(x);
    const char* ba = static_cast<const char*>(b);
    if (xa < ba + bytes && ba < xa + bytes) return fail(ctx, MRHS_ERR_INVALID_ARG, "x and b overlap");
  }
  SolverState* st;
  mrhs_status s = state_of(mg, &st);
  if (s == MRHS_OK) s = ensure_levels(mg, st, nrhs);
  if (s == MRHS_OK) s = join_ctx_stream(mg, st);
  if (s != MRHS_OK) return s;
  st->timing = false;
  SOLVER_HIP(launch_zero(x, bytes, st->stream));
  SOLVER_HIP(hipMemcpyAsync(st->lr[level].p, b, bytes, hipMemcpyDeviceToDevice, st->stream));
  SOLVER_HIP(mr_steps(mg, st, level, x, st->lr[level].p, st->lp[level].p, nrhs, iters, prec));
  SOLVER_HIP(hipStreamSynchronize(st->stream));
  return MRHS_OK;
}

mrhs_status mrhs_mg_setup(mrhs_mg mg, const mrhs_setup_params* prm) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  if (!prm) return fail(ctx, MRHS_ERR_INVALID_ARG, "null parameters");
  const int setup_iters = prm->setup_iters, smooth_steps = prm->smooth_steps, adapt_iters = prm->adapt_iters;
  if (!ctx->have_gauge || !ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "fine operator not set");
  if (setup_iters < 0 || smooth_steps < 0 || setup_iters > 100 || smooth_steps > 1000 || adapt_iters < 0 ||
      adapt_iters > 50)
    return fail(ctx, MRHS_ERR_INVALID_ARG, "setup iteration counts out of range");
  if (adapt_iters > 0) {
    mrhs_status sv = check_vc(mg, &prm->vc);
    if (sv != MRHS_OK) return sv;
  }
  for (int l = 0; l + 1 < mg->nlevels; ++l)
    if (!mg->lv[l].have_basis) return fail(ctx, MRHS_ERR_STATE, "starting vectors of level %d not set", l);
  SolverState* st;
  mrhs_status s = state_of(mg, &st);
  if (s != MRHS_OK) return s;
  int nmax = 0;
  for (int l = 0; l + 1 < mg->nlevels; ++l) nmax = std::max(nmax, mg->lv[l].nv);
  s = ensure_levels(mg, st, nmax);
  if (s == MRHS_OK && adapt_iters > 0) s = prepare_eo(mg, st, nmax, prm->vc);
  if (s != MRHS_OK) return s;
  st->timing = false;
  st->evused = 0;
  s = join_ctx_stream(mg, st);
  if (s != MRHS_OK) return s;
  hipStream_t ss = st->stream;
  std::vector<double> minus(MRHS_MAX_NRHS, -1.0);
  for (int l = 0; l + 1 < mg->nlevels; ++l) {
    LevelData& L = mg->lv[l];
    const int n = L.nv;
    const long rows = level_rows(mg, l);
    // the internal basis [site][ncomp][nv] is a level-l field with nv columns
    void* v = L.basis32.p;
    void* r = st->lr[l].p;
    void* p = st->lp[l].p;
    for (int it = 0; it < setup_iters; ++it) {
      SOLVER_HIP(apply_level(mg, l, r, v, n, MRHS_F32, ss));
      SOLVER_HIP(hipMemcpyAsync(st->scl.p, minus.data(), n * 8, hipMemcpyHostToDevice, ss));
      SOLVER_HIP(launch_scale_cols(0, r, r, static_cast<const double*>(st->scl.p), rows, n, ss));
      SOLVER_HIP(mr_steps(mg, st, l, v, r, p, n, smooth_steps, MRHS_F32));
      SOLVER_HIP(hipStreamSynchronize(ss));  // the host array `minus` is reused next sweep
      s = orthonormalise_columns(mg, st, v, rows, n);
      if (s != MRHS_OK) return s;
    }
    s = rebuild_next(mg, st, l);
    if (s != MRHS_OK) return s;
  }
  // adaptive passes: inverse iteration v <- K v on every level, K the V-cycle
  // from that level down (an approximate inverse of D, so the low modes grow)
  for (int a = 0; a < adapt_iters; ++a) {
    for (int l = 0; l + 1 < mg->nlevels; ++l) {
      LevelData& L = mg->lv[l];
      const int n = L.nv;
      const long rows = level_rows(mg, l);
      void* v = L.basis32.p;
      if (prm->vc.coarse_prec == MRHS_BF16) {
        s = ensure_basis_bf16(mg, l);
        if (s != MRHS_OK) return s;
      }
      SOLVER_HIP(hipMemcpyAsync(st->lb[l].p, v, (size_t)rows * n * 8, hipMemcpyDeviceToDevice, ss));
      SOLVER_HIP(vcycle(mg, st, l, n, prm->vc));
      SOLVER_HIP(hipMemcpyAsync(v, st->lx[l].p, (size_t)rows * n * 8, hipMemcpyDeviceToDevice, ss));
      s = orthonormalise_columns(mg, st, v, rows, n);
      if (s != MRHS_OK) return s;
      s = rebuild_next(mg, st, l);
      if (s != MRHS_OK) return s;
    }
  }
  drop_graphs(st);  // the graphs only hold pointers into rebuilt operators, but keep it simple
  return MRHS_OK;
}

mrhs_status mrhs_mg_solve(mrhs_mg mg, void* x, const void* b, int32_t nrhs, const mrhs_solve_params* prm,
                          mrhs_solve_stats* stats) {
  if (!mg) return MRHS_ERR_INVALID_ARG;
  mrhs_ctx ctx = mg->ctx;
  if (!x || !b || !aligned16(x) || !aligned16(b)) return fail(ctx, MRHS_ERR_INVALID_ARG, "null or misaligned field");
  if (!prm) return fail(ctx, MRHS_ERR_INVALID_ARG, "null parameters");
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  const int m = prm->restart;
  if (m < 1 || m >= kMaxMultiDot) return fail(ctx, MRHS_ERR_INVALID_ARG, "restart %d outside [1, %d]", m, kMaxMultiDot - 1);
  if (!(prm->tol > 0.0) || prm->max_iters < 1) return fail(ctx, MRHS_ERR_INVALID_ARG, "bad tol or max_iters");
  if (!(prm->reorth_eta >= 0.0 && prm->reorth_eta <= 1.0))
    return fail(ctx, MRHS_ERR_INVALID_ARG, "reorth_eta must lie in [0, 1]");
  if (prm->krylov_prec != MRHS_F64 && prm->krylov_prec != MRHS_F32)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "Krylov basis precision %d not supported", (int)prm->krylov_prec);
  mrhs_status s = MRHS_OK;
  if (prm->precondition) {
    s = check_vc(mg, &prm->vc);
    if (s == MRHS_OK) s = check_ready(mg);
  } else if (!ctx->have_gauge || !ctx->have_clover) {
    s = fail(ctx, MRHS_ERR_STATE, "fine operator not set");
  }
  if (s != MRHS_OK) return s;
  const long rows = level_rows(mg, 0);
  {
    const char* xa = static_cast<const char*>(x);
    const char* ba = static_cast<const char*>(b);
    const size_t bytes = (size_t)rows * nrhs * 16;
    if (xa < ba + bytes && ba < xa + bytes) return fail(ctx, MRHS_ERR_INVALID_ARG, "x and b overlap");
  }
  SolverState* st;
  s = state_of(mg, &st);
  if (s == MRHS_OK) s = ensure_levels(mg, st, nrhs);
  if (s == MRHS_OK && prm->precondition) s = prepare_eo(mg, st, nrhs, prm->vc);
  if (s != MRHS_OK) return s;
  const int n = nrhs;
  const bool k32 = prm->krylov_prec == MRHS_F32;
  const size_t f64 = (size_t)rows * n * 16, f32 = (size_t)rows * n * 8;
  const size_t fv = k32 ? f32 : f64;  // one basis vector
  if (st->m < m || st->on < n || st->kprec != (int)k32) {
    drop_graphs(st);  // they read V and write into Z, which are reallocated
    release(st->V64);
    release(st->Z32);
    release(st->w32);
    s = ensure(ctx, st->V64, (size_t)(m + 1) * fv);
    if (s == MRHS_OK) s = ensure(ctx, st->Z32, (size_t)m * f32);
    if (s == MRHS_OK) s = ensure(ctx, st->w64, f64);
    if (s == MRHS_OK && k32) s = ensure(ctx, st->w32, f32);
    if (s != MRHS_OK) return s;
    st->m = m;
    st->on = n;
    st->kprec = k32;
  }
  st->timing = prm->timers != 0;
  st->evused = 0;
  st->marks.clear();
  if (prm->precondition && prm->vc.coarse_prec == MRHS_BF16) s = ensure_basis_bf16(mg, 0);
  if (s == MRHS_OK) s = join_ctx_stream(mg, st);
  if (s != MRHS_OK) return s;
  hipStream_t ss = st->stream;
  const auto t0 = std::chrono::steady_clock::now();
  double t_pre = 0.0;

  auto Vj = [&](int j) { return static_cast<void*>(static_cast<char*>(st->V64.p) + (size_t)j * fv); };
  auto Zj = [&](int j) { return static_cast<void*>(static_cast<char*>(st->Z32.p) + (size_t)j * f32); };
  auto D64 = [&](void* out, const void* in) {
    return launch_fine_f64(ctx->g, ctx->t_bc, 0, ctx->kappa, ctx->U64.p, ctx->A64.p, in, out, n, ss,
                           &ctx->f64_walk[n]);
  };
  auto norms = [&](const void* a, std::vector<double>& q, int prec64 = 1) -> mrhs_status {
    SOLVER_HIP(launch_dot(prec64, 1, a, a, rows, n, st->qn.p, st->part.p, ss));
    SOLVER_HIP(hipMemcpyAsync(q.data(), st->qn.p, n * 8, hipMemcpyDeviceToHost, ss));
    SOLVER_HIP(hipStreamSynchronize(ss));
    return MRHS_OK;
  };
  // The Krylov vectors are stored unnormalised: V64[i] holds u_i = hv_i v_i
  // with v_i the orthonormal vector and hv_i = ||u_i|| (per RHS, on the host),
  // and Z32[i] holds M u_i, so that z_i = (M u_i) / hv_i.  No pass over a
  // field is spent on scaling: every 1 / hv factor lives in the host scalars
  // (Hessenberg entries, solution coefficients) or in the per-(i, RHS) factors
  // 1 / hv_i^2 the Gram-Schmidt update reads from the device.
  //
  // With krylov_prec = MRHS_F32 the basis is stored in FP32 (the Gram-Schmidt
  // arithmetic and the inner products stay FP64) and D z_j is the FP32
  // operator: every cycle is then an FP32 Krylov solve of the FP64 residual,
  // whose relative accuracy (about 1e-6) far exceeds the reduction a cycle of
  // a few preconditioned steps achieves, and the restarts (FP64 true residual,
  // FP64 x) carry the solution to the FP64 tolerance, as in iterative
  // refinement.  It halves the outer solver's memory traffic; the V-cycle
  // reads each FP32 basis vector in place.
  //
  // u_{j+1} = yin - sum_i <u_i, yin> / hv_i^2 u_i into V[j + 1] (and, for an
  // FP64 basis, its FP32 rounding into the V-cycle's input), q = ||u_{j+1}||^2
  // per RHS, one pass; the first nprod products of the multi-dot are copied to hout
  auto project_out = [&](const void* yin, const std::vector<const void*>& vs, int cnt, int nprod, void* yout,
                         std::vector<std::complex<double>>& hout, std::vector<double>& qout) -> mrhs_status {
    SOLVER_HIP(launch_multi_axpy_norm(k32 ? 0 : 1, yout, (!k32 && prm->precondition) ? st->lb[0].p : nullptr, yin,
                                      st->coef.p, st->scl.p, vs.data(), cnt, -1.0, rows, n, st->qn.p, st->part.p,
                                      ss));
    SOLVER_HIP(hipMemcpyAsync(hout.data(), st->coef.p, (size_t)nprod * n * 16, hipMemcpyDeviceToHost, ss));
    SOLVER_HIP(hipMemcpyAsync(qout.data(), st->qn.p, n * 8, hipMemcpyDeviceToHost, ss));
    SOLVER_HIP(hipStreamSynchronize(ss));
    return MRHS_OK;
  };

  using cd = std::complex<double>;
  std::vector<double> bn(n), q(n), rel(n, 1.0);
  s = norms(b, bn);
  if (s != MRHS_OK) return s;
  for (int k = 0; k < n; ++k) bn[k] = std::sqrt(bn[k]);
  std::vector<int> done(n, 0);
  std::vector<cd> H((size_t)n * (m + 1) * m), g((size_t)n * (m + 1)), cs((size_t)n * m), sn((size_t)n * m);
  std::vector<cd> hc((size_t)(m + 2) * n), hc2((size_t)(m + 2) * n), y((size_t)m * n);
  // ih[i][k] = 1 / hv_i of column k (0 for a converged column or a zero vector);
  // ih2 = ih^2, the factors of the Gram-Schmidt update
  std::vector<double> ih((size_t)(m + 1) * n), ih2((size_t)(m + 1) * n);
  int iters = 0, cycles = 0, reorth = 0;
  bool all_done = false;
  auto Hel = [&](int k, int i, int j) -> cd& { return H[((size_t)k * (m + 1) + i) * m + j]; };

  while (true) {
    // true residual r = b - D x in FP64, straight into V[0] = u_0 (and its
    // FP32 rounding into the V-cycle's input); with an FP32 basis r stays in
    // w64 for the convergence test and u_0 is its FP32 rounding
    SOLVER_HIP(D64(st->w64.p, x));
    std::vector<double> qtrue(n);
    if (k32) {
      SOLVER_HIP(launch_sub_dual(st->w64.p, Vj(0), b, st->w64.p, rows * n, ss));
      s = norms(st->w64.p, qtrue);
      if (s == MRHS_OK) s = norms(Vj(0), q, 0);
    } else {
      SOLVER_HIP(launch_sub_dual(Vj(0), prm->precondition ? st->lb[0].p : nullptr, b, st->w64.p, rows * n, ss));
      s = norms(Vj(0), q);
      qtrue = q;
    }
    if (s != MRHS_OK) return s;
    all_done = true;
    for (int k = 0; k < n; ++k) {
      const double beta = std::sqrt(q[k]);
      rel[k] = bn[k] > 0 ? std::sqrt(qtrue[k]) / bn[k] : 0.0;
      done[k] = rel[k] <= prm->tol;
      all_done = all_done && done[k];
      ih[k] = (beta > 0 && !done[k]) ? 1.0 / beta : 0.0;
      ih2[k] = ih[k] * ih[k];
      g[(size_t)k * (m + 1)] = done[k] ? 0.0 : beta;
      for (int i = 1; i <= m; ++i) g[(size_t)k * (m + 1) + i] = 0.0;
    }
    if (all_done || iters >= prm->max_iters) break;
    ++cycles;
    int jdone = 0;
    for (int j = 0; j < m && iters < prm->max_iters; ++j) {
      ++iters;
      // Z32[j] = M u_j
      {
        auto tp = std::chrono::steady_clock::now();
        if (prm->precondition) {  // lb[0] already holds FP32(u_j), written with u_j; an FP32 u_j is read in place
          st->b0 = k32 ? Vj(j) : nullptr;
          s = run_vcycle(mg, st, n, prm->vc, prm->use_graph != 0, Zj(j), j);
          st->b0 = nullptr;
          if (s != MRHS_OK) return s;
        } else if (k32) {
          SOLVER_HIP(hipMemcpyAsync(Zj(j), Vj(j), f32, hipMemcpyDeviceToDevice, ss));
        } else {
          SOLVER_HIP(launch_convert_f64_to_f32(static_cast<const double*>(Vj(j)), static_cast<float*>(Zj(j)),
                                               2 * rows * n, ss));
        }
        if (st->timing) {
          SOLVER_HIP(hipStreamSynchronize(ss));
          t_pre += std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count();
        }
      }
      // w_hat = D Z32[j] in FP64, reading the FP32 direction directly (exact
      // widening), or the FP32 operator for an FP32 basis; D z_j = w_hat ih_j
      void* w = k32 ? st->w32.p : st->w64.p;
      if (k32)
        SOLVER_HIP(launch_fine_f32(ctx->g, ctx->t_bc, 0, (float)ctx->kappa, ctx->U32.p, ctx->A32.p, Zj(j), w, n, ss,
                                   &ctx->fine_cfg[n]));
      else
        SOLVER_HIP(launch_fine_f64_in32(ctx->g, ctx->kappa, ctx->U64.p, ctx->A64.p, Zj(j), w, n, ss,
                                        &ctx->fine_cfg[n]));
      // classical Gram-Schmidt; the first pass also yields ||w_hat||^2 (w_hat is
      // the last vector of the multi-dot), and a second pass is made only when
      // the projection removed more than 1 - reorth_eta of it for some RHS
      SOLVER_HIP(hipMemcpyAsync(st->scl.p, ih2.data(), (size_t)(j + 1) * n * 8, hipMemcpyHostToDevice, ss));
      std::vector<const void*> vs(j + 2);
      for (int i = 0; i <= j; ++i) vs[i] = Vj(i);
      vs[j + 1] = w;
      SOLVER_HIP(launch_multi_dot(k32 ? 0 : 1, vs.data(), j + 2, w, rows, n, st->coef.p, st->part.p, ss));
      s = project_out(w, vs, j + 1, j + 2, Vj(j + 1), hc, q);  // the last of the j + 2 products is ||w_hat||^2
      if (s != MRHS_OK) return s;
      bool again = false;
      for (int k = 0; k < n; ++k)
        if (!done[k] && q[k] < prm->reorth_eta * hc[(size_t)(j + 1) * n + k].real()) again = true;
      std::fill(hc2.begin(), hc2.end(), cd(0.0));
      if (again) {
        SOLVER_HIP(launch_multi_dot(k32 ? 0 : 1, vs.data(), j + 1, Vj(j + 1), rows, n, st->coef.p, st->part.p, ss));
        s = project_out(Vj(j + 1), vs, j + 1, j + 1, Vj(j + 1), hc2, q);
        if (s != MRHS_OK) return s;
        ++reorth;
      }
      bool all_conv = true;
      for (int k = 0; k < n; ++k) {
        const double ihj = ih[(size_t)j * n + k];
        for (int i = 0; i <= j; ++i)
          Hel(k, i, j) = (hc[(size_t)i * n + k] + hc2[(size_t)i * n + k]) * (ih[(size_t)i * n + k] * ihj);
        const double un = std::sqrt(q[k]);
        Hel(k, j + 1, j) = un * ihj;
        ih[(size_t)(j + 1) * n + k] = (un > 0 && !done[k]) ? 1.0 / un : 0.0;
        ih2[(size_t)(j + 1) * n + k] = ih[(size_t)(j + 1) * n + k] * ih[(size_t)(j + 1) * n + k];
        // apply the previous rotations to column j, then a new one
        for (int i = 0; i < j; ++i) {
          const cd a = Hel(k, i, j), c = Hel(k, i + 1, j);
          const cd ci = cs[(size_t)k * m + i], si = sn[(size_t)k * m + i];
          Hel(k, i, j) = std::conj(ci) * a + std::conj(si) * c;
          Hel(k, i + 1, j) = -si * a + ci * c;
        }
        const cd a = Hel(k, j, j), c = Hel(k, j + 1, j);
        const double den = std::sqrt(std::norm(a) + std::norm(c));
        cd ci = 1.0, si = 0.0;
        if (den > 0) {
          ci = a / den;
          si = c / den;
        }
        cs[(size_t)k * m + j] = ci;
        sn[(size_t)k * m + j] = si;
        Hel(k, j, j) = std::conj(ci) * a + std::conj(si) * c;
        Hel(k, j + 1, j) = 0.0;
        const cd gj = g[(size_t)k * (m + 1) + j];
        g[(size_t)k * (m + 1) + j] = std::conj(ci) * gj;
        g[(size_t)k * (m + 1) + j + 1] = -si * gj;
        const double est = bn[k] > 0 ? std::abs(g[(size_t)k * (m + 1) + j + 1]) / bn[k] : 0.0;
        if (!done[k] && est > prm->tol) all_conv = false;
      }
      jdone = j + 1;
      if (all_conv) break;
    }
    // y = R^{-1} g per RHS, x += sum_i y_i z_i = sum_i (y_i ih_i) Z32[i]
    for (int k = 0; k < n; ++k) {
      for (int i = jdone - 1; i >= 0; --i) {
        cd acc = g[(size_t)k * (m + 1) + i];
        for (int l = i + 1; l < jdone; ++l) acc -= Hel(k, i, l) * y[(size_t)l * n + k];
        const cd d = Hel(k, i, i);
        y[(size_t)i * n + k] = (done[k] || std::abs(d) == 0.0) ? cd(0.0) : acc / d;
      }
    }
    if (jdone > 0) {
      std::vector<cd> yz((size_t)jdone * n);
      for (int i = 0; i < jdone; ++i)
        for (int k = 0; k < n; ++k) yz[(size_t)i * n + k] = y[(size_t)i * n + k] * ih[(size_t)i * n + k];
      SOLVER_HIP(hipMemcpyAsync(st->coef.p, yz.data(), (size_t)jdone * n * 16, hipMemcpyHostToDevice, ss));
      std::vector<const void*> zs(jdone);
      for (int i = 0; i < jdone; ++i) zs[i] = Zj(i);
      SOLVER_HIP(launch_multi_axpy(0, x, st->coef.p, zs.data(), jdone, 1.0, rows, n, ss));
      SOLVER_HIP(hipStreamSynchronize(ss));  // yz is host memory
    }
  }
  SOLVER_HIP(hipStreamSynchronize(ss));
  const double t_tot = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->nrhs = n;
    stats->iters = iters;
    stats->cycles = cycles;
    stats->reorth = reorth;
    for (int k = 0; k < n; ++k) {
      stats->converged[k] = done[k];
      stats->rel_resid[k] = rel[k];
    }
    stats->seconds_total = t_tot;
    stats->seconds_precond = t_pre;
    if (st->timing) {
      for (auto& mk : st->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, mk.second.first, mk.second.second) == hipSuccess)
          stats->seconds_phase[mk.first] += ms * 1e-3;
      }
    }
  }
  st->marks.clear();
  if (!all_done) return fail(ctx, MRHS_ERR_NOT_CONVERGED, "not converged after %d iterations", iters);
  return MRHS_OK;
}

}  // extern "C"
