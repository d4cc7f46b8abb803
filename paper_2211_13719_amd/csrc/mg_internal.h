// Multigrid hierarchy object shared by the multigrid translation units.
#pragma once

#include "internal.h"

namespace mrhs {

// One level of the hierarchy.  Level 0 is the fine lattice (12 spinor
// components); level l >= 1 has ncomp = 2 n_v(l-1) components per site.
struct LevelData {
  Geom g{};
  int ncomp = 0;
  // basis prolongating from level + 1 (internal layout [site][ncomp][nv])
  int nv = 0;
  AggGeom agg{};
  Buffer basis64, basis32;
  bool have_basis = false;
  // BF16 copy of basis32 for the matrix-core intergrid kernels (n_v = 16),
  // built on demand and dropped whenever basis32 changes
  Buffer Wbf16;
  bool bf16_ok = false;
  // stencil blocks (levels >= 1): FP64 master [site][9][i][j], transposed
  // copies [site][9][j][i] for the vector-ALU kernels, MFMA packs
  Buffer B64, BT32, BT64, Bbf16, Bf16, Bf32p;
  bool have_blocks = false;
  // inverses of the self blocks (FP64 [site][Nb][Nb]) and their MFMA packs,
  // built on first use by the even-odd calls, dropped when the blocks change
  Buffer Sinv64, SinvBf16, SinvF16, SinvF32p;
  bool have_sinv = false;
  // FP32 stencil kernel per Nrhs, set by mrhs_mg_tune: 0 the FP32 matrix
  // cores (default for Nb = 32), 1 the vector-ALU kernel
  signed char f32_valu[MRHS_MAX_NRHS + 1] = {};
  // launch shape of the BF16 / FP16 stencil per Nrhs (launch_coarse_mfma's
  // cfg), set by mrhs_mg_tune; 0 until tuned
  signed char lowp_cfg[MRHS_MAX_NRHS + 1] = {};
  // launch shape of the fused BF16 MR step per Nrhs (same encoding), set by
  // mrhs_mg_tune on levels small enough for it; 0 until tuned
  signed char mr_cfg[MRHS_MAX_NRHS + 1] = {};
};

struct SolverState;

}  // namespace mrhs

struct mrhs_mg_s {
  mrhs_ctx ctx = nullptr;
  int nlevels = 0;
  mrhs::LevelData lv[MRHS_MAX_LEVELS];
  mrhs::Buffer tmpA, tmpB, tmpC;  // setup scratch
  mrhs::Buffer colscale;          // per-RHS FP16 scales and their reduction words
  int* flag = nullptr;            // device flag (rank deficiency)
  mrhs::SolverState* solver = nullptr;
};

namespace mrhs {

mrhs_status refresh_blocks(mrhs_mg mg, int level);
// Inverted self blocks of a level and their MFMA packs, built on first use
// (synchronises; not under graph capture).
mrhs_status ensure_self_inverse(mrhs_mg mg, int level);
// FP32 stencil D_l in -> out with the kernel mrhs_mg_tune chose for n (Nb = 32:
// matrix cores unless the vector-ALU kernel measured faster)
hipError_t coarse_apply_f32(mrhs_mg mg, int level, const void* in, void* out, int n, hipStream_t s);
// per-RHS FP16 scales and their reduction words (zeroed when first allocated)
mrhs_status ensure_colscale(mrhs_mg mg);
mrhs_status refresh_basis32(mrhs_mg mg, int level);
// Builds the BF16 basis copy of every level >= from (where the matrix-core
// intergrid kernels apply) unless current; synchronises the context stream.
mrhs_status ensure_basis_bf16(mrhs_mg mg, int from);
// basis32 of `level` was modified in place: drop its BF16 copy
inline void basis32_changed(mrhs_mg mg, int level) { mg->lv[level].bf16_ok = false; }

// intergrid_mfma.hip (n_v = 16, FP32 fields, BF16 basis and operands, FP32 accumulation)
bool intergrid_mfma_supported(const AggGeom& a, int h, int nv);
hipError_t launch_pack_basis_bf16(const void* basis32, void* out, long ncomplex, hipStream_t s);
hipError_t launch_restrict_bf16(const AggGeom& a, int h, int nrhs, const void* Wbf16, const void* f, void* y,
                                hipStream_t s);
hipError_t launch_prolong_bf16(const AggGeom& a, int h, int nrhs, const void* Wbf16, const void* y, void* f,
                               hipStream_t s);

// coarse_mfma.hip
bool mfma_supported(int nb);
size_t mfma_pack_bytes(long nsite);
mrhs_status pack_blocks_mfma(mrhs_mg mg, int level);
hipError_t launch_pack_blocks(int f16, const void* B64, void* packed, long nsite, hipStream_t s);
// scale[k] for FP16 operands; work holds nrhs 32-bit words, zero on entry and exit
hipError_t launch_column_scale(const void* in, long rows, int nrhs, void* work, float* scale, hipStream_t s);
// cfg (0..3): bit 0 eight wavefronts per workgroup (else four), bit 1 two
// 32-column tiles per workgroup (else one)
hipError_t launch_coarse_mfma(int f16, const Geom& g, int nb, int nrhs, const void* packed, const void* in, void* out,
                              const float* scale, hipStream_t s, int cfg = 0);
// One fused minimal-residual step with the BF16 stencil (see the kernel;
// two launches): part holds coarse_mr_part_bytes(V) bytes.
size_t coarse_mr_part_bytes(long nsite);
// Levels that take the fused MR step: Nb = 32 and at most this many sites.
constexpr int kFusedMrMaxSites = 1024;
hipError_t launch_coarse_mr_step(const Geom& g, int nb, int nrhs, const void* packed, const void* rold, const void* pold,
                                 void* rnew, void* pnew, void* x, const void* aold, void* anew, void* part, int first,
                                 int cfg, hipStream_t s);
// x += a r and, if rout is given, rout = r - a p (the end of a fused MR sweep)
hipError_t launch_mr_finish(void* x, const void* r, const void* p, void* rout, const void* alpha, long rows, int nrhs,
                            hipStream_t s);
// FP32 operands on the FP32 matrix cores (Nb = 32)
hipError_t launch_coarse_mfma_f32(const Geom& g, int nb, int nrhs, const void* packed, const void* in, void* out,
                                  hipStream_t s);

// even-odd modes of the stencil (coarse_mfma.hip): prec 0 FP32, 1 BF16, 2 FP16;
// eo 1 the eight hop directions into parity p, eo 2 per-site blocks on parity p
// (bstride 9: the stencil pack's self blocks, 1: a pack of one block per site)
hipError_t launch_coarse_mfma_eo(int prec, int eo, int parity, const Geom& g, int nb, int nrhs, const void* packed,
                                 int bstride, const void* in, void* out, const float* scale, hipStream_t s);
hipError_t launch_self_invert(long nsite, const void* B64, void* out, int* flag, hipStream_t s);
// out = S_p in - H_{p,1-p} in2 on parity p (BF16 operands), and the parity-row
// gather / scatter-add between full and checkerboard coarse fields
hipError_t launch_coarse_schur(int parity, const Geom& g, int nb, int nrhs, const void* packed, const void* in,
                               const void* in2, void* out, hipStream_t s);
hipError_t launch_coarse_cb_rows(int parity, const Geom& g, int nb, int nrhs, const void* src, void* dst, int scatter_add,
                                 hipStream_t s);
// kind 0 FP32 pack, 1 BF16, 2 FP16, of nblk FP64 Nb x Nb blocks
hipError_t launch_pack_block_list(int kind, const void* B64, void* packed, long nblk, hipStream_t s);

// solver (mg_solve.hip)
void mg_solver_release(mrhs_mg mg);

}  // namespace mrhs
