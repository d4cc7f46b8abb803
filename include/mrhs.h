/*
 * mrhs.h -- C interface of libmrhs, the MI355X (gfx950) library that applies
 * the Wilson-clover operator and the pieces of an aggregation multigrid to a
 * block of Nrhs right-hand sides at once.
 *
 * What is computed follows Richtmann, Meyer, Wettig, "MRHS multigrid solver
 * for Wilson-clover fermions" (LATTICE2022): the fine hopping and clover
 * terms (Sec. 4), the intergrid project/promote operators (Sec. 5), the
 * coarse-level hopping term (Sec. 6) and simultaneous inner products
 * (Sec. 7), each acting on Nrhs fields in one call (Sec. 2: gauge links are
 * loaded once and reused for every right-hand side).  The paper prints no
 * operator formula; the conventions below are the standard ones and are
 * stated with each call.
 *
 * Conventions shared by every call
 * --------------------------------
 *  Lattice   dims = (Lx, Ly, Lz, Lt); site s = x + Lx*(y + Ly*(z + Lz*t)).
 *            Directions mu = 0..3 are x, y, z, t.
 *  Spinor    12 complex components per site, index 3*spin + colour, in the
 *            chiral gamma basis (gamma_5 = diag(1, 1, -1, -1)): components
 *            0..5 have chirality +, 6..11 chirality -.
 *  Fields    [site][component][rhs], complex interleaved (re, im), i.e.
 *            element (s, c, k) sits at complex offset (s*ncomp + c)*nrhs + k.
 *            FP32 fields are float pairs, FP64 fields double pairs.
 *  Gauge     [site][mu][3][3] complex, U_mu(x)[a][b] row-major; links are
 *            periodic.  Fermion hops across the t boundary are multiplied by
 *            t_bc (+1 periodic, -1 antiperiodic).
 *  Clover    [site][chirality][36] real: the Hermitian 6x6 block A_chi of
 *            A = 1 + C, packed as its 6 real diagonal entries followed by the
 *            15 strictly-lower entries (1,0), (2,0), (2,1), (3,0), ... (5,4)
 *            as (re, im).
 *  Nrhs      1 <= nrhs <= 64, otherwise MRHS_ERR_SHAPE.
 *
 *  Memory    Pointers marked "device" are HIP device pointers (any allocator,
 *            e.g. PyTorch tensors), 16-byte aligned.  The caller owns them;
 *            the library keeps no reference once a call returns.  Gauge and
 *            clover data are copied into library-owned device memory.
 *  Streams   Every compute call is enqueued on the context's stream and
 *            returns without waiting, unless its comment says it synchronises.
 *  Errors    Every call returns an mrhs_status.  Arguments are checked on the
 *            host before anything is launched; on failure nothing is launched
 *            and mrhs_last_error(ctx) describes the problem.  HIP runtime
 *            errors map to MRHS_ERR_HIP with the HIP message.  No C++
 *            exception crosses this interface.
 *  Threads   A context is used by one host thread at a time.
 */
#ifndef MRHS_H
#define MRHS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRHS_MAX_NRHS 64
#define MRHS_MAX_LEVELS 3

typedef struct mrhs_ctx_s* mrhs_ctx;

typedef enum {
  MRHS_OK = 0,
  MRHS_ERR_INVALID_ARG = 1, /* null/misaligned pointer, bad enum, bad parameter */
  MRHS_ERR_SHAPE = 2,       /* lattice, nrhs or component count out of range */
  MRHS_ERR_UNSUPPORTED = 3, /* precision not offered for this call */
  MRHS_ERR_STATE = 4,       /* called before the data it needs was set */
  MRHS_ERR_OOM = 5,         /* device allocation failed */
  MRHS_ERR_HIP = 6,         /* HIP runtime error */
  MRHS_ERR_NOT_CONVERGED = 7
} mrhs_status;

typedef enum { MRHS_F64 = 0, MRHS_F32 = 1, MRHS_BF16 = 2, MRHS_F16 = 3 } mrhs_prec;

/* ---- context -------------------------------------------------------------
 * mrhs_create: a context for one lattice on one GPU.  dims[4] = (Lx, Ly, Lz,
 * Lt), each >= 2 and V = Lx*Ly*Lz*Lt < 2^31 / 64; t_bc = +1 or -1 is the
 * fermion boundary factor in time (the paper's Sec. 4 benchmarks and the
 * U101 solve of Sec. 8 use lattices of this form); device is the HIP device
 * ordinal; stream is a hipStream_t (NULL = the default stream) on which all
 * work is enqueued.  On success *ctx receives the new context. */
mrhs_status mrhs_create(mrhs_ctx* ctx, const int32_t dims[4], int32_t t_bc, int32_t device,
                        void* stream);
/* Frees everything the context owns.  NULL is ignored. */
void mrhs_destroy(mrhs_ctx ctx);
/* Message of the last failed call on ctx ("" if none); with ctx == NULL the
 * last failure of mrhs_create on this thread.  Never NULL; valid until the
 * next call on the same context. */
const char* mrhs_last_error(mrhs_ctx ctx);
/* Replaces the stream work is enqueued on. */
mrhs_status mrhs_set_stream(mrhs_ctx ctx, void* stream);
/* Blocks until all work on the context's stream has finished. */
mrhs_status mrhs_synchronize(mrhs_ctx ctx);

/* ---- fine-level operator (paper Sec. 4) ----------------------------------
 * mrhs_set_gauge: copies the links U (layout above, prec MRHS_F64 or
 * MRHS_F32, host memory if on_device == 0 else device memory) into the
 * context, which keeps an FP64 and an FP32 copy.  Synchronises. */
mrhs_status mrhs_set_gauge(mrhs_ctx ctx, const void* U, mrhs_prec prec, int32_t on_device);

/* mrhs_build_clover: computes the clover blocks on the GPU, in FP64, from the
 * links already set:  A = 1 + i csw kappa sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu},
 * sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], F_{mu nu} = (Q - Q^dag)/8 with
 * Q the sum of the four mu-nu plaquette leaves at x (the "precomputed
 * clover term" of Sec. 4).  Stores kappa for the operator calls below.
 * MRHS_ERR_STATE without links.  Synchronises. */
mrhs_status mrhs_build_clover(mrhs_ctx ctx, double csw, double kappa);

/* mrhs_set_clover: copies packed clover blocks (layout above, MRHS_F64 or
 * MRHS_F32, host or device) and sets kappa.  Synchronises. */
mrhs_status mrhs_set_clover(mrhs_ctx ctx, const void* A, mrhs_prec prec, int32_t on_device,
                            double kappa);

/* mrhs_get_clover: copies the context's clover blocks out, in prec
 * (MRHS_F64 or MRHS_F32), to host (on_device == 0) or device memory.
 * Synchronises. */
mrhs_status mrhs_get_clover(mrhs_ctx ctx, void* A, mrhs_prec prec, int32_t on_device);

/* mrhs_dwc_apply: out = D in for nrhs fields at once, with
 *   D = A - kappa H,
 *   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *              + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu),
 * i.e. the fine hopping term (D_hop of Sec. 4) fused with the clover term
 * (M_ooee of Sec. 4).  in/out: device fields [V][12][nrhs] in prec
 * (MRHS_F32 or MRHS_F64); they must not overlap.  The launch configuration
 * is the one mrhs_tune chose for nrhs (FP32: mrhs_get_tuning; FP64:
 * mrhs_get_f64_walk), else a default; every configuration gives the same
 * bits.  MRHS_ERR_STATE before links and clover are set. */
mrhs_status mrhs_dwc_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec);
/* mrhs_hop_apply: out = H in (hopping term only, Sec. 4 D_hop). */
mrhs_status mrhs_hop_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec);
/* mrhs_clover_apply: out = A in (clover term only, Sec. 4 M_ooee on the
 * full lattice). */
mrhs_status mrhs_clover_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs,
                              mrhs_prec prec);

/* Even-odd (checkerboard) pieces of the fine operator, Sec. 4: M_eooe (the
 * hopping term between the checkerboarded lattices) and M_ooee (the clover
 * term on one checkerboard) with its inverse.  Parity p(x) = (x+y+z+t) mod 2;
 * every lattice extent must be even (MRHS_ERR_SHAPE otherwise), so that each
 * hop joins the two parities.  A field on one parity is a device array
 * [V/2][12][nrhs] in prec (MRHS_F32 or MRHS_F64) whose entry i is the site
 * of that parity among the lattice sites 2i and 2i + 1.  in and out must not
 * overlap.  Index tables (and, for the inverse, the inverted blocks) are
 * built on the first call and kept by the context. */
/* mrhs_hop_eo_apply: out (parity out_parity) = H in (parity 1 - out_parity),
 * H the hopping term of mrhs_hop_apply restricted to those two parities.
 * MRHS_ERR_STATE before the links are set. */
mrhs_status mrhs_hop_eo_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, int32_t out_parity,
                              mrhs_prec prec);
/* mrhs_set_eo_walk: launch shape of the FP32 checkerboard hop (mrhs_hop_eo_apply,
 * mrhs_schur_apply and the even-odd smoother) for nrhs right-hand sides:
 * tile = (Bx, By, Bz, Ts) selects the t-walk kernel (each thread walks Ts
 * output sites of one site of a Bx x By x Bz spatial block, every second
 * time slice, carrying the backward t-hop in registers; Bx By Bz >= 16, the
 * block must divide the spatial extents and Ts divide Lt / 2) with
 * rhs_per_thread 1 or 2 (0: two for even nrhs, else one); tile = NULL
 * selects the tiled kernel.  mrhs_tune chooses it by timing (lattices with
 * even extents).  The fields computed are bit-identical either way.  An
 * invalid shape gets MRHS_ERR_INVALID_ARG. */
mrhs_status mrhs_set_eo_walk(mrhs_ctx ctx, int32_t nrhs, const int32_t* tile, int32_t rhs_per_thread);
/* mrhs_get_eo_walk: the shape in use for nrhs (*on = 0: tiled kernel), and
 * the times the last mrhs_tune measured for it and for the tiled kernel
 * (microseconds, 0 if not measured).  Any output pointer may be NULL. */
mrhs_status mrhs_get_eo_walk(mrhs_ctx ctx, int32_t nrhs, int32_t* on, int32_t* rhs_per_thread, int32_t tile[4],
                             float* us, float* us_tiled);
/* mrhs_clover_eo_apply: out = A_p in (inverse = 0) or out = A_p^-1 in
 * (inverse = 1) on parity p, A_p the chiral 6x6 clover blocks of the parity-p
 * sites.  The inverse blocks are computed once per clover term in FP64
 * (Gauss-Jordan with partial pivoting); MRHS_ERR_STATE before the clover
 * term is set or when a block is singular.  Synchronises on the first
 * inverse call after a new clover term. */
mrhs_status mrhs_clover_eo_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, int32_t parity,
                                 int32_t inverse, mrhs_prec prec);
/* mrhs_schur_apply: out = (A_e - kappa^2 H_eo A_o^-1 H_oe) in on the even
 * sites, the Schur complement of D = A - kappa H with respect to the odd
 * sites (D x = b is equivalent to applying it to x_e with right-hand side
 * b_e + kappa H_eo A_o^-1 b_o).  in and out are even-parity fields; the
 * odd-parity intermediate A_o^-1 H_oe in lives in a context-owned workspace
 * field, grown on demand. */
mrhs_status mrhs_schur_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec);

/* ---- batched level-1 operations (paper Sec. 7) ---------------------------
 * A field here is any [nsites][ncomp][nrhs] complex array in device memory,
 * prec MRHS_F32 or MRHS_F64 (fine spinors have ncomp = 12, coarse vectors
 * ncomp = Nb).  Each operation acts on the nrhs columns independently and
 * makes one pass over the data for all of them: the simultaneous inner
 * products of Sec. 7, which replace one global reduction per right-hand side
 * by one for the whole block.  FP32 inputs are widened to FP64 before they
 * are multiplied and all sums are taken in FP64, in an order fixed by
 * (nsites, ncomp, nrhs) alone, so results repeat bit for bit.
 * nsites*ncomp >= 1, 1 <= nrhs <= 64.
 *
 * mrhs_dot: out[2k] + i out[2k+1] = <a_k, b_k> = sum_{s,c} conj(a[s][c][k]) b[s][c][k].
 *   out holds 2*nrhs doubles in host memory (out_on_device = 0: the call
 *   synchronises) or device memory (out_on_device = 1: asynchronous). */
mrhs_status mrhs_dot(mrhs_ctx ctx, double* out, const void* a, const void* b, int64_t nsites, int32_t ncomp,
                     int32_t nrhs, mrhs_prec prec, int32_t out_on_device);
/* mrhs_norm2: out[k] = ||a_k||^2, nrhs doubles, same rules as mrhs_dot. */
mrhs_status mrhs_norm2(mrhs_ctx ctx, double* out, const void* a, int64_t nsites, int32_t ncomp, int32_t nrhs,
                       mrhs_prec prec, int32_t out_on_device);
/* mrhs_multi_dot: out[2(j*nrhs + k)] + i out[2(j*nrhs + k) + 1] = <v_j,k, w_k> for
 * j < m, 1 <= m <= 16: the m inner products of one Gram-Schmidt step, reading
 * w once.  v is a host array of m device field pointers (all of the shape of
 * w).  out: 2*m*nrhs doubles, host or device as for mrhs_dot. */
mrhs_status mrhs_multi_dot(mrhs_ctx ctx, double* out, const void* const* v, int32_t m, const void* w,
                           int64_t nsites, int32_t ncomp, int32_t nrhs, mrhs_prec prec, int32_t out_on_device);
/* mrhs_multi_dot_noalloc: mrhs_multi_dot for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, same kernels and bit-identical
 * results, but no allocation of any kind.  Its partial sums (and, with
 * out_on_device = 0, the staged result) live in a fixed device array of
 * 16 MiB + 16 KiB per device, held until the process ends; its address is
 * looked up when a context is first created on the device.  Limits: m <= 16
 * and nrhs <= 64 (the array holds 1024 x m x nrhs partials at the maximum);
 * larger requests get MRHS_ERR_SHAPE.  Every call on one device shares that
 * array: calls that overlap in time on one device (other host threads or
 * streams) race and must be serialised by the caller. */
mrhs_status mrhs_multi_dot_noalloc(mrhs_ctx ctx, double* out, const void* const* v, int32_t m, const void* w,
                                   int64_t nsites, int32_t ncomp, int32_t nrhs, mrhs_prec prec,
                                   int32_t out_on_device);

/* mrhs_read_probe: measurement helper for the rooflines of kernels bound by
 * their L2 misses.  Reads the device buffer buf (bytes, a multiple of 16)
 * `sweeps` times with `grid` workgroups of 256 threads, each thread reading
 * 16-byte words in a grid-stride loop, `depth` (1, 2, 4 or 8) independent
 * words in flight per thread (after one untimed sweep), and returns the
 * elapsed time in *ms (HIP events on the context stream).  The bytes read per
 * second tell which level serves a working set of that size (the L2s, 4 MiB
 * per XCD; the Infinity Cache; HBM) and, across depths, whether the rate is
 * bound by bandwidth or by the latency of too few loads in flight.  Bad
 * sizes, sweeps, grid or depth get MRHS_ERR_INVALID_ARG.  Synchronises. */
mrhs_status mrhs_read_probe(mrhs_ctx ctx, const void* buf, int64_t bytes, int32_t sweeps, int32_t grid, int32_t depth,
                            float* ms);

/* mrhs_axpy: y_k <- y_k + alpha_k x_k per column, alpha_k = alpha[2k] + i alpha[2k+1]
 * (FP64, host memory if alpha_on_device = 0, else device memory); the update
 * is computed in FP64 and rounded to prec.  x and y must not overlap. */
mrhs_status mrhs_axpy(mrhs_ctx ctx, void* y, const double* alpha, const void* x, int64_t nsites, int32_t ncomp,
                      int32_t nrhs, mrhs_prec prec, int32_t alpha_on_device);

/* ---- multigrid hierarchy (paper Secs. 5 and 6) ---------------------------
 * Levels are numbered from 0 (the fine lattice of the context, 12 spinor
 * components per site) to nlevels - 1.  Coarsening step l (level l -> l + 1)
 * groups the sites of level l into aggregates of extent block[l] (x, y, z, t)
 * and keeps n_v[l] basis vectors, each split by chirality, so level l + 1 has
 * the lattice dims(l) / block[l] and ncomp(l + 1) = Nb = 2 n_v[l] components
 * per site ("nbasis = twice the number of basis vectors", Sec. 5).  On every
 * level the first half of the components has chirality + and the second
 * half chirality -; aggregate A = X + Cx (Y + Cy (Z + Cz T)) is the coarse
 * site.  Fields on level l are [site][ncomp(l)][nrhs] complex, like fine
 * fields.  Supported: n_v in {4, 8, 16}; the matrix-core stencil needs Nb = 32.
 */
typedef struct mrhs_mg_s* mrhs_mg;

typedef struct {
  int32_t nlevels;      /* 2 or 3 */
  int32_t block[2][4];  /* aggregate extent of step l; must divide dims(l) */
  int32_t n_v[2];       /* basis vectors per step */
} mrhs_mg_params;

/* Creates the hierarchy on ctx's lattice (ctx must outlive it).  MRHS_ERR_SHAPE
 * if a block does not divide its lattice, MRHS_ERR_UNSUPPORTED for n_v
 * outside the supported set. */
mrhs_status mrhs_mg_create(mrhs_ctx ctx, const mrhs_mg_params* params, mrhs_mg* mg);
void mrhs_mg_destroy(mrhs_mg mg);
/* Lattice extents and components per site of a level. */
mrhs_status mrhs_mg_level_info(mrhs_mg mg, int32_t level, int32_t dims[4], int32_t* ncomp);

/* mrhs_mg_set_basis: the n_v[level] basis vectors of step `level` (0 <= level
 * < nlevels - 1) as [site][n_v][ncomp(level)] complex (vector i at site s,
 * component c at (s n_v + i) ncomp + c), prec MRHS_F64 or MRHS_F32, host or
 * device.  Copied in; the library keeps an FP64 master and an FP32 copy.
 * Synchronises.  Invalidates the blocks of the coarser levels. */
mrhs_status mrhs_mg_set_basis(mrhs_mg mg, int32_t level, const void* vecs, mrhs_prec prec, int32_t on_device);
/* Copies the (current) basis out in the layout above.  Synchronises. */
mrhs_status mrhs_mg_get_basis(mrhs_mg mg, int32_t level, void* vecs, mrhs_prec prec, int32_t on_device);
/* mrhs_mg_block_orthonormalise: for every aggregate A and chirality chi the
 * n_v vectors restricted to (A, chi) are replaced by the Q factor of their
 * thin QR decomposition with real positive diagonal of R (unique), computed
 * on the GPU in FP64 by Gram-Schmidt applied twice.  MRHS_ERR_STATE if some
 * (A, chi) block is rank-deficient.  Synchronises. */
mrhs_status mrhs_mg_block_orthonormalise(mrhs_mg mg, int32_t level);

/* mrhs_restrict ("project", Sec. 5): coarse = P^dag fine for nrhs fields,
 *   coarse(A, chi n_v + i, k) = sum_{x in A} sum_{c in chi} conj(v_i(x)_c) fine(x, c, k),
 * fine on level `level`, coarse on level + 1.  prec MRHS_F32 or MRHS_F64:
 * both fields and the sums in that precision (vector ALU).  prec MRHS_BF16:
 * FP32 fields, the basis and the input rounded to BF16 (nearest even) and
 * multiplied on the matrix cores with FP32 accumulation; needs n_v = 16 and
 * aggregates of a multiple of 16 sites, at most 4096, else
 * MRHS_ERR_UNSUPPORTED. */
mrhs_status mrhs_restrict(mrhs_mg mg, int32_t level, void* coarse, const void* fine, int32_t nrhs, mrhs_prec prec);
/* mrhs_prolong ("promote", Sec. 5): fine = P coarse,
 *   fine(x, c, k) = sum_i v_i(x)_c coarse(A(x), chi(c) n_v + i, k);
 * precisions as for mrhs_restrict. */
mrhs_status mrhs_prolong(mrhs_mg mg, int32_t level, void* fine, const void* coarse, int32_t nrhs, mrhs_prec prec);
/* mrhs_block_normalise: for every RHS k, aggregate A of step `level` and
 * chirality chi, divides the (A, chi) block of field k by its 2-norm (a zero
 * block stays zero).  norms: optional device array [A][chi][k] of FP64 norms
 * (may be NULL).  Norms are summed in FP64. */
mrhs_status mrhs_block_normalise(mrhs_mg mg, int32_t level, void* fields, int32_t nrhs, mrhs_prec prec,
                                 double* norms);

/* mrhs_coarse_set_blocks: stencil blocks of coarse level `level` (>= 1) as
 * [site][d][i][j] complex, d in (self, +x, -x, +y, -y, +z, -z, +t, -t),
 * i, j < ncomp(level), prec MRHS_F64 or MRHS_F32, host or device; the
 * operator is (D_c e)(A) = sum_d B_d(A) e(A + d), periodic, no boundary
 * phase.  Synchronises. */
mrhs_status mrhs_coarse_set_blocks(mrhs_mg mg, int32_t level, const void* blocks, mrhs_prec prec, int32_t on_device);
/* Copies the FP64 blocks out (prec must be MRHS_F64).  Synchronises. */
mrhs_status mrhs_coarse_get_blocks(mrhs_mg mg, int32_t level, void* blocks, mrhs_prec prec, int32_t on_device);
/* mrhs_mg_build_coarse: Galerkin blocks of level `level` from level - 1,
 * B_d(A) = sum_{x in A} W(x)^dag (D_d W)(x), with W the chirality-split basis
 * of step level - 1 and D_d the piece of the level - 1 operator that couples
 * A to A + d: for d = self the clover/self term and the hops that stay inside
 * A, for d = +-mu the hops that leave A through its +-mu face (so with a
 * coarse extent of 2 the +mu and -mu blocks stay distinct).  The fine
 * operator is the context's D = A - kappa H.  FP64 throughout.  Synchronises. */
mrhs_status mrhs_mg_build_coarse(mrhs_mg mg, int32_t level);
/* mrhs_coarse_apply (Sec. 6): out = D_c in on coarse level `level`.
 * prec MRHS_F64: FP64 fields and arithmetic; MRHS_F32: FP32 fields and
 * arithmetic (on the FP32 matrix cores for Nb = 32, else the vector ALU); MRHS_BF16 / MRHS_F16: FP32 fields, blocks and vectors rounded
 * to BF16 / FP16 (nearest even; blocks via FP32) and multiplied on the
 * matrix cores with FP32 accumulation (Nb = 32 only; FP16 vectors are scaled
 * per RHS by a power of two first, exactly undone on output). */
mrhs_status mrhs_coarse_apply(mrhs_mg mg, int32_t level, void* out, const void* in, int32_t nrhs, mrhs_prec prec);

/* mrhs_mg_tune: for every coarse level with Nb = 32 and blocks set, and each
 * nrhs in nrhs_list (count entries), times on the device (a) the two FP32
 * stencil kernels (FP32 matrix cores, vector ALU) and keeps the faster one for
 * mrhs_coarse_apply with MRHS_F32 and for V-cycles with FP32 coarse levels
 * (untuned: the matrix cores), and (b) the launch shapes of the BF16/FP16
 * matrix-core stencil (four or eight wavefronts per site, one or two
 * 32-column tiles of right-hand sides per workgroup, the two as separate or
 * interleaved columns; untuned: four and one), used for BF16 and FP16 applies
 * and V-cycles, and (c) on levels of at most 1024 sites the shapes without
 * interleaving for the fused BF16 minimal-residual step of the coarsest-level
 * solve.  Synchronises; drops the solver's captured V-cycles
 * and work buffers, which the next solve rebuilds. */
mrhs_status mrhs_mg_tune(mrhs_mg mg, const int32_t* nrhs_list, int32_t count);
/* mrhs_mg_get_tuning: *f32_valu = 1 when level uses the vector-ALU FP32
 * stencil for nrhs (always for Nb != 32), 0 for the FP32 matrix cores;
 * *lowp_cfg (if not NULL) = the BF16/FP16 stencil's launch shape, bit 0 eight
 * wavefronts per site (else four), cfg >> 1 the column tiling: 0 one
 * 32-column tile per workgroup, 1 two, 2 two tiles of interleaved column
 * pairs read with 16-byte loads (even nrhs; run as 1 otherwise). */
mrhs_status mrhs_mg_get_tuning(mrhs_mg mg, int32_t level, int32_t nrhs, int32_t* f32_valu, int32_t* lowp_cfg);
/* mrhs_mg_set_lowp_cfg: sets the BF16/FP16 stencil's launch shape (and that
 * of the fused MR step, which has no column-pair form: 4 / 5 give it 2 / 3)
 * for level and nrhs by hand (0..5, as in mrhs_mg_get_tuning), e.g. to
 * restore a persisted tuning; every shape computes the same operator.
 * Captured V-cycles are recaptured. */
mrhs_status mrhs_mg_set_lowp_cfg(mrhs_mg mg, int32_t level, int32_t nrhs, int32_t cfg);

/* Even-odd pieces of the coarse stencil, Sec. 6 (the coarse-level M_eooe):
 * on a level whose extents are all even, with the checkerboard layout of the
 * fine even-odd calls (FP32 complex device fields [V/2][Nb][nrhs], entry i the
 * site of that parity among 2i, 2i + 1), and Nb = 32.  prec selects the
 * arithmetic: MRHS_F32 (FP32 matrix cores), MRHS_BF16 or
 * MRHS_F16 (matrix cores, FP32 accumulation, FP16 with a per-RHS power-of-two
 * scale as in mrhs_coarse_apply).  MRHS_ERR_SHAPE for odd extents,
 * MRHS_ERR_STATE before the level's blocks exist. */
/* mrhs_coarse_hop_eo_apply: out (parity out_parity) = the eight hop directions
 * of D_c applied to in (parity 1 - out_parity); the self blocks do not enter. */
mrhs_status mrhs_coarse_hop_eo_apply(mrhs_mg mg, int32_t level, void* out, const void* in, int32_t nrhs,
                                     int32_t out_parity, mrhs_prec prec);
/* mrhs_coarse_self_eo_apply: out = S_p in (inverse = 0) or S_p^-1 in
 * (inverse = 1) on parity p, S the self blocks B_self.  The inverses are
 * computed once per set of blocks in FP64 (Gauss-Jordan with partial
 * pivoting, one workgroup per site) and rounded to the operand precision;
 * the first inverse call synchronises, MRHS_ERR_STATE for a singular block. */
mrhs_status mrhs_coarse_self_eo_apply(mrhs_mg mg, int32_t level, void* out, const void* in, int32_t nrhs,
                                      int32_t parity, int32_t inverse, mrhs_prec prec);

/* ---- multigrid-preconditioned solve (paper Sec. 8) -----------------------
 * The paper solves with FGMRES preconditioned by multigrid, on many RHS at
 * once; it does not describe its smoother, cycle or setup, so the ones below
 * are this library's.  All of them act on Nrhs columns at once with one
 * independent Krylov space / scalar set per column.
 *
 * V-cycle (the preconditioner, FP32 fields): on each level above the
 * coarsest, nu_pre minimal-residual (MR) steps x += a r, r -= a D r with
 * a = <D r, r> / ||D r||^2 per column, the coarse-grid correction
 * x += P V(R r), the residual r = b - D x and nu_post MR steps; on the
 * coarsest level coarsest_iters MR steps from x = 0.  The fine operator runs
 * in FP32; coarse levels in coarse_prec (MRHS_F32 vector ALU or FP32 matrix
 * cores, MRHS_BF16 or MRHS_F16 matrix cores with FP32 accumulation,
 * Nb = 32).  With MRHS_BF16 the restriction and prolongation of a step with
 * n_v = 16 run on the BF16 matrix cores too, otherwise in FP32.
 * With fine_eo = 1 (every extent even) a fine-level smoothing pass of nu
 * steps computes its correction e ~ D^-1 r from the Schur complement
 * Dhat = A_e - kappa^2 H_eo A_o^-1 H_oe (see mrhs_schur_apply): nu MR steps
 * on Dhat e_e = r_e + kappa H_eo A_o^-1 r_o from e_e = 0, then
 * e_o = A_o^-1 (r_o + kappa H_oe e_e) and x += e (then r = b - D x when the
 * residual is still needed, i.e. after the pre-smoothing pass).
 * With coarse_eo the same elimination on a coarse level, D_c = [[S_e, H_eo],
 * [H_oe, S_o]] with S the self blocks and H the eight hop directions: nu MR
 * steps on (S_e - H_eo S_o^-1 H_oe) e_e = r_e - H_eo S_o^-1 r_o from e_e = 0,
 * then e_o = S_o^-1 (r_o - H_oe e_e), x += e.
 * With fine_sap (Sec. 9 outlook, Schwarz smoothing) the fine lattice is cut
 * into the level-0 aggregates as blocks, coloured (X + Y + Z + T) mod 2 (the
 * block counts L / b must all be even); one SAP cycle is, for colour c = 0
 * then 1: r = b - D x, on every block B of colour c sap_iters MR steps on
 * D_B e_B = r|_B from zero (D_B: D on B with the hops across the block
 * boundary dropped; step length from the block's own inner products), and
 * x += e_B. */
typedef struct {
  int32_t nu_pre;
  int32_t nu_post;
  int32_t coarsest_iters;
  mrhs_prec coarse_prec;
  int32_t fine_eo; /* 1: the fine-level smoothing steps run on the even-odd
                      Schur complement (see below); 0: on D */
  int32_t coarse_eo; /* 1: on every coarse level above the coarsest whose
                        extents are all even (Nb = 32, BF16 coarse_prec) the
                        smoothing steps run on the coarse Schur complement
                        S_e - H_eo S_o^-1 H_oe (Sec. 6, the coarse M_eooe;
                        see below); 0: on D_c */
  int32_t fine_sap;  /* 1: the fine level smooths with the Schwarz alternating
                        procedure instead (not together with fine_eo; see
                        below): nu_pre / nu_post count SAP cycles */
  int32_t sap_iters; /* MR steps per block solve of a SAP cycle, 1..64 */
} mrhs_vcycle_params;

typedef struct {
  double tol;           /* stop when ||b_k - D x_k|| / ||b_k|| <= tol for every k (FP64 true residual) */
  int32_t restart;      /* FGMRES cycle length m, 1 <= m <= 15 */
  int32_t max_iters;    /* total preconditioned steps */
  int32_t precondition; /* 1: V-cycle; 0: none (plain restarted GMRES with FP32-rounded directions) */
  int32_t use_graph;    /* 1: replay the V-cycle from a captured HIP graph */
  int32_t timers;       /* 1: per-phase device timers (no graph; slower) */
  mrhs_vcycle_params vc;
  double reorth_eta;    /* second Gram-Schmidt pass when the first left less than reorth_eta times
                           ||w||^2 for some RHS: 0.5 is the classical "twice is enough" test, 0 never;
                           one FP64 pass loses about eps / sqrt(reorth_eta) of orthogonality, so 1e-2
                           (the Python default) costs nothing in convergence at FP64 */
  int32_t krylov_prec;  /* storage of the Krylov basis: MRHS_F64 (0), or MRHS_F32: basis vectors in
                           FP32 (inner products and updates computed in FP64) and the FP32 operator
                           in the Arnoldi step, each cycle an FP32 Krylov solve of the FP64 residual;
                           the restarts (FP64 true residual, FP64 x) reach the same FP64 tolerance,
                           with half the outer solver's memory traffic and basis footprint */
} mrhs_solve_params;

typedef struct {
  int32_t nrhs;
  int32_t iters;                    /* preconditioned steps (shared by all columns) */
  int32_t cycles;                   /* restart cycles */
  int32_t reorth;                   /* Gram-Schmidt steps that needed a second pass */
  int32_t converged[MRHS_MAX_NRHS]; /* 1 if column k met tol */
  double rel_resid[MRHS_MAX_NRHS];  /* final true ||b_k - D x_k|| / ||b_k||, FP64 */
  double seconds_total;             /* host wall clock of the call */
  double seconds_precond;           /* V-cycles (with timers) */
  double seconds_phase[4];          /* with timers: fine level, restrict, prolong, coarse levels (device) */
} mrhs_solve_stats;

/* mrhs_mg_precondition: z = V-cycle(v) for nrhs FP32 fine fields (device,
 * [V][12][nrhs]).  Needs the bases and coarse operators of every level.
 * Synchronises. */
mrhs_status mrhs_mg_precondition(mrhs_mg mg, void* z, const void* v, int32_t nrhs, const mrhs_vcycle_params* vc);
/* mrhs_coarse_mr_solve: x ~ D_c^-1 b on coarse level `level` (>= 1) by
 * `iters` minimal-residual steps from x = 0, alpha_k = <D r_k, r_k> /
 * ||D r_k||^2 per right-hand side: the coarsest-level solve of the V-cycle
 * (Sec. 6).  x, b: FP32 device fields [V_level][Nb][nrhs] (x is
 * overwritten; b is read only).  prec: the stencil's arithmetic, MRHS_F32,
 * MRHS_BF16 or MRHS_F16; with BF16 on a level of Nb = 32 and at most 1024
 * sites every step is two launches (stencil fused with the previous step's
 * update and the per-site inner products; the step length).  Synchronises. */
mrhs_status mrhs_coarse_mr_solve(mrhs_mg mg, int32_t level, void* x, const void* b, int32_t nrhs, int32_t iters,
                                 mrhs_prec prec);
typedef struct {
  int32_t setup_iters;    /* smoothing sweeps per level, 0..100 */
  int32_t smooth_steps;   /* MR steps per sweep, 0..1000 */
  int32_t adapt_iters;    /* adaptive passes (below), 0..50 */
  mrhs_vcycle_params vc;  /* cycle the adaptive passes use */
} mrhs_setup_params;

/* mrhs_mg_setup: near-null-space setup of the hierarchy (not specified by
 * the paper).  From the starting vectors already set with mrhs_mg_set_basis
 * on every step (e.g. Gaussian), level by level: setup_iters sweeps of
 * smooth_steps MR steps on D x = 0 starting from the vectors (which damps
 * their high modes), column normalisation, block orthonormalisation (FP64)
 * and the Galerkin operator of the next level.  Then adapt_iters passes of
 * inverse iteration with the hierarchy itself: on every level l, each
 * vector becomes K v with K the V-cycle from level l down (an approximate
 * inverse of D, so the low modes grow); the vectors are renormalised and
 * re-orthonormalised and the next level rebuilt.
 * Synchronises. */
mrhs_status mrhs_mg_setup(mrhs_mg mg, const mrhs_setup_params* params);
/* mrhs_mg_solve: solves D x_k = b_k for the context's fine operator
 * D = A - kappa H (for the mass form D_m = D / (2 kappa) pass 2 kappa b), by
 * FGMRES(m) in FP64 with the V-cycle as preconditioner (the Krylov basis in
 * FP64 or, with params->krylov_prec = MRHS_F32, in FP32 between FP64
 * restarts).  x: device FP64 [V][12][nrhs], in: initial guess, out: solution;
 * b: device FP64, not overlapping x.  Returns MRHS_ERR_NOT_CONVERGED (stats
 * filled, x holds the last iterate) if max_iters is reached first; an
 * unsupported krylov_prec gets MRHS_ERR_UNSUPPORTED.  Synchronises. */
mrhs_status mrhs_mg_solve(mrhs_mg mg, void* x, const void* b, int32_t nrhs, const mrhs_solve_params* params,
                          mrhs_solve_stats* stats);

/* ---- autotuning ----------------------------------------------------------
 * mrhs_tune: for each nrhs in nrhs_list (count entries), times the FP32 fine
 * operator (mrhs_dwc_apply and the smoother) in every supported launch
 * configuration -- right-hand sides per thread 1, 2 or 4, a set of site
 * traversal tiles that divide the lattice (including slabs of Lt / 8 time
 * slices, one per XCD, and columns of the full time extent), two tile orders
 * (lexicographic, Morton), or the t-walk kernel (each thread walks a run of
 * time slices of one site of a spatial block, carrying its t-neighbours in
 * registers) with its block and run length, the right-hand sides split into 1, 2 or 4 chunks
 * swept one after the other, at most 1, 2 or 3 workgroups per CU or no limit,
 * two register budgets (the compiler's, and one that admits 4 wavefronts per
 * SIMD) and ordinary or non-temporal output stores -- on
 * scratch fields, and keeps the
 * fastest for later FP32 applies of that nrhs on this context.  All
 * configurations give bit-identical results.  On lattices with even extents
 * it also chooses the checkerboard hop's kernel (tiled or t-walk, see
 * mrhs_set_eo_walk) per nrhs, by timing, every call, and, when the FP64
 * links and clover are present, the FP64 operator's kernel (tiled or t-walk,
 * see mrhs_set_f64_walk), also timed every call.  cache_path (may be NULL) names
 * a text file: existing entries for this device architecture, lattice and
 * nrhs are used without timing, new choices are appended.  Needs links and
 * clover.  Synchronises. */
mrhs_status mrhs_tune(mrhs_ctx ctx, const int32_t* nrhs_list, int32_t count, const char* cache_path);
/* mrhs_get_tuning: the configuration in use for nrhs: right-hand sides per
 * thread (0 = untuned default), tile[4] (0 = default tile; for the t-walk
 * kernel its spatial block and time slices per thread), variant = tile
 * order (0 lexicographic, 1 Morton) + 2 if compiled for at least 4
 * wavefronts per SIMD + 4 if the output is written with non-temporal
 * stores + 8 log2(RHS chunks) + 32 (workgroups-per-CU limit, 0 = none)
 * + 128 for the t-walk kernel, measured microseconds (0 if untuned).  Any
 * output pointer may be NULL. */
mrhs_status mrhs_get_tuning(mrhs_ctx ctx, int32_t nrhs, int32_t* rhs_per_thread, int32_t tile[4], int32_t* curve,
                            float* us);
/* mrhs_set_f64_walk: kernel of the FP64 operator A - kappa H (mrhs_dwc_apply
 * with MRHS_F64 and the outer solver's residuals) for nrhs right-hand sides:
 * tile = (Bx, By, Bz, Ts) selects the t-walk kernel, one right-hand side per
 * thread (each thread walks Ts consecutive time slices of one site of a
 * Bx x By x Bz spatial block, carrying its t-neighbours in registers; the
 * block must divide the spatial extents and Ts the time extent); variant
 * bit 0: non-temporal output stores, bit 1: the register budget of two
 * workgroups per CU (else the compiler's); tile = NULL selects the tiled
 * kernel.  The fields computed are bit-identical either way.  A shape that
 * does not divide the lattice gets MRHS_ERR_INVALID_ARG. */
mrhs_status mrhs_set_f64_walk(mrhs_ctx ctx, int32_t nrhs, const int32_t* tile, int32_t variant);
/* mrhs_get_f64_walk: the FP64 operator's kernel for nrhs (*on = 0: tiled),
 * its tile and variant bits, and the times the last mrhs_tune measured for
 * it and for the tiled kernel (microseconds, 0 if not measured).  Any output
 * pointer may be NULL. */
mrhs_status mrhs_get_f64_walk(mrhs_ctx ctx, int32_t nrhs, int32_t* on, int32_t tile[4], int32_t* variant,
                              float* us, float* us_tiled);

#ifdef __cplusplus
}
#endif

#endif /* MRHS_H */
