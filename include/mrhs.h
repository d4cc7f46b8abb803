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
 * (MRHS_F32 or MRHS_F64); they must not overlap.  MRHS_ERR_STATE before
 * links and clover are set. */
mrhs_status mrhs_dwc_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec);
/* mrhs_hop_apply: out = H in (hopping term only, Sec. 4 D_hop). */
mrhs_status mrhs_hop_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs, mrhs_prec prec);
/* mrhs_clover_apply: out = A in (clover term only, Sec. 4 M_ooee on the
 * full lattice). */
mrhs_status mrhs_clover_apply(mrhs_ctx ctx, void* out, const void* in, int32_t nrhs,
                              mrhs_prec prec);

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
/* mrhs_axpy: y_k <- y_k + alpha_k x_k per column, alpha_k = alpha[2k] + i alpha[2k+1]
 * (FP64, host memory if alpha_on_device = 0, else device memory); the update
 * is computed in FP64 and rounded to prec.  x and y must not overlap. */
mrhs_status mrhs_axpy(mrhs_ctx ctx, void* y, const double* alpha, const void* x, int64_t nsites, int32_t ncomp,
                      int32_t nrhs, mrhs_prec prec, int32_t alpha_on_device);

#ifdef __cplusplus
}
#endif

#endif /* MRHS_H */
