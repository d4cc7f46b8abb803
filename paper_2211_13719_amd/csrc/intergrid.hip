// Aggregation-multigrid intergrid operators on Nrhs fields at once (paper
// Sec. 5: "project" = restriction, "promote" = prolongation; the coarse
// spinor has nbasis = 2 n_v components because every basis vector is split by
// chirality).
//
// A level has sites s (geometry Geom) and ncomp = 2h components per site, the
// first h of chirality +, the last h of chirality -.  Aggregates are blocks
// b = (bx, by, bz, bt) of sites; aggregate A = X + Cx (Y + Cy (Z + Cz T)).
// The basis of a level is held in the internal layout [site][ncomp][n_v]
// (basis index fastest), so the n_v values a thread needs at one (site,
// component) are contiguous.  With v_i(x)_c that basis,
//
//   restrict: y(A, chi n_v + i, k) = sum_{x in A} sum_{c in chi} conj(v_i(x)_c) f(x)_{c,k}
//   prolong:  f(x)_{c,k}           = sum_i v_i(x)_c y(A(x), chi(c) n_v + i, k)
//
// and block orthonormalisation makes, for every (aggregate, chirality), the
// n_v restricted vectors orthonormal: the Q factor of their thin QR with real
// positive diagonal, by classical Gram-Schmidt applied twice, in FP64.
#include "agg.h"
#include "internal.h"

namespace mrhs {
namespace {

template <typename T>
struct cx;
template <>
struct cx<float> {
  using type = float2;
};
template <>
struct cx<double> {
  using type = double2;
};
template <typename T>
using cplx = typename cx<T>::type;

template <typename T>
__device__ __forceinline__ cplx<T> mk(T a, T b) {
  cplx<T> z;
  z.x = a;
  z.y = b;
  return z;
}

// ---- restriction ----------------------------------------------------------------
// One workgroup per aggregate.  A thread owns a 4 (basis index) x 4 (RHS)
// output tile of one chirality and a slice of the aggregate's sites; the
// slices are summed through LDS at the end in a fixed order.
constexpr int kRI = 4, kRR = 4;

template <typename T, int NV>
__global__ __launch_bounds__(256) void restrict_kernel(AggGeom a, int h, int nrhs,
                                                       const cplx<T>* __restrict__ basis,
                                                       const cplx<T>* __restrict__ f, cplx<T>* __restrict__ y) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* red = reinterpret_cast<cplx<T>*>(smem_raw);
  const int A = blockIdx.x;
  const int ncomp = 2 * h;
  const int G = (nrhs + kRR - 1) / kRR;
  const int ntile = 2 * (NV / kRI) * G;
  const int S = max(1, 256 / ntile);
  const int t = threadIdx.x;
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];

  cplx<T> acc[kRI][kRR];
#pragma unroll
  for (int i = 0; i < kRI; ++i)
#pragma unroll
    for (int k = 0; k < kRR; ++k) acc[i][k] = mk<T>(0, 0);

  const int tile = t % ntile;
  const int slice = t / ntile;
  const int kg = tile % G;
  const int ig = (tile / G) % (NV / kRI);
  const int chi = tile / (G * (NV / kRI));
  const int k0 = kg * kRR, i0 = ig * kRI;
  if (slice < S) {
    for (int l = slice; l < nsa; l += S) {
      const int s = agg_site(a, A, l);
      const cplx<T>* fb = f + ((size_t)s * ncomp + chi * h) * nrhs + k0;
      const cplx<T>* bb = basis + ((size_t)s * ncomp + chi * h) * NV + i0;
      for (int c = 0; c < h; ++c) {
        cplx<T> fv[kRR], bv[kRI];
#pragma unroll
        for (int k = 0; k < kRR; ++k) fv[k] = (k0 + k < nrhs) ? fb[(size_t)c * nrhs + k] : mk<T>(0, 0);
#pragma unroll
        for (int i = 0; i < kRI; ++i) bv[i] = bb[(size_t)c * NV + i];
#pragma unroll
        for (int i = 0; i < kRI; ++i)
#pragma unroll
          for (int k = 0; k < kRR; ++k) {
            // conj(b) * f
            acc[i][k].x = fma(bv[i].x, fv[k].x, acc[i][k].x);
            acc[i][k].x = fma(bv[i].y, fv[k].y, acc[i][k].x);
            acc[i][k].y = fma(bv[i].x, fv[k].y, acc[i][k].y);
            acc[i][k].y = fma(-bv[i].y, fv[k].x, acc[i][k].y);
          }
      }
    }
    // red[slice][tile][16]
#pragma unroll
    for (int i = 0; i < kRI; ++i)
#pragma unroll
      for (int k = 0; k < kRR; ++k) red[((size_t)slice * ntile + tile) * (kRI * kRR) + i * kRR + k] = acc[i][k];
  }
  __syncthreads();
  const int nout = ntile * kRI * kRR;
  for (int o = t; o < nout; o += 256) {
    cplx<T> sum = red[o];
    for (int q = 1; q < S; ++q) {
      const cplx<T> v = red[(size_t)q * nout + o];
      sum.x += v.x;
      sum.y += v.y;
    }
    const int tl = o / (kRI * kRR);
    const int ii = (o / kRR) % kRI;
    const int kk = o % kRR;
    const int kgo = tl % G, igo = (tl / G) % (NV / kRI), cho = tl / (G * (NV / kRI));
    const int k = kgo * kRR + kk;
    if (k < nrhs) y[((size_t)A * 2 * NV + cho * NV + igo * kRI + ii) * nrhs + k] = sum;
  }
}

// ---- prolongation -------------------------------------------------------------------
// One thread per (fine site, chirality, group of R right-hand sides).
template <typename T, int NV, int H, int R>
__global__ __launch_bounds__(256) void prolong_kernel(AggGeom a, int nrhs, const cplx<T>* __restrict__ basis,
                                                      const cplx<T>* __restrict__ y, cplx<T>* __restrict__ f) {
  const int G = (nrhs + R - 1) / R;
  const long gid = (long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (long)a.V * 2 * G) return;
  const int kg = (int)(gid % G);
  const int chi = (int)((gid / G) % 2);
  const int s = (int)(gid / (2 * G));
  const int k0 = kg * R;
  const int A = site_agg(a, s);
  constexpr int ncomp = 2 * H;
  cplx<T> acc[H][R];
#pragma unroll
  for (int c = 0; c < H; ++c)
#pragma unroll
    for (int k = 0; k < R; ++k) acc[c][k] = mk<T>(0, 0);
  const cplx<T>* yb = y + ((size_t)A * 2 * NV + chi * NV) * nrhs + k0;
  const cplx<T>* bb = basis + ((size_t)s * ncomp + chi * H) * NV;
#pragma unroll 4
  for (int i = 0; i < NV; ++i) {
    cplx<T> yv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) yv[k] = (k0 + k < nrhs) ? yb[(size_t)i * nrhs + k] : mk<T>(0, 0);
#pragma unroll
    for (int c = 0; c < H; ++c) {
      const cplx<T> b = bb[(size_t)c * NV + i];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        acc[c][k].x = fma(b.x, yv[k].x, acc[c][k].x);
        acc[c][k].x = fma(-b.y, yv[k].y, acc[c][k].x);
        acc[c][k].y = fma(b.x, yv[k].y, acc[c][k].y);
        acc[c][k].y = fma(b.y, yv[k].x, acc[c][k].y);
      }
    }
  }
  cplx<T>* fb = f + ((size_t)s * ncomp + chi * H) * nrhs + k0;
#pragma unroll
  for (int c = 0; c < H; ++c)
#pragma unroll
    for (int k = 0; k < R; ++k)
      if (k0 + k < nrhs) fb[(size_t)c * nrhs + k] = acc[c][k];
}

// Few right-hand sides (nrhs <= 2): one thread per fine row (site, component),
// so that a wavefront reads 64 consecutive basis rows (n_v contiguous values
// each) instead of 64 rows' worth of scattered single values; the coarse
// values of the aggregate are shared through the cache.  Same arithmetic and
// order per output as prolong_kernel.
template <typename T, int NV, int NR>
__global__ __launch_bounds__(256) void prolong_row_kernel(AggGeom a, int h, const cplx<T>* __restrict__ basis,
                                                          const cplx<T>* __restrict__ y, cplx<T>* __restrict__ f) {
  const int ncomp = 2 * h;
  const long row = (long)blockIdx.x * 256 + threadIdx.x;
  if (row >= (long)a.V * ncomp) return;
  const int s = (int)(row / ncomp);
  const int c = (int)(row - (long)s * ncomp);
  const int chi = c / h;
  const int A = site_agg(a, s);
  const cplx<T>* bb = basis + row * NV;
  const cplx<T>* yb = y + ((size_t)A * 2 * NV + chi * NV) * NR;
  cplx<T> acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const cplx<T> b = bb[i];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const cplx<T> yv = yb[(size_t)i * NR + k];
      acc[k].x = fma(b.x, yv.x, acc[k].x);
      acc[k].x = fma(-b.y, yv.y, acc[k].x);
      acc[k].y = fma(b.x, yv.y, acc[k].y);
      acc[k].y = fma(b.y, yv.x, acc[k].y);
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) f[row * NR + k] = acc[k];
}

// ---- block orthonormalisation (FP64) --------------------------------------------------
// A (aggregate, chirality) block is rank-deficient when the part of v_i left
// after projecting out v_0..v_{i-1} is below kRankTol times |v_i|.
constexpr double kRankTol = 1e-10;

__device__ double2 block_sum(double2 v, double2* lds) {
  // wavefront reduction, then across the 4 wavefronts of the workgroup
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double2 s = lds[0];
  for (int q = 1; q < 4; ++q) {
    s.x += lds[q].x;
    s.y += lds[q].y;
  }
  return s;
}

// One workgroup of 256 threads per (aggregate, chirality).  Vector i of the
// block is v_i(x)_c for x in A, c in chi; the kernel overwrites the basis in
// place with the orthonormal Q and reports a rank deficiency through *flag.
__global__ __launch_bounds__(256) void block_gs_kernel(AggGeom a, int h, int nv, double2* __restrict__ basis,
                                                       int* __restrict__ flag) {
  __shared__ double2 lds[4];
  __shared__ double2 r[64];
  const int A = blockIdx.x >> 1;
  const int chi = blockIdx.x & 1;
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  const int dim = nsa * h;
  const int ncomp = 2 * h;
  auto elem = [&](int e, int i) -> double2* {
    const int s = agg_site(a, A, e / h);
    const int c = chi * h + e % h;
    return basis + ((size_t)s * ncomp + c) * nv + i;
  };
  for (int i = 0; i < nv; ++i) {
    double2 p0 = make_double2(0.0, 0.0);
    for (int e = threadIdx.x; e < dim; e += 256) {
      const double2 v = *elem(e, i);
      p0.x = fma(v.x, v.x, p0.x);
      p0.x = fma(v.y, v.y, p0.x);
    }
    const double nrm0 = sqrt(block_sum(p0, lds).x);
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < i; ++j) {
        double2 p = make_double2(0.0, 0.0);
        for (int e = threadIdx.x; e < dim; e += 256) {
          const double2 q = *elem(e, j), v = *elem(e, i);
          p.x = fma(q.x, v.x, p.x);
          p.x = fma(q.y, v.y, p.x);
          p.y = fma(q.x, v.y, p.y);
          p.y = fma(-q.y, v.x, p.y);
        }
        const double2 s = block_sum(p, lds);
        if (threadIdx.x == 0) r[j] = s;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < dim; e += 256) {
        double2 v = *elem(e, i);
        for (int j = 0; j < i; ++j) {
          const double2 q = *elem(e, j);
          const double2 c = r[j];
          v.x -= c.x * q.x - c.y * q.y;
          v.y -= c.x * q.y + c.y * q.x;
        }
        *elem(e, i) = v;
      }
      __syncthreads();
    }
    double2 p = make_double2(0.0, 0.0);
    for (int e = threadIdx.x; e < dim; e += 256) {
      const double2 v = *elem(e, i);
      p.x = fma(v.x, v.x, p.x);
      p.x = fma(v.y, v.y, p.x);
    }
    const double nrm = sqrt(block_sum(p, lds).x);
    // rank deficiency: what is left after the projections is rounding-sized
    if (!(nrm > kRankTol * nrm0)) {
      if (threadIdx.x == 0) *flag = 1;
      return;  // uniform across the workgroup
    }
    const double inv = 1.0 / nrm;
    for (int e = threadIdx.x; e < dim; e += 256) {
      double2* pv = elem(e, i);
      pv->x *= inv;
      pv->y *= inv;
    }
    __syncthreads();
  }
}

// ---- block normalisation -----------------------------------------------------------------
// One workgroup per aggregate; thread t accumulates |f|^2 for one (chirality,
// RHS) pair over a slice of sites, the slices are summed in LDS in a fixed
// order, and the same workgroup then scales the block.
template <typename T, int W>
__global__ __launch_bounds__(256) void block_norm_kernel(AggGeom a, int h, int nrhs, cplx<T>* __restrict__ f,
                                                         double* __restrict__ norms) {
  // Thread (slice, chi, g) owns right-hand sides g W .. g W + W - 1 of one
  // chirality on the sites l = slice, slice + S, ... of the aggregate: it
  // sums their squares (FP64), the slices are combined in a fixed order,
  // and then the same thread rescales the same elements.
  __shared__ double part[256 * W];
  __shared__ double inv[2 * 64];
  const int A = blockIdx.x;
  const int ncomp = 2 * h;
  const int G = nrhs / W;
  const int np = 2 * G;
  const int S = 256 / np;
  const int t = threadIdx.x;
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  const int pair = t % np, slice = t / np;
  const int chi = pair / G, k0 = (pair % G) * W;
  double acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0.0;
  if (slice < S) {
    for (int l = slice; l < nsa; l += S) {
      const cplx<T>* fb = f + ((size_t)agg_site(a, A, l) * ncomp + chi * h) * nrhs + k0;
      for (int c = 0; c < h; ++c) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const cplx<T> v = fb[(size_t)c * nrhs + w];
          acc[w] = fma((double)v.x, (double)v.x, acc[w]);
          acc[w] = fma((double)v.y, (double)v.y, acc[w]);
        }
      }
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) part[t * W + w] = acc[w];
  __syncthreads();
  if (t < np) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      double s2 = 0.0;
      for (int q = 0; q < S; ++q) s2 += part[(q * np + t) * W + w];
      const double n = sqrt(s2);
      inv[chi * nrhs + k0 + w] = n > 0.0 ? 1.0 / n : 0.0;
      if (norms) norms[((size_t)A * 2 + chi) * nrhs + k0 + w] = n;
    }
  }
  __syncthreads();
  if (slice < S) {
    T sc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) sc[w] = (T)inv[chi * nrhs + k0 + w];
    for (int l = slice; l < nsa; l += S) {
      cplx<T>* fb = f + ((size_t)agg_site(a, A, l) * ncomp + chi * h) * nrhs + k0;
      for (int c = 0; c < h; ++c) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          cplx<T> v = fb[(size_t)c * nrhs + w];
          v.x *= sc[w];
          v.y *= sc[w];
          fb[(size_t)c * nrhs + w] = v;
        }
      }
    }
  }
}

// Single-pass variant for FP32 fields with an even number of RHS: workgroups
// of 1024 threads keep a whole (aggregate, chirality) block, or a range of its
// RHS columns, in registers, so the field is read once and written once (the
// kernel above reads it twice).  The norms are per column, so the C = nrhs /
// parts columns of each part are independent; the parts of one block get
// workgroup indices 8 apart (workgroups go round-robin over the eight XCDs),
// which keeps them on one XCD, where they share the L2 lines that their column
// ranges have in common.  Thread (slice, g) holds columns 2g, 2g + 1 of its
// part for the rows r = slice, slice + S, ... (r = l h + c: site offset l,
// component c), at most MAXR of them; with MAXR = 10 and WPE = 8 a workgroup
// fits in 64 VGPRs per lane and two share a CU, so one's loads overlap the
// other's reduction and stores.  The squares are summed in FP64 per thread,
// then over the slices in a fixed order (eight interleaved partial sums, then
// those eight), so the result does not depend on timing.
template <int MAXR, int WPE>
__global__ __launch_bounds__(1024, WPE) void block_norm_reg_kernel(AggGeom a, int h, int nrhs, int parts, int nac,
                                                                   float2* __restrict__ f,
                                                                   double* __restrict__ norms) {
  __shared__ double part[1024 * 2];
  __shared__ double red[8 * 64];
  __shared__ double inv[64];
  const int q8 = blockIdx.x >> 3;
  const int ac = (q8 / parts) * 8 + (blockIdx.x & 7);
  if (ac >= nac) return;  // whole workgroup
  const int pc = q8 % parts;
  const int A = ac >> 1, chi = ac & 1;
  const int ncomp = 2 * h;
  const int C = nrhs / parts;
  const int G = C / 2;
  const int S = 1024 / G;
  const int t = threadIdx.x;
  const int g = t % G, slice = t / G;
  const int k0 = pc * C + 2 * g;
  const int nrow = a.b[0] * a.b[1] * a.b[2] * a.b[3] * h;
  auto offset = [&](int r) {
    const int l = r / h, c = r - (r / h) * h;
    return ((size_t)agg_site(a, A, l) * ncomp + chi * h + c) * nrhs + k0;
  };
  float4 v[MAXR];
  // all loads first: a row past the end reads row 0 (a valid address) and
  // counts zero; the value is used either way, so no load sits in a branch
#pragma unroll
  for (int q = 0; q < MAXR; ++q) {
    const int r = slice + q * S;
    v[q] = *reinterpret_cast<const float4*>(f + offset(slice < S && r < nrow ? r : 0));
  }
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
  for (int q = 0; q < MAXR; ++q) {
    const int r = slice + q * S;
    const double m = (slice < S && r < nrow) ? 1.0 : 0.0;
    acc0 = fma(m * (double)v[q].x, (double)v[q].x, acc0);
    acc0 = fma(m * (double)v[q].y, (double)v[q].y, acc0);
    acc1 = fma(m * (double)v[q].z, (double)v[q].z, acc1);
    acc1 = fma(m * (double)v[q].w, (double)v[q].w, acc1);
  }
  // column o = 2 g + w of slice q sits at part[2 q G + o]
  part[2 * t] = acc0;
  part[2 * t + 1] = acc1;
  __syncthreads();
  if (t < 16 * G) {
    const int o = t % (2 * G), j = t / (2 * G);
    double s2 = 0.0;
    for (int q = j; q < S; q += 8) s2 += part[2 * q * G + o];
    red[j * 2 * G + o] = s2;
  }
  __syncthreads();
  if (t < 2 * G) {
    double s2 = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s2 += red[j * 2 * G + t];
    const double n = sqrt(s2);
    inv[t] = n > 0.0 ? 1.0 / n : 0.0;
    if (norms) norms[((size_t)A * 2 + chi) * nrhs + pc * C + t] = n;
  }
  __syncthreads();
  const float sc0 = (float)inv[2 * g], sc1 = (float)inv[2 * g + 1];
#pragma unroll
  for (int q = 0; q < MAXR; ++q) {
    const int r = slice + q * S;
    if (slice < S && r < nrow)
      *reinterpret_cast<float4*>(f + offset(r)) = make_float4(v[q].x * sc0, v[q].y * sc0, v[q].z * sc1, v[q].w * sc1);
  }
}

constexpr int kNormRegRows = 20, kNormRegRowsSplit = 6;

// Number of column parts for the MAXR = 10 variant: the fewest that fit, each
// of at least 8 columns (64-byte row segments) unless the block fits whole.
int norm_reg_parts(long nrow, int nrhs) {
  if (nrhs % 2) return 0;
  for (int p = 1; p <= nrhs / 2; ++p) {
    if ((nrhs / 2) % p || (p > 1 && nrhs / p < 8)) continue;
    const int G = nrhs / 2 / p;
    if (nrow <= (long)kNormRegRowsSplit * (1024 / G)) return p;
  }
  return 0;
}

// ---- layout conversion between [site][n_v][ncomp] (interface) and [site][ncomp][n_v] --------
template <typename Tin, typename Tout>
__global__ void basis_transpose(const cplx<Tin>* __restrict__ in, cplx<Tout>* __restrict__ out, long nsite, int nv,
                                int ncomp, int to_internal) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long per = (long)nv * ncomp;
  if (e >= nsite * per) return;
  const long s = e / per;
  const int r = (int)(e % per);
  long src, dst;
  if (to_internal) {  // e enumerates the interface layout (i, c)
    const int i = r / ncomp, c = r % ncomp;
    src = e;
    dst = s * per + (long)c * nv + i;
  } else {  // e enumerates the interface layout of the output
    const int i = r / ncomp, c = r % ncomp;
    dst = e;
    src = s * per + (long)c * nv + i;
  }
  const cplx<Tin> v = in[src];
  out[dst] = mk<Tout>((Tout)v.x, (Tout)v.y);
}

template <typename T, int NV>
hipError_t restrict_nv(const AggGeom& a, int h, int nrhs, const void* basis, const void* f, void* y, hipStream_t s) {
  const int G = (nrhs + kRR - 1) / kRR;
  const int ntile = 2 * (NV / kRI) * G;
  if (ntile > 256) return hipErrorInvalidValue;
  const int S = std::max(1, 256 / ntile);
  const size_t shmem = (size_t)S * ntile * kRI * kRR * sizeof(cplx<T>);
  hipLaunchKernelGGL((restrict_kernel<T, NV>), dim3(a.Vc), dim3(256), shmem, s, a, h, nrhs,
                     static_cast<const cplx<T>*>(basis), static_cast<const cplx<T>*>(f), static_cast<cplx<T>*>(y));
  return hipGetLastError();
}

template <typename T, int NV, int H>
hipError_t prolong_nvh(const AggGeom& a, int nrhs, const void* basis, const void* y, void* f, hipStream_t s) {
  if (nrhs <= 2) {
    const long rows = (long)a.V * 2 * H;
    const int nb = (int)((rows + 255) / 256);
    if (nrhs == 1)
      hipLaunchKernelGGL((prolong_row_kernel<T, NV, 1>), dim3(nb), dim3(256), 0, s, a, H,
                         static_cast<const cplx<T>*>(basis), static_cast<const cplx<T>*>(y),
                         static_cast<cplx<T>*>(f));
    else
      hipLaunchKernelGGL((prolong_row_kernel<T, NV, 2>), dim3(nb), dim3(256), 0, s, a, H,
                         static_cast<const cplx<T>*>(basis), static_cast<const cplx<T>*>(y),
                         static_cast<cplx<T>*>(f));
    return hipGetLastError();
  }
  constexpr int R = (H > 8) ? 2 : 4;
  const long threads = (long)a.V * 2 * ((nrhs + R - 1) / R);
  const int nb = (int)((threads + 255) / 256);
  hipLaunchKernelGGL((prolong_kernel<T, NV, H, R>), dim3(nb), dim3(256), 0, s, a, nrhs,
                     static_cast<const cplx<T>*>(basis), static_cast<const cplx<T>*>(y), static_cast<cplx<T>*>(f));
  return hipGetLastError();
}

template <typename T, int NV>
hipError_t prolong_nv(const AggGeom& a, int h, int nrhs, const void* basis, const void* y, void* f, hipStream_t s) {
  switch (h) {
    case 4:
      return prolong_nvh<T, NV, 4>(a, nrhs, basis, y, f, s);
    case 6:
      return prolong_nvh<T, NV, 6>(a, nrhs, basis, y, f, s);
    case 8:
      return prolong_nvh<T, NV, 8>(a, nrhs, basis, y, f, s);
    case 16:
      return prolong_nvh<T, NV, 16>(a, nrhs, basis, y, f, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

bool intergrid_supported(int nv, int h) {
  return (nv == 4 || nv == 8 || nv == 16) && (h == 4 || h == 6 || h == 8 || h == 16);
}

hipError_t launch_restrict(int prec64, const AggGeom& a, int h, int nv, int nrhs, const void* basis, const void* f,
                           void* y, hipStream_t s) {
  if (prec64) {
    switch (nv) {
      case 4:
        return restrict_nv<double, 4>(a, h, nrhs, basis, f, y, s);
      case 8:
        return restrict_nv<double, 8>(a, h, nrhs, basis, f, y, s);
      case 16:
        return restrict_nv<double, 16>(a, h, nrhs, basis, f, y, s);
    }
  } else {
    // from 4 right-hand sides on, n_v = 16 goes to the FP32 matrix cores
    if (nv == 16 && nrhs >= 4 && intergrid_mfma_supported(a, h, nv))
      return launch_restrict_f32mfma(a, h, nrhs, basis, f, y, s);
    switch (nv) {
      case 4:
        return restrict_nv<float, 4>(a, h, nrhs, basis, f, y, s);
      case 8:
        return restrict_nv<float, 8>(a, h, nrhs, basis, f, y, s);
      case 16:
        return restrict_nv<float, 16>(a, h, nrhs, basis, f, y, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_prolong(int prec64, const AggGeom& a, int h, int nv, int nrhs, const void* basis, const void* y,
                          void* f, hipStream_t s) {
  if (prec64) {
    switch (nv) {
      case 4:
        return prolong_nv<double, 4>(a, h, nrhs, basis, y, f, s);
      case 8:
        return prolong_nv<double, 8>(a, h, nrhs, basis, y, f, s);
      case 16:
        return prolong_nv<double, 16>(a, h, nrhs, basis, y, f, s);
    }
  } else {
    if (nv == 16 && nrhs >= 4 && intergrid_mfma_supported(a, h, nv))
      return launch_prolong_f32mfma(a, h, nrhs, basis, y, f, s);
    switch (nv) {
      case 4:
        return prolong_nv<float, 4>(a, h, nrhs, basis, y, f, s);
      case 8:
        return prolong_nv<float, 8>(a, h, nrhs, basis, y, f, s);
      case 16:
        return prolong_nv<float, 16>(a, h, nrhs, basis, y, f, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_block_gs(const AggGeom& a, int h, int nv, void* basis64, int* flag_dev, hipStream_t s) {
  if (nv > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(block_gs_kernel, dim3(2 * a.Vc), dim3(256), 0, s, a, h, nv, static_cast<double2*>(basis64),
                     flag_dev);
  return hipGetLastError();
}

hipError_t launch_block_normalise(int prec64, const AggGeom& a, int h, int nrhs, void* f, double* norms,
                                  hipStream_t s) {
  if (2 * nrhs > 256) return hipErrorInvalidValue;
  const long nrow = (long)a.b[0] * a.b[1] * a.b[2] * a.b[3] * h;
  const int nac = 2 * a.Vc;
  if (prec64)
    hipLaunchKernelGGL((block_norm_kernel<double, 1>), dim3(a.Vc), dim3(256), 0, s, a, h, nrhs,
                       static_cast<double2*>(f), norms);
  else if (const int p = norm_reg_parts(nrow, nrhs); p > 0)
    hipLaunchKernelGGL((block_norm_reg_kernel<kNormRegRowsSplit, 8>), dim3((nac + 7) / 8 * 8 * p), dim3(1024), 0, s,
                       a, h, nrhs, p, nac, static_cast<float2*>(f), norms);
  else if (nrhs % 2 == 0 && nrow <= (long)kNormRegRows * (1024 / (nrhs / 2)))
    hipLaunchKernelGGL((block_norm_reg_kernel<kNormRegRows, 4>), dim3((nac + 7) / 8 * 8), dim3(1024), 0, s, a, h,
                       nrhs, 1, nac, static_cast<float2*>(f), norms);
  else if (nrhs % 2 == 0)
    hipLaunchKernelGGL((block_norm_kernel<float, 2>), dim3(a.Vc), dim3(256), 0, s, a, h, nrhs,
                       static_cast<float2*>(f), norms);
  else
    hipLaunchKernelGGL((block_norm_kernel<float, 1>), dim3(a.Vc), dim3(256), 0, s, a, h, nrhs,
                       static_cast<float2*>(f), norms);
  return hipGetLastError();
}

// in_prec64 / out_prec64 select double2 or float2 on each side.
hipError_t launch_basis_convert(const void* in, int in_prec64, void* out, int out_prec64, long nsite, int nv, int ncomp,
                                int to_internal, hipStream_t s) {
  const long n = nsite * nv * ncomp;
  const int nb = (int)((n + 255) / 256);
  if (in_prec64 && out_prec64)
    hipLaunchKernelGGL((basis_transpose<double, double>), dim3(nb), dim3(256), 0, s, static_cast<const double2*>(in),
                       static_cast<double2*>(out), nsite, nv, ncomp, to_internal);
  else if (in_prec64)
    hipLaunchKernelGGL((basis_transpose<double, float>), dim3(nb), dim3(256), 0, s, static_cast<const double2*>(in),
                       static_cast<float2*>(out), nsite, nv, ncomp, to_internal);
  else if (out_prec64)
    hipLaunchKernelGGL((basis_transpose<float, double>), dim3(nb), dim3(256), 0, s, static_cast<const float2*>(in),
                       static_cast<double2*>(out), nsite, nv, ncomp, to_internal);
  else
    hipLaunchKernelGGL((basis_transpose<float, float>), dim3(nb), dim3(256), 0, s, static_cast<const float2*>(in),
                       static_cast<float2*>(out), nsite, nv, ncomp, to_internal);
  return hipGetLastError();
}

}  // namespace mrhs
