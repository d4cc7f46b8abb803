// Coarse-level 9-point stencil on the matrix cores (paper Sec. 6), for
// Nb = 32 components per site: with many right-hand sides the coarse operator
// becomes, site by site, a sum of nine dense complex 32 x 32 by 32 x Nrhs
// products, which gfx950 runs as BF16 or FP16 MFMA with FP32 accumulation.
//
// Complex arithmetic is split into real products,
//   Re O += Re B Re E - Im B Im E,   Im O += Re B Im E + Im B Re E,
// four v_mfma_f32_32x32x16 per 16-wide slice of the contraction index j.
// One workgroup owns one site and one or two 32-column tiles of right-hand
// sides (two tiles either as columns c0.. and c0 + 32.., or interleaved, even
// columns in one tile and odd in the other, so that a lane reads a column pair
// with one 16-byte load).  The 18 units of work of a site (nine directions,
// two 16-wide slices of j) are dealt to its four or eight wavefronts in turn,
// and their partial sums are added through LDS in a fixed order, which gives
// the latency-bound small coarse lattices several wavefronts per site.  Rows
// of the 32 x 32 output are the 32 coarse components i, columns the
// right-hand sides.
//
// Operand layouts of v_mfma_f32_32x32x16_{bf16,f16} (lane l, 8 values each):
//   A (blocks):  A[i = l % 32][j = 8 (l / 32) + q], q = 0..7
//   B (vectors): B[j = 8 (l / 32) + q][col = l % 32]
//   D (output):  D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in accumulator r = 0..15
// Blocks are pre-packed once per level in exactly the A order,
// [site][d][j-slice][re|im][lane][8], so every A load is one 16-byte load per
// lane and 1 KiB contiguous per wavefront.  Vectors stay FP32 in memory
// ([site][j][rhs]); each lane reads its eight values (256-byte contiguous runs
// across the wavefront) and rounds them from FP32 to BF16/FP16 on the fly
// (hardware conversion, round to nearest even; the one-time block pack,
// which starts from FP64, uses the explicit conversions of rounding.h).
// FP16 operands are first scaled per right-hand side by a power of two,
// 2^-E with max_k |x| = m 2^E, m in [0.5, 1), and the output is scaled back in
// FP32; the power of two keeps the scaling exact.
#include "mg_internal.h"
#include "rounding.h"

namespace mrhs {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kNb = 32;

__device__ __forceinline__ unsigned short bf16_rne(float f) { return bf16_rne_bits(__float_as_uint(f)); }
__device__ __forceinline__ unsigned short f16_rne(float f) { return f16_rne_bits(__float_as_uint(f)); }

template <bool F16>
struct Op;
template <>
struct Op<false> {
  using vec = bf16x8;
  static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  // FP32 -> BF16 by the hardware conversion, which rounds to nearest even
  // (checked on exact ties; the parity tests compare with the emulation)
  static __device__ __forceinline__ vec cvt(const float (&x)[8]) {
    vec v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (__bf16)x[q];
    return v;
  }
};
template <>
struct Op<true> {
  using vec = f16x8;
  static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ vec cvt(const float (&x)[8]) {
    vec v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (_Float16)x[q];
    return v;
  }
};

// Workgroups are dealt round-robin to the 8 XCDs; remap so that every XCD
// works on one contiguous range of sites (and keeps their neighbours' vectors
// in its own L2).  The grid is a multiple of 8; surplus workgroups get an
// index past the end and exit.
__device__ __forceinline__ int xcd_block(int nblocks) {
  const int b = blockIdx.x;
  const int per = (nblocks + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// Adds the partial accumulators of the four wavefronts as (0 + 2) + (1 + 3),
// through 16 KiB of LDS.  Returns false on the wavefronts that have nothing
// left to do.
__device__ __forceinline__ bool reduce_waves(f32x16& accR, f32x16& accI) {
  __shared__ float red[2][64][32];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (wv >= 2) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      red[wv - 2][l][r] = accR[r];
      red[wv - 2][l][16 + r] = accI[r];
    }
  }
  __syncthreads();
  if (wv < 2) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accR[r] += red[wv][l][r];
      accI[r] += red[wv][l][16 + r];
    }
  }
  __syncthreads();
  if (wv == 1) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      red[0][l][r] = accR[r];
      red[0][l][16 + r] = accI[r];
    }
  }
  __syncthreads();
  if (wv != 0) return false;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accR[r] += red[0][l][r];
    accI[r] += red[0][l][16 + r];
  }
  return true;
}

// Sum of the WV wavefronts' accumulators into wavefront 0 in a fixed order, a
// halving tree through LDS (wavefront w + h is added into w for h = WV / 2,
// WV / 4, ..., 1; for WV = 4 that is (0 + 2) + (1 + 3)).  Every thread of the
// workgroup must call it.
template <int WV>
__device__ __forceinline__ void reduce_waves_t(f32x16& accR, f32x16& accI, float (*red)[64][32]) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int h = WV / 2; h >= 1; h >>= 1) {
    if (wv >= h && wv < 2 * h) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        red[wv - h][l][r] = accR[r];
        red[wv - h][l][16 + r] = accI[r];
      }
    }
    __syncthreads();
    if (wv < h) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[r] += red[wv][l][r];
        accI[r] += red[wv][l][16 + r];
      }
    }
    __syncthreads();
  }
}

// Even-odd modes of the stencil kernels (all coarse extents even; a field on
// one parity is [V/2][Nb][nrhs], entry i the site of that parity among 2i,
// 2i + 1): EO = 1 applies the eight hop directions from parity 1 - p to p,
// EO = 2 the self blocks (or the packed blocks bstride = 1 of their
// inverses) on parity p.  EO = 0 is the full stencil.
__device__ __forceinline__ int cb_site(const Geom& g, int i, int p) {
  const int s2 = 2 * i;
  int r = s2;
  int sum = 0;
  for (int m = 0; m < 4; ++m) {
    sum += r % g.L[m];
    r /= g.L[m];
  }
  return (sum & 1) == p ? s2 : s2 + 1;
}

// Neighbour of site s (coordinates x) in direction d of the stencil
// (self, +x, -x, +y, -y, +z, -z, +t, -t), periodic.  Only constant indices
// into the geometry: indexed by a per-lane direction it is read from memory,
// and every such read waits for all loads issued before it, which would
// serialise the units of a wavefront.
__device__ __forceinline__ int stencil_nbr(const Geom& g, int s, const int (&x)[4], int d) {
  int off = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int fw = x[m] + 1 < g.L[m] ? g.stride[m] : g.stride[m] * (1 - g.L[m]);
    const int bw = x[m] > 0 ? -g.stride[m] : g.stride[m] * (g.L[m] - 1);
    off = d == 2 * m + 1 ? fw : off;
    off = d == 2 * m + 2 ? bw : off;
  }
  return s + off;
}

// The stencil's work on one site, split into units (d, kc) = (direction,
// 16-wide slice of the contraction index): unit u = 2 d + kc.  Wavefront w of
// WV takes units u0 + w, u0 + w + WV, ... (balanced: 18 units over four
// wavefronts are 5, 5, 4, 4), each unit four v_mfma_f32_32x32x16 per
// 32-column tile of the NT tiles the workgroup covers, so a block slice is
// loaded once for all its right-hand sides.  A unit past the end is computed
// on a valid unit with zero operands (straight-line loads, no branch).
// fetch(row, e, t, d) returns the FP32 operand at row `row` (of the input
// field of direction d), element offset e = j nrhs + column, for tile t.
// PAIR (with NT = 2): tile 0 holds the even and tile 1 the odd columns of a
// 64-column group, lane l columns c0 + 2 (l % 32) and the next, so each
// operand row is one 16-byte load fetch4(row, e, d) of the column pair at
// element offset e (colc[0] the even column) instead of two 8-byte loads.
template <bool F16, int WV, int NT, bool PAIR = false, class Fetch, class Fetch4>
__device__ __forceinline__ void stencil_units(const Geom& g, int s, int io, int EOmode, int nrhs, const uint4* Bp,
                                              int bstride, const int (&colc)[NT], const bool (&colok)[NT],
                                              const float (&sc)[NT], Fetch&& fetch, Fetch4&& fetch4,
                                              f32x16 (&accR)[NT], f32x16 (&accI)[NT]) {
  static_assert(!PAIR || NT == 2, "column pairs fill two tiles");
  using O = Op<F16>;
  using vec = typename O::vec;
  // the wavefront index, and with it each unit's direction, is uniform
  const int l = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int jh = 8 * (l >> 5);
  int x[4];
  {
    int r = s;
    x[0] = r % g.L[0];
    r /= g.L[0];
    x[1] = r % g.L[1];
    r /= g.L[1];
    x[2] = r % g.L[2];
    x[3] = r / g.L[2];
  }
  const int u0 = EOmode == 1 ? 2 : 0, u1 = EOmode == 2 ? 2 : 18;
  constexpr int KMAX = (18 + WV - 1) / WV;
  // units are handled in batches: every load of a batch is issued before its
  // first matrix instruction, so a wavefront waits for memory once per batch
  // instead of once per unit (with one tile all of a wavefront's units form
  // one batch; with two tiles batches of three bound the registers, and for
  // column pairs smaller batches buy occupancy: one-unit batches on four
  // wavefronts measured fastest, 3 wavefronts per SIMD against 2)
  constexpr int PB = NT == 1 ? KMAX : (PAIR ? (WV == 4 ? 1 : 2) : 3);
#pragma unroll
  for (int k0 = 0; k0 < KMAX; k0 += PB) {
    uint4 br[PB], bi[PB];
    float2 ev[PB][NT][8];
    bool live[PB];
#pragma unroll
    for (int kk = 0; kk < PB; ++kk) {
      const int u = u0 + wv + (k0 + kk) * WV;
      live[kk] = (k0 + kk < KMAX) && u < u1;
      const int uc = live[kk] ? u : u0;
      const int d = uc >> 1, kc = uc & 1;
      const int nbr = stencil_nbr(g, s, x, d);
      // input row: EO 1 the neighbour's checkerboard index, EO 2 the output
      // row, EO 3 both (self term on the output row, hops on the neighbours')
      const int ii = EOmode == 1 ? nbr / 2 : (EOmode == 2 ? io : (EOmode == 3 ? (d == 0 ? io : nbr / 2) : nbr));
      const uint4* bp = Bp + ((size_t)s * bstride + d) * 256;
      br[kk] = bp[(kc * 2 + 0) * 64 + l];
      bi[kk] = bp[(kc * 2 + 1) * 64 + l];
      if constexpr (PAIR) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 v = fetch4(ii, (size_t)(kc * 16 + jh + q) * nrhs + colc[0], d);
          ev[kk][0][q] = make_float2(v.x, v.y);
          ev[kk][NT - 1][q] = make_float2(v.z, v.w);
        }
      } else {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 8; ++q) ev[kk][t][q] = fetch(ii, (size_t)(kc * 16 + jh + q) * nrhs + colc[t], t, d);
      }
    }
#pragma unroll
    for (int kk = 0; kk < PB; ++kk) {
      const uint4 b_i = bi[kk];
      const uint4 nbi =
          make_uint4(b_i.x ^ 0x80008000u, b_i.y ^ 0x80008000u, b_i.z ^ 0x80008000u, b_i.w ^ 0x80008000u);
      const vec ar = __builtin_bit_cast(vec, br[kk]);
      const vec ai = __builtin_bit_cast(vec, b_i);
      const vec an = __builtin_bit_cast(vec, nbi);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        float er[8], ei[8];
        const bool on = live[kk] && colok[t];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          er[q] = on ? ev[kk][t][q].x * sc[t] : 0.f;
          ei[q] = on ? ev[kk][t][q].y * sc[t] : 0.f;
        }
        const vec vr = O::cvt(er), vi = O::cvt(ei);
        accR[t] = O::mma(ar, vr, accR[t]);
        accR[t] = O::mma(an, vi, accR[t]);
        accI[t] = O::mma(ar, vi, accI[t]);
        accI[t] = O::mma(ai, vr, accI[t]);
      }
    }
  }
}

// One workgroup of WV wavefronts per (output site, group of NT 32-column
// tiles of right-hand sides).
// EO = 3 (the coarse Schur complement's outer product, all extents even):
// out = S_p in - H_{p,1-p} in2 on parity p, in on parity p, in2 on 1 - p.
template <bool F16, int EO, int WV, int NT, bool PAIR = false>
__global__ __launch_bounds__(64 * WV) void coarse_mfma_kernel(Geom g, int nrhs, const uint4* __restrict__ Bp,
                                                              const float2* __restrict__ in, float2* __restrict__ out,
                                                              const float* __restrict__ scale, int nblocks,
                                                              int parity, int bstride,
                                                              const float2* __restrict__ in2 = nullptr) {
  __shared__ float red[WV / 2][64][32];
  const int l = threadIdx.x & 63;
  const int ngroups = (nrhs + 32 * NT - 1) / (32 * NT);
  const long w = xcd_block(nblocks);
  const int nsite = EO ? g.V / 2 : g.V;
  if (w >= (long)nsite * ngroups) return;  // whole workgroup
  const int io = (int)(w / ngroups);  // output row
  const int s = EO ? cb_site(g, io, parity) : io;
  const int c0 = (int)(w % ngroups) * 32 * NT;
  int col[NT], colc[NT];
  bool colok[NT];
  float sc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    // PAIR: lane l owns the column pair c0 + 2 (l % 32), + 1 (nrhs even)
    col[t] = PAIR ? c0 + 2 * (l & 31) + t : c0 + 32 * t + (l & 31);
    colok[t] = col[t] < nrhs;
    colc[t] = colok[t] ? col[t] : (PAIR ? nrhs - 2 + t : nrhs - 1);
    sc[t] = (F16 && colok[t]) ? scale[col[t]] : 1.0f;
  }
  f32x16 accR[NT], accI[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accR[t] = f32x16{};
    accI[t] = f32x16{};
  }
  stencil_units<F16, WV, NT, PAIR>(
      g, s, io, EO, nrhs, Bp, bstride, colc, colok, sc,
      // EO 3: minus the hop term, read from the second field (the field is
      // selected before the load, so no branch separates the loads)
      [&](int ii, size_t e, int, int d) {
        const bool hop = EO == 3 && d > 0;
        const float2 v = (hop ? in2 : in)[(size_t)ii * kNb * nrhs + e];
        return hop ? make_float2(-v.x, -v.y) : v;
      },
      [&](int ii, size_t e, int d) {
        const bool hop = EO == 3 && d > 0;
        const float4 v = *reinterpret_cast<const float4*>((hop ? in2 : in) + (size_t)ii * kNb * nrhs + e);
        return hop ? make_float4(-v.x, -v.y, -v.z, -v.w) : v;
      },
      accR, accI);
#pragma unroll
  for (int t = 0; t < NT; ++t) reduce_waves_t<WV>(accR[t], accI[t], red);
  if ((threadIdx.x >> 6) != 0) return;
  if constexpr (PAIR) {
    if (!colok[0]) return;
    const float inv0 = F16 ? 1.0f / sc[0] : 1.0f, inv1 = F16 ? 1.0f / sc[1] : 1.0f;
    float4* o = reinterpret_cast<float4*>(out + (size_t)io * kNb * nrhs + col[0]);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
      o[(size_t)row * nrhs / 2] =
          make_float4(accR[0][r] * inv0, accI[0][r] * inv0, accR[1][r] * inv1, accI[1][r] * inv1);
    }
  } else {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (!colok[t]) continue;
      const float inv = F16 ? 1.0f / sc[t] : 1.0f;  // exact: sc is a power of two
      float2* o = out + (size_t)io * kNb * nrhs + col[t];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
        o[(size_t)row * nrhs] = make_float2(accR[t][r] * inv, accI[t][r] * inv);
      }
    }
  }
}

// r_k - a_k p_k in FP32 with the rounding of the separate MR update kernel
// (a_k rounded to FP32 first).
__device__ __forceinline__ float2 mr_residual(float2 rv, float2 pv, float ar, float ai) {
  float2 rn;
  rn.x = fmaf(-ar, pv.x, fmaf(ai, pv.y, rv.x));
  rn.y = fmaf(-ar, pv.y, fmaf(-ai, pv.x, rv.y));
  return rn;
}

// One minimal-residual step on a coarse level with BF16 operands in two
// launches (paper Sec. 6: the coarsest level is latency-bound, so a step
// should be as few kernels as possible, not a stencil, two reductions and an
// update):
//   r_i = r_{i-1} - a_{i-1} p_{i-1}   recomputed on the fly wherever the
//                                     stencil reads it, stored for the own site
//   x_i = x_{i-1} + a_{i-1} r_{i-1}   own site, in place
//   p_i = D r_i                       stored
//   per (site, column): <p_i, r_i> and ||p_i||^2 over the site's Nb rows (FP64),
//   which a second small launch (mr_site_alpha_kernel) sums over the sites in
//   a fixed order into a_i = <p_i, r_i> / ||p_i||^2 per column.
// first: step 0, r_0 = rold as given, x untouched.  Fields [V][Nb][nrhs] FP32;
// rold / pold and rnew / pnew are different buffers (ping-pong across steps).
// The step is a template parameter: a run-time flag around the operand loads
// becomes a branch per load, each waiting for the loads before it.
template <int WV, int NT, bool first>
__global__ __launch_bounds__(64 * WV) void coarse_mr_step_kernel(
    Geom g, int nrhs, const uint4* __restrict__ Bp, const float2* __restrict__ rold, const float2* __restrict__ pold,
    float2* __restrict__ rnew, float2* __restrict__ pnew, float2* __restrict__ x, const double2* __restrict__ aold,
    double4* __restrict__ part, int nblocks) {
  __shared__ float red[WV / 2][64][32];
  __shared__ double4 dred[64];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ngroups = (nrhs + 32 * NT - 1) / (32 * NT);
  const long w = xcd_block(nblocks);
  const long nwork = (long)g.V * ngroups;
  if (w >= nwork) return;  // whole workgroup
  const int s = (int)(w / ngroups);
  const int c0 = (int)(w % ngroups) * 32 * NT;
  int col[NT], colc[NT];
  bool colok[NT];
  float sc[NT], ar[NT], ai[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    col[t] = c0 + 32 * t + (l & 31);
    colok[t] = col[t] < nrhs;
    colc[t] = colok[t] ? col[t] : nrhs - 1;
    sc[t] = 1.0f;
    const double2 a = first ? make_double2(0.0, 0.0) : aold[colc[t]];
    ar[t] = (float)a.x;
    ai[t] = (float)a.y;
  }
  f32x16 accR[NT], accI[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accR[t] = f32x16{};
    accI[t] = f32x16{};
  }
  stencil_units<false, WV, NT>(g, s, s, 0, nrhs, Bp, 9, colc, colok, sc,
                               [&](int ii, size_t e, int t, int) {
                                 const size_t o = (size_t)ii * kNb * nrhs + e;
                                 const float2 rv = rold[o];
                                 if constexpr (first) return rv;
                                 else return mr_residual(rv, pold[o], ar[t], ai[t]);
                               },
                               [](int, size_t, int) { return make_float4(0.f, 0.f, 0.f, 0.f); }, accR, accI);
#pragma unroll
  for (int t = 0; t < NT; ++t) reduce_waves_t<WV>(accR[t], accI[t], red);
  // epilogue on wavefront 0: own-site r_i, x_i, p_i and the partial sums
  double4 sum[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) sum[t] = make_double4(0.0, 0.0, 0.0, 0.0);
  if (wv == 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // the loads of eight rows first (clamped column), then their arithmetic
      // and stores: interleaved, each load would wait for the stores before
      // it; eight rows at a time bound the registers
      const size_t base = (size_t)s * kNb * nrhs + colc[t];
#pragma unroll
      for (int h = 0; h < 16; h += 8) {
        float2 rv[8], pv[8], xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int r = h + q;
          const size_t o = base + (size_t)(8 * (r >> 2) + 4 * (l >> 5) + (r & 3)) * nrhs;
          rv[q] = rold[o];
          if constexpr (!first) {
            pv[q] = pold[o];
            xv[q] = x[o];
          }
        }
        if (colok[t]) {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int r = h + q;
            const size_t o = base + (size_t)(8 * (r >> 2) + 4 * (l >> 5) + (r & 3)) * nrhs;
            float2 ri = rv[q];
            if constexpr (!first) {
              ri = mr_residual(rv[q], pv[q], ar[t], ai[t]);
              float2 xn = xv[q];
              xn.x = fmaf(ar[t], rv[q].x, fmaf(-ai[t], rv[q].y, xn.x));
              xn.y = fmaf(ar[t], rv[q].y, fmaf(ai[t], rv[q].x, xn.y));
              x[o] = xn;
              rnew[o] = ri;
            }
            const float2 p = make_float2(accR[t][r], accI[t][r]);
            pnew[o] = p;
            const double px = p.x, py = p.y, rx = ri.x, ry = ri.y;
            sum[t].x = fma(px, rx, fma(py, ry, sum[t].x));
            sum[t].y = fma(px, ry, fma(-py, rx, sum[t].y));
            sum[t].z = fma(px, px, fma(py, py, sum[t].z));
          }
        }
      }
    }
  }
  // lanes l and l + 32 of wavefront 0 hold the two row halves of a column
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (wv == 0 && l >= 32) dred[l - 32] = sum[t];
    __syncthreads();
    if (wv == 0 && l < 32 && colok[t]) {
      const double4 o = dred[l];
      part[(size_t)s * nrhs + col[t]] =
          make_double4(sum[t].x + o.x, sum[t].y + o.y, sum[t].z + o.z, 0.0);
    }
    __syncthreads();
  }
}

// Step length of the fused MR step: one workgroup per column sums the
// per-site partials in a fixed order (strided by thread, then a tree) and
// writes a = <p, r> / ||p||^2.
__global__ __launch_bounds__(256) void mr_site_alpha_kernel(const double4* __restrict__ part, int nsite, int nrhs,
                                                            double2* __restrict__ anew) {
  __shared__ double4 red[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
  int site = t;
  for (; site + 3 * 256 < nsite; site += 4 * 256) {
    double4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[(size_t)(site + u * 256) * nrhs + k];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc.x += v[u].x;
      acc.y += v[u].y;
      acc.z += v[u].z;
    }
  }
  for (; site < nsite; site += 256) {
    const double4 v = part[(size_t)site * nrhs + k];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
  }
  red[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      red[t].x += red[t + w].x;
      red[t].y += red[t + w].y;
      red[t].z += red[t + w].z;
    }
    __syncthreads();
  }
  if (t == 0) {
    const double4 a = red[0];
    anew[k] = a.z > 0.0 ? make_double2(a.x / a.z, a.y / a.z) : make_double2(0.0, 0.0);
  }
}

// After the last fused step: x += a r and, if rout is given, rout = r - a p
// (FP32, the separate update kernel's rounding).  rout may be r itself.
__global__ __launch_bounds__(256) void mr_finish_kernel(float2* __restrict__ x, const float2* r,
                                                        const float2* __restrict__ p, float2* rout,
                                                        const double2* __restrict__ alpha, long n, int nrhs) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double2 a = alpha[e % nrhs];
  const float ar = (float)a.x, ai = (float)a.y;
  const float2 rv = r[e];
  float2 xv = x[e];
  xv.x = fmaf(ar, rv.x, fmaf(-ai, rv.y, xv.x));
  xv.y = fmaf(ar, rv.y, fmaf(ai, rv.x, xv.y));
  x[e] = xv;
  if (rout) rout[e] = mr_residual(rv, p[e], ar, ai);
}

// FP32 operands on v_mfma_f32_32x32x2_f32 (full-rate FP32 matrix cores):
//   A[i = l % 32][k = l / 32], B[k = l / 32][col = l % 32], D as above,
// so one instruction contracts two values of j.  Blocks are packed
// [site][d][re|im][lane][16] with element q of lane l holding
// B[i = l % 32][j = 2 q + l / 32]: four 16-byte loads per lane per part.
template <int EO>
__global__ __launch_bounds__(256) void coarse_mfma_f32_kernel(Geom g, int nrhs, const float4* __restrict__ Bp,
                                                              const float2* __restrict__ in,
                                                              float2* __restrict__ out, int nblocks, int parity,
                                                              int bstride) {
  const int l = threadIdx.x & 63;
  const int ntiles = (nrhs + 31) >> 5;
  const long w = xcd_block(nblocks);
  const int nsite = EO ? g.V / 2 : g.V;
  if (w >= (long)nsite * ntiles) return;  // whole workgroup
  const int io = (int)(w / ntiles);  // output row
  const int s = EO ? cb_site(g, io, parity) : io;
  const int col = (int)(w % ntiles) * 32 + (l & 31);
  const bool colok = col < nrhs;
  const int colc = colok ? col : nrhs - 1;
  const int jh = l >> 5;
  int x[4];
  {
    int r = s;
    x[0] = r % g.L[0];
    r /= g.L[0];
    x[1] = r % g.L[1];
    r /= g.L[1];
    x[2] = r % g.L[2];
    x[3] = r / g.L[2];
  }
  f32x16 accR = {}, accI = {};
  const int d0 = EO == 1 ? 1 : 0, d1 = EO == 2 ? 1 : 9;
  for (int d = d0 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); d < d1; d += 4) {
    const int nbr = stencil_nbr(g, s, x, d);
    const int ii = EO == 1 ? nbr / 2 : (EO == 2 ? io : nbr);  // input row
    const float4* bp = Bp + ((size_t)s * bstride + d) * 2 * 64 * 4;
    float br[16], bi[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 a = bp[(0 * 64 + l) * 4 + q], b = bp[(1 * 64 + l) * 4 + q];
      br[4 * q] = a.x;
      br[4 * q + 1] = a.y;
      br[4 * q + 2] = a.z;
      br[4 * q + 3] = a.w;
      bi[4 * q] = b.x;
      bi[4 * q + 1] = b.y;
      bi[4 * q + 2] = b.z;
      bi[4 * q + 3] = b.w;
    }
    // all vector loads first, from a clamped column (no branch around the
    // loads); columns past nrhs are zeroed and never stored
    const float2* e = in + (size_t)ii * kNb * nrhs + colc;
    float2 ev[16];
#pragma unroll
    for (int kc = 0; kc < 16; ++kc) ev[kc] = e[(size_t)(2 * kc + jh) * nrhs];
#pragma unroll
    for (int kc = 0; kc < 16; ++kc) {
      const float2 v = colok ? ev[kc] : make_float2(0.f, 0.f);
      accR = __builtin_amdgcn_mfma_f32_32x32x2f32(br[kc], v.x, accR, 0, 0, 0);
      accR = __builtin_amdgcn_mfma_f32_32x32x2f32(-bi[kc], v.y, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_32x32x2f32(br[kc], v.y, accI, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_32x32x2f32(bi[kc], v.x, accI, 0, 0, 0);
    }
  }
  if (!reduce_waves(accR, accI) || !colok) return;
  float2* o = out + (size_t)io * kNb * nrhs + col;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    o[(size_t)row * nrhs] = make_float2(accR[r], accI[r]);
  }
}

__global__ void pack_f32_kernel(const double2* __restrict__ B, float* __restrict__ P, long nblk) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= nblk * kNb * kNb) return;
  const long blk = e / (kNb * kNb);
  const int r = (int)(e % (kNb * kNb));
  const int i = r / kNb, j = r % kNb;
  const int lane = i + 32 * (j & 1), q = j >> 1;
  const double2 v = B[e];
  float* base = P + blk * (2 * 64 * 16);
  base[(0 * 64 + lane) * 16 + q] = (float)v.x;
  base[(1 * 64 + lane) * 16 + q] = (float)v.y;
}

// FP64 blocks [site][9][32][32] complex -> packed A-operand order; the value is
// rounded to FP32 first, then to BF16/FP16 (nearest even).
template <bool F16>
__global__ void pack_kernel(const double2* __restrict__ B, unsigned short* __restrict__ P, long nblk) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;  // one thread per packed element pair (re, im)
  if (e >= nblk * kNb * kNb) return;
  const long blk = e / (kNb * kNb);
  const int r = (int)(e % (kNb * kNb));
  const int i = r / kNb, j = r % kNb;
  const int kc = j / 16, jj = j % 16;
  const int lane = i + 32 * (jj / 8), q = jj % 8;
  const double2 v = B[e];
  const float fr = (float)v.x, fi = (float)v.y;
  unsigned short hr, hi;
  if constexpr (F16) {
    hr = f16_rne(fr);
    hi = f16_rne(fi);
  } else {
    hr = bf16_rne(fr);
    hi = bf16_rne(fi);
  }
  unsigned short* base = P + blk * (2 * 2 * 64 * 8);
  base[((kc * 2 + 0) * 64 + lane) * 8 + q] = hr;
  base[((kc * 2 + 1) * 64 + lane) * 8 + q] = hi;
}

// scale[k] = 2^-E with max over the column of |re|, |im| = m 2^E, m in [0.5, 1); 1 for a zero column.
__global__ void colmax_kernel(const float2* __restrict__ in, long rows, int nrhs, unsigned int* __restrict__ m) {
  const long e0 = (long)blockIdx.x * 256 + threadIdx.x;
  const long n = rows * nrhs;
  const long stride = (long)gridDim.x * 256;
  // the stride is a multiple of nrhs when launched as below, so the column is fixed
  const int k = (int)(e0 % nrhs);
  float mx = 0.f;
  // four loads in flight per thread; an index past the end reads this
  // thread's own first element (valid, as e0 < n inside the loop) and counts
  // zero, so no load sits in a branch
  constexpr int U = 4;
  for (long e = e0; e < n; e += U * stride) {
    float2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = in[e + u * stride < n ? e + u * stride : e0];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float a = fmaxf(fabsf(v[u].x), fabsf(v[u].y));
      mx = fmaxf(mx, e + u * stride < n ? a : 0.f);
    }
  }
  // one atomic per (workgroup, column): thread j < nrhs combines the threads
  // t = j, j + nrhs, ... of the workgroup, which all hold column k(j)
  __shared__ float smax[256];
  smax[threadIdx.x] = mx;
  __syncthreads();
  if ((int)threadIdx.x < nrhs) {
    float c = 0.f;
    for (int t = threadIdx.x; t < 256; t += nrhs) c = fmaxf(c, smax[t]);
    atomicMax(m + k, __float_as_uint(c));  // non-negative floats order as their bit patterns
  }
}
// Also clears the reduction words, so that the next call starts from zero
// without a separate launch.
__global__ void colmax_to_scale(unsigned int* __restrict__ m, float* __restrict__ scale, int nrhs) {
  const int k = threadIdx.x;
  if (k >= nrhs) return;
  const float mx = __uint_as_float(m[k]);
  int E = 0;
  (void)frexpf(mx, &E);
  scale[k] = mx > 0.f ? ldexpf(1.0f, -E) : 1.0f;
  m[k] = 0u;
}

}  // namespace

bool mfma_supported(int nb) { return nb == kNb; }

size_t mfma_pack_bytes(long nsite) { return (size_t)nsite * 9 * kNb * kNb * 2 * 2; }

hipError_t launch_pack_blocks(int f16, const void* B64, void* packed, long nsite, hipStream_t s) {
  const long n = nsite * 9 * kNb * kNb;
  const int blocks = (int)((n + 255) / 256);
  if (f16)
    hipLaunchKernelGGL((pack_kernel<true>), dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(B64),
                       static_cast<unsigned short*>(packed), nsite * 9);
  else
    hipLaunchKernelGGL((pack_kernel<false>), dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(B64),
                       static_cast<unsigned short*>(packed), nsite * 9);
  return hipGetLastError();
}

// work: nrhs 32-bit words that are zero on entry (and are left zero).
hipError_t launch_column_scale(const void* in, long rows, int nrhs, void* work, float* scale, hipStream_t s) {
  unsigned int* m = static_cast<unsigned int*>(work);
  // workgroup stride must be a multiple of nrhs: use blocks of 256 threads and
  // a grid such that 256 * grid % nrhs == 0 (a few hundred workgroups: every
  // one ends in nrhs atomics on the same nrhs words)
  int grid = 256;
  while ((256L * grid) % nrhs) ++grid;
  hipLaunchKernelGGL(colmax_kernel, dim3(grid), dim3(256), 0, s, static_cast<const float2*>(in), rows, nrhs, m);
  hipLaunchKernelGGL(colmax_to_scale, dim3(1), dim3(64), 0, s, m, scale, nrhs);
  return hipGetLastError();
}

namespace {

template <bool F16, int WV, int NT, bool PAIR = false>
hipError_t launch_stencil_t(const Geom& g, int nrhs, const void* packed, const void* in, void* out, const float* scale,
                            hipStream_t s) {
  const int blocks = (int)((long)g.V * ((nrhs + 32 * NT - 1) / (32 * NT)));
  const int grid = ((blocks + 7) / 8) * 8;
  hipLaunchKernelGGL((coarse_mfma_kernel<F16, 0, WV, NT, PAIR>), dim3(grid), dim3(64 * WV), 0, s, g, nrhs,
                     static_cast<const uint4*>(packed), static_cast<const float2*>(in), static_cast<float2*>(out),
                     scale, blocks, 0, 9, nullptr);
  return hipGetLastError();
}

template <int WV, int NT>
hipError_t launch_mr_t(const Geom& g, int nrhs, const void* packed, const void* rold, const void* pold, void* rnew,
                       void* pnew, void* x, const void* aold, void* anew, void* part, int first, hipStream_t s) {
  const int blocks = (int)((long)g.V * ((nrhs + 32 * NT - 1) / (32 * NT)));
  const int grid = ((blocks + 7) / 8) * 8;
  auto k = first ? coarse_mr_step_kernel<WV, NT, true> : coarse_mr_step_kernel<WV, NT, false>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WV), 0, s, g, nrhs, static_cast<const uint4*>(packed),
                     static_cast<const float2*>(rold), static_cast<const float2*>(pold), static_cast<float2*>(rnew),
                     static_cast<float2*>(pnew), static_cast<float2*>(x), static_cast<const double2*>(aold),
                     static_cast<double4*>(part), blocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mr_site_alpha_kernel, dim3(nrhs), dim3(256), 0, s, static_cast<const double4*>(part), g.V, nrhs,
                     static_cast<double2*>(anew));
  return hipGetLastError();
}

}  // namespace

// cfg: launch shape of the BF16/FP16 stencil, bit 0 eight wavefronts per
// workgroup (else four); cfg >> 1 the column tiling: 0 one 32-column tile per
// workgroup, 1 two, 2 two tiles as interleaved column pairs read with 16-byte
// loads (fields are 16-byte aligned, which the entry points check).  The pair
// form needs an even nrhs; for an odd one cfg 4 / 5 run as cfg 2 / 3 (the same
// result).
hipError_t launch_coarse_mfma(int f16, const Geom& g, int nb, int nrhs, const void* packed, const void* in, void* out,
                              const float* scale, hipStream_t s, int cfg) {
  if (nb != kNb || cfg < 0 || cfg >= kLowpCfgs) return hipErrorInvalidValue;
  if (cfg >= 4 && (nrhs & 1)) cfg -= 2;
  if (f16) {
    switch (cfg) {
      case 0: return launch_stencil_t<true, 4, 1>(g, nrhs, packed, in, out, scale, s);
      case 1: return launch_stencil_t<true, 8, 1>(g, nrhs, packed, in, out, scale, s);
      case 2: return launch_stencil_t<true, 4, 2>(g, nrhs, packed, in, out, scale, s);
      case 3: return launch_stencil_t<true, 8, 2>(g, nrhs, packed, in, out, scale, s);
      case 4: return launch_stencil_t<true, 4, 2, true>(g, nrhs, packed, in, out, scale, s);
      default: return launch_stencil_t<true, 8, 2, true>(g, nrhs, packed, in, out, scale, s);
    }
  }
  switch (cfg) {
    case 0: return launch_stencil_t<false, 4, 1>(g, nrhs, packed, in, out, scale, s);
    case 1: return launch_stencil_t<false, 8, 1>(g, nrhs, packed, in, out, scale, s);
    case 2: return launch_stencil_t<false, 4, 2>(g, nrhs, packed, in, out, scale, s);
    case 3: return launch_stencil_t<false, 8, 2>(g, nrhs, packed, in, out, scale, s);
    case 4: return launch_stencil_t<false, 4, 2, true>(g, nrhs, packed, in, out, scale, s);
    default: return launch_stencil_t<false, 8, 2, true>(g, nrhs, packed, in, out, scale, s);
  }
}

size_t coarse_mr_part_bytes(long nsite) { return (size_t)nsite * MRHS_MAX_NRHS * sizeof(double4); }

hipError_t launch_coarse_mr_step(const Geom& g, int nb, int nrhs, const void* packed, const void* rold, const void* pold,
                                 void* rnew, void* pnew, void* x, const void* aold, void* anew, void* part, int first,
                                 int cfg, hipStream_t s) {
  if (nb != kNb || cfg < 0 || cfg > 3 || nrhs < 1 || nrhs > MRHS_MAX_NRHS) return hipErrorInvalidValue;
  switch (cfg) {
    case 0: return launch_mr_t<4, 1>(g, nrhs, packed, rold, pold, rnew, pnew, x, aold, anew, part, first, s);
    case 1: return launch_mr_t<8, 1>(g, nrhs, packed, rold, pold, rnew, pnew, x, aold, anew, part, first, s);
    case 2: return launch_mr_t<4, 2>(g, nrhs, packed, rold, pold, rnew, pnew, x, aold, anew, part, first, s);
    default: return launch_mr_t<8, 2>(g, nrhs, packed, rold, pold, rnew, pnew, x, aold, anew, part, first, s);
  }
}

hipError_t launch_mr_finish(void* x, const void* r, const void* p, void* rout, const void* alpha, long rows, int nrhs,
                            hipStream_t s) {
  const long n = rows * nrhs;
  hipLaunchKernelGGL(mr_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, static_cast<float2*>(x),
                     static_cast<const float2*>(r), static_cast<const float2*>(p), static_cast<float2*>(rout),
                     static_cast<const double2*>(alpha), n, nrhs);
  return hipGetLastError();
}

// Even-odd modes (see cb_site): prec 0 FP32, 1 BF16, 2 FP16 (scale needed);
// eo 1 hop to parity p, eo 2 per-site blocks (bstride 9: the self blocks of
// the stencil pack, 1: a pack of single blocks per site).
hipError_t launch_coarse_mfma_eo(int prec, int eo, int parity, const Geom& g, int nb, int nrhs, const void* packed,
                                 int bstride, const void* in, void* out, const float* scale, hipStream_t s) {
  if (nb != kNb || (eo != 1 && eo != 2) || (parity != 0 && parity != 1)) return hipErrorInvalidValue;
  for (int m = 0; m < 4; ++m)
    if (g.L[m] % 2) return hipErrorInvalidValue;
  const int blocks = (int)((long)(g.V / 2) * ((nrhs + 31) / 32));
  const dim3 grid((unsigned)(((blocks + 7) / 8) * 8));
  const auto* x = static_cast<const float2*>(in);
  auto* y = static_cast<float2*>(out);
  if (prec == 0) {
    const auto* b = static_cast<const float4*>(packed);
    if (eo == 1)
      hipLaunchKernelGGL((coarse_mfma_f32_kernel<1>), grid, dim3(256), 0, s, g, nrhs, b, x, y, blocks, parity,
                         bstride);
    else
      hipLaunchKernelGGL((coarse_mfma_f32_kernel<2>), grid, dim3(256), 0, s, g, nrhs, b, x, y, blocks, parity,
                         bstride);
  } else {
    const auto* b = static_cast<const uint4*>(packed);
    if (prec == 2 && eo == 1)
      hipLaunchKernelGGL((coarse_mfma_kernel<true, 1, 4, 1>), grid, dim3(256), 0, s, g, nrhs, b, x, y, scale, blocks,
                         parity, bstride, nullptr);
    else if (prec == 2)
      hipLaunchKernelGGL((coarse_mfma_kernel<true, 2, 4, 1>), grid, dim3(256), 0, s, g, nrhs, b, x, y, scale, blocks,
                         parity, bstride, nullptr);
    else if (eo == 1)
      hipLaunchKernelGGL((coarse_mfma_kernel<false, 1, 4, 1>), grid, dim3(256), 0, s, g, nrhs, b, x, y, scale, blocks,
                         parity, bstride, nullptr);
    else
      hipLaunchKernelGGL((coarse_mfma_kernel<false, 2, 4, 1>), grid, dim3(256), 0, s, g, nrhs, b, x, y, scale, blocks,
                         parity, bstride, nullptr);
  }
  return hipGetLastError();
}

// The coarse Schur complement's outer product on parity p with BF16 operands:
// out = S_p in - H_{p,1-p} in2 (in, out on parity p; in2 on 1 - p).
hipError_t launch_coarse_schur(int parity, const Geom& g, int nb, int nrhs, const void* packed, const void* in,
                               const void* in2, void* out, hipStream_t s) {
  if (nb != kNb || (parity != 0 && parity != 1)) return hipErrorInvalidValue;
  for (int m = 0; m < 4; ++m)
    if (g.L[m] % 2) return hipErrorInvalidValue;
  const int blocks = (int)((long)(g.V / 2) * ((nrhs + 31) / 32));
  hipLaunchKernelGGL((coarse_mfma_kernel<false, 3, 4, 1>), dim3((unsigned)(((blocks + 7) / 8) * 8)), dim3(256), 0, s,
                     g, nrhs, static_cast<const uint4*>(packed), static_cast<const float2*>(in),
                     static_cast<float2*>(out), nullptr, blocks, parity, 9, static_cast<const float2*>(in2));
  return hipGetLastError();
}

// Rows of one parity between a full coarse field [V][Nb][nrhs] and a
// checkerboard one [V/2][Nb][nrhs] (entry i: the site of that parity among
// 2i, 2i + 1): half = full rows (gather), or full rows += half (scatter_add).
__global__ __launch_bounds__(256) void cb_rows_kernel(const Geom g, int parity, long rowlen, const float2* __restrict__ src,
                                                      float2* __restrict__ dst, int scatter_add) {
  const int i = blockIdx.y;
  const int s = cb_site(g, i, parity);
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < rowlen; e += (long)gridDim.x * 256) {
    if (scatter_add) {
      float2 v = dst[(size_t)s * rowlen + e];
      const float2 h = src[(size_t)i * rowlen + e];
      v.x += h.x;
      v.y += h.y;
      dst[(size_t)s * rowlen + e] = v;
    } else {
      dst[(size_t)i * rowlen + e] = src[(size_t)s * rowlen + e];
    }
  }
}

hipError_t launch_coarse_cb_rows(int parity, const Geom& g, int nb, int nrhs, const void* src, void* dst, int scatter_add,
                                 hipStream_t s) {
  if (g.V / 2 > 65535) return hipErrorInvalidValue;
  const long rowlen = (long)nb * nrhs;
  const dim3 grid((unsigned)((rowlen + 255) / 256), (unsigned)(g.V / 2));
  hipLaunchKernelGGL(cb_rows_kernel, grid, dim3(256), 0, s, g, parity, rowlen, static_cast<const float2*>(src),
                     static_cast<float2*>(dst), scatter_add);
  return hipGetLastError();
}

// Inverse of every Nb x Nb self block (FP64 Gauss-Jordan with partial
// pivoting, one workgroup per site, [M | 1] in LDS).  B64 is the stencil
// master [site][9][Nb][Nb]; out [site][Nb][Nb]; a vanishing pivot sets *flag.
__global__ __launch_bounds__(256) void self_invert_kernel(const double2* __restrict__ B64,
                                                          double2* __restrict__ out, int* __restrict__ flag) {
  __shared__ double2 M[kNb][2 * kNb];
  __shared__ int piv;
  const int site = blockIdx.x;
  const double2* b = B64 + (size_t)site * 9 * kNb * kNb;  // direction 0
  for (int e = threadIdx.x; e < kNb * 2 * kNb; e += 256) {
    const int r = e / (2 * kNb), c = e % (2 * kNb);
    M[r][c] = c < kNb ? b[r * kNb + c] : make_double2(c - kNb == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < kNb; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = -1.0;
      for (int r = k; r < kNb; ++r) {
        const double m = M[r][k].x * M[r][k].x + M[r][k].y * M[r][k].y;
        if (m > best) {
          best = m;
          p = r;
        }
      }
      piv = best > 0.0 ? p : -1;
    }
    __syncthreads();
    const int p = piv;
    if (p < 0) {
      if (threadIdx.x == 0) atomicOr(flag, 1);
      return;  // uniform across the workgroup
    }
    if (p != k && threadIdx.x < 2 * kNb) {
      const double2 t = M[k][threadIdx.x];
      M[k][threadIdx.x] = M[p][threadIdx.x];
      M[p][threadIdx.x] = t;
    }
    __syncthreads();
    const double2 a = M[k][k];
    const double n2 = a.x * a.x + a.y * a.y;
    const double2 ia = make_double2(a.x / n2, -a.y / n2);
    __syncthreads();
    if (threadIdx.x < 2 * kNb) {
      const double2 v = M[k][threadIdx.x];
      M[k][threadIdx.x] = make_double2(v.x * ia.x - v.y * ia.y, v.x * ia.y + v.y * ia.x);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kNb * 2 * kNb; e += 256) {
      const int r = e / (2 * kNb), c = e % (2 * kNb);
      if (r == k) continue;
      const double2 f = M[r][k], v = M[k][c];
      // M[r][k] itself is read by every column of row r: update it last
      if (c == k) continue;
      M[r][c] = make_double2(M[r][c].x - (f.x * v.x - f.y * v.y), M[r][c].y - (f.x * v.y + f.y * v.x));
    }
    __syncthreads();
    if (threadIdx.x < kNb && threadIdx.x != k) M[threadIdx.x][k] = make_double2(0.0, 0.0);
    __syncthreads();
  }
  double2* o = out + (size_t)site * kNb * kNb;
  for (int e = threadIdx.x; e < kNb * kNb; e += 256) o[e] = M[e / kNb][kNb + e % kNb];
}

hipError_t launch_self_invert(long nsite, const void* B64, void* out, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(self_invert_kernel, dim3((unsigned)nsite), dim3(256), 0, s, static_cast<const double2*>(B64),
                     static_cast<double2*>(out), flag);
  return hipGetLastError();
}

// Packs nblk FP64 Nb x Nb blocks into the BF16 / FP16 (f16) or FP32 operand orders.
hipError_t launch_pack_block_list(int kind, const void* B64, void* packed, long nblk, hipStream_t s) {
  const long n = nblk * kNb * kNb;
  const int blocks = (int)((n + 255) / 256);
  if (kind == 0)
    hipLaunchKernelGGL(pack_f32_kernel, dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(B64),
                       static_cast<float*>(packed), nblk);
  else if (kind == 2)
    hipLaunchKernelGGL((pack_kernel<true>), dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(B64),
                       static_cast<unsigned short*>(packed), nblk);
  else
    hipLaunchKernelGGL((pack_kernel<false>), dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(B64),
                       static_cast<unsigned short*>(packed), nblk);
  return hipGetLastError();
}

hipError_t launch_coarse_mfma_f32(const Geom& g, int nb, int nrhs, const void* packed, const void* in, void* out,
                                  hipStream_t s) {
  if (nb != kNb) return hipErrorInvalidValue;
  const int blocks = (int)((long)g.V * ((nrhs + 31) / 32));  // one workgroup per (site, 32-column tile)
  const int grid = ((blocks + 7) / 8) * 8;
  hipLaunchKernelGGL((coarse_mfma_f32_kernel<0>), dim3(grid), dim3(256), 0, s, g, nrhs,
                     static_cast<const float4*>(packed), static_cast<const float2*>(in), static_cast<float2*>(out),
                     blocks, 0, 9);
  return hipGetLastError();
}

// Packs both low-precision copies of a level's blocks from the FP64 master.
mrhs_status pack_blocks_mfma(mrhs_mg mg, int level) {
  LevelData& L = mg->lv[level];
  if (!mfma_supported(L.ncomp)) return MRHS_OK;
  mrhs_ctx ctx = mg->ctx;
  const size_t bytes = mfma_pack_bytes(L.g.V);
  mrhs_status st = ensure(ctx, L.Bbf16, bytes);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, L.Bf16, bytes);
  if (st != MRHS_OK) return st;
  st = ensure(ctx, L.Bf32p, 2 * bytes);
  if (st != MRHS_OK) return st;
  MRHS_HIP(ctx, launch_pack_blocks(0, L.B64.p, L.Bbf16.p, L.g.V, ctx->stream));
  MRHS_HIP(ctx, launch_pack_blocks(1, L.B64.p, L.Bf16.p, L.g.V, ctx->stream));
  const long n = (long)L.g.V * 9 * kNb * kNb;
  hipLaunchKernelGGL(pack_f32_kernel, dim3((int)((n + 255) / 256)), dim3(256), 0, ctx->stream,
                     static_cast<const double2*>(L.B64.p), static_cast<float*>(L.Bf32p.p), (long)L.g.V * 9);
  MRHS_HIP(ctx, hipGetLastError());
  return MRHS_OK;
}

}  // namespace mrhs
