// Restriction and prolongation on the matrix cores (paper Sec. 5, with
// n_v = 16 basis vectors per chirality): with Nrhs right-hand sides both are,
// per (aggregate A, chirality chi), complex GEMMs
//
//   restrict:  Y = W^dag F     (16 x R) = (16 x R_A)^dag (R_A x Nrhs)
//   prolong:   F = W Y         (R_A x Nrhs) = (R_A x 16) (16 x Nrhs)
//
// where R_A = (sites of A) x (h components of chi) and W holds the 16 basis
// vectors restricted to (A, chi).  They run as v_mfma_f32_32x32x16_bf16 with
// FP32 accumulation on the real form of the complex product:
//
//   restrict: rows 0..15 of the 32 x 32 output are Re y_i, rows 16..31 Im y_i,
//             A'[i][(r, re)] = Re w_ri, A'[i][(r, im)] = Im w_ri,
//             A'[16 + i][(r, re)] = -Im w_ri, A'[16 + i][(r, im)] = Re w_ri,
//             B'[(r, re|im)][k] = Re|Im f_rk;
//   prolong:  rows 0..15 are Re f_r, rows 16..31 Im f_r of 16 consecutive r,
//             A'[r][(i, re)] = Re w_ri, A'[r][(i, im)] = -Im w_ri,
//             A'[16 + r][(i, re)] = Im w_ri, A'[16 + r][(i, im)] = Re w_ri,
//             B'[(i, re|im)][k] = Re|Im y_ik.
//
// With the MFMA layouts A[l % 32][8 (l / 32) + q], B[8 (l / 32) + q][l % 32]
// and D[8 (p / 4) + 4 (l / 32) + p % 4][l % 32] (accumulator p), the real and
// imaginary part of one output sit in accumulators p and p + 8 of the same
// lane, so every store is one complex value and 32 lanes write 256
// contiguous bytes.  Rows r of (A, chi) are ordered component-major,
// r = c * (sites of A) + l, so a lane's consecutive rows are consecutive
// sites of one component.
//
// The basis is a BF16 copy of the FP32 basis (round to nearest even, one
// 32-bit word per complex value, re in the low half); the fine and coarse
// fields stay FP32 in memory and are rounded to BF16 on the fly by the
// hardware conversion (round to nearest even).  Products of BF16 values are
// exact in FP32, so the only other rounding is the FP32 accumulation.
//
// The FP32 variants use v_mfma_f32_32x32x2_f32 on the FP32 basis with the
// same real form: one contraction step is one row r (restrict) or one basis
// index i (prolong) with its real and imaginary part as the two k values,
// A[l % 32][k = l / 32], B[k = l / 32][l % 32].
#include "agg.h"
#include "internal.h"
#include "rounding.h"

namespace mrhs {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

constexpr int kNV = 16;

// The fine sites of aggregate A are computed once per workgroup into LDS:
// the site of an offset takes a chain of integer divisions by run-time
// extents, which per use would cost more vector instructions than the matrix
// products.  Aggregates of up to kAggTab sites (8^4) take these kernels.
constexpr int kAggTab = 4096;

struct AggSites {
  const int* tab;
  __device__ __forceinline__ int operator()(int l) const { return tab[l]; }
};

// Fills tab (every thread of the workgroup takes part; ends with a barrier).
__device__ __forceinline__ AggSites agg_sites(const AggGeom& a, int A, int nsa, int* tab) {
  for (int l = threadIdx.x; l < nsa; l += blockDim.x) tab[l] = agg_site(a, A, l);
  __syncthreads();
  return AggSites{tab};
}

__device__ __forceinline__ bf16x8 to_bf16(const float (&x)[8]) {
  bf16x8 v;
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = (__bf16)x[q];
  return v;
}

// One workgroup per (aggregate, chirality, 32-column tile); its four
// wavefronts take a quarter of the rows each and are summed through LDS in a
// fixed order.
__global__ __launch_bounds__(256) void restrict_bf16_kernel(AggGeom a, int h, int nrhs, int ntile,
                                                            const unsigned* __restrict__ W,
                                                            const float2* __restrict__ f, float2* __restrict__ y) {
  __shared__ float red[3][64][16];
  const int bid = blockIdx.x;
  const int tile = bid % ntile;
  const int chi = (bid / ntile) & 1;
  const int A = bid / ntile >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 31, g = lane >> 5;
  const int ncomp = 2 * h;
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  const int per_c = nsa / 8;  // MFMA steps per component
  const int steps = h * per_c;
  const int s0 = wave * steps / 4, s1 = (wave + 1) * steps / 4;
  const int k = tile * 32 + m;
  const bool kin = k < nrhs;
  const int i = m & 15;
  const bool imrow = m >= 16;
  __shared__ int stab[kAggTab];
  const AggSites site_of = agg_sites(a, A, nsa, stab);
  f32x16 acc = {};
  // four MFMA steps' loads in flight together, from clamped addresses with
  // the operands zeroed instead of branching (steps past the end and
  // columns past nrhs add zero products)
  constexpr int U = 4;
  const int kc = kin ? k : nrhs - 1;
  for (int s = s0; s < s1; s += U) {
    u32x4 av[U];
    float bv[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = s + u < s1;
      const int su = in ? s + u : s0;
      const int c = su / per_c;
      const int l0 = (su - c * per_c) * 8 + 4 * g;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int site = site_of(l0 + j);
        const size_t row = (size_t)site * ncomp + chi * h + c;
        const unsigned w = W[row * kNV + i];
        const float2 v = f[row * nrhs + kc];
        const unsigned x = imrow ? (((w >> 16) ^ 0x8000u) | (w << 16)) : w;
        av[u][j] = in ? x : 0u;
        bv[u][2 * j] = (in && kin) ? v.x : 0.f;
        bv[u][2 * j + 1] = (in && kin) ? v.y : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[u]), to_bf16(bv[u]), acc, 0, 0, 0);
  }
  if (wave > 0) {
#pragma unroll
    for (int p = 0; p < 16; ++p) red[wave - 1][lane][p] = acc[p];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int p = 0; p < 16; ++p) acc[p] += red[w][lane][p];
    if (kin) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int row = 8 * (p / 4) + 4 * g + (p % 4);
        y[((size_t)A * 2 * kNV + chi * kNV + row) * nrhs + k] = make_float2(acc[p], acc[p + 8]);
      }
    }
  }
}

// One workgroup per (aggregate, chirality, 32-column tile); the coarse
// values are loaded once, and the four wavefronts walk the 16-row tiles of
// the aggregate in turn.
__global__ __launch_bounds__(256) void prolong_bf16_kernel(AggGeom a, int h, int nrhs, int ntile,
                                                           const unsigned* __restrict__ W,
                                                           const float2* __restrict__ y, float2* __restrict__ f) {
  const int bid = blockIdx.x;
  const int tile = bid % ntile;
  const int chi = (bid / ntile) & 1;
  const int A = bid / ntile >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 31, g = lane >> 5;
  const int ncomp = 2 * h;
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  const int k = tile * 32 + m;
  const bool kin = k < nrhs;
  const bool imrow = m >= 16;
  __shared__ int stab[kAggTab];
  const AggSites site_of = agg_sites(a, A, nsa, stab);
  bf16x8 B[2];
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    float bv[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = st * 8 + 4 * g + j;
      // clamped column, zeroed past nrhs (no branch around the loads)
      const float2 v = y[((size_t)A * 2 * kNV + chi * kNV + i) * nrhs + (kin ? k : nrhs - 1)];
      bv[2 * j] = kin ? v.x : 0.f;
      bv[2 * j + 1] = kin ? v.y : 0.f;
    }
    B[st] = to_bf16(bv);
  }
  const int ntr = h * nsa / 16;
  // Software pipeline over the row tiles of the wavefront (t, t + 4, ...):
  // the basis loads of the next tile are issued before the matrix
  // instructions of the current one.  A tile past the end loads the first
  // tile's rows again and writes nothing.
  auto load = [&](int t, u32x4 (&wt)[2]) {
    const int tc = t < ntr ? t : wave;
    const int r0 = tc * 16;
    const int c = r0 / nsa;
    const int l0 = r0 - c * nsa;
    // A operand: row r0 + (m & 15)
    const size_t arow = (size_t)site_of(l0 + (m & 15)) * ncomp + chi * h + c;
#pragma unroll
    for (int st = 0; st < 2; ++st) wt[st] = *reinterpret_cast<const u32x4*>(W + arow * kNV + st * 8 + 4 * g);
  };
  auto row_tile = [&](int t, const u32x4 (&wt)[2]) {
    const int r0 = t * 16;
    const int c = r0 / nsa;
    const int l0 = r0 - c * nsa;
    f32x16 acc = {};
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      u32x4 w = wt[st];
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = imrow ? ((w[j] >> 16) | (w[j] << 16)) : (w[j] ^ 0x80000000u);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, w), B[st], acc, 0, 0, 0);
    }
    if (kin && t < ntr) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int lb = l0 + 8 * half + 4 * g;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int site = site_of(lb + j);
          const int p = 4 * half + j;
          f[((size_t)site * ncomp + chi * h + c) * nrhs + k] = make_float2(acc[p], acc[p + 8]);
        }
      }
    }
  };
  u32x4 wA[2], wB[2];
  if (wave < ntr) load(wave, wA);
  for (int t = wave; t < ntr; t += 8) {
    load(t + 4, wB);
    row_tile(t, wA);
    load(t + 8, wA);
    row_tile(t + 4, wB);
  }
}

// FP32 restrict on the FP32 matrix cores; workgroup and wavefront split as
// in restrict_bf16_kernel, the rows of (A, chi) taken site by site (all h
// components of a site in turn).  H > 0 fixes h at compile time, so that the
// loads of a site are issued together (H = 0: any h).
template <int H>
__global__ __launch_bounds__(256) void restrict_f32_kernel(AggGeom a, int h, int nrhs, int ntile,
                                                           const float2* __restrict__ W,
                                                           const float2* __restrict__ f, float2* __restrict__ y) {
  __shared__ float red[3][64][16];
  const int bid = blockIdx.x;
  const int tile = bid % ntile;
  const int chi = (bid / ntile) & 1;
  const int A = bid / ntile >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 31, g = lane >> 5;
  const int ncomp = 2 * h;
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  const int l0 = wave * nsa / 4, l1 = (wave + 1) * nsa / 4;
  const int k = tile * 32 + m;
  const bool kin = k < nrhs;
  const int i = m & 15;
  const bool imrow = m >= 16;
  __shared__ int stab[kAggTab];
  const AggSites site_of = agg_sites(a, A, nsa, stab);
  f32x16 acc = {};
  if constexpr (H > 0) {
    // Software pipeline over the sites of the wavefront: the loads of the
    // next US sites are issued before the matrix instructions of the current
    // ones (the compiler does not unroll a loop around the matrix
    // instruction by itself).  Addresses are clamped to valid ones and the
    // operands zeroed instead of branching, so a site past the end and a
    // column past nrhs add zero products.
    constexpr int US = H <= 8 ? 2 : 1;
    const int kc = kin ? k : nrhs - 1;
    auto load = [&](int lb, float2 (&w)[US][H], float2 (&v)[US][H]) {
#pragma unroll
      for (int u = 0; u < US; ++u) {
        const size_t row0 = (size_t)site_of(lb + u < l1 ? lb + u : l0) * ncomp + chi * H;
#pragma unroll
        for (int c = 0; c < H; ++c) {
          w[u][c] = W[(row0 + c) * kNV + i];
          v[u][c] = f[(row0 + c) * nrhs + kc];
        }
      }
    };
    auto mma = [&](int lb, const float2 (&w)[US][H], const float2 (&v)[US][H]) {
#pragma unroll
      for (int u = 0; u < US; ++u) {
        const bool in = lb + u < l1;
#pragma unroll
        for (int c = 0; c < H; ++c) {
          // g = 0: coefficient of Re f, g = 1: of Im f
          const float x = imrow ? (g ? w[u][c].x : -w[u][c].y) : (g ? w[u][c].y : w[u][c].x);
          const float av = in ? x : 0.f;
          const float bv = (in && kin) ? (g ? v[u][c].y : v[u][c].x) : 0.f;
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
      }
    };
    float2 wA[US][H], vA[US][H], wB[US][H], vB[US][H];
    if (l0 < l1) load(l0, wA, vA);
    for (int l = l0; l < l1; l += 2 * US) {
      load(l + US, wB, vB);
      mma(l, wA, vA);
      load(l + 2 * US, wA, vA);
      mma(l + US, wB, vB);
    }
  } else {
    for (int l = l0; l < l1; ++l) {
      const size_t row0 = (size_t)site_of(l) * ncomp + chi * h;
      for (int c = 0; c < h; ++c) {
        const float2 wc = W[(row0 + c) * kNV + i];
        const float2 vc = kin ? f[(row0 + c) * nrhs + k] : make_float2(0.f, 0.f);
        const float av = imrow ? (g ? wc.x : -wc.y) : (g ? wc.y : wc.x);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, g ? vc.y : vc.x, acc, 0, 0, 0);
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int p = 0; p < 16; ++p) red[wave - 1][lane][p] = acc[p];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int p = 0; p < 16; ++p) acc[p] += red[w][lane][p];
    if (kin) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int r = 8 * (p / 4) + 4 * g + (p % 4);
        y[((size_t)A * 2 * kNV + chi * kNV + r) * nrhs + k] = make_float2(acc[p], acc[p + 8]);
      }
    }
  }
}

// FP32 prolong on the FP32 matrix cores: as prolong_bf16_kernel, sixteen
// contraction steps (one per basis index) per 16-row tile.
__global__ __launch_bounds__(256) void prolong_f32_kernel(AggGeom a, int h, int nrhs, int ntile,
                                                          const float2* __restrict__ W,
                                                          const float2* __restrict__ y, float2* __restrict__ f) {
  const int bid = blockIdx.x;
  const int tile = bid % ntile;
  const int chi = (bid / ntile) & 1;
  const int A = bid / ntile >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 31, g = lane >> 5;
  const int ncomp = 2 * h;
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  const int k = tile * 32 + m;
  const bool kin = k < nrhs;
  const bool imrow = m >= 16;
  __shared__ int stab[kAggTab];
  const AggSites site_of = agg_sites(a, A, nsa, stab);
  float bv[kNV];
#pragma unroll
  for (int i = 0; i < kNV; ++i) {
    // a column past nrhs reads column nrhs - 1: B column k feeds only output
    // column k, which is not stored (and a select here would let the
    // compiler put each load behind a branch of its own)
    const float2 v = y[((size_t)A * 2 * kNV + chi * kNV + i) * nrhs + (kin ? k : nrhs - 1)];
    bv[i] = g ? v.y : v.x;
  }
  const int ntr = h * nsa / 16;
  // Software pipeline over the row tiles of the wavefront (t, t + 4, ...):
  // the basis loads of the next tile are issued before the matrix
  // instructions of the current one.  A tile past the end loads the first
  // tile's rows again and writes nothing.
  auto load = [&](int t, float4 (&wt)[kNV / 2]) {
    const int tc = t < ntr ? t : wave;
    const int r0 = tc * 16;
    const int c = r0 / nsa;
    const int lb0 = r0 - c * nsa;
    const size_t arow = (size_t)site_of(lb0 + (m & 15)) * ncomp + chi * h + c;
    const float4* wr = reinterpret_cast<const float4*>(W + arow * kNV);
#pragma unroll
    for (int q = 0; q < kNV / 2; ++q) wt[q] = wr[q];  // basis values i = 2q and 2q + 1
  };
  auto row_tile = [&](int t, const float4 (&wt)[kNV / 2]) {
    const int r0 = t * 16;
    const int c = r0 / nsa;
    const int lb0 = r0 - c * nsa;
    f32x16 acc = {};
#pragma unroll
    for (int q = 0; q < kNV / 2; ++q) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float wre = e ? wt[q].z : wt[q].x, wim = e ? wt[q].w : wt[q].y;
        // g = 0: coefficient of Re y, g = 1: of Im y
        const float av = imrow ? (g ? wre : wim) : (g ? -wim : wre);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[2 * q + e], acc, 0, 0, 0);
      }
    }
    if (kin && t < ntr) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int lb = lb0 + 8 * half + 4 * g;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int site = site_of(lb + j);
          const int p = 4 * half + j;
          f[((size_t)site * ncomp + chi * h + c) * nrhs + k] = make_float2(acc[p], acc[p + 8]);
        }
      }
    }
  };
  float4 wA[kNV / 2], wB[kNV / 2];
  if (wave < ntr) load(wave, wA);
  for (int t = wave; t < ntr; t += 8) {
    load(t + 4, wB);
    row_tile(t, wA);
    load(t + 8, wA);
    row_tile(t + 4, wB);
  }
}

// FP32 basis [site][ncomp][16] complex -> BF16 pairs (round to nearest even).
__global__ __launch_bounds__(256) void pack_basis_bf16_kernel(const float2* __restrict__ in, unsigned* __restrict__ out,
                                                              long n) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float2 v = in[e];
  out[e] = (unsigned)bf16_rne_bits(__float_as_uint(v.x)) | ((unsigned)bf16_rne_bits(__float_as_uint(v.y)) << 16);
}

}  // namespace

bool intergrid_mfma_supported(const AggGeom& a, int h, int nv) {
  const int nsa = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  return nv == kNV && h >= 1 && nsa % 16 == 0 && nsa <= kAggTab;
}

hipError_t launch_pack_basis_bf16(const void* basis32, void* out, long ncomplex, hipStream_t s) {
  hipLaunchKernelGGL(pack_basis_bf16_kernel, dim3((unsigned)((ncomplex + 255) / 256)), dim3(256), 0, s,
                     static_cast<const float2*>(basis32), static_cast<unsigned*>(out), ncomplex);
  return hipGetLastError();
}

hipError_t launch_restrict_bf16(const AggGeom& a, int h, int nrhs, const void* Wbf16, const void* f, void* y,
                                hipStream_t s) {
  if (!intergrid_mfma_supported(a, h, kNV)) return hipErrorInvalidValue;
  const int ntile = (nrhs + 31) / 32;
  hipLaunchKernelGGL(restrict_bf16_kernel, dim3((unsigned)(a.Vc * 2 * ntile)), dim3(256), 0, s, a, h, nrhs, ntile,
                     static_cast<const unsigned*>(Wbf16), static_cast<const float2*>(f), static_cast<float2*>(y));
  return hipGetLastError();
}

hipError_t launch_prolong_bf16(const AggGeom& a, int h, int nrhs, const void* Wbf16, const void* y, void* f,
                               hipStream_t s) {
  if (!intergrid_mfma_supported(a, h, kNV)) return hipErrorInvalidValue;
  const int ntile = (nrhs + 31) / 32;
  hipLaunchKernelGGL(prolong_bf16_kernel, dim3((unsigned)(a.Vc * 2 * ntile)), dim3(256), 0, s, a, h, nrhs, ntile,
                     static_cast<const unsigned*>(Wbf16), static_cast<const float2*>(y), static_cast<float2*>(f));
  return hipGetLastError();
}

hipError_t launch_restrict_f32mfma(const AggGeom& a, int h, int nrhs, const void* W32, const void* f, void* y,
                                   hipStream_t s) {
  if (!intergrid_mfma_supported(a, h, kNV)) return hipErrorInvalidValue;
  const int ntile = (nrhs + 31) / 32;
  const dim3 grid((unsigned)(a.Vc * 2 * ntile));
  const auto* w = static_cast<const float2*>(W32);
  const auto* fi = static_cast<const float2*>(f);
  auto* yo = static_cast<float2*>(y);
  if (h == 6)
    hipLaunchKernelGGL(restrict_f32_kernel<6>, grid, dim3(256), 0, s, a, h, nrhs, ntile, w, fi, yo);
  else if (h == 16)
    hipLaunchKernelGGL(restrict_f32_kernel<16>, grid, dim3(256), 0, s, a, h, nrhs, ntile, w, fi, yo);
  else
    hipLaunchKernelGGL(restrict_f32_kernel<0>, grid, dim3(256), 0, s, a, h, nrhs, ntile, w, fi, yo);
  return hipGetLastError();
}

hipError_t launch_prolong_f32mfma(const AggGeom& a, int h, int nrhs, const void* W32, const void* y, void* f,
                                  hipStream_t s) {
  if (!intergrid_mfma_supported(a, h, kNV)) return hipErrorInvalidValue;
  const int ntile = (nrhs + 31) / 32;
  hipLaunchKernelGGL(prolong_f32_kernel, dim3((unsigned)(a.Vc * 2 * ntile)), dim3(256), 0, s, a, h, nrhs, ntile,
                     static_cast<const float2*>(W32), static_cast<const float2*>(y), static_cast<float2*>(f));
  return hipGetLastError();
}

}  // namespace mrhs
