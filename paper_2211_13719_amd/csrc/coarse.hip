// Coarse-level operator on Nrhs vectors at once (paper Sec. 6: the coarse
// hopping term and the coarse clover term, which on an aggregation level form
// one 9-point stencil of dense Nb x Nb complex blocks):
//
//   (D_c e)(A) = sum_d B_d(A) e(A + d),   d in (self, +x, -x, +y, -y, +z, -z, +t, -t),
//
// periodic in every direction with no boundary phase (the fine antiperiodic
// factor is already inside the blocks).  This file holds the vector-ALU path
// for FP32 and FP64 operands; the BF16/FP16 matrix-core path is in
// coarse_mfma.hip.
//
// Blocks are kept transposed, [site][d][j][i] (column index j outer), so the
// four rows a thread needs at one j are one contiguous load.  A thread owns a
// 4 (rows) x 4 (RHS) output tile of one site and accumulates all nine
// directions in a fixed order.
//
// The same kernel applies the direction-resolved pieces the Galerkin
// construction of the next level needs (filter below): with the next level's
// aggregate extent b, sign 0 keeps the self block and every hop whose source
// stays inside the aggregate of the output site, sign +1 (-1) with direction
// mu keeps only the +mu (-mu) hops that leave the aggregate through its +mu
// (-mu) face.
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

constexpr int kTI = 4, kTR = 4;

__device__ __forceinline__ bool keep_dir(const DirFilter& f, int d, const int (&x)[4]) {
  if (f.sign == 2) return true;
  if (d == 0) return f.sign == 0;
  const int mu = (d - 1) >> 1;
  const bool fwd = ((d - 1) & 1) == 0;
  const int c = x[mu] % f.b[mu];
  const bool on_face = fwd ? (c == f.b[mu] - 1) : (c == 0);
  if (f.sign == 0) return !on_face;
  if (f.mu != mu) return false;
  return (fwd ? f.sign == 1 : f.sign == -1) && on_face;
}

template <typename T>
__global__ __launch_bounds__(256) void coarse_valu_kernel(Geom g, int nb, int nrhs, const cplx<T>* __restrict__ BT,
                                                          const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                          DirFilter f) {
  const int G = (nrhs + kTR - 1) / kTR;
  const int IG = nb / kTI;
  const long gid = (long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (long)g.V * IG * G) return;
  const int kg = (int)(gid % G);
  const int ig = (int)((gid / G) % IG);
  const int s = (int)(gid / ((long)G * IG));
  const int k0 = kg * kTR, i0 = ig * kTI;
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
  cplx<T> acc[kTI][kTR];
#pragma unroll
  for (int i = 0; i < kTI; ++i)
#pragma unroll
    for (int k = 0; k < kTR; ++k) acc[i][k] = mk<T>(0, 0);

  for (int d = 0; d < 9; ++d) {
    if (!keep_dir(f, d, x)) continue;
    int nbr = s;
    if (d > 0) {
      const int mu = (d - 1) >> 1;
      const int step = ((d - 1) & 1) ? -1 : 1;
      const int c = x[mu] + step;
      const int cw = c < 0 ? g.L[mu] - 1 : (c >= g.L[mu] ? 0 : c);
      nbr = s + (cw - x[mu]) * g.stride[mu];
    }
    const cplx<T>* bp = BT + ((size_t)s * 9 + d) * nb * nb + i0;
    const cplx<T>* ep = in + (size_t)nbr * nb * nrhs + k0;
    for (int j = 0; j < nb; ++j) {
      cplx<T> bv[kTI], ev[kTR];
#pragma unroll
      for (int i = 0; i < kTI; ++i) bv[i] = bp[(size_t)j * nb + i];
#pragma unroll
      for (int k = 0; k < kTR; ++k) ev[k] = (k0 + k < nrhs) ? ep[(size_t)j * nrhs + k] : mk<T>(0, 0);
#pragma unroll
      for (int i = 0; i < kTI; ++i)
#pragma unroll
        for (int k = 0; k < kTR; ++k) {
          acc[i][k].x = fma(bv[i].x, ev[k].x, acc[i][k].x);
          acc[i][k].x = fma(-bv[i].y, ev[k].y, acc[i][k].x);
          acc[i][k].y = fma(bv[i].x, ev[k].y, acc[i][k].y);
          acc[i][k].y = fma(bv[i].y, ev[k].x, acc[i][k].y);
        }
    }
  }
  cplx<T>* op = out + ((size_t)s * nb + i0) * nrhs + k0;
#pragma unroll
  for (int i = 0; i < kTI; ++i)
#pragma unroll
    for (int k = 0; k < kTR; ++k)
      if (k0 + k < nrhs) op[(size_t)i * nrhs + k] = acc[i][k];
}

// [site][9][i][j] (interface) <-> [site][9][j][i] (transposed), with a precision change.
template <typename Tin, typename Tout>
__global__ void block_transpose(const cplx<Tin>* __restrict__ in, cplx<Tout>* __restrict__ out, long nblk, int nb) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long per = (long)nb * nb;
  if (e >= nblk * per) return;
  const long q = e / per;
  const int r = (int)(e % per);
  const int i = r / nb, j = r % nb;
  const cplx<Tin> v = in[e];
  out[q * per + (long)j * nb + i] = mk<Tout>((Tout)v.x, (Tout)v.y);
}

// Columns of the chirality-split basis as an Nb-column field: W[s][c][chi*nv + j] =
// v_j(s)_c if component c has chirality chi, else 0.  basis is [s][ncomp][nv].
template <typename T>
__global__ void basis_columns(const cplx<T>* __restrict__ basis, cplx<T>* __restrict__ W, long nsite, int ncomp,
                              int nv) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const int nbc = 2 * nv;
  if (e >= nsite * ncomp * nbc) return;
  const int col = (int)(e % nbc);
  const int c = (int)((e / nbc) % ncomp);
  const long s = e / ((long)nbc * ncomp);
  const int chi = col / nv, j = col % nv;
  const int h = ncomp / 2;
  W[e] = (c / h == chi) ? basis[(s * ncomp + c) * nv + j] : mk<T>(0, 0);
}

}  // namespace

hipError_t launch_coarse_valu(int prec64, const Geom& g, int nb, int nrhs, const void* BT, const void* in, void* out,
                              const DirFilter& f, hipStream_t s) {
  if (nb % kTI) return hipErrorInvalidValue;
  const long threads = (long)g.V * (nb / kTI) * ((nrhs + kTR - 1) / kTR);
  const int blocks = (int)((threads + 255) / 256);
  if (prec64)
    hipLaunchKernelGGL((coarse_valu_kernel<double>), dim3(blocks), dim3(256), 0, s, g, nb, nrhs,
                       static_cast<const double2*>(BT), static_cast<const double2*>(in), static_cast<double2*>(out), f);
  else
    hipLaunchKernelGGL((coarse_valu_kernel<float>), dim3(blocks), dim3(256), 0, s, g, nb, nrhs,
                       static_cast<const float2*>(BT), static_cast<const float2*>(in), static_cast<float2*>(out), f);
  return hipGetLastError();
}

hipError_t launch_block_transpose(const void* in, int in64, void* out, int out64, long nblk, int nb, hipStream_t s) {
  const long n = nblk * nb * nb;
  const int blocks = (int)((n + 255) / 256);
  if (in64 && out64)
    hipLaunchKernelGGL((block_transpose<double, double>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const double2*>(in), static_cast<double2*>(out), nblk, nb);
  else if (in64)
    hipLaunchKernelGGL((block_transpose<double, float>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const double2*>(in), static_cast<float2*>(out), nblk, nb);
  else if (out64)
    hipLaunchKernelGGL((block_transpose<float, double>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const float2*>(in), static_cast<double2*>(out), nblk, nb);
  else
    hipLaunchKernelGGL((block_transpose<float, float>), dim3(blocks), dim3(256), 0, s, static_cast<const float2*>(in),
                       static_cast<float2*>(out), nblk, nb);
  return hipGetLastError();
}

hipError_t launch_basis_columns(int prec64, const void* basis, void* W, long nsite, int ncomp, int nv, hipStream_t s) {
  const long n = nsite * ncomp * 2 * nv;
  const int blocks = (int)((n + 255) / 256);
  if (prec64)
    hipLaunchKernelGGL((basis_columns<double>), dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(basis),
                       static_cast<double2*>(W), nsite, ncomp, nv);
  else
    hipLaunchKernelGGL((basis_columns<float>), dim3(blocks), dim3(256), 0, s, static_cast<const float2*>(basis),
                       static_cast<float2*>(W), nsite, ncomp, nv);
  return hipGetLastError();
}

}  // namespace mrhs
