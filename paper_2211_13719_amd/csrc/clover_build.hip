// Construction of the site-diagonal clover term in FP64 (paper Sec. 4: the
// "precomputed clover term" that M_ooee applies).
//
//   A(x) = 1 + i csw kappa sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x),
//   F_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / 8,
//
// Q the sum of the four plaquettes in the mu-nu plane that start and end at
// x.  In the chiral basis sigma_{mu nu} = diag(s+_{mu nu}, s-_{mu nu}) with
// 2x2 blocks: for spatial j < k both blocks are -eps_{jkl} sigma_l, and for
// (k, t) they are +sigma_k and -sigma_k.  A therefore splits into two
// Hermitian 6x6 blocks A_chi (index 3*spin + colour within the chirality),
// stored packed as 6 real diagonal entries and the 15 strictly-lower entries.
//
// Two kernels: one thread per (site, plane) computes F into a scratch array,
// then one thread per (site, chirality) assembles and packs A_chi and writes
// both an FP64 and an FP32 copy.
#include "internal.h"

namespace mrhs {
namespace {

struct c64 {
  double re, im;
};

__device__ __forceinline__ c64 cm(c64 a, c64 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c64 cmc(c64 a, c64 b) {  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

struct M3 {
  c64 e[3][3];
};

__device__ __forceinline__ M3 load_link(const c64* __restrict__ U, int site, int mu) {
  M3 m;
  const c64* p = U + ((size_t)site * 4 + mu) * 9;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) m.e[a][b] = p[3 * a + b];
  return m;
}

// C = A B, C = A B^dag, C = A^dag B
__device__ __forceinline__ M3 mul(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      c64 z = {0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        c64 t = cm(A.e[a][k], B.e[k][b]);
        z.re += t.re;
        z.im += t.im;
      }
      C.e[a][b] = z;
    }
  return C;
}
__device__ __forceinline__ M3 mul_nd(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      c64 z = {0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        c64 t = cmc(B.e[b][k], A.e[a][k]);  // A[a][k] * conj(B[b][k])
        z.re += t.re;
        z.im += t.im;
      }
      C.e[a][b] = z;
    }
  return C;
}
__device__ __forceinline__ M3 mul_dn(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      c64 z = {0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        c64 t = cmc(A.e[k][a], B.e[k][b]);
        z.re += t.re;
        z.im += t.im;
      }
      C.e[a][b] = z;
    }
  return C;
}

__device__ __forceinline__ M3 dag(const M3& A) {
  M3 C;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) C.e[a][b] = {A.e[b][a].re, -A.e[b][a].im};
  return C;
}

__device__ __forceinline__ int step(const Geom& g, int site, int mu, int d) {
  // site index of x + d*mu (d = +1 or -1), periodic
  int r = site;
  int c = 0;
  for (int m = 0; m < 4; ++m) {
    if (m == mu) c = r % g.L[m];
    r /= g.L[m];
  }
  if (d > 0) return (c == g.L[mu] - 1) ? site - (g.L[mu] - 1) * g.stride[mu] : site + g.stride[mu];
  return (c == 0) ? site + (g.L[mu] - 1) * g.stride[mu] : site - g.stride[mu];
}

// plane p = 0..5 <-> (mu, nu) = (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__constant__ int kPlaneMu[6] = {0, 0, 0, 1, 1, 2};
__constant__ int kPlaneNu[6] = {1, 2, 3, 2, 3, 3};

__global__ __launch_bounds__(256) void field_strength_kernel(Geom g, const c64* __restrict__ U,
                                                             c64* __restrict__ F) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)g.V * 6) return;
  const int x = (int)(gid / 6);
  const int p = (int)(gid % 6);
  const int mu = kPlaneMu[p], nu = kPlaneNu[p];
  const int xpm = step(g, x, mu, +1), xpn = step(g, x, nu, +1);
  const int xmm = step(g, x, mu, -1), xmn = step(g, x, nu, -1);
  const int xmm_pn = step(g, xmm, nu, +1), xmm_mn = step(g, xmm, nu, -1);
  const int xpm_mn = step(g, xpm, nu, -1);

  // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
  M3 Q = mul_nd(mul_nd(mul(load_link(U, x, mu), load_link(U, xpm, nu)), load_link(U, xpn, mu)),
                load_link(U, x, nu));
  // leaf 2: U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
  M3 L = mul(mul_nd(mul_nd(load_link(U, x, nu), load_link(U, xmm_pn, mu)), load_link(U, xmm, nu)),
             load_link(U, xmm, mu));
  // leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
  //       = (U_nu(x-mu-nu) U_mu(x-mu))^dag U_mu(x-mu-nu) U_nu(x-nu)
  M3 L3 = mul(mul(dag(mul(load_link(U, xmm_mn, nu), load_link(U, xmm, mu))), load_link(U, xmm_mn, mu)),
              load_link(U, xmn, nu));
  // leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
  M3 L4 = mul_nd(mul(mul_dn(load_link(U, xmn, nu), load_link(U, xmn, mu)), load_link(U, xpm_mn, nu)),
                 load_link(U, x, mu));

  c64* out = F + ((size_t)x * 6 + p) * 9;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const c64 q = {Q.e[a][b].re + L.e[a][b].re + L3.e[a][b].re + L4.e[a][b].re,
                     Q.e[a][b].im + L.e[a][b].im + L3.e[a][b].im + L4.e[a][b].im};
      const c64 qt = {Q.e[b][a].re + L.e[b][a].re + L3.e[b][a].re + L4.e[b][a].re,
                      Q.e[b][a].im + L.e[b][a].im + L3.e[b][a].im + L4.e[b][a].im};
      // (Q - Q^dag)_{ab} / 8
      out[3 * a + b] = {(q.re - qt.re) * 0.125, (q.im + qt.im) * 0.125};
    }
}

// 2x2 chiral pieces of sigma_{mu nu} per plane and chirality, as
// (re, im) of entries [s][t].
__device__ __forceinline__ c64 sigma_piece(int p, int chi, int s, int t) {
  // Pauli matrices
  auto pauli = [](int k, int s, int t) -> c64 {
    if (k == 0) return (s != t) ? c64{1, 0} : c64{0, 0};
    if (k == 1) {
      if (s == 0 && t == 1) return {0, -1};
      if (s == 1 && t == 0) return {0, 1};
      return {0, 0};
    }
    if (s != t) return {0, 0};
    return (s == 0) ? c64{1, 0} : c64{-1, 0};
  };
  switch (p) {
    case 0: {  // (x,y): -sigma_z on both
      c64 v = pauli(2, s, t);
      return {-v.re, -v.im};
    }
    case 1: {  // (x,z): -eps_{x z y} sigma_y = +sigma_y
      return pauli(1, s, t);
    }
    case 3: {  // (y,z): -sigma_x
      c64 v = pauli(0, s, t);
      return {-v.re, -v.im};
    }
    default: {  // (k,t): +sigma_k for chi=+, -sigma_k for chi=-
      const int k = (p == 2) ? 0 : (p == 4) ? 1 : 2;
      c64 v = pauli(k, s, t);
      return chi == 0 ? v : c64{-v.re, -v.im};
    }
  }
}

__global__ __launch_bounds__(256) void clover_pack_kernel(int V, double csw, double kappa,
                                                          const c64* __restrict__ F,
                                                          double* __restrict__ A64,
                                                          float* __restrict__ A32) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)V * 2) return;
  const int x = (int)(gid >> 1);
  const int chi = (int)(gid & 1);
  const double ck = csw * kappa;
  const c64* f = F + (size_t)x * 6 * 9;
  // entry (i, j) of A_chi, i = 3s + a, j = 3t + b:
  //   delta_ij + i ck sum_p sigma_p[s][t] F_p[a][b]
  auto entry = [&](int i, int j) -> c64 {
    const int s = i / 3, a = i % 3, t = j / 3, b = j % 3;
    c64 z = {0, 0};
    for (int p = 0; p < 6; ++p) {
      const c64 sg = sigma_piece(p, chi, s, t);
      if (sg.re == 0 && sg.im == 0) continue;
      const c64 v = cm(sg, f[p * 9 + 3 * a + b]);
      z.re += v.re;
      z.im += v.im;
    }
    // multiply by i*ck
    c64 r = {-ck * z.im, ck * z.re};
    if (i == j) r.re += 1.0;
    return r;
  };
  double* o64 = A64 + (size_t)gid * 36;
  float* o32 = A32 + (size_t)gid * 36;
  for (int i = 0; i < 6; ++i) {
    const double d = entry(i, i).re;
    o64[i] = d;
    o32[i] = (float)d;
  }
  int k = 6;
  for (int i = 1; i < 6; ++i)
    for (int j = 0; j < i; ++j) {
      const c64 e = entry(i, j);
      o64[k] = e.re;
      o64[k + 1] = e.im;
      o32[k] = (float)e.re;
      o32[k + 1] = (float)e.im;
      k += 2;
    }
}

__global__ void convert_kernel_d2f(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void convert_kernel_f2d(const float* __restrict__ in, double* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

}  // namespace

hipError_t launch_clover_build(const Geom& g, double csw, double kappa, const void* U64, void* F_scratch,
                               void* A64, void* A32, hipStream_t s) {
  const long n1 = (long)g.V * 6;
  hipLaunchKernelGGL(field_strength_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, g,
                     reinterpret_cast<const c64*>(U64), reinterpret_cast<c64*>(F_scratch));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long n2 = (long)g.V * 2;
  hipLaunchKernelGGL(clover_pack_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, g.V, csw, kappa,
                     reinterpret_cast<const c64*>(F_scratch), reinterpret_cast<double*>(A64),
                     reinterpret_cast<float*>(A32));
  return hipGetLastError();
}

hipError_t launch_convert_f64_to_f32(const double* in, float* out, size_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(convert_kernel_d2f, dim3(blocks ? blocks : 1), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_convert_f32_to_f64(const float* in, double* out, size_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(convert_kernel_f2d, dim3(blocks ? blocks : 1), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

namespace {
__global__ void fold_phase_kernel(int nslice, int base, double2* __restrict__ U64, float2* __restrict__ U32,
                                  double ph) {
  const int e = blockIdx.x * 256 + threadIdx.x;  // (site of the last slice, colour pair)
  if (e >= nslice * 9) return;
  const size_t off = ((size_t)(base + e / 9) * 4 + 3) * 9 + e % 9;
  double2 a = U64[off];
  U64[off] = make_double2(ph * a.x, ph * a.y);
  float2 b = U32[off];
  U32[off] = make_float2((float)ph * b.x, (float)ph * b.y);
}
}  // namespace

hipError_t launch_fold_boundary_phase(const Geom& g, int t_bc, void* U64, void* U32, hipStream_t s) {
  if (t_bc == 1) return hipSuccess;
  const int nslice = g.stride[3];  // sites per time slice
  const int base = (g.L[3] - 1) * nslice;
  hipLaunchKernelGGL(fold_phase_kernel, dim3((nslice * 9 + 255) / 256), dim3(256), 0, s, nslice, base,
                     static_cast<double2*>(U64), static_cast<float2*>(U32), (double)t_bc);
  return hipGetLastError();
}

}  // namespace mrhs
