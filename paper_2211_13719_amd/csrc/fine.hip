// Fine-level Wilson-clover operator on Nrhs right-hand sides at once
// (paper Sec. 4: the hopping term D_hop and the clover term M_ooee).
//
//   out = A psi - kappa H psi,   A = 1 + C in two Hermitian 6x6 chiral blocks,
//   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu).
//
// Work decomposition: one thread owns one site and R consecutive right-hand
// sides (R in 1, 2, 4 and the traversal tile below are chosen per Nrhs by the
// autotuner; untuned: R = 2 for even Nrhs in FP32, else 1), or, in the t-walk
// kernels further down, one site of a spatial block, R right-hand sides and a
// run of time slices.  Fields are [site][12][nrhs] complex, so the nrhs/R
// threads of a site are adjacent lanes that read contiguous memory for every
// component, and all
// of them share the site's links and clover blocks (one cache line serves the
// whole group: the gauge-field reuse of Sec. 2).  Each neighbour spinor is
// spin-projected to a half spinor (2 spins x 3 colours) before the SU(3)
// product, which halves the link arithmetic.
//
// The gamma matrices are the chiral basis, gamma_k = [[0, -i s_k], [i s_k, 0]],
// gamma_4 = [[0, 1], [1, 0]].  Writing psi = (u0, u1, l0, l1) in spin, the
// projection (1 -+ gamma_mu) psi has upper half h = (h0, h1) and lower half a
// fixed multiple of h, listed per direction in project()/reconstruct().
#include <type_traits>

#include "internal.h"

namespace mrhs {
namespace {

template <typename T>
struct cplx_t;
template <>
struct cplx_t<float> {
  using type = float2;
};
template <>
struct cplx_t<double> {
  using type = double2;
};

template <typename T>
using cplx = typename cplx_t<T>::type;

template <typename T>
__device__ __forceinline__ cplx<T> mk(T re, T im) {
  cplx<T> z;
  z.x = re;
  z.y = im;
  return z;
}
template <typename T>
__device__ __forceinline__ cplx<T> add(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> sub(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x - b.x, a.y - b.y);
}
// a + i b, a - i b
template <typename T>
__device__ __forceinline__ cplx<T> addi(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x - b.y, a.y + b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> subi(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x + b.y, a.y - b.x);
}
// acc += a * b ; acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cmac(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ void cmac_conj(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// Load R consecutive complex numbers starting at p (R-aligned element offset).
template <typename T, int R>
__device__ __forceinline__ void load_r(const cplx<T>* __restrict__ p, cplx<T> (&v)[R]) {
  if constexpr (sizeof(T) == 4 && R % 2 == 0) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int j = 0; j < R / 2; ++j) {
      float4 w = q[j];
      v[2 * j] = mk<T>(w.x, w.y);
      v[2 * j + 1] = mk<T>(w.z, w.w);
    }
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = p[j];
  }
}

// Load R consecutive input values stored as P (the compute type's complex,
// or FP32 complex widened exactly to FP64 for the mixed-precision FP64 apply).
template <typename T, int R, typename P>
__device__ __forceinline__ void load_in(const P* __restrict__ p, cplx<T> (&v)[R]) {
  if constexpr (std::is_same<P, cplx<T>>::value) {
    load_r<T, R>(p, v);
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const P w = p[j];
      v[j] = mk<T>((T)w.x, (T)w.y);
    }
  }
}

typedef float f32x4_nt __attribute__((ext_vector_type(4)));
typedef float f32x2_nt __attribute__((ext_vector_type(2)));

// nt: non-temporal store (the output is not read again by this kernel, so it
// should not displace neighbour spinors from the caches).
template <typename T, int R>
__device__ __forceinline__ void store_r(cplx<T>* __restrict__ p, const cplx<T> (&v)[R], bool nt = false) {
  if constexpr (sizeof(T) == 4 && R % 2 == 0) {
    float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
    for (int j = 0; j < R / 2; ++j) {
      if (nt) {
        const f32x4_nt w = {v[2 * j].x, v[2 * j].y, v[2 * j + 1].x, v[2 * j + 1].y};
        __builtin_nontemporal_store(w, reinterpret_cast<f32x4_nt*>(q + j));
      } else {
        q[j] = make_float4(v[2 * j].x, v[2 * j].y, v[2 * j + 1].x, v[2 * j + 1].y);
      }
    }
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (nt) {
        const f32x2_nt w = {v[j].x, v[j].y};
        __builtin_nontemporal_store(w, reinterpret_cast<f32x2_nt*>(p + j));
      } else {
        p[j] = v[j];
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) p[j] = v[j];
  }
}

// Half spinor of (1 - s*gamma_mu) psi, s = +1 (forward hop) or -1 (backward hop).
// psi[spin][colour][rhs] -> h[2][3][R]
template <typename T, int R, int MU, int S>
__device__ __forceinline__ void project(const cplx<T> (&p)[4][3][R], cplx<T> (&h)[2][3][R]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if constexpr (MU == 0) {  // gamma_1: h0 = u0 +- i l1, h1 = u1 +- i l0
        h[0][c][j] = S > 0 ? addi<T>(p[0][c][j], p[3][c][j]) : subi<T>(p[0][c][j], p[3][c][j]);
        h[1][c][j] = S > 0 ? addi<T>(p[1][c][j], p[2][c][j]) : subi<T>(p[1][c][j], p[2][c][j]);
      } else if constexpr (MU == 1) {  // gamma_2: h0 = u0 +- l1, h1 = u1 -+ l0
        h[0][c][j] = S > 0 ? add<T>(p[0][c][j], p[3][c][j]) : sub<T>(p[0][c][j], p[3][c][j]);
        h[1][c][j] = S > 0 ? sub<T>(p[1][c][j], p[2][c][j]) : add<T>(p[1][c][j], p[2][c][j]);
      } else if constexpr (MU == 2) {  // gamma_3: h0 = u0 +- i l0, h1 = u1 -+ i l1
        h[0][c][j] = S > 0 ? addi<T>(p[0][c][j], p[2][c][j]) : subi<T>(p[0][c][j], p[2][c][j]);
        h[1][c][j] = S > 0 ? subi<T>(p[1][c][j], p[3][c][j]) : addi<T>(p[1][c][j], p[3][c][j]);
      } else {  // gamma_4: h0 = u0 -+ l0, h1 = u1 -+ l1
        h[0][c][j] = S > 0 ? sub<T>(p[0][c][j], p[2][c][j]) : add<T>(p[0][c][j], p[2][c][j]);
        h[1][c][j] = S > 0 ? sub<T>(p[1][c][j], p[3][c][j]) : add<T>(p[1][c][j], p[3][c][j]);
      }
    }
}

// Spin components that the two halves of (1 - s*gamma_mu) psi combine:
// half 0 uses (0, SA0), half 1 uses (1, SA1) with the lower spin index given
// below (x, y: 3 and 2; z, t: 2 and 3).
template <int MU>
struct HalfPair {
  static constexpr int lo0 = (MU <= 1) ? 3 : 2;
  static constexpr int lo1 = (MU <= 1) ? 2 : 3;
};

// h = half `HALF` of (1 - s*gamma_mu) psi from the upper spin u = psi[HALF]
// and the lower spin l it combines with (see project()).
template <typename T, int R, int MU, int S, int HALF>
__device__ __forceinline__ void project_half(const cplx<T> (&u)[3][R], const cplx<T> (&l)[3][R],
                                             cplx<T> (&h)[3][R]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if constexpr (MU == 0) {  // h0 = u0 +- i l1, h1 = u1 +- i l0
        h[c][j] = S > 0 ? addi<T>(u[c][j], l[c][j]) : subi<T>(u[c][j], l[c][j]);
      } else if constexpr (MU == 1) {  // h0 = u0 +- l1, h1 = u1 -+ l0
        if constexpr (HALF == 0)
          h[c][j] = S > 0 ? add<T>(u[c][j], l[c][j]) : sub<T>(u[c][j], l[c][j]);
        else
          h[c][j] = S > 0 ? sub<T>(u[c][j], l[c][j]) : add<T>(u[c][j], l[c][j]);
      } else if constexpr (MU == 2) {  // h0 = u0 +- i l0, h1 = u1 -+ i l1
        if constexpr (HALF == 0)
          h[c][j] = S > 0 ? addi<T>(u[c][j], l[c][j]) : subi<T>(u[c][j], l[c][j]);
        else
          h[c][j] = S > 0 ? subi<T>(u[c][j], l[c][j]) : addi<T>(u[c][j], l[c][j]);
      } else {  // h0 = u0 -+ l0, h1 = u1 -+ l1
        h[c][j] = S > 0 ? sub<T>(u[c][j], l[c][j]) : add<T>(u[c][j], l[c][j]);
      }
    }
}

// Half spinor h of the neighbour at site nb, loading only the two spin
// components each half needs (keeps half as many values live as loading the
// whole spinor first).
template <typename T, int R, int MU, int S, typename P>
__device__ __forceinline__ void load_project(const P* __restrict__ in, int nb, int nrhs, int k0,
                                             cplx<T> (&h)[2][3][R]) {
  const P* base = in + (size_t)nb * 12 * nrhs + k0;
  {
    cplx<T> u[3][R], l[3][R];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      load_in<T, R>(base + (0 * 3 + c) * nrhs, u[c]);
      load_in<T, R>(base + (HalfPair<MU>::lo0 * 3 + c) * nrhs, l[c]);
    }
    project_half<T, R, MU, S, 0>(u, l, h[0]);
  }
  {
    cplx<T> u[3][R], l[3][R];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      load_in<T, R>(base + (1 * 3 + c) * nrhs, u[c]);
      load_in<T, R>(base + (HalfPair<MU>::lo1 * 3 + c) * nrhs, l[c]);
    }
    project_half<T, R, MU, S, 1>(u, l, h[1]);
  }
}

// One link U_mu(x) (3 x 3 complex, 72 bytes at [site][mu]).  In FP32 the
// matrix starts on a 16-byte boundary for even mu and 8 bytes past one for
// odd mu, so it is read as four 16-byte loads and one 8-byte load.
template <typename T, int MU>
__device__ __forceinline__ void load_link(const cplx<T>* __restrict__ u, cplx<T> (&uu)[3][3]) {
  if constexpr (sizeof(T) == 4) {
    float v[18];
    if constexpr (MU % 2 == 0) {
      const float4* q = reinterpret_cast<const float4*>(u);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float4 w = q[i];
        v[4 * i] = w.x;
        v[4 * i + 1] = w.y;
        v[4 * i + 2] = w.z;
        v[4 * i + 3] = w.w;
      }
      const cplx<T> t = u[8];
      v[16] = t.x;
      v[17] = t.y;
    } else {
      const cplx<T> t = u[0];
      v[0] = t.x;
      v[1] = t.y;
      const float4* q = reinterpret_cast<const float4*>(u + 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float4 w = q[i];
        v[2 + 4 * i] = w.x;
        v[3 + 4 * i] = w.y;
        v[4 + 4 * i] = w.z;
        v[5 + 4 * i] = w.w;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) uu[a][b] = mk<T>(v[2 * (3 * a + b)], v[2 * (3 * a + b) + 1]);
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) uu[a][b] = u[3 * a + b];
  }
}

// acc += (1 - s*gamma_mu)-reconstruction of the transported half spinor w.
template <typename T, int R, int MU, int S>
__device__ __forceinline__ void reconstruct(cplx<T> (&acc)[4][3][R], const cplx<T> (&w)[2][3][R]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const cplx<T> a = w[0][c][j], b = w[1][c][j];
      acc[0][c][j] = add<T>(acc[0][c][j], a);
      acc[1][c][j] = add<T>(acc[1][c][j], b);
      if constexpr (MU == 0) {  // l0 = -+ i h1, l1 = -+ i h0
        acc[2][c][j] = S > 0 ? subi<T>(acc[2][c][j], b) : addi<T>(acc[2][c][j], b);
        acc[3][c][j] = S > 0 ? subi<T>(acc[3][c][j], a) : addi<T>(acc[3][c][j], a);
      } else if constexpr (MU == 1) {  // l0 = -+ h1, l1 = +- h0
        acc[2][c][j] = S > 0 ? sub<T>(acc[2][c][j], b) : add<T>(acc[2][c][j], b);
        acc[3][c][j] = S > 0 ? add<T>(acc[3][c][j], a) : sub<T>(acc[3][c][j], a);
      } else if constexpr (MU == 2) {  // l0 = -+ i h0, l1 = +- i h1
        acc[2][c][j] = S > 0 ? subi<T>(acc[2][c][j], a) : addi<T>(acc[2][c][j], a);
        acc[3][c][j] = S > 0 ? addi<T>(acc[3][c][j], b) : subi<T>(acc[3][c][j], b);
      } else {  // l0 = -+ h0, l1 = -+ h1
        acc[2][c][j] = S > 0 ? sub<T>(acc[2][c][j], a) : add<T>(acc[2][c][j], a);
        acc[3][c][j] = S > 0 ? sub<T>(acc[3][c][j], b) : add<T>(acc[3][c][j], b);
      }
    }
}

// Forces the accumulator to be materialised here.  Without it the compiler
// sinks all arithmetic below the loads of all eight neighbours, which keeps
// eight spinors live at once and exhausts the register file.
template <typename T, int R>
__device__ __forceinline__ void pin(cplx<T> (&acc)[4][3][R]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < R; ++j) asm volatile("" : "+v"(acc[sp][c][j].x), "+v"(acc[sp][c][j].y));
}

template <typename T, int R, typename P>
__device__ __forceinline__ void load_spinor(const P* __restrict__ in, int site, int nrhs, int k0,
                                            cplx<T> (&p)[4][3][R]) {
  const P* base = in + (size_t)site * 12 * nrhs + k0;
  if constexpr (R == 1 && sizeof(T) == 4 && std::is_same<P, cplx<T>>::value) {
    if (nrhs == 1) {  // the whole 96-byte spinor is contiguous: six 16-byte loads
      const float4* q = reinterpret_cast<const float4*>(base);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const float4 w = q[i];
        p[(2 * i) / 3][(2 * i) % 3][0] = mk<T>(w.x, w.y);
        p[(2 * i + 1) / 3][(2 * i + 1) % 3][0] = mk<T>(w.z, w.w);
      }
      return;
    }
  }
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) load_in<T, R>(base + (3 * sp + c) * nrhs, p[sp][c]);
}

// One direction mu, both hops, accumulated into acc.  nbf / nbb are the
// sites x + mu and x - mu.  The fermion boundary factor is already folded
// into the links (see fold_boundary_phase), so no hop needs a phase here.
// lbb, when given, is the site whose link U_mu carries the backward hop (on a
// checkerboarded field the spinor index nbb and the lattice site differ).
template <typename T, int R, int MU, bool SPLIT, typename P>
__device__ __forceinline__ void hop_dir(int site, int nbf, int nbb, int nrhs, int k0, const cplx<T>* __restrict__ U,
                                        const P* __restrict__ in, cplx<T> (&acc)[4][3][R], bool inc_f = true,
                                        bool inc_b = true, int lbb = -1) {
  // With one FP32 right-hand side the whole 96-byte spinor is contiguous and
  // six 16-byte loads fetch it, half the load instructions of the split path
  // (twelve 8-byte loads), so that case projects after a full load.
  const bool split = SPLIT && !(R == 1 && sizeof(T) == 4 && std::is_same<P, cplx<T>>::value && nrhs == 1);
  // forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
  if (inc_f) {
    cplx<T> h[2][3][R];
    if (split) {
      load_project<T, R, MU, +1>(in, nbf, nrhs, k0, h);
    } else {
      cplx<T> p[4][3][R];
      load_spinor<T, R>(in, nbf, nrhs, k0, p);
      project<T, R, MU, +1>(p, h);
    }
    cplx<T> uu[3][3];
    load_link<T, MU>(U + ((size_t)site * 4 + MU) * 9, uu);
    cplx<T> w[2][3][R];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int j = 0; j < R; ++j)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          cplx<T> z = mk<T>(0, 0);
#pragma unroll
          for (int b = 0; b < 3; ++b) cmac<T>(z, uu[a][b], h[s][b][j]);
          w[s][a][j] = z;
        }
    reconstruct<T, R, MU, +1>(acc, w);
    pin<T, R>(acc);
  }
  // backward: (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
  if (inc_b) {
    cplx<T> h[2][3][R];
    if (split) {
      load_project<T, R, MU, -1>(in, nbb, nrhs, k0, h);
    } else {
      cplx<T> p[4][3][R];
      load_spinor<T, R>(in, nbb, nrhs, k0, p);
      project<T, R, MU, -1>(p, h);
    }
    cplx<T> uu[3][3];
    load_link<T, MU>(U + ((size_t)(lbb < 0 ? nbb : lbb) * 4 + MU) * 9, uu);
    cplx<T> w[2][3][R];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int j = 0; j < R; ++j)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          cplx<T> z = mk<T>(0, 0);
#pragma unroll
          for (int b = 0; b < 3; ++b) cmac_conj<T>(z, uu[b][a], h[s][b][j]);
          w[s][a][j] = z;
        }
    reconstruct<T, R, MU, -1>(acc, w);
    pin<T, R>(acc);
  }
}

// One chiral 6x6 block times six components (R right-hand sides each).
template <typename T, int R>
__device__ __forceinline__ void clover_block(const T* __restrict__ a, const cplx<T> (&x)[6][R],
                                             cplx<T> (&y)[6][R]) {
  T m[36];
  if constexpr (sizeof(T) == 4) {
    const float4* q = reinterpret_cast<const float4*>(a);  // 144-byte blocks, 16-byte aligned
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float4 w = q[i];
      m[4 * i] = w.x;
      m[4 * i + 1] = w.y;
      m[4 * i + 2] = w.z;
      m[4 * i + 3] = w.w;
    }
  } else {
    const double2* q = reinterpret_cast<const double2*>(a);
#pragma unroll
    for (int i = 0; i < 18; ++i) {
      const double2 w = q[i];
      m[2 * i] = w.x;
      m[2 * i + 1] = w.y;
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) y[i][j] = mk<T>(m[i] * x[i][j].x, m[i] * x[i][j].y);
  int idx = 6;
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < i; ++k) {
      const cplx<T> l = mk<T>(m[idx], m[idx + 1]);
      idx += 2;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        cmac<T>(y[i][j], l, x[k][j]);
        cmac_conj<T>(y[k][j], l, x[i][j]);
      }
    }
}

// Which hops into a site whose coordinate along mu is c the direction-resolved
// operator of the Galerkin construction keeps (aggregate extent b along mu).
__device__ __forceinline__ void galerkin_keep(const DirFilter& f, int mu, int c, bool& inc_f, bool& inc_b) {
  const int r = c % f.b[mu];
  const bool fface = (r == f.b[mu] - 1), bface = (r == 0);
  if (f.sign == 0) {
    inc_f = !fface;
    inc_b = !bface;
  } else {
    inc_f = (f.sign == 1 && f.mu == mu && fface);
    inc_b = (f.sign == -1 && f.mu == mu && bface);
  }
}

// MODE 0: out = A psi - kappa H psi ; MODE 1: out = H psi ; MODE 2: out = A psi.
// MODE 3: the direction-resolved piece D_d of MODE 0 selected by the filter
// (sign 0: A psi and the hops that stay inside the aggregate; sign +-1: only
// the -kappa hops that cross the +-mu face), used to build coarse blocks.
// OCC > 0 asks the compiler for at least OCC wavefronts per SIMD (it then
// keeps the register count at or below 512 / OCC, spilling if it must); the
// autotuner measures whether that pays.
template <typename T, int R, int MODE, bool XCD, bool SPLIT, int OCC, typename P = cplx<T>>
__global__ __launch_bounds__(256, (OCC > 0 ? OCC : 1)) void fine_kernel(Geom g, int nrhs, T kappa, const int* __restrict__ order,
                                                   const cplx<T>* __restrict__ U,
                                                   const T* __restrict__ A,
                                                   const P* __restrict__ in,
                                                   cplx<T>* __restrict__ out, int nblocks, DirFilter filt,
                                                   int nt_out, int nc) {
  int b = blockIdx.x;
  int chunk = 0;
  if constexpr (XCD) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
    // contiguous range of the traversal so that neighbour re-reads hit its
    // own L2.  The right-hand sides are split into chunks of nc that are
    // swept one after the other (the launch has nblocks workgroups per
    // chunk), which shrinks the bytes per site that one sweep keeps in L2.
    const int per = (nblocks + 7) >> 3;
    const int j = b >> 3;
    chunk = j / per;
    b = (b & 7) * per + (j - chunk * per);
    if (b >= nblocks) return;
  }
  const int groups = nc / R;
  const long gid = (long)b * 256 + threadIdx.x;
  if (gid >= (long)g.V * groups) return;
  // Sites are visited in the order of the traversal table (tile by tile),
  // so that the eight neighbours of the sites in flight on one XCD are
  // mostly still in its L2; neighbour indices come from a per-site table.
  const int p = (int)(gid / groups);
  const int k0 = chunk * nc + (int)(gid - (long)p * groups) * R;
  const int site = order[p];
  const int4 n0 = g.nbr[2 * site], n1 = g.nbr[2 * site + 1];  // +x -x +y -y | +z -z +t -t

  cplx<T> acc[4][3][R];
  if constexpr (MODE != 2) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[sp][c][j] = mk<T>(0, 0);
    if constexpr (MODE == 3) {
      int r = site;
      const int x = r % g.L[0];
      r /= g.L[0];
      const int y = r % g.L[1];
      r /= g.L[1];
      const int z = r % g.L[2];
      const int t = r / g.L[2];
      if (filt.color >= 0 && ((x / filt.b[0] + y / filt.b[1] + z / filt.b[2] + t / filt.b[3]) & 1) != filt.color) return;
      bool f0, b0, f1, b1, f2, b2, f3, b3;
      galerkin_keep(filt, 0, x, f0, b0);
      galerkin_keep(filt, 1, y, f1, b1);
      galerkin_keep(filt, 2, z, f2, b2);
      galerkin_keep(filt, 3, t, f3, b3);
      hop_dir<T, R, 0, SPLIT>(site, n0.x, n0.y, nrhs, k0, U, in, acc, f0, b0);
      hop_dir<T, R, 1, SPLIT>(site, n0.z, n0.w, nrhs, k0, U, in, acc, f1, b1);
      hop_dir<T, R, 2, SPLIT>(site, n1.x, n1.y, nrhs, k0, U, in, acc, f2, b2);
      hop_dir<T, R, 3, SPLIT>(site, n1.z, n1.w, nrhs, k0, U, in, acc, f3, b3);
    } else {
      hop_dir<T, R, 0, SPLIT>(site, n0.x, n0.y, nrhs, k0, U, in, acc);
      hop_dir<T, R, 1, SPLIT>(site, n0.z, n0.w, nrhs, k0, U, in, acc);
      hop_dir<T, R, 2, SPLIT>(site, n1.x, n1.y, nrhs, k0, U, in, acc);
      hop_dir<T, R, 3, SPLIT>(site, n1.z, n1.w, nrhs, k0, U, in, acc);
    }
  }

  cplx<T>* o = out + (size_t)site * 12 * nrhs + k0;
  if constexpr (MODE == 1) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) store_r<T, R>(o + (3 * sp + c) * nrhs, acc[sp][c], nt_out);
  } else {
    const P* base = in + (size_t)site * 12 * nrhs + k0;
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
      cplx<T> xin[6][R], yout[6][R];
#pragma unroll
      for (int i = 0; i < 6; ++i) load_in<T, R>(base + (6 * chi + i) * nrhs, xin[i]);
      if (MODE != 3 || filt.sign == 0) {
        clover_block<T, R>(A + ((size_t)site * 2 + chi) * 36, xin, yout);
      } else {
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
          for (int j = 0; j < R; ++j) yout[i][j] = mk<T>(0, 0);
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        if constexpr (MODE == 0 || MODE == 3) {
          const int sp = 2 * chi + i / 3, c = i % 3;
#pragma unroll
          for (int j = 0; j < R; ++j) {
            yout[i][j].x = fma(-kappa, acc[sp][c][j].x, yout[i][j].x);
            yout[i][j].y = fma(-kappa, acc[sp][c][j].y, yout[i][j].y);
          }
        }
        store_r<T, R>(o + (6 * chi + i) * nrhs, yout[i], nt_out);
      }
    }
  }
}

// chunks: RHS chunks swept in turn (nrhs / chunks must be a multiple of R);
// lds: dynamic LDS reserved per workgroup (unused by the kernel) to cap the
// number of workgroups resident on one CU.
template <typename T, int R, int MODE, int OCC = 0, typename P = cplx<T>>
hipError_t launch_r(const Geom& g, const int* order, T kappa, const void* U, const void* A, const void* in,
                    void* out, int nrhs, hipStream_t s, const DirFilter& f = DirFilter{}, int nt = 0,
                    int chunks = 1, unsigned lds = 0) {
  if (!g.nbr || !order) return hipErrorInvalidValue;
  if (chunks < 1 || nrhs % chunks || (nrhs / chunks) % R) return hipErrorInvalidValue;
  const int nc = nrhs / chunks;
  const long threads = (long)g.V * (nc / R);
  const int nblocks = (int)((threads + 255) / 256);
  const long grid = (long)((nblocks + 7) / 8) * 8 * chunks;
  if (grid > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fine_kernel<T, R, MODE, true, true, OCC, P>), dim3((unsigned)grid), dim3(256), lds, s, g, nrhs,
                     kappa, order, reinterpret_cast<const cplx<T>*>(U), reinterpret_cast<const T*>(A),
                     reinterpret_cast<const P*>(in), reinterpret_cast<cplx<T>*>(out), nblocks, f, nt, nc);
  return hipGetLastError();
}

// ---- t-walk variant of D = A - kappa H (FP32; FP64 with one RHS per thread) ----
// Every thread owns one site of a spatial block (Bx x By x Bz), R right-hand
// sides, and a run of Ts consecutive time slices that it visits in turn.  The
// spinor psi(x, t+1) that slice t loads for its forward t-hop stays in
// registers: it is the clover input of slice t+1, and transported by
// U_t(x, t)^dag it is the backward t-hop of slice t+1.  So no t-neighbour is
// read twice, whatever the cache holds.  (Keeping only the transported half
// spinor and reading the slice's own spinor again takes fewer registers, 166
// instead of 224 at R = 2, but measured slower at every Nrhs.)  The threads
// of one block walk together, a slice at a time, and read each other's
// spinors as spatial neighbours within about one slice step of their load,
// so more of those re-reads hit the L2 than in the tiled kernel; rows that
// cross a block face, or whose owner has drifted a step away, still come
// from memory.
//
// Work units are (RHS chunk, t-run, spatial block), numbered with the block
// fastest; each XCD takes one contiguous range of their workgroups.  The
// hops are accumulated in the order of fine_kernel (x, y, z, t; forward
// before backward) with the same arithmetic, so both kernels give
// bit-identical results.
struct WalkShape {
  int B[3];       // spatial block extents
  int Ts;         // time slices per thread
  int nc;         // right-hand sides per chunk
  int groups;     // threads per site and chunk (nc / R)
  int bs;         // sites per block
  int nb[2];      // blocks along x, y
  int nblk;       // blocks per slice run
  int nseg;       // t-runs (Lt / Ts)
  int wg_unit;    // workgroups per unit
  long total_wg;  // workgroups of the whole launch
  long per;       // workgroups per XCD
};

template <int R, typename T>
__device__ __forceinline__ void transport_dag(const cplx<T> (&uu)[3][3], const cplx<T> (&h)[2][3][R],
                                              cplx<T> (&w)[2][3][R]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cplx<T> z = mk<T>(0, 0);
#pragma unroll
        for (int b = 0; b < 3; ++b) cmac_conj<T>(z, uu[b][a], h[s][b][j]);
        w[s][a][j] = z;
      }
}

template <int R, typename T>
__device__ __forceinline__ void transport(const cplx<T> (&uu)[3][3], const cplx<T> (&h)[2][3][R],
                                          cplx<T> (&w)[2][3][R]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cplx<T> z = mk<T>(0, 0);
#pragma unroll
        for (int b = 0; b < 3; ++b) cmac<T>(z, uu[a][b], h[s][b][j]);
        w[s][a][j] = z;
      }
}

// The walk in precision T (fields, links, clover and arithmetic).  RES:
// out = bres - D in (the residual), the subtraction after the operator in the
// same precision, exactly as a separate pass would do it.
template <typename T, int R, bool RES>
__device__ __forceinline__ void walk_body(const Geom& g, int nrhs, T kappa, const cplx<T>* __restrict__ U,
                                          const T* __restrict__ A, const cplx<T>* __restrict__ in,
                                          cplx<T>* __restrict__ out, const WalkShape& w, int nt_out,
                                          const cplx<T>* __restrict__ bres) {
  const int hw = blockIdx.x;
  const long wgi = (long)(hw & 7) * w.per + (hw >> 3);
  if (wgi >= w.total_wg) return;
  const int unit = (int)(wgi / w.wg_unit);
  const int tid = (int)(wgi - (long)unit * w.wg_unit) * 256 + (int)threadIdx.x;
  if (tid >= w.bs * w.groups) return;
  const int sb = tid / w.groups;
  const int blk = unit % w.nblk, rest = unit / w.nblk;
  const int seg = rest % w.nseg, chunk = rest / w.nseg;
  const int k0 = chunk * w.nc + (tid - sb * w.groups) * R;
  const int x = (blk % w.nb[0]) * w.B[0] + sb % w.B[0];
  const int y = ((blk / w.nb[0]) % w.nb[1]) * w.B[1] + (sb / w.B[0]) % w.B[1];
  const int z = (blk / (w.nb[0] * w.nb[1])) * w.B[2] + sb / (w.B[0] * w.B[1]);
  const int xs = x + g.L[0] * (y + g.L[1] * z);
  const int Vs = g.stride[3];
  const int dxf = x + 1 < g.L[0] ? 1 : 1 - g.L[0], dxb = x > 0 ? -1 : g.L[0] - 1;
  const int dyf = y + 1 < g.L[1] ? g.stride[1] : g.stride[1] * (1 - g.L[1]);
  const int dyb = y > 0 ? -g.stride[1] : g.stride[1] * (g.L[1] - 1);
  const int dzf = z + 1 < g.L[2] ? g.stride[2] : g.stride[2] * (1 - g.L[2]);
  const int dzb = z > 0 ? -g.stride[2] : g.stride[2] * (g.L[2] - 1);

  const int t0 = seg * w.Ts;
  cplx<T> self[4][3][R], bwd[2][3][R];
  {
    const int sm = xs + Vs * ((t0 == 0 ? g.L[3] : t0) - 1);
    cplx<T> p[4][3][R], h[2][3][R], uu[3][3];
    load_spinor<T, R>(in, sm, nrhs, k0, p);
    project<T, R, 3, -1>(p, h);
    load_link<T, 3>(U + ((size_t)sm * 4 + 3) * 9, uu);
    transport_dag<R, T>(uu, h, bwd);
    load_spinor<T, R>(in, xs + Vs * t0, nrhs, k0, self);
  }
  for (int i = 0; i < w.Ts; ++i) {
    const int t = t0 + i;
    const int site = xs + Vs * t;
    cplx<T> acc[4][3][R];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[sp][c][j] = mk<T>(0, 0);
    hop_dir<T, R, 0, true>(site, site + dxf, site + dxb, nrhs, k0, U, in, acc);
    hop_dir<T, R, 1, true>(site, site + dyf, site + dyb, nrhs, k0, U, in, acc);
    hop_dir<T, R, 2, true>(site, site + dzf, site + dzb, nrhs, k0, U, in, acc);
    cplx<T> nxt[4][3][R];
    load_spinor<T, R>(in, xs + Vs * (t + 1 == g.L[3] ? 0 : t + 1), nrhs, k0, nxt);
    cplx<T> uu[3][3];
    load_link<T, 3>(U + ((size_t)site * 4 + 3) * 9, uu);
    {
      cplx<T> h[2][3][R], wv[2][3][R];
      project<T, R, 3, +1>(nxt, h);
      transport<R, T>(uu, h, wv);
      reconstruct<T, R, 3, +1>(acc, wv);
      pin<T, R>(acc);
    }
    reconstruct<T, R, 3, -1>(acc, bwd);
    pin<T, R>(acc);
    {
      cplx<T> h[2][3][R];
      project<T, R, 3, -1>(self, h);
      transport_dag<R, T>(uu, h, bwd);
    }
    cplx<T>* o = out + (size_t)site * 12 * nrhs + k0;
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
      cplx<T> xin[6][R], yout[6][R];
#pragma unroll
      for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int j = 0; j < R; ++j) xin[q][j] = self[(6 * chi + q) / 3][(6 * chi + q) % 3][j];
      clover_block<T, R>(A + ((size_t)site * 2 + chi) * 36, xin, yout);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int sp = 2 * chi + q / 3, c = q % 3;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          yout[q][j].x = fma(-kappa, acc[sp][c][j].x, yout[q][j].x);
          yout[q][j].y = fma(-kappa, acc[sp][c][j].y, yout[q][j].y);
        }
        if constexpr (RES) {
          cplx<T> bv[R];
          load_r<T, R>(bres + (size_t)site * 12 * nrhs + k0 + (6 * chi + q) * nrhs, bv);
#pragma unroll
          for (int j = 0; j < R; ++j) yout[q][j] = sub<T>(bv[j], yout[q][j]);
        }
        store_r<T, R>(o + (6 * chi + q) * nrhs, yout[q], nt_out);
      }
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < R; ++j) self[sp][c][j] = nxt[sp][c][j];
  }
}

template <int R, int OCC, bool RES = false>
__global__ __launch_bounds__(256, (OCC > 0 ? OCC : 1)) void fine_walk_kernel(Geom g, int nrhs, float kappa,
                                                                           const cplx<float>* __restrict__ U,
                                                                           const float* __restrict__ A,
                                                                           const cplx<float>* __restrict__ in,
                                                                           cplx<float>* __restrict__ out, WalkShape w,
                                                                           int nt_out,
                                                                           const cplx<float>* __restrict__ bres = nullptr) {
  walk_body<float, R, RES>(g, nrhs, kappa, U, A, in, out, w, nt_out, bres);
}

// The FP64 operator of the outer solver's residuals, one RHS per thread.
template <int OCC>
__global__ __launch_bounds__(256, (OCC > 0 ? OCC : 1)) void fine_walk_f64_kernel(Geom g, int nrhs, double kappa,
                                                            const cplx<double>* __restrict__ U,
                                                            const double* __restrict__ A,
                                                            const cplx<double>* __restrict__ in,
                                                            cplx<double>* __restrict__ out, WalkShape w, int nt_out) {
  walk_body<double, 1, false>(g, nrhs, kappa, U, A, in, out, w, nt_out, nullptr);
}

// Shape of a t-walk launch for tile T = (Bx, By, Bz, Ts) and nc = nrhs / chunks
// right-hand sides per chunk; false if the tile does not divide the lattice.
bool walk_shape(const Geom& g, const int T[4], int nrhs, int R, int chunks, WalkShape& w) {
  for (int m = 0; m < 4; ++m)
    if (T[m] < 1 || g.L[m] % T[m]) return false;
  if (chunks < 1 || nrhs % chunks || (nrhs / chunks) % R) return false;
  for (int m = 0; m < 3; ++m) w.B[m] = T[m];
  w.Ts = T[3];
  w.nc = nrhs / chunks;
  w.groups = w.nc / R;
  w.bs = T[0] * T[1] * T[2];
  w.nb[0] = g.L[0] / T[0];
  w.nb[1] = g.L[1] / T[1];
  w.nblk = w.nb[0] * w.nb[1] * (g.L[2] / T[2]);
  w.nseg = g.L[3] / T[3];
  w.wg_unit = (w.bs * w.groups + 255) / 256;
  const long units = (long)chunks * w.nseg * w.nblk;
  w.total_wg = units * w.wg_unit;
  w.per = (w.total_wg + 7) / 8;
  return w.per * 8 <= 0x7fffffffL;
}

template <int R, int OCC, bool RES>
hipError_t launch_walk_r(const Geom& g, const FineCfg& c, float kappa, const void* U, const void* A, const void* in,
                         void* out, int nrhs, hipStream_t s, const void* bres) {
  WalkShape w;
  if (!walk_shape(g, c.T, nrhs, R, c.chunks, w)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fine_walk_kernel<R, OCC, RES>), dim3((unsigned)(w.per * 8)), dim3(256), c.lds, s, g, nrhs,
                     kappa, reinterpret_cast<const cplx<float>*>(U), reinterpret_cast<const float*>(A),
                     reinterpret_cast<const cplx<float>*>(in), reinterpret_cast<cplx<float>*>(out), w, c.nt,
                     reinterpret_cast<const cplx<float>*>(bres));
  return hipGetLastError();
}

// bres given: out = bres - D in
template <bool RES>
hipError_t launch_walk_res(const Geom& g, const FineCfg& c, float kappa, const void* U, const void* A, const void* in,
                           void* out, int nrhs, hipStream_t s, const void* bres) {
  if (c.occ == 4) {
    if (c.R == 2) return launch_walk_r<2, 4, RES>(g, c, kappa, U, A, in, out, nrhs, s, bres);
    if (c.R == 1) return launch_walk_r<1, 4, RES>(g, c, kappa, U, A, in, out, nrhs, s, bres);
  } else {
    if (c.R == 2) return launch_walk_r<2, 0, RES>(g, c, kappa, U, A, in, out, nrhs, s, bres);
    if (c.R == 1) return launch_walk_r<1, 0, RES>(g, c, kappa, U, A, in, out, nrhs, s, bres);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_walk(const Geom& g, const FineCfg& c, float kappa, const void* U, const void* A, const void* in,
                       void* out, int nrhs, hipStream_t s, const void* bres = nullptr) {
  if (bres) return launch_walk_res<true>(g, c, kappa, U, A, in, out, nrhs, s, bres);
  return launch_walk_res<false>(g, c, kappa, U, A, in, out, nrhs, s, nullptr);
}

template <typename T, int MODE>
hipError_t launch_mode(const Geom& g, int t_bc, T kappa, const void* U, const void* A, const void* in,
                       void* out, int nrhs, hipStream_t s, const FineCfg* cfg) {
  (void)t_bc;  // folded into the links
  const int* order = (cfg && cfg->R > 0 && cfg->order) ? cfg->order : g.order;
  int R = (cfg && cfg->R > 0) ? cfg->R : 0;
  if constexpr (sizeof(T) == 4) {
    // Untuned default: two right-hand sides per thread (one 16-byte load per
    // component) for even Nrhs, one otherwise.
    if (R == 0) R = (nrhs % 2 == 0) ? 2 : 1;
    const bool occ4 = MODE == 0 && cfg && cfg->occ == 4;
    const bool tuned = cfg && cfg->R > 0;
    const int nt = tuned ? cfg->nt : 0;
    int ch = tuned ? cfg->chunks : 1;
    const unsigned lds = tuned ? cfg->lds : 0u;
    if (R == 4 && nrhs % 4) R = 2;
    if (R == 2 && nrhs % 2) R = 1;
    if (ch < 1 || nrhs % ch || (nrhs / ch) % R) ch = 1;
    const DirFilter f;
    if constexpr (MODE == 0) {
      if (tuned && cfg->walk) return launch_walk(g, *cfg, kappa, U, A, in, out, nrhs, s);
      if (occ4) {
        if (R == 4) return launch_r<T, 4, MODE, 4>(g, order, kappa, U, A, in, out, nrhs, s, f, nt, ch, lds);
        if (R == 2) return launch_r<T, 2, MODE, 4>(g, order, kappa, U, A, in, out, nrhs, s, f, nt, ch, lds);
        return launch_r<T, 1, MODE, 4>(g, order, kappa, U, A, in, out, nrhs, s, f, nt, ch, lds);
      }
    }
    if (R == 4) return launch_r<T, 4, MODE>(g, order, kappa, U, A, in, out, nrhs, s, f, nt, ch, lds);
    if (R == 2) return launch_r<T, 2, MODE>(g, order, kappa, U, A, in, out, nrhs, s, f, nt, ch, lds);
    return launch_r<T, 1, MODE>(g, order, kappa, U, A, in, out, nrhs, s, f, nt, ch, lds);
  }
  return launch_r<T, 1, MODE>(g, order, kappa, U, A, in, out, nrhs, s);
}

template <typename T>
hipError_t launch_fine(const Geom& g, int t_bc, int mode, T kappa, const void* U, const void* A,
                       const void* in, void* out, int nrhs, hipStream_t s, const FineCfg* cfg) {
  switch (mode) {
    case 0:
      return launch_mode<T, 0>(g, t_bc, kappa, U, A, in, out, nrhs, s, cfg);
    case 1:
      return launch_mode<T, 1>(g, t_bc, kappa, U, A, in, out, nrhs, s, cfg);
    default:
      return launch_mode<T, 2>(g, t_bc, kappa, U, A, in, out, nrhs, s, cfg);
  }
}

// ---- checkerboarded pieces (paper Sec. 4: M_eooe and M_ooee) ----------------------------
// A field on one parity is [V/2][12][nrhs]; entry i is the site of that parity
// among s = 2i, 2i + 1.  Per checkerboard index the table holds four int4:
// the checkerboard indices of the neighbours (+x, -x, +y, -y), (+z, -z, +t,
// -t) on the other parity, then the lattice site of i itself and of its
// backward neighbours (self, -x, -y, -z), (-t, -, -, -), which index the links
// and clover blocks.

// M_eooe: out (parity p) = H in (parity 1 - p), R right-hand sides per thread.
// Sites are visited in the order of a traversal table (the parity-p sites of
// the full kernel's tiled order), each XCD taking one contiguous range of it,
// so that neighbour rows are re-read from its own L2 as in fine_kernel.
// EPI selects what is stored, with h = H in, Ablk the clover blocks (or their
// inverses) of the output sites and in2 a field on the output parity:
//   0: h;  1: Ablk h;  2: Ablk in2 + coef h;  3: in2 + coef h;
//   4: Ablk (in2 + coef h).
// 1 and 2 fuse the Schur complement's clover factors into the hops, 3 and 4
// the even-odd smoother's right-hand side and odd-site reconstruction.  FULL2
// reads in2 from a full-lattice field (row = lattice site) instead of a
// checkerboard one; ADDF adds the result into a full-lattice out.  DOT (with
// EPI 2, the minimal-residual step p = Dhat r, in2 = r) also writes per
// workgroup b and column k the partial sums (Re <p, r>, Im <p, r>, ||p||^2)
// in FP64 to part[b][k], summed over the workgroup's threads in a fixed order.
// The stores of one output site of hop_eo_kernel / hop_eo_walk_kernel (EPI,
// FULL2, ADDF as there): i its checkerboard index, site its lattice site,
// acc = (H in) at the site; with DOT the site's terms of the partial sums are
// added to dre, dim, dpp (nothing is stored for an invalid thread).
template <typename T, int R, int EPI, bool FULL2, bool ADDF, bool DOT>
__device__ __forceinline__ void hop_eo_epilogue(int i, int site, int nrhs, int k0, bool valid,
                                                const cplx<T> (&acc)[4][3][R], cplx<T>* __restrict__ out,
                                                const T* __restrict__ Ablk, const cplx<T>* __restrict__ in2, T coef,
                                                double (&dre)[R], double (&dim)[R], double (&dpp)[R]) {
  cplx<T>* o = out + (size_t)(ADDF ? site : i) * 12 * nrhs + k0;
  const cplx<T>* q = in2 + (size_t)(FULL2 ? site : i) * 12 * nrhs + k0;
  // y = the stored value of component r of chirality chi
  auto put = [&](cplx<T>* dst, const cplx<T> (&y)[R]) {
    if constexpr (DOT) {
      if (!valid) return;
    }
    if constexpr (ADDF) {
      cplx<T> a[R], sum[R];
      load_r<T, R>(dst, a);
#pragma unroll
      for (int j = 0; j < R; ++j) sum[j] = add<T>(a[j], y[j]);
      store_r<T, R>(dst, sum);
    } else {
      store_r<T, R>(dst, y);
    }
  };
  if constexpr (EPI == 0 || EPI == 3) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cplx<T> y[R];
        if constexpr (EPI == 3) {
          load_r<T, R>(q + (3 * sp + c) * nrhs, y);
#pragma unroll
          for (int j = 0; j < R; ++j) {
            y[j].x = fma(coef, acc[sp][c][j].x, y[j].x);
            y[j].y = fma(coef, acc[sp][c][j].y, y[j].y);
          }
        } else {
#pragma unroll
          for (int j = 0; j < R; ++j) y[j] = acc[sp][c][j];
        }
        put(o + (3 * sp + c) * nrhs, y);
      }
  } else {
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
      cplx<T> xin[6][R], yout[6][R];
      if constexpr (EPI == 1) {
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int j = 0; j < R; ++j) xin[r][j] = acc[2 * chi + r / 3][r % 3][j];
      } else {
#pragma unroll
        for (int r = 0; r < 6; ++r) load_r<T, R>(q + (6 * chi + r) * nrhs, xin[r]);
        if constexpr (EPI == 4) {
#pragma unroll
          for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int j = 0; j < R; ++j) {
              xin[r][j].x = fma(coef, acc[2 * chi + r / 3][r % 3][j].x, xin[r][j].x);
              xin[r][j].y = fma(coef, acc[2 * chi + r / 3][r % 3][j].y, xin[r][j].y);
            }
        }
      }
      clover_block<T, R>(Ablk + ((size_t)site * 2 + chi) * 36, xin, yout);
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        if constexpr (EPI == 2) {
#pragma unroll
          for (int j = 0; j < R; ++j) {
            yout[r][j].x = fma(coef, acc[2 * chi + r / 3][r % 3][j].x, yout[r][j].x);
            yout[r][j].y = fma(coef, acc[2 * chi + r / 3][r % 3][j].y, yout[r][j].y);
          }
        }
        if constexpr (DOT) {
#pragma unroll
          for (int j = 0; j < R; ++j) {
            const double px = yout[r][j].x, py = yout[r][j].y, qx = xin[r][j].x, qy = xin[r][j].y;
            dre[j] = fma(px, qx, fma(py, qy, dre[j]));
            dim[j] = fma(px, qy, fma(-py, qx, dim[j]));
            dpp[j] = fma(px, px, fma(py, py, dpp[j]));
          }
        }
        put(o + (6 * chi + r) * nrhs, yout[r]);
      }
    }
  }
}

// DOT: per-workgroup partial sums in a fixed order.  Thread u of the
// workgroup holds column group (first + u) mod groups (first = the group
// index of its thread 0); columns k < nrhs go to row[k].
template <int R>
__device__ __forceinline__ void hop_eo_dot_store(const double (&dre)[R], const double (&dim)[R],
                                                 const double (&dpp)[R], bool valid, long first, int groups,
                                                 int nrhs, double4* __restrict__ row) {
  __shared__ double red[256 * R * 3];
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    red[(t * R + j) * 3 + 0] = valid ? dre[j] : 0.0;
    red[(t * R + j) * 3 + 1] = valid ? dim[j] : 0.0;
    red[(t * R + j) * 3 + 2] = valid ? dpp[j] : 0.0;
  }
  __syncthreads();
  if (t < nrhs) {
    const int gi = t / R, j = t - (t / R) * R;
    int u = gi - (int)(first % groups);
    if (u < 0) u += groups;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (; u < 256; u += groups) {
      s0 += red[(u * R + j) * 3 + 0];
      s1 += red[(u * R + j) * 3 + 1];
      s2 += red[(u * R + j) * 3 + 2];
    }
    row[t] = make_double4(s0, s1, s2, 0.0);
  }
}

template <typename T, int R, int EPI, bool FULL2, bool ADDF, bool DOT = false>
__global__ __launch_bounds__(256) void hop_eo_kernel(int nhalf, int nrhs, const int4* __restrict__ tab,
                                                     const int* __restrict__ order, int nblocks,
                                                     const cplx<T>* __restrict__ U, const cplx<T>* __restrict__ in,
                                                     cplx<T>* __restrict__ out, const T* __restrict__ Ablk,
                                                     const cplx<T>* __restrict__ in2, T coef,
                                                     double4* __restrict__ part = nullptr) {
  static_assert(!DOT || (EPI == 2 && !ADDF), "the MR partial sums go with the second Schur hop");
  const int per = (nblocks + 7) >> 3;
  const int b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (b >= nblocks) return;  // the whole workgroup
  const int groups = nrhs / R;
  const long gid = (long)b * 256 + threadIdx.x;
  const long total = (long)nhalf * groups;
  // with DOT every thread reaches the workgroup's barrier: one past the end
  // recomputes the last entry, stores nothing and adds zeros
  const bool valid = gid < total;
  if (!DOT && !valid) return;
  const long gv = valid ? gid : total - 1;
  const int pidx = (int)(gv / groups);
  const int k0 = (int)(gv - (long)pidx * groups) * R;
  double dre[R], dim[R], dpp[R];
#pragma unroll
  for (int j = 0; j < R; ++j) dre[j] = dim[j] = dpp[j] = 0.0;
  const int i = order[pidx];
  const int4 n0 = tab[4 * i], n1 = tab[4 * i + 1], s0 = tab[4 * i + 2], s1 = tab[4 * i + 3];
  cplx<T> acc[4][3][R];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < R; ++j) acc[sp][c][j] = mk<T>(0, 0);
  hop_dir<T, R, 0, true>(s0.x, n0.x, n0.y, nrhs, k0, U, in, acc, true, true, s0.y);
  hop_dir<T, R, 1, true>(s0.x, n0.z, n0.w, nrhs, k0, U, in, acc, true, true, s0.z);
  hop_dir<T, R, 2, true>(s0.x, n1.x, n1.y, nrhs, k0, U, in, acc, true, true, s0.w);
  hop_dir<T, R, 3, true>(s0.x, n1.z, n1.w, nrhs, k0, U, in, acc, true, true, s1.x);
  hop_eo_epilogue<T, R, EPI, FULL2, ADDF, DOT>(i, s0.x, nrhs, k0, valid, acc, out, Ablk, in2, coef, dre, dim, dpp);
  if constexpr (DOT) hop_eo_dot_store<R>(dre, dim, dpp, valid, (long)b * 256, groups, nrhs, part + (long)b * nrhs);
}

// t-walk form of hop_eo_kernel (FP32): a thread owns one site of a spatial
// block, R right-hand sides and a run of Ts output sites of its parity along
// t (every second time slice).  The input spinor at t + 1 that the forward
// t-hop of output t loads is, transported by U_t(x, t + 1)^dag, the backward
// t-hop of output t + 2: it is carried in registers instead of read again.
// Hops are accumulated in the order of hop_eo_kernel (x, y, z, t; forward
// before backward) with the same arithmetic, and the stores are the same
// epilogue, so both kernels give bit-identical fields (DOT partials are per
// workgroup, so the sums' grouping differs).  Work units and the XCD split
// are those of fine_walk_kernel; `parity` is the output parity.
template <int R, int EPI, bool FULL2, bool ADDF, bool DOT>
__global__ __launch_bounds__(256) void hop_eo_walk_kernel(Geom g, int parity, int nrhs, WalkShape w,
                                                          const cplx<float>* __restrict__ U,
                                                          const cplx<float>* __restrict__ in,
                                                          cplx<float>* __restrict__ out, const float* __restrict__ Ablk,
                                                          const cplx<float>* __restrict__ in2, float coef,
                                                          double4* __restrict__ part) {
  static_assert(!DOT || (EPI == 2 && !ADDF), "the MR partial sums go with the second Schur hop");
  const int hw = blockIdx.x;
  const long wgi = (long)(hw & 7) * w.per + (hw >> 3);
  if (wgi >= w.total_wg) return;  // the whole workgroup
  const int unit = (int)(wgi / w.wg_unit);
  const int wl = (int)(wgi - (long)unit * w.wg_unit);
  const int tid = wl * 256 + (int)threadIdx.x;
  // with DOT every thread reaches the workgroup's barrier; a thread past the
  // unit's end walks the unit's last site, stores nothing and adds zeros
  const bool valid = tid < w.bs * w.groups;
  if (!DOT && !valid) return;
  const int tv = valid ? tid : w.bs * w.groups - 1;
  const int sb = tv / w.groups;
  const int blk = unit % w.nblk, seg = unit / w.nblk;
  const int k0 = (tv - sb * w.groups) * R;
  const int x = (blk % w.nb[0]) * w.B[0] + sb % w.B[0];
  const int y = ((blk / w.nb[0]) % w.nb[1]) * w.B[1] + (sb / w.B[0]) % w.B[1];
  const int z = (blk / (w.nb[0] * w.nb[1])) * w.B[2] + sb / (w.B[0] * w.B[1]);
  const int xs = x + g.L[0] * (y + g.L[1] * z);
  const int Vs = g.stride[3];
  const int dxf = x + 1 < g.L[0] ? 1 : 1 - g.L[0], dxb = x > 0 ? -1 : g.L[0] - 1;
  const int dyf = y + 1 < g.L[1] ? g.stride[1] : g.stride[1] * (1 - g.L[1]);
  const int dyb = y > 0 ? -g.stride[1] : g.stride[1] * (g.L[1] - 1);
  const int dzf = z + 1 < g.L[2] ? g.stride[2] : g.stride[2] * (1 - g.L[2]);
  const int dzb = z > 0 ? -g.stride[2] : g.stride[2] * (g.L[2] - 1);
  // output times t = t0 + 2 q, q < Ts, of this site's parity
  const int t0 = (parity ^ ((x + y + z) & 1)) + 2 * seg * w.Ts;
  double dre[R], dim[R], dpp[R];
#pragma unroll
  for (int j = 0; j < R; ++j) dre[j] = dim[j] = dpp[j] = 0.0;
  cplx<float> bwd[2][3][R];
  {
    const int sm = xs + Vs * ((t0 == 0 ? g.L[3] : t0) - 1);
    cplx<float> p[4][3][R], h[2][3][R], uu[3][3];
    load_spinor<float, R>(in, sm >> 1, nrhs, k0, p);
    project<float, R, 3, -1>(p, h);
    load_link<float, 3>(U + ((size_t)sm * 4 + 3) * 9, uu);
    transport_dag<R, float>(uu, h, bwd);
  }
  for (int q = 0; q < w.Ts; ++q) {
    const int t = t0 + 2 * q;
    const int site = xs + Vs * t;
    cplx<float> acc[4][3][R];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[sp][c][j] = mk<float>(0, 0);
    hop_dir<float, R, 0, true>(site, (site + dxf) >> 1, (site + dxb) >> 1, nrhs, k0, U, in, acc, true, true,
                               site + dxb);
    hop_dir<float, R, 1, true>(site, (site + dyf) >> 1, (site + dyb) >> 1, nrhs, k0, U, in, acc, true, true,
                               site + dyb);
    hop_dir<float, R, 2, true>(site, (site + dzf) >> 1, (site + dzb) >> 1, nrhs, k0, U, in, acc, true, true,
                               site + dzb);
    const int sp1 = xs + Vs * (t + 1 == g.L[3] ? 0 : t + 1);
    {
      cplx<float> p[4][3][R], hf[2][3][R], hb[2][3][R], uu[3][3], wv[2][3][R];
      load_spinor<float, R>(in, sp1 >> 1, nrhs, k0, p);
      project<float, R, 3, +1>(p, hf);
      project<float, R, 3, -1>(p, hb);
      load_link<float, 3>(U + ((size_t)site * 4 + 3) * 9, uu);
      transport<R, float>(uu, hf, wv);
      reconstruct<float, R, 3, +1>(acc, wv);
      pin<float, R>(acc);
      reconstruct<float, R, 3, -1>(acc, bwd);
      pin<float, R>(acc);
      // the backward t-hop of output t + 2: U_t(x, t + 1)^dag P psi(t + 1)
      load_link<float, 3>(U + ((size_t)sp1 * 4 + 3) * 9, uu);
      transport_dag<R, float>(uu, hb, bwd);
    }
    hop_eo_epilogue<float, R, EPI, FULL2, ADDF, DOT>(site >> 1, site, nrhs, k0, valid, acc, out, Ablk, in2, coef,
                                                     dre, dim, dpp);
  }
  if constexpr (DOT) hop_eo_dot_store<R>(dre, dim, dpp, valid, (long)wl * 256, w.groups, nrhs, part + wgi * nrhs);
}

// Shape of a checkerboard t-walk: spatial block B, Ts output sites per run
// (2 Ts time slices); false unless B divides the spatial extents and Ts
// divides Lt / 2.
bool eo_walk_shape(const Geom& g, const int B[3], int Ts, int nrhs, int R, WalkShape& w) {
  for (int m = 0; m < 3; ++m)
    if (B[m] < 1 || g.L[m] % B[m]) return false;
  if (Ts < 1 || g.L[3] % 2 || (g.L[3] / 2) % Ts || nrhs % R) return false;
  for (int m = 0; m < 3; ++m) w.B[m] = B[m];
  w.Ts = Ts;
  w.nc = nrhs;
  w.groups = nrhs / R;
  w.bs = B[0] * B[1] * B[2];
  w.nb[0] = g.L[0] / B[0];
  w.nb[1] = g.L[1] / B[1];
  w.nblk = w.nb[0] * w.nb[1] * (g.L[2] / B[2]);
  w.nseg = (g.L[3] / 2) / Ts;
  w.wg_unit = (w.bs * w.groups + 255) / 256;
  w.total_wg = (long)w.nseg * w.nblk * w.wg_unit;
  w.per = (w.total_wg + 7) / 8;
  return w.per * 8 <= 0x7fffffffL;
}

// M_ooee (or its inverse, given the inverse blocks): out = A in + coef add on
// one parity (add may be null).
// FULLIN: in is a full-lattice field (row = lattice site).
template <typename T, int R, bool FULLIN>
__global__ __launch_bounds__(256) void clover_eo_kernel(int nhalf, int nrhs, const int4* __restrict__ tab,
                                                        const T* __restrict__ A, const cplx<T>* __restrict__ in,
                                                        const cplx<T>* __restrict__ add, T coef,
                                                        cplx<T>* __restrict__ out) {
  const int groups = nrhs / R;
  const long gid = (long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (long)nhalf * groups) return;
  const int i = (int)(gid / groups);
  const int k0 = (int)(gid - (long)i * groups) * R;
  const int site = tab[4 * i + 2].x;
  const size_t base = (size_t)i * 12 * nrhs + k0;
  const size_t ibase = (size_t)(FULLIN ? site : i) * 12 * nrhs + k0;
#pragma unroll
  for (int chi = 0; chi < 2; ++chi) {
    cplx<T> xin[6][R], yout[6][R];
#pragma unroll
    for (int r = 0; r < 6; ++r) load_r<T, R>(in + ibase + (6 * chi + r) * nrhs, xin[r]);
    clover_block<T, R>(A + ((size_t)site * 2 + chi) * 36, xin, yout);
    if (add) {
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        cplx<T> a[R];
        load_r<T, R>(add + base + (6 * chi + r) * nrhs, a);
#pragma unroll
        for (int j = 0; j < R; ++j) {
          yout[r][j].x = fma(coef, a[j].x, yout[r][j].x);
          yout[r][j].y = fma(coef, a[j].y, yout[r][j].y);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) store_r<T, R>(out + base + (6 * chi + r) * nrhs, yout[r]);
  }
}

// Inverse of every Hermitian 6x6 chiral clover block (FP64, Gauss-Jordan
// elimination with partial pivoting), packed like the blocks: six real
// diagonal entries, then the strictly lower triangle row by row as (re, im).
// A block whose pivot vanishes sets *flag.
__global__ __launch_bounds__(256) void clover_invert_kernel(long nblk, const double* __restrict__ A,
                                                            double* __restrict__ Ai64, float* __restrict__ Ai32,
                                                            int* __restrict__ flag) {
  const long b = (long)blockIdx.x * 256 + threadIdx.x;
  if (b >= nblk) return;
  const double* a = A + b * 36;
  double2 M[6][6], X[6][6];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) X[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  for (int r = 0; r < 6; ++r) M[r][r] = make_double2(a[r], 0.0);
  int k = 6;
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < r; ++c) {
      M[r][c] = make_double2(a[k], a[k + 1]);
      M[c][r] = make_double2(a[k], -a[k + 1]);
      k += 2;
    }
  bool ok = true;
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    double best = -1.0;
    for (int r = col; r < 6; ++r) {
      const double m = M[r][col].x * M[r][col].x + M[r][col].y * M[r][col].y;
      if (m > best) {
        best = m;
        piv = r;
      }
    }
    if (!(best > 0.0)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int c = 0; c < 6; ++c) {
        const double2 t = M[col][c];
        M[col][c] = M[piv][c];
        M[piv][c] = t;
        const double2 u = X[col][c];
        X[col][c] = X[piv][c];
        X[piv][c] = u;
      }
    // 1 / pivot
    const double2 p = M[col][col];
    const double2 ip = make_double2(p.x / best, -p.y / best);
    for (int c = 0; c < 6; ++c) {
      const double2 m = M[col][c], x = X[col][c];
      M[col][c] = make_double2(m.x * ip.x - m.y * ip.y, m.x * ip.y + m.y * ip.x);
      X[col][c] = make_double2(x.x * ip.x - x.y * ip.y, x.x * ip.y + x.y * ip.x);
    }
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      const double2 f = M[r][col];
      for (int c = 0; c < 6; ++c) {
        const double2 m = M[col][c], x = X[col][c];
        M[r][c] = make_double2(M[r][c].x - (f.x * m.x - f.y * m.y), M[r][c].y - (f.x * m.y + f.y * m.x));
        X[r][c] = make_double2(X[r][c].x - (f.x * x.x - f.y * x.y), X[r][c].y - (f.x * x.y + f.y * x.x));
      }
    }
  }
  if (!ok) {
    atomicOr(flag, 1);
    return;
  }
  double* o64 = Ai64 + b * 36;
  float* o32 = Ai32 + b * 36;
  for (int r = 0; r < 6; ++r) {
    o64[r] = X[r][r].x;
    o32[r] = (float)X[r][r].x;
  }
  k = 6;
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < r; ++c) {
      o64[k] = X[r][c].x;
      o64[k + 1] = X[r][c].y;
      o32[k] = (float)X[r][c].x;
      o32[k + 1] = (float)X[r][c].y;
      k += 2;
    }
}

// Row copies between a full-lattice FP32 field and one parity's checkerboard
// field: one thread per (checkerboard site, component, pair of RHS values).
template <bool ADD>
__global__ __launch_bounds__(256) void eo_rows_kernel(int nhalf, int nrhs, const int4* __restrict__ tab,
                                                      float2* __restrict__ full, float2* __restrict__ half) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long per = 12L * nrhs;
  if (e >= (long)nhalf * per) return;
  const int i = (int)(e / per);
  const long r = e - (long)i * per;
  const size_t f = (size_t)tab[4 * i + 2].x * per + r;
  if (ADD) {
    const float2 a = full[f], b = half[e];
    full[f] = make_float2(a.x + b.x, a.y + b.y);
  } else {
    half[e] = full[f];
  }
}

template <typename T, int R, int EPI, bool FULL2, bool ADDF>
hipError_t launch_hop_eo_k(int nhalf, int nrhs, const int4* tab, const int* order, const void* U, const void* in,
                           void* out, const void* Ablk, const void* in2, double coef, hipStream_t s) {
  const long threads = (long)nhalf * (nrhs / R);
  const int nblocks = (int)((threads + 255) / 256);
  const dim3 grid((unsigned)(((nblocks + 7) / 8) * 8));
  hipLaunchKernelGGL((hop_eo_kernel<T, R, EPI, FULL2, ADDF>), grid, dim3(256), 0, s, nhalf, nrhs, tab, order, nblocks,
                     static_cast<const cplx<T>*>(U), static_cast<const cplx<T>*>(in), static_cast<cplx<T>*>(out),
                     static_cast<const T*>(Ablk), static_cast<const cplx<T>*>(in2), (T)coef);
  return hipGetLastError();
}

template <int R>
hipError_t launch_hop_eo_dot_r(int nhalf, int nrhs, const int4* tab, const int* order, const void* U, const void* in,
                               void* out, const void* Ablk, const void* in2, double coef, void* part, int* nblk,
                               hipStream_t s) {
  const long threads = (long)nhalf * (nrhs / R);
  const int nblocks = (int)((threads + 255) / 256);
  const dim3 grid((unsigned)(((nblocks + 7) / 8) * 8));
  hipLaunchKernelGGL((hop_eo_kernel<float, R, 2, false, false, true>), grid, dim3(256), 0, s, nhalf, nrhs, tab, order,
                     nblocks, static_cast<const float2*>(U), static_cast<const float2*>(in),
                     static_cast<float2*>(out), static_cast<const float*>(Ablk), static_cast<const float2*>(in2),
                     (float)coef, static_cast<double4*>(part));
  *nblk = nblocks;
  return hipGetLastError();
}

template <int R, int EPI, bool FULL2, bool ADDF, bool DOT>
hipError_t launch_hop_eo_walk_k(const Geom& g, int parity, int nrhs, const EoWalk& ew, const void* U, const void* in,
                                void* out, const void* Ablk, const void* in2, double coef, void* part, long* nblk,
                                hipStream_t s) {
  WalkShape w;
  if (!eo_walk_shape(g, ew.B, ew.Ts, nrhs, R, w)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((hop_eo_walk_kernel<R, EPI, FULL2, ADDF, DOT>), dim3((unsigned)(w.per * 8)), dim3(256), 0, s, g,
                     parity, nrhs, w, static_cast<const float2*>(U), static_cast<const float2*>(in),
                     static_cast<float2*>(out), static_cast<const float*>(Ablk), static_cast<const float2*>(in2),
                     (float)coef, static_cast<double4*>(part));
  if (nblk) *nblk = w.total_wg;
  return hipGetLastError();
}

template <int R>
hipError_t launch_hop_eo_walk_r(int epi, const Geom& g, int parity, int nrhs, const EoWalk& ew, const void* U,
                                const void* in, void* out, const void* Ablk, const void* in2, double coef,
                                hipStream_t s) {
  switch (epi) {
    case 0:
      return launch_hop_eo_walk_k<R, 0, false, false, false>(g, parity, nrhs, ew, U, in, out, Ablk, in2, coef,
                                                             nullptr, nullptr, s);
    case 1:
      return launch_hop_eo_walk_k<R, 1, false, false, false>(g, parity, nrhs, ew, U, in, out, Ablk, in2, coef,
                                                             nullptr, nullptr, s);
    case 2:
      return launch_hop_eo_walk_k<R, 2, false, false, false>(g, parity, nrhs, ew, U, in, out, Ablk, in2, coef,
                                                             nullptr, nullptr, s);
    case 3:
      return launch_hop_eo_walk_k<R, 3, true, false, false>(g, parity, nrhs, ew, U, in, out, Ablk, in2, coef,
                                                            nullptr, nullptr, s);
    case 4:
      return launch_hop_eo_walk_k<R, 4, true, true, false>(g, parity, nrhs, ew, U, in, out, Ablk, in2, coef,
                                                           nullptr, nullptr, s);
    default:
      return hipErrorInvalidValue;
  }
}

// epi 0..2 on checkerboard fields (FP32 and FP64); the smoother's forms 3
// (in2 full-lattice) and 4 (in2 full-lattice, added into a full-lattice out)
// in FP32 only.
template <typename T, int R>
hipError_t launch_hop_eo_r(int epi, int nhalf, int nrhs, const int4* tab, const int* order, const void* U,
                           const void* in, void* out, const void* Ablk, const void* in2, double coef, hipStream_t s) {
  switch (epi) {
    case 0:
      return launch_hop_eo_k<T, R, 0, false, false>(nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
    case 1:
      return launch_hop_eo_k<T, R, 1, false, false>(nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
    case 2:
      return launch_hop_eo_k<T, R, 2, false, false>(nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
    default:
      break;
  }
  if constexpr (sizeof(T) == 4) {
    if (epi == 3)
      return launch_hop_eo_k<T, R, 3, true, false>(nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
    if (epi == 4)
      return launch_hop_eo_k<T, R, 4, true, true>(nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int R>
hipError_t launch_clover_eo_r(int nhalf, int nrhs, const int4* tab, const void* A, const void* in, const void* add,
                              double coef, void* out, bool full_in, hipStream_t s) {
  const long threads = (long)nhalf * (nrhs / R);
  const dim3 grid((unsigned)((threads + 255) / 256));
  if (full_in)
    hipLaunchKernelGGL((clover_eo_kernel<T, R, true>), grid, dim3(256), 0, s, nhalf, nrhs, tab,
                       static_cast<const T*>(A), static_cast<const cplx<T>*>(in), static_cast<const cplx<T>*>(add),
                       (T)coef, static_cast<cplx<T>*>(out));
  else
    hipLaunchKernelGGL((clover_eo_kernel<T, R, false>), grid, dim3(256), 0, s, nhalf, nrhs, tab,
                       static_cast<const T*>(A), static_cast<const cplx<T>*>(in), static_cast<const cplx<T>*>(add),
                       (T)coef, static_cast<cplx<T>*>(out));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fine_f32(const Geom& g, int t_bc, int mode, float kappa, const void* U, const void* A,
                           const void* in, void* out, int nrhs, hipStream_t s, const FineCfg* cfg) {
  return launch_fine<float>(g, t_bc, mode, kappa, U, A, in, out, nrhs, s, cfg);
}

// r = b - D x in FP32 in one launch when the tuned configuration of nrhs is
// the t-walk kernel; false (nothing launched) otherwise.
bool launch_fine_residual_f32(const Geom& g, float kappa, const void* U, const void* A, const void* x, const void* b,
                              void* r, int nrhs, hipStream_t s, const FineCfg* cfg, hipError_t* err) {
  if (!cfg || cfg->R <= 0 || !cfg->walk || !b) return false;
  *err = launch_walk(g, *cfg, kappa, U, A, x, r, nrhs, s, b);
  return true;
}

bool f64_walk_fits(const Geom& g, const int tile[4], int nrhs) {
  WalkShape w;
  return walk_shape(g, tile, nrhs, 1, 1, w);
}

hipError_t launch_fine_f64(const Geom& g, int t_bc, int mode, double kappa, const void* U, const void* A,
                           const void* in, void* out, int nrhs, hipStream_t s, const F64Walk* fw) {
  if (mode == 0 && fw && fw->on) {
    const int tile[4] = {fw->B[0], fw->B[1], fw->B[2], fw->Ts};
    WalkShape w;
    if (!walk_shape(g, tile, nrhs, 1, 1, w)) return hipErrorInvalidValue;
    auto k = fw->occ == 2 ? fine_walk_f64_kernel<2> : fine_walk_f64_kernel<0>;
    hipLaunchKernelGGL(k, dim3((unsigned)(w.per * 8)), dim3(256), 0, s, g, nrhs, kappa,
                       static_cast<const cplx<double>*>(U), static_cast<const double*>(A),
                       static_cast<const cplx<double>*>(in), static_cast<cplx<double>*>(out), w, fw->nt);
    return hipGetLastError();
  }
  return launch_fine<double>(g, t_bc, mode, kappa, U, A, in, out, nrhs, s, nullptr);
}

hipError_t launch_fine_f64_in32(const Geom& g, double kappa, const void* U, const void* A, const void* in, void* out,
                                int nrhs, hipStream_t s, const FineCfg* cfg) {
  // the traversal order (tile) the autotuner chose for the FP32 kernel at
  // this Nrhs, one RHS per thread
  const bool tuned = cfg && cfg->R > 0 && cfg->order;
  return launch_r<double, 1, 0, 0, float2>(g, tuned ? cfg->order : g.order, kappa, U, A, in, out, nrhs, s);
}

hipError_t launch_fine_dir_f64(const Geom& g, int t_bc, double kappa, const void* U, const void* A, const void* in,
                               void* out, int nrhs, const DirFilter& f, hipStream_t s) {
  (void)t_bc;  // folded into the links
  return launch_r<double, 1, 3>(g, g.order, kappa, U, A, in, out, nrhs, s, f);
}

hipError_t launch_fine_dir_f32(const Geom& g, float kappa, const void* U, const void* A, const void* in, void* out,
                               int nrhs, const DirFilter& f, hipStream_t s) {
  if (nrhs % 2 == 0) return launch_r<float, 2, 3>(g, g.order, kappa, U, A, in, out, nrhs, s, f);
  return launch_r<float, 1, 3>(g, g.order, kappa, U, A, in, out, nrhs, s, f);
}

// FP32: two right-hand sides per thread for even nrhs; FP64: one.  With a
// t-walk configuration (g, parity and ew->on given; FP32 only) the walk
// kernel runs instead of the tiled one, on the same fields.
hipError_t launch_hop_eo(int prec64, int nhalf, const int4* tab, const int* order, const void* U, const void* in,
                         void* out, int nrhs, hipStream_t s, int epi, const void* Ablk, const void* in2,
                         double coef, const Geom* g, int parity, const EoWalk* ew) {
  const bool need_a = epi == 1 || epi == 2 || epi == 4, need_in2 = epi >= 2;
  if (!tab || !order || epi < 0 || epi > 4 || (need_a && !Ablk) || (need_in2 && !in2)) return hipErrorInvalidValue;
  if (!prec64 && g && ew && ew->on) {
    const int R = ew->R ? ew->R : (nrhs % 2 == 0 ? 2 : 1);
    if (R == 2) return launch_hop_eo_walk_r<2>(epi, *g, parity, nrhs, *ew, U, in, out, Ablk, in2, coef, s);
    if (R == 1) return launch_hop_eo_walk_r<1>(epi, *g, parity, nrhs, *ew, U, in, out, Ablk, in2, coef, s);
    return hipErrorInvalidValue;
  }
  if (prec64) return launch_hop_eo_r<double, 1>(epi, nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
  if (nrhs % 2 == 0) return launch_hop_eo_r<float, 2>(epi, nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
  return launch_hop_eo_r<float, 1>(epi, nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, s);
}

bool eo_walk_fits(const Geom& g, const int tile[4], int nrhs, int R) {
  WalkShape w;
  if (R == 0) R = nrhs % 2 == 0 ? 2 : 1;
  return (R == 1 || R == 2) && tile[0] * tile[1] * tile[2] >= kEoWalkMinBlock &&
         eo_walk_shape(g, tile, tile[3], nrhs, R, w);
}

// FP32 epi 2 with the minimal-residual partial sums (see hop_eo_kernel).
// The partials of one launch: sized for one RHS per thread, which bounds
// every nrhs' <= nrhs as well, plus one workgroup per work unit of a t-walk
// whose spatial block has at least kEoWalkMinBlock sites (the walk's units
// may end in a partial workgroup).
size_t hop_eo_dot_scratch_bytes(int nhalf, int nrhs) {
  const long nblocks = ((long)nhalf * nrhs + 255) / 256 + nhalf / kEoWalkMinBlock + 1;
  return (size_t)nblocks * nrhs * sizeof(double4);
}

hipError_t launch_hop_eo_dot(int nhalf, const int4* tab, const int* order, const void* U, const void* in, void* out,
                             const void* Ablk, const void* in2, double coef, int nrhs, void* part, int* nblk,
                             hipStream_t s, const Geom* g, int parity, const EoWalk* ew) {
  if (!tab || !order || !Ablk || !in2 || !part || !nblk || nrhs < 1 || nrhs > 256) return hipErrorInvalidValue;
  if (g && ew && ew->on) {
    if (ew->B[0] * ew->B[1] * ew->B[2] < kEoWalkMinBlock) return hipErrorInvalidValue;
    long nb = 0;
    const int R = ew->R ? ew->R : (nrhs % 2 == 0 ? 2 : 1);
    if (R != 1 && R != 2) return hipErrorInvalidValue;
    hipError_t e = R == 2 ? launch_hop_eo_walk_k<2, 2, false, false, true>(*g, parity, nrhs, *ew, U, in, out, Ablk,
                                                                           in2, coef, part, &nb, s)
                          : launch_hop_eo_walk_k<1, 2, false, false, true>(*g, parity, nrhs, *ew, U, in, out, Ablk,
                                                                           in2, coef, part, &nb, s);
    *nblk = (int)nb;
    return e;
  }
  if (nrhs % 2 == 0)
    return launch_hop_eo_dot_r<2>(nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, part, nblk, s);
  return launch_hop_eo_dot_r<1>(nhalf, nrhs, tab, order, U, in, out, Ablk, in2, coef, part, nblk, s);
}

hipError_t launch_clover_eo(int prec64, int nhalf, const int4* tab, const void* A, const void* in, const void* add,
                            double coef, void* out, int nrhs, hipStream_t s, bool full_in) {
  if (prec64) return launch_clover_eo_r<double, 1>(nhalf, nrhs, tab, A, in, add, coef, out, full_in, s);
  if (nrhs % 2 == 0) return launch_clover_eo_r<float, 2>(nhalf, nrhs, tab, A, in, add, coef, out, full_in, s);
  return launch_clover_eo_r<float, 1>(nhalf, nrhs, tab, A, in, add, coef, out, full_in, s);
}

hipError_t launch_eo_gather(int nhalf, const int4* tab, const void* full, void* half, int nrhs, hipStream_t s) {
  const long n = (long)nhalf * 12 * nrhs;
  hipLaunchKernelGGL(eo_rows_kernel<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nhalf, nrhs, tab,
                     const_cast<float2*>(static_cast<const float2*>(full)), static_cast<float2*>(half));
  return hipGetLastError();
}

hipError_t launch_eo_scatter_add(int nhalf, const int4* tab, void* full, const void* half, int nrhs, hipStream_t s) {
  const long n = (long)nhalf * 12 * nrhs;
  hipLaunchKernelGGL(eo_rows_kernel<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nhalf, nrhs, tab,
                     static_cast<float2*>(full), const_cast<float2*>(static_cast<const float2*>(half)));
  return hipGetLastError();
}

hipError_t launch_clover_invert(long nblk, const void* A64, void* Ai64, void* Ai32, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(clover_invert_kernel, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, s, nblk,
                     static_cast<const double*>(A64), static_cast<double*>(Ai64), static_cast<float*>(Ai32), flag);
  return hipGetLastError();
}

}  // namespace mrhs
