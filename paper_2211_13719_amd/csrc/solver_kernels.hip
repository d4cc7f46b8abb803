// Level-1 kernels of the solver on MRHS fields [rows][nrhs] (rows = sites x
// components), every right-hand side with its own scalars, which live in
// device memory so that a whole smoothing sweep runs without the host.
//
//   minimal-residual step (smoother):  alpha_k = <p_k, r_k> / ||p_k||^2,
//                                      x_k += alpha_k r_k,  r_k -= alpha_k p_k
//   Gram-Schmidt update (outer Krylov): y_k += s sum_i c_{i,k} x_{i,k}
//   column scaling, normalisation, differences, zero fill.
//
// Reductions are deterministic (fixed-order partials, then a fixed tree),
// with FP64 sums.
#include "internal.h"

namespace mrhs {
namespace {

constexpr int kB = 256;
constexpr int kMaxPart = 1024;

template <typename T>
struct c2;
template <>
struct c2<float> {
  using type = float2;
};
template <>
struct c2<double> {
  using type = double2;
};

int tpb_of(int nrhs) { return (kB / nrhs) * nrhs; }
int nblk_of(long rows, int nrhs) {
  const long rpb = tpb_of(nrhs) / nrhs;
  long nb = (rows + rpb - 1) / rpb;
  if (nb > kMaxPart) nb = kMaxPart;
  return (int)(nb < 1 ? 1 : nb);
}

// partial[b][k] = (Re <p,r>, Im <p,r>, ||p||^2, 0)
__global__ __launch_bounds__(kB) void mr_partial(const float2* __restrict__ p, const float2* __restrict__ r, long rows,
                                                 int nrhs, int tpb, double4* __restrict__ part) {
  __shared__ double4 red[kB];
  const int t = threadIdx.x;
  double4 acc = make_double4(0, 0, 0, 0);
  if (t < tpb) {
    const int k = t % nrhs;
    const int rpb = tpb / nrhs;
    const long step = (long)gridDim.x * rpb;
    for (long row = (long)blockIdx.x * rpb + t / nrhs; row < rows; row += step) {
      const long e = row * nrhs + k;
      const float2 a = p[e], b = r[e];
      const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
      acc.x = fma(ax, bx, fma(ay, by, acc.x));
      acc.y = fma(ax, by, fma(-ay, bx, acc.y));
      acc.z = fma(ax, ax, fma(ay, ay, acc.z));
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t < nrhs) {
    double4 s = red[t];
    for (int j = t + nrhs; j < tpb; j += nrhs) {
      s.x += red[j].x;
      s.y += red[j].y;
      s.z += red[j].z;
    }
    part[(long)blockIdx.x * nrhs + t] = s;
  }
}

__global__ __launch_bounds__(kB) void mr_final(const double4* __restrict__ part, int nblk, int nrhs,
                                               double2* __restrict__ alpha) {
  __shared__ double4 red[kB];
  const int k = blockIdx.x, t = threadIdx.x;
  double4 s = make_double4(0, 0, 0, 0);
  auto add = [&](const double4& v) {
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
  };
  // four loads in flight; the sum keeps the order j = t, t + kB, ...
  int j = t;
  for (; j + 3 * kB < nblk; j += 4 * kB) {
    double4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[(long)(j + u * kB) * nrhs + k];
#pragma unroll
    for (int u = 0; u < 4; ++u) add(v[u]);
  }
  for (; j < nblk; j += kB) add(part[(long)j * nrhs + k]);
  red[t] = s;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if (t < w) {
      red[t].x += red[t + w].x;
      red[t].y += red[t + w].y;
      red[t].z += red[t + w].z;
    }
    __syncthreads();
  }
  if (t == 0) {
    const double pp = red[0].z;
    alpha[k] = pp > 0.0 ? make_double2(red[0].x / pp, red[0].y / pp) : make_double2(0.0, 0.0);
  }
}

// x += alpha r ; r -= alpha p  (FP32 fields)
__global__ __launch_bounds__(kB) void mr_update(float2* __restrict__ x, float2* __restrict__ r,
                                                const float2* __restrict__ p, const double2* __restrict__ alpha,
                                                long n, int nrhs) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  const double2 a = alpha[e % nrhs];
  const float ar = (float)a.x, ai = (float)a.y;
  const float2 rv = r[e], pv = p[e];
  float2 xv = x[e];
  xv.x = fmaf(ar, rv.x, fmaf(-ai, rv.y, xv.x));
  xv.y = fmaf(ar, rv.y, fmaf(ai, rv.x, xv.y));
  float2 rn;
  rn.x = fmaf(-ar, pv.x, fmaf(ai, pv.y, rv.x));
  rn.y = fmaf(-ar, pv.y, fmaf(-ai, pv.x, rv.y));
  x[e] = xv;
  r[e] = rn;
}

// y_k += s sum_i c[i][k] x_i   (y FP64; x_i FP32 or FP64)
struct Ptrs {
  const void* p[kMaxMultiDot];
};
template <typename TX>
__global__ __launch_bounds__(kB) void multi_axpy(double2* __restrict__ y, const double2* __restrict__ c, Ptrs xs,
                                                 int m, double s, long n, int nrhs) {
  using CX = typename c2<TX>::type;
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  const int k = (int)(e % nrhs);
  double2 acc = y[e];
#pragma unroll 4
  for (int i = 0; i < m; ++i) {
    const CX xv = static_cast<const CX*>(xs.p[i])[e];
    const double2 ci = c[i * nrhs + k];
    const double cr = s * ci.x, cim = s * ci.y;
    acc.x = fma(cr, (double)xv.x, fma(-cim, (double)xv.y, acc.x));
    acc.y = fma(cr, (double)xv.y, fma(cim, (double)xv.x, acc.y));
  }
  y[e] = acc;
}

// y_k = yin_k + s sum_i c[i][k] x_i (y, yin, x_i all FP64 or all FP32, the
// arithmetic in FP64; y may be yin) and, in the same pass, the FP32 rounding
// of an FP64 y into y32 (if given) and the partial sums of ||y_k||^2 of the
// stored y: partial[b][k], fixed order.
// cs (if given): a real factor per (i, column), cs[i * nrhs + k], multiplying c.
template <typename T>
__global__ __launch_bounds__(kB) void multi_axpy_norm(typename c2<T>::type* y, float2* __restrict__ y32,
                                                      const typename c2<T>::type* yin,
                                                      const double2* __restrict__ c, const double* __restrict__ cs,
                                                      Ptrs xs, int m, double s, long rows, int nrhs, int tpb,
                                                      double* __restrict__ part) {
  using CT = typename c2<T>::type;
  __shared__ double red[kB];
  const int t = threadIdx.x;
  double acc2 = 0.0;
  if (t < tpb) {
    const int k = t % nrhs;
    const int rpb = tpb / nrhs;
    const long step = (long)gridDim.x * rpb;
    for (long row = (long)blockIdx.x * rpb + t / nrhs; row < rows; row += step) {
      const long e = row * nrhs + k;
      const CT y0 = yin[e];
      double2 acc = make_double2((double)y0.x, (double)y0.y);
#pragma unroll 4
      for (int i = 0; i < m; ++i) {
        const CT xv = static_cast<const CT*>(xs.p[i])[e];
        const double2 ci = c[i * nrhs + k];
        const double f = cs ? s * cs[i * nrhs + k] : s;
        const double cr = f * ci.x, cim = f * ci.y;
        acc.x = fma(cr, (double)xv.x, fma(-cim, (double)xv.y, acc.x));
        acc.y = fma(cr, (double)xv.y, fma(cim, (double)xv.x, acc.y));
      }
      CT out;
      out.x = (T)acc.x;
      out.y = (T)acc.y;
      y[e] = out;
      if constexpr (sizeof(T) == 8) {
        if (y32) y32[e] = make_float2((float)acc.x, (float)acc.y);
      }
      acc2 = fma((double)out.x, (double)out.x, fma((double)out.y, (double)out.y, acc2));
    }
  }
  red[t] = acc2;
  __syncthreads();
  if (t < nrhs) {
    double v = red[t];
    for (int j = t + nrhs; j < tpb; j += nrhs) v += red[j];
    part[(long)blockIdx.x * nrhs + t] = v;
  }
}

// multi_axpy_norm for FP32 fields of even nrhs: each thread owns a pair of
// adjacent columns, read and written as one 16-byte word per row (twice the
// bytes in flight per load of the one-column kernel); same arithmetic per
// element, partials part[b][k] in the same layout.
__global__ __launch_bounds__(kB) void multi_axpy_norm_pair(float4* y, const float4* yin,
                                                           const double2* __restrict__ c, const double* __restrict__ cs,
                                                           Ptrs xs, int m, double s, long rows, int npair, int tpb,
                                                           double* __restrict__ part) {
  __shared__ double red[kB];
  const int t = threadIdx.x;
  const int nrhs = 2 * npair;
  double acc2[2] = {0.0, 0.0};
  if (t < tpb) {
    const int kp = t % npair;
    const int rpb = tpb / npair;
    const long step = (long)gridDim.x * rpb;
    const int k0 = 2 * kp;
    for (long row = (long)blockIdx.x * rpb + t / npair; row < rows; row += step) {
      const long e = row * npair + kp;
      const float4 y0 = yin[e];
      double2 a0 = make_double2((double)y0.x, (double)y0.y), a1 = make_double2((double)y0.z, (double)y0.w);
#pragma unroll 4
      for (int i = 0; i < m; ++i) {
        const float4 xv = static_cast<const float4*>(xs.p[i])[e];
        const double2 c0 = c[i * nrhs + k0], c1 = c[i * nrhs + k0 + 1];
        const double f0 = cs ? s * cs[i * nrhs + k0] : s, f1 = cs ? s * cs[i * nrhs + k0 + 1] : s;
        const double r0 = f0 * c0.x, i0 = f0 * c0.y, r1 = f1 * c1.x, i1 = f1 * c1.y;
        a0.x = fma(r0, (double)xv.x, fma(-i0, (double)xv.y, a0.x));
        a0.y = fma(r0, (double)xv.y, fma(i0, (double)xv.x, a0.y));
        a1.x = fma(r1, (double)xv.z, fma(-i1, (double)xv.w, a1.x));
        a1.y = fma(r1, (double)xv.w, fma(i1, (double)xv.z, a1.y));
      }
      const float4 out = make_float4((float)a0.x, (float)a0.y, (float)a1.x, (float)a1.y);
      y[e] = out;
      acc2[0] = fma((double)out.x, (double)out.x, fma((double)out.y, (double)out.y, acc2[0]));
      acc2[1] = fma((double)out.z, (double)out.z, fma((double)out.w, (double)out.w, acc2[1]));
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    red[t] = acc2[h];
    __syncthreads();
    if (t < npair) {
      double v = red[t];
      for (int j = t + npair; j < tpb; j += npair) v += red[j];
      part[(long)blockIdx.x * nrhs + 2 * t + h] = v;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kB) void col_sum_final(const double* __restrict__ part, int nblk, int nrhs,
                                                    double* __restrict__ out) {
  __shared__ double red[kB];
  const int k = blockIdx.x, t = threadIdx.x;
  double v = 0.0;
  for (int j = t; j < nblk; j += kB) v += part[(long)j * nrhs + k];
  red[t] = v;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[k] = red[0];
}

// y_k = s_k x_k, s real per column (device array)
template <typename T>
__global__ __launch_bounds__(kB) void scale_cols(typename c2<T>::type* __restrict__ y,
                                                 const typename c2<T>::type* __restrict__ x,
                                                 const double* __restrict__ s, long n, int nrhs) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  const T f = (T)s[e % nrhs];
  typename c2<T>::type v = x[e];
  v.x *= f;
  v.y *= f;
  y[e] = v;
}

// s_k = f / sqrt(q_k)  (0 if q_k == 0)
__global__ void inv_sqrt_cols(const double* __restrict__ q, double* __restrict__ s, int nrhs, double f) {
  const int k = threadIdx.x;
  if (k < nrhs) s[k] = q[k] > 0.0 ? f / sqrt(q[k]) : 0.0;
}

template <typename T>
__global__ __launch_bounds__(kB) void sub_fields(typename c2<T>::type* __restrict__ out,
                                                 const typename c2<T>::type* __restrict__ a,
                                                 const typename c2<T>::type* __restrict__ b, long n) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  typename c2<T>::type u = a[e], v = b[e];
  u.x -= v.x;
  u.y -= v.y;
  out[e] = u;
}

// out = a - b in FP64 and, if out32 is given, its FP32 rounding too
// out = a - b in FP64 (out may be b) and its FP32 rounding into out32 (if given)
__global__ __launch_bounds__(kB) void sub_dual(double2* out, float2* __restrict__ out32,
                                               const double2* __restrict__ a, const double2* b, long n) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  double2 u = a[e];
  const double2 v = b[e];
  u.x -= v.x;
  u.y -= v.y;
  out[e] = u;
  if (out32) out32[e] = make_float2((float)u.x, (float)u.y);
}

__global__ __launch_bounds__(kB) void add_f32(float2* __restrict__ y, const float2* __restrict__ x, long n) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  float2 u = y[e];
  const float2 v = x[e];
  u.x += v.x;
  u.y += v.y;
  y[e] = u;
}

// y += c x for n complex FP32 values (real c).
__global__ __launch_bounds__(kB) void axpy_f32(float2* __restrict__ y, const float2* __restrict__ x, float c, long n) {
  for (long e = (long)blockIdx.x * kB + threadIdx.x; e < n; e += (long)gridDim.x * kB) {
    const float2 a = y[e], b = x[e];
    y[e] = make_float2(fmaf(c, b.x, a.x), fmaf(c, b.y, a.y));
  }
}

__global__ __launch_bounds__(kB) void zero_words(uint4* __restrict__ p, long n16) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e < n16) p[e] = make_uint4(0, 0, 0, 0);
}

int grid_of(long n) { return (int)((n + kB - 1) / kB); }

// One minimal-residual step of the Schwarz block solves on the blocks of one
// colour, one workgroup per block (its whole block in one workgroup, so the
// step length needs no global reduction): with q = D_B rho,
//   alpha = <q, rho>_B / ||q||^2_B per column (FP64 sums over the block's sites
//   and components, fixed order),  x += alpha rho,  rho -= alpha q  (FP32).
// Blocks are the aggregates of a (extent a.b, a.C blocks per direction).
__global__ __launch_bounds__(kB) void sap_block_mr(AggGeom a, int nrhs, int color, float2* __restrict__ x,
                                                   float2* __restrict__ rho, const float2* __restrict__ q) {
  __shared__ double4 red[kB];
  __shared__ double2 al[kB];
  const int B = blockIdx.x;
  const int X = B % a.C[0], Y = (B / a.C[0]) % a.C[1], Z = (B / (a.C[0] * a.C[1])) % a.C[2],
            T = B / (a.C[0] * a.C[1] * a.C[2]);
  if (((X + Y + Z + T) & 1) != color) return;  // whole workgroup
  const int nsb = a.b[0] * a.b[1] * a.b[2] * a.b[3];
  const long rows = (long)nsb * 12;
  const int tpb = (kB / nrhs) * nrhs, rpb = tpb / nrhs;
  const int t = threadIdx.x, k = t % nrhs;
  // element offset of block row j (local site j / 12, component j % 12), column k
  auto elem = [&](long j) {
    int ls = (int)(j / 12);
    const int c = (int)(j % 12);
    const int lx = ls % a.b[0];
    ls /= a.b[0];
    const int ly = ls % a.b[1];
    ls /= a.b[1];
    const int lz = ls % a.b[2];
    const int lt = ls / a.b[2];
    const long s = (long)(X * a.b[0] + lx) +
                   (long)a.L[0] * ((Y * a.b[1] + ly) + (long)a.L[1] * ((Z * a.b[2] + lz) + (long)a.L[2] * (T * a.b[3] + lt)));
    return (s * 12 + c) * nrhs + k;
  };
  double4 acc = make_double4(0, 0, 0, 0);
  if (t < tpb) {
    for (long j = t / nrhs; j < rows; j += rpb) {
      const long e = elem(j);
      const float2 qv = q[e], rv = rho[e];
      const double qx = qv.x, qy = qv.y, rx = rv.x, ry = rv.y;
      acc.x = fma(qx, rx, fma(qy, ry, acc.x));
      acc.y = fma(qx, ry, fma(-qy, rx, acc.y));
      acc.z = fma(qx, qx, fma(qy, qy, acc.z));
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t < nrhs) {
    double4 sm = red[t];
    for (int j = t + nrhs; j < tpb; j += nrhs) {
      sm.x += red[j].x;
      sm.y += red[j].y;
      sm.z += red[j].z;
    }
    al[t] = sm.z > 0.0 ? make_double2(sm.x / sm.z, sm.y / sm.z) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (t >= tpb) return;
  const double2 av = al[k];
  const float ar = (float)av.x, ai = (float)av.y;
  for (long j = t / nrhs; j < rows; j += rpb) {
    const long e = elem(j);
    const float2 rv = rho[e], qv = q[e];
    float2 xv = x[e];
    xv.x = fmaf(ar, rv.x, fmaf(-ai, rv.y, xv.x));
    xv.y = fmaf(ar, rv.y, fmaf(ai, rv.x, xv.y));
    x[e] = xv;
    float2 rn;
    rn.x = fmaf(-ar, qv.x, fmaf(ai, qv.y, rv.x));
    rn.y = fmaf(-ar, qv.y, fmaf(-ai, qv.x, rv.y));
    rho[e] = rn;
  }
}

// Gram matrix of the nv <= 16 columns of one field, G[a][b] = sum_rows
// conj(v_a) v_b: workgroup partials over row ranges (rows staged in LDS,
// thread (a, b) accumulates one entry in FP64), then a fixed-order sum.
constexpr int kGramRows = 64;

__global__ __launch_bounds__(kB) void col_gram_partial(const float2* __restrict__ v, long rows, int nv, long per,
                                                       double2* __restrict__ part) {
  __shared__ float2 tile[kGramRows * 16];
  const int a = threadIdx.x >> 4, b = threadIdx.x & 15;
  const long r0 = (long)blockIdx.x * per, r1 = min(rows, r0 + per);
  double re = 0.0, im = 0.0;
  for (long base = r0; base < r1; base += kGramRows) {
    const int nr = (int)min((long)kGramRows, r1 - base);
    for (int e = threadIdx.x; e < nr * nv; e += kB) tile[(e / nv) * 16 + e % nv] = v[base * nv + e];
    __syncthreads();
    if (a < nv && b < nv) {
      for (int r = 0; r < nr; ++r) {
        const float2 x = tile[r * 16 + a], y = tile[r * 16 + b];
        re += (double)x.x * y.x + (double)x.y * y.y;
        im += (double)x.x * y.y - (double)x.y * y.x;
      }
    }
    __syncthreads();
  }
  part[(size_t)blockIdx.x * 256 + threadIdx.x] = make_double2(re, im);
}

__global__ __launch_bounds__(kB) void col_gram_final(const double2* __restrict__ part, int nblk,
                                                     double2* __restrict__ g) {
  double re = 0.0, im = 0.0;
  for (int i = 0; i < nblk; ++i) {
    const double2 p = part[(size_t)i * 256 + threadIdx.x];
    re += p.x;
    im += p.y;
  }
  g[threadIdx.x] = make_double2(re, im);
}

// v <- v T for an upper-triangular nv x nv matrix T (row a, column b at 16 a + b).
__global__ __launch_bounds__(kB) void col_transform(float2* __restrict__ v, long rows, int nv,
                                                    const float2* __restrict__ T) {
  __shared__ float2 t[256];
  t[threadIdx.x] = T[threadIdx.x];
  __syncthreads();
  const long r = (long)blockIdx.x * kB + threadIdx.x;
  if (r >= rows) return;
  float2 x[16], y[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) x[a] = a < nv ? v[r * nv + a] : make_float2(0.f, 0.f);
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int a = 0; a <= b; ++a) {
      const float2 c = t[16 * a + b];
      re = fmaf(x[a].x, c.x, fmaf(-x[a].y, c.y, re));
      im = fmaf(x[a].x, c.y, fmaf(x[a].y, c.x, im));
    }
    y[b] = make_float2(re, im);
  }
#pragma unroll
  for (int b = 0; b < 16; ++b)
    if (b < nv) v[r * nv + b] = y[b];
}

}  // namespace

size_t solver_scratch_bytes(int nrhs) { return (size_t)kMaxPart * nrhs * sizeof(double4); }

hipError_t launch_mr_alpha(const void* p, const void* r, long rows, int nrhs, void* alpha, void* scratch,
                           hipStream_t s) {
  const int tpb = tpb_of(nrhs), nb = nblk_of(rows, nrhs);
  hipLaunchKernelGGL(mr_partial, dim3(nb), dim3(kB), 0, s, static_cast<const float2*>(p),
                     static_cast<const float2*>(r), rows, nrhs, tpb, static_cast<double4*>(scratch));
  hipLaunchKernelGGL(mr_final, dim3(nrhs), dim3(kB), 0, s, static_cast<const double4*>(scratch), nb, nrhs,
                     static_cast<double2*>(alpha));
  return hipGetLastError();
}

hipError_t launch_mr_final(const void* part, int nblk, int nrhs, void* alpha, hipStream_t s) {
  hipLaunchKernelGGL(mr_final, dim3(nrhs), dim3(kB), 0, s, static_cast<const double4*>(part), nblk, nrhs,
                     static_cast<double2*>(alpha));
  return hipGetLastError();
}

hipError_t launch_mr_update(void* x, void* r, const void* p, const void* alpha, long rows, int nrhs, hipStream_t s) {
  const long n = rows * nrhs;
  hipLaunchKernelGGL(mr_update, dim3(grid_of(n)), dim3(kB), 0, s, static_cast<float2*>(x), static_cast<float2*>(r),
                     static_cast<const float2*>(p), static_cast<const double2*>(alpha), n, nrhs);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(int x64, void* y, const void* coef, const void* const* xs, int m, double sgn, long rows,
                             int nrhs, hipStream_t s) {
  if (m < 1 || m > kMaxMultiDot) return hipErrorInvalidValue;
  Ptrs P{};
  for (int i = 0; i < m; ++i) P.p[i] = xs[i];
  const long n = rows * nrhs;
  if (x64)
    hipLaunchKernelGGL((multi_axpy<double>), dim3(grid_of(n)), dim3(kB), 0, s, static_cast<double2*>(y),
                       static_cast<const double2*>(coef), P, m, sgn, n, nrhs);
  else
    hipLaunchKernelGGL((multi_axpy<float>), dim3(grid_of(n)), dim3(kB), 0, s, static_cast<double2*>(y),
                       static_cast<const double2*>(coef), P, m, sgn, n, nrhs);
  return hipGetLastError();
}

hipError_t launch_scale_cols(int prec64, void* y, const void* x, const double* sdev, long rows, int nrhs,
                             hipStream_t s) {
  const long n = rows * nrhs;
  if (prec64)
    hipLaunchKernelGGL((scale_cols<double>), dim3(grid_of(n)), dim3(kB), 0, s, static_cast<double2*>(y),
                       static_cast<const double2*>(x), sdev, n, nrhs);
  else
    hipLaunchKernelGGL((scale_cols<float>), dim3(grid_of(n)), dim3(kB), 0, s, static_cast<float2*>(y),
                       static_cast<const float2*>(x), sdev, n, nrhs);
  return hipGetLastError();
}

hipError_t launch_inv_sqrt(const double* q, double* sdev, int nrhs, double f, hipStream_t s) {
  hipLaunchKernelGGL(inv_sqrt_cols, dim3(1), dim3(64), 0, s, q, sdev, nrhs, f);
  return hipGetLastError();
}

hipError_t launch_sub(int prec64, void* out, const void* a, const void* b, long n, hipStream_t s) {
  if (prec64)
    hipLaunchKernelGGL((sub_fields<double>), dim3(grid_of(n)), dim3(kB), 0, s, static_cast<double2*>(out),
                       static_cast<const double2*>(a), static_cast<const double2*>(b), n);
  else
    hipLaunchKernelGGL((sub_fields<float>), dim3(grid_of(n)), dim3(kB), 0, s, static_cast<float2*>(out),
                       static_cast<const float2*>(a), static_cast<const float2*>(b), n);
  return hipGetLastError();
}

hipError_t launch_sap_block_mr(const AggGeom& a, int nrhs, int color, void* x, void* rho, const void* q, hipStream_t s) {
  if (nrhs < 1 || nrhs > kB || (color != 0 && color != 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sap_block_mr, dim3((unsigned)a.Vc), dim3(kB), 0, s, a, nrhs, color, static_cast<float2*>(x),
                     static_cast<float2*>(rho), static_cast<const float2*>(q));
  return hipGetLastError();
}

hipError_t launch_sub_dual(void* out, void* out32, const void* a, const void* b, long n, hipStream_t s) {
  hipLaunchKernelGGL(sub_dual, dim3(grid_of(n)), dim3(kB), 0, s, static_cast<double2*>(out), static_cast<float2*>(out32),
                     static_cast<const double2*>(a), static_cast<const double2*>(b), n);
  return hipGetLastError();
}

hipError_t launch_add_f32(void* y, const void* x, long n, hipStream_t s) {
  hipLaunchKernelGGL(add_f32, dim3(grid_of(n)), dim3(kB), 0, s, static_cast<float2*>(y), static_cast<const float2*>(x),
                     n);
  return hipGetLastError();
}

hipError_t launch_axpy_f32(void* y, const void* x, double c, long n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_f32, dim3(grid_of(n)), dim3(kB), 0, s, static_cast<float2*>(y), static_cast<const float2*>(x),
                     (float)c, n);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes % 16) return hipErrorInvalidValue;
  const long n16 = (long)(bytes / 16);
  hipLaunchKernelGGL(zero_words, dim3(grid_of(n16)), dim3(kB), 0, s, static_cast<uint4*>(p), n16);
  return hipGetLastError();
}

}  // namespace mrhs

namespace mrhs {

size_t col_gram_scratch_bytes() { return (size_t)kMaxPart * 256 * sizeof(double2); }

hipError_t launch_col_gram(const void* v, long rows, int nv, void* scratch, void* g, hipStream_t s) {
  if (nv < 1 || nv > 16) return hipErrorInvalidValue;
  long nb = (rows + kGramRows - 1) / kGramRows;
  if (nb > kMaxPart) nb = kMaxPart;
  if (nb < 1) nb = 1;
  const long per = ((rows + nb - 1) / nb + kGramRows - 1) / kGramRows * kGramRows;
  nb = (rows + per - 1) / per;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(col_gram_partial, dim3((unsigned)nb), dim3(kB), 0, s, static_cast<const float2*>(v), rows, nv,
                     per, static_cast<double2*>(scratch));
  hipLaunchKernelGGL(col_gram_final, dim3(1), dim3(kB), 0, s, static_cast<const double2*>(scratch), (int)nb,
                     static_cast<double2*>(g));
  return hipGetLastError();
}

hipError_t launch_col_transform(void* v, long rows, int nv, const void* T, hipStream_t s) {
  if (nv < 1 || nv > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(col_transform, dim3((unsigned)((rows + kB - 1) / kB)), dim3(kB), 0, s, static_cast<float2*>(v),
                     rows, nv, static_cast<const float2*>(T));
  return hipGetLastError();
}

// prec64: y, yin and the x_i FP64 (y32 optional), else all FP32 (y32 unused)
hipError_t launch_multi_axpy_norm(int prec64, void* y, void* y32, const void* yin, const void* coef,
                                 const void* cscale, const void* const* xs, int m, double sgn, long rows, int nrhs,
                                 void* norms, void* scratch, hipStream_t s) {
  if (m < 1 || m > kMaxMultiDot || nrhs < 1 || nrhs > kB || (!prec64 && y32)) return hipErrorInvalidValue;
  Ptrs p{};
  for (int i = 0; i < m; ++i) p.p[i] = xs[i];
  const int tpb = tpb_of(nrhs), nb = nblk_of(rows, nrhs);
  if (prec64)
    hipLaunchKernelGGL(multi_axpy_norm<double>, dim3(nb), dim3(kB), 0, s, static_cast<double2*>(y),
                       static_cast<float2*>(y32), static_cast<const double2*>(yin), static_cast<const double2*>(coef),
                       static_cast<const double*>(cscale), p, m, sgn, rows, nrhs, tpb, static_cast<double*>(scratch));
  else if (nrhs % 2 == 0) {
    const int npair = nrhs / 2, tpb2 = tpb_of(npair), nb2 = nblk_of(rows, npair);
    hipLaunchKernelGGL(multi_axpy_norm_pair, dim3(nb2), dim3(kB), 0, s, static_cast<float4*>(y),
                       static_cast<const float4*>(yin), static_cast<const double2*>(coef),
                       static_cast<const double*>(cscale), p, m, sgn, rows, npair, tpb2,
                       static_cast<double*>(scratch));
    hipLaunchKernelGGL(col_sum_final, dim3(nrhs), dim3(kB), 0, s, static_cast<const double*>(scratch), nb2, nrhs,
                       static_cast<double*>(norms));
    return hipGetLastError();
  } else
    hipLaunchKernelGGL(multi_axpy_norm<float>, dim3(nb), dim3(kB), 0, s, static_cast<float2*>(y), nullptr,
                       static_cast<const float2*>(yin), static_cast<const double2*>(coef),
                       static_cast<const double*>(cscale), p, m, sgn, rows, nrhs, tpb, static_cast<double*>(scratch));
  hipLaunchKernelGGL(col_sum_final, dim3(nrhs), dim3(kB), 0, s, static_cast<const double*>(scratch), nb, nrhs,
                     static_cast<double*>(norms));
  return hipGetLastError();
}



}  // namespace mrhs
