// Batched level-1 linear algebra on MRHS fields (paper Sec. 7: the inner
// products of all right-hand sides are computed simultaneously, in one pass
// over the data, instead of one reduction per right-hand side).
//
// A field is viewed as a row-major matrix of `rows` = nsites*ncomp rows and
// `nrhs` columns of complex numbers; every operation acts column by column.
// Inner products are conjugate-linear in the first argument, products and
// sums are formed in FP64 (FP32 inputs are widened before multiplying), and
// the reduction is deterministic: pass 1 writes one partial per (workgroup,
// column) in a fixed order, pass 2 sums the partials of each column in a
// fixed order.  The result therefore does not depend on timing.
//
// Thread mapping: a workgroup of T = (256 / nrhs) * nrhs threads (or 256 for
// nrhs > 256, which the interface never asks for) covers T / nrhs consecutive
// rows, so thread t always owns column t % nrhs and the loads of a wavefront
// are contiguous in memory.
#include "internal.h"

namespace mrhs {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartialBlocks = 1024;

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

template <typename T>
__device__ __forceinline__ double2 widen(typename c2<T>::type z) {
  return make_double2((double)z.x, (double)z.y);
}

// Pass 1.  MODE 0: <a, b>; MODE 1: ||a||^2 (real part only).
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void dot_partial(const typename c2<T>::type* __restrict__ a,
                                                      const typename c2<T>::type* __restrict__ b, long rows,
                                                      int nrhs, int tpb, double2* __restrict__ partial) {
  __shared__ double2 red[kBlock];
  const int t = threadIdx.x;
  const int rpb = tpb / nrhs;  // rows per sweep of this workgroup
  double2 acc = make_double2(0.0, 0.0);
  if (t < tpb) {
    const int k = t % nrhs;
    const long r0 = (long)blockIdx.x * rpb + t / nrhs;
    const long step = (long)gridDim.x * rpb;
    auto add = [&](const typename c2<T>::type& av, const typename c2<T>::type& bv) {
      const double2 x = widen<T>(av);
      if constexpr (MODE == 0) {
        const double2 y = widen<T>(bv);
        acc.x = fma(x.x, y.x, acc.x);
        acc.x = fma(x.y, y.y, acc.x);
        acc.y = fma(x.x, y.y, acc.y);
        acc.y = fma(-x.y, y.x, acc.y);
      } else {
        acc.x = fma(x.x, x.x, acc.x);
        acc.x = fma(x.y, x.y, acc.x);
      }
    };
    long r = r0;
    // several rows' loads in flight at once (four for one input, two for
    // two inputs); the sums keep the row order
    constexpr int UN = MODE == 0 ? 2 : 4;
    for (; r + (UN - 1) * step < rows; r += UN * step) {
      typename c2<T>::type av[UN], bv[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const long e = (r + u * step) * nrhs + k;
        av[u] = a[e];
        bv[u] = MODE == 0 ? b[e] : av[u];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) add(av[u], bv[u]);
    }
    for (; r < rows; r += step) {
      const long e = r * nrhs + k;
      add(a[e], MODE == 0 ? b[e] : a[e]);
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t < nrhs) {
    double2 s = red[t];
    for (int j = t + nrhs; j < tpb; j += nrhs) {
      s.x += red[j].x;
      s.y += red[j].y;
    }
    partial[(long)blockIdx.x * nrhs + t] = s;
  }
}

// Pass 2: one workgroup per column sums the partials of its column with a
// fixed-shape tree.  MODE 1 writes the real part only (to a double array).
template <int MODE>
__global__ __launch_bounds__(kBlock) void dot_final(const double2* __restrict__ partial, int nblk, int nrhs,
                                                   void* __restrict__ out) {
  __shared__ double2 red[kBlock];
  const int k = blockIdx.x;
  const int t = threadIdx.x;
  double2 s = make_double2(0.0, 0.0);
  for (int j = t; j < nblk; j += kBlock) {
    s.x += partial[(long)j * nrhs + k].x;
    s.y += partial[(long)j * nrhs + k].y;
  }
  red[t] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
      red[t].x += red[t + w].x;
      red[t].y += red[t + w].y;
    }
    __syncthreads();
  }
  if (t == 0) {
    if constexpr (MODE == 0)
      static_cast<double2*>(out)[k] = red[0];
    else
      static_cast<double*>(out)[k] = red[0].x;
  }
}

// y_k <- y_k + alpha_k x_k, alpha complex FP64 per column (device array).
template <typename T>
__global__ __launch_bounds__(kBlock) void axpy_kernel(typename c2<T>::type* __restrict__ y,
                                                      const double2* __restrict__ alpha,
                                                      const typename c2<T>::type* __restrict__ x, long n,
                                                      int nrhs) {
  const long e = (long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const double2 al = alpha[e % nrhs];
  const double2 xv = widen<T>(x[e]);
  const double2 yv = widen<T>(y[e]);
  typename c2<T>::type r;
  r.x = (T)(yv.x + al.x * xv.x - al.y * xv.y);
  r.y = (T)(yv.y + al.x * xv.y + al.y * xv.x);
  y[e] = r;
}

// Multi-dot pass 1: <v_j, w>_k for j < m, reading w once.
struct PtrList {
  const void* p[kMaxMultiDot];
};

template <typename T>
__global__ __launch_bounds__(kBlock) void multidot_partial(PtrList v, int m,
                                                           const typename c2<T>::type* __restrict__ w,
                                                           long rows, int nrhs, int tpb,
                                                           double2* __restrict__ partial) {
  __shared__ double2 red[kBlock];
  using C = typename c2<T>::type;
  const int t = threadIdx.x;
  const int rpb = tpb / nrhs;
  double2 acc[kMaxMultiDot];
#pragma unroll
  for (int j = 0; j < kMaxMultiDot; ++j) acc[j] = make_double2(0.0, 0.0);
  if (t < tpb) {
    const int k = t % nrhs;
    const long r0 = (long)blockIdx.x * rpb + t / nrhs;
    const long step = (long)gridDim.x * rpb;
    for (long r = r0; r < rows; r += step) {
      const long e = r * nrhs + k;
      const double2 y = widen<T>(w[e]);
#pragma unroll
      for (int j = 0; j < kMaxMultiDot; ++j) {
        if (j < m) {
          const double2 x = widen<T>(static_cast<const C*>(v.p[j])[e]);
          acc[j].x = fma(x.x, y.x, acc[j].x);
          acc[j].x = fma(x.y, y.y, acc[j].x);
          acc[j].y = fma(x.x, y.y, acc[j].y);
          acc[j].y = fma(-x.y, y.x, acc[j].y);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxMultiDot; ++j) {
    if (j < m) {  // m is uniform across the workgroup, so the barriers are too
      red[t] = acc[j];
      __syncthreads();
      if (t < nrhs) {
        double2 s = red[t];
        for (int i = t + nrhs; i < tpb; i += nrhs) {
          s.x += red[i].x;
          s.y += red[i].y;
        }
        partial[((long)blockIdx.x * m + j) * nrhs + t] = s;
      }
      __syncthreads();
    }
  }
}

// Multi-dot pass 1 for FP32 fields of even nrhs: each thread owns a pair of
// adjacent columns and reads them as one 16-byte word per row, so a
// wavefront has twice the bytes of the one-column kernel in flight per load
// (that kernel is bound by the latency of its 8-byte loads).  Thread t owns
// columns 2 (t % (nrhs / 2)) and the next; the partial layout is the
// one-column kernel's.  MMAX >= m bounds the accumulators kept in registers.
template <int MMAX>
__global__ __launch_bounds__(kBlock) void multidot_partial_pair(PtrList v, int m, const float4* __restrict__ w,
                                                                long rows, int npair, int tpb,
                                                                double2* __restrict__ partial) {
  __shared__ double2 red[kBlock];
  const int t = threadIdx.x;
  const int rpb = tpb / npair;
  double2 acc[MMAX][2];
#pragma unroll
  for (int j = 0; j < MMAX; ++j) acc[j][0] = acc[j][1] = make_double2(0.0, 0.0);
  if (t < tpb) {
    const int kp = t % npair;
    const long r0 = (long)blockIdx.x * rpb + t / npair;
    const long step = (long)gridDim.x * rpb;
    for (long r = r0; r < rows; r += step) {
      const long e = r * npair + kp;
      const float4 y = w[e];
#pragma unroll
      for (int j = 0; j < MMAX; ++j) {
        if (j < m) {
          const float4 x = static_cast<const float4*>(v.p[j])[e];
          acc[j][0].x = fma((double)x.x, (double)y.x, acc[j][0].x);
          acc[j][0].x = fma((double)x.y, (double)y.y, acc[j][0].x);
          acc[j][0].y = fma((double)x.x, (double)y.y, acc[j][0].y);
          acc[j][0].y = fma(-(double)x.y, (double)y.x, acc[j][0].y);
          acc[j][1].x = fma((double)x.z, (double)y.z, acc[j][1].x);
          acc[j][1].x = fma((double)x.w, (double)y.w, acc[j][1].x);
          acc[j][1].y = fma((double)x.z, (double)y.w, acc[j][1].y);
          acc[j][1].y = fma(-(double)x.w, (double)y.z, acc[j][1].y);
        }
      }
    }
  }
  const int nrhs = 2 * npair;
#pragma unroll
  for (int j = 0; j < MMAX; ++j) {
    if (j < m) {  // m is uniform across the workgroup, so the barriers are too
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        red[t] = acc[j][c];
        __syncthreads();
        if (t < npair) {
          double2 s = red[t];
          for (int i = t + npair; i < tpb; i += npair) {
            s.x += red[i].x;
            s.y += red[i].y;
          }
          partial[((long)blockIdx.x * m + j) * nrhs + 2 * t + c] = s;
        }
        __syncthreads();
      }
    }
  }
}

int threads_per_block(int nrhs) { return nrhs >= kBlock ? kBlock : (kBlock / nrhs) * nrhs; }

int partial_blocks(long rows, int nrhs) {
  const long rpb = threads_per_block(nrhs) / nrhs;
  long nb = (rows + rpb - 1) / rpb;
  // enough workgroups to fill the chip several times; fewer partials keep pass 2 short
  if (nb > kMaxPartialBlocks) nb = kMaxPartialBlocks;
  return (int)(nb < 1 ? 1 : nb);
}

}  // namespace

size_t blas_scratch_bytes(int nrhs, int m) { return (size_t)kMaxPartialBlocks * nrhs * (m < 1 ? 1 : m) * 16; }

hipError_t launch_dot(int prec64, int mode, const void* a, const void* b, long rows, int nrhs, void* out,
                      void* scratch, hipStream_t s) {
  const int tpb = threads_per_block(nrhs);
  const int nb = partial_blocks(rows, nrhs);
  double2* part = static_cast<double2*>(scratch);
  if (prec64) {
    if (mode == 0)
      hipLaunchKernelGGL((dot_partial<double, 0>), dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const double2*>(a), static_cast<const double2*>(b), rows, nrhs, tpb, part);
    else
      hipLaunchKernelGGL((dot_partial<double, 1>), dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const double2*>(a), static_cast<const double2*>(a), rows, nrhs, tpb, part);
  } else {
    if (mode == 0)
      hipLaunchKernelGGL((dot_partial<float, 0>), dim3(nb), dim3(kBlock), 0, s, static_cast<const float2*>(a),
                         static_cast<const float2*>(b), rows, nrhs, tpb, part);
    else
      hipLaunchKernelGGL((dot_partial<float, 1>), dim3(nb), dim3(kBlock), 0, s, static_cast<const float2*>(a),
                         static_cast<const float2*>(a), rows, nrhs, tpb, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == 0)
    hipLaunchKernelGGL((dot_final<0>), dim3(nrhs), dim3(kBlock), 0, s, part, nb, nrhs, out);
  else
    hipLaunchKernelGGL((dot_final<1>), dim3(nrhs), dim3(kBlock), 0, s, part, nb, nrhs, out);
  return hipGetLastError();
}

hipError_t launch_multi_dot(int prec64, const void* const* v, int m, const void* w, long rows, int nrhs,
                            void* out, void* scratch, hipStream_t s) {
  if (m < 1 || m > kMaxMultiDot) return hipErrorInvalidValue;
  PtrList pl{};
  for (int j = 0; j < m; ++j) pl.p[j] = v[j];
  const int tpb = threads_per_block(nrhs);
  const int nb = partial_blocks(rows, nrhs);
  double2* part = static_cast<double2*>(scratch);
  if (prec64) {
    hipLaunchKernelGGL((multidot_partial<double>), dim3(nb), dim3(kBlock), 0, s, pl, m,
                       static_cast<const double2*>(w), rows, nrhs, tpb, part);
  } else if (nrhs % 2 == 0) {
    // column pairs as 16-byte words; at most as many workgroups as the one-column kernel
    const int npair = nrhs / 2;
    const int tpb2 = threads_per_block(npair);
    const int nb2 = partial_blocks(rows, npair);
    if (m <= 4)
      hipLaunchKernelGGL((multidot_partial_pair<4>), dim3(nb2), dim3(kBlock), 0, s, pl, m,
                         static_cast<const float4*>(w), rows, npair, tpb2, part);
    else if (m <= 10)
      hipLaunchKernelGGL((multidot_partial_pair<10>), dim3(nb2), dim3(kBlock), 0, s, pl, m,
                         static_cast<const float4*>(w), rows, npair, tpb2, part);
    else
      hipLaunchKernelGGL((multidot_partial_pair<kMaxMultiDot>), dim3(nb2), dim3(kBlock), 0, s, pl, m,
                         static_cast<const float4*>(w), rows, npair, tpb2, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((dot_final<0>), dim3(m * nrhs), dim3(kBlock), 0, s, part, nb2, m * nrhs, out);
    return hipGetLastError();
  } else {
    hipLaunchKernelGGL((multidot_partial<float>), dim3(nb), dim3(kBlock), 0, s, pl, m,
                       static_cast<const float2*>(w), rows, nrhs, tpb, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the partials of (block, j) for column k sit at ((block * m + j) * nrhs + k): viewed as
  // nb blocks of m*nrhs columns, pass 2 is the ordinary column sum
  hipLaunchKernelGGL((dot_final<0>), dim3(m * nrhs), dim3(kBlock), 0, s, part, nb, m * nrhs, out);
  return hipGetLastError();
}

hipError_t launch_axpy(int prec64, void* y, const void* alpha_dev, const void* x, long rows, int nrhs,
                       hipStream_t s) {
  const long n = rows * nrhs;
  const int nb = (int)((n + kBlock - 1) / kBlock);
  if (prec64)
    hipLaunchKernelGGL((axpy_kernel<double>), dim3(nb), dim3(kBlock), 0, s, static_cast<double2*>(y),
                       static_cast<const double2*>(alpha_dev), static_cast<const double2*>(x), n, nrhs);
  else
    hipLaunchKernelGGL((axpy_kernel<float>), dim3(nb), dim3(kBlock), 0, s, static_cast<float2*>(y),
                       static_cast<const double2*>(alpha_dev), static_cast<const float2*>(x), n, nrhs);
  return hipGetLastError();
}

}  // namespace mrhs
