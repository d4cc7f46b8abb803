// Site <-> aggregate index maps of the aggregation multigrid, shared by the
// intergrid kernels.  Aggregates are blocks b = (bx, by, bz, bt) of sites,
// A = X + Cx (Y + Cy (Z + Cz T)); inside an aggregate, sites are numbered
// lexicographically with x fastest.
#pragma once

#include "internal.h"

namespace mrhs {

// Fine site of local offset l inside aggregate A.
__device__ __forceinline__ int agg_site(const AggGeom& a, int A, int l) {
  const int X = A % a.C[0];
  int r = A / a.C[0];
  const int Y = r % a.C[1];
  r /= a.C[1];
  const int Z = r % a.C[2];
  const int Tt = r / a.C[2];
  const int lx = l % a.b[0];
  int q = l / a.b[0];
  const int ly = q % a.b[1];
  q /= a.b[1];
  const int lz = q % a.b[2];
  const int lt = q / a.b[2];
  const int x = X * a.b[0] + lx, y = Y * a.b[1] + ly, z = Z * a.b[2] + lz, t = Tt * a.b[3] + lt;
  return x + a.L[0] * (y + a.L[1] * (z + a.L[2] * t));
}

__device__ __forceinline__ int site_agg(const AggGeom& a, int s) {
  const int x = s % a.L[0];
  int r = s / a.L[0];
  const int y = r % a.L[1];
  r /= a.L[1];
  const int z = r % a.L[2];
  const int t = r / a.L[2];
  return x / a.b[0] + a.C[0] * (y / a.b[1] + a.C[1] * (z / a.b[2] + a.C[2] * (t / a.b[3])));
}

// Matrix-core intergrid launchers (intergrid_mfma.hip): n_v = 16, aggregates
// of a multiple of 16 sites, at most 4096; FP32 fields with either the FP32 basis on the
// FP32 matrix cores or the packed BF16 basis on the BF16 ones.
bool intergrid_mfma_supported(const AggGeom& a, int h, int nv);
hipError_t launch_restrict_f32mfma(const AggGeom& a, int h, int nrhs, const void* W32, const void* f, void* y,
                                   hipStream_t s);
hipError_t launch_prolong_f32mfma(const AggGeom& a, int h, int nrhs, const void* W32, const void* y, void* f,
                                  hipStream_t s);

}  // namespace mrhs
