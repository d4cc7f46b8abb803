// Autotuner of the FP32 fine Wilson-clover kernel: for each requested Nrhs it
// times every supported launch configuration -- right-hand sides per thread
// (1, 2, 4) times traversal tile -- on scratch fields of the context's
// lattice and keeps the fastest for all later FP32 applies of that Nrhs
// (the configurations compute bit-identical results: each output element
// sees the same operations in the same order).  Choices can be persisted in
// a plain text cache, one line per (device architecture, lattice, Nrhs):
//
//   <arch> <Lx> <Ly> <Lz> <Lt> <nrhs> <R> <Tx> <Ty> <Tz> <Tt> <curve> <occupancy> <microseconds>
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace mrhs;

namespace {

struct Cand {
  int R;
  int T[4];
  int curve;
  int occ;
};

bool divides(const Geom& g, const int T[4]) {
  for (int m = 0; m < 4; ++m)
    if (T[m] < 1 || g.L[m] % T[m]) return false;
  return true;
}

// RHS per thread x tile x tile order.  The tiles with a t-extent of Lt / 8
// give every XCD its own slab of time slices.
std::vector<Cand> candidates(const Geom& g, int nrhs) {
  std::vector<std::array<int, 4>> tiles = {{8, 4, 4, 4}, {4, 4, 4, 4}, {6, 6, 6, 6}, {8, 8, 2, 2},
                                           {2, 2, 2, 2}, {1, 1, 1, 1}};
  if (g.L[3] % 8 == 0) {
    const int st = g.L[3] / 8;
    for (auto t : {std::array<int, 4>{8, 4, 4, st}, {4, 4, 4, st}, {6, 6, 3, st}, {8, 8, 2, st}, {4, 4, 2, st},
                   {12, 4, 4, st}})
      tiles.push_back(t);
  }
  std::vector<Cand> out;
  for (int R : {1, 2, 4}) {
    if (nrhs % R) continue;
    for (auto& t : tiles)
      for (int curve : {0, 1})
        for (int occ : {0, 4}) {
          Cand c{R, {t[0], t[1], t[2], t[3]}, curve, occ};
          if (divides(g, c.T)) out.push_back(c);
        }
  }
  return out;
}

std::string arch_name(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

bool cache_lookup(const char* path, const std::string& arch, const Geom& g, int nrhs, FineCfg& out) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char a[64];
  int L[4], n, R, T[4], curve, occ;
  float us;
  bool found = false;
  while (std::fscanf(f, "%63s %d %d %d %d %d %d %d %d %d %d %d %d %f", a, &L[0], &L[1], &L[2], &L[3], &n, &R, &T[0],
                     &T[1], &T[2], &T[3], &curve, &occ, &us) == 14) {
    if (arch == a && n == nrhs && L[0] == g.L[0] && L[1] == g.L[1] && L[2] == g.L[2] && L[3] == g.L[3] &&
        (R == 1 || R == 2 || R == 4) && nrhs % R == 0 && divides(g, T) && (curve == 0 || curve == 1) &&
        (occ == 0 || occ == 4)) {
      out.R = R;
      for (int m = 0; m < 4; ++m) out.T[m] = T[m];
      out.curve = curve;
      out.occ = occ;
      out.us = us;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_append(const char* path, const std::string& arch, const Geom& g, int nrhs, const FineCfg& c) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %d %.2f\n", arch.c_str(), g.L[0], g.L[1], g.L[2], g.L[3],
               nrhs, c.R, c.T[0], c.T[1], c.T[2], c.T[3], c.curve, c.occ, c.us);
  std::fclose(f);
}

}  // namespace

extern "C" {

mrhs_status mrhs_tune(mrhs_ctx ctx, const int32_t* nrhs_list, int32_t count, const char* cache_path) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (!nrhs_list || count < 1 || count > 64) return fail(ctx, MRHS_ERR_INVALID_ARG, "bad nrhs list");
  for (int i = 0; i < count; ++i)
    if (nrhs_list[i] < 1 || nrhs_list[i] > MRHS_MAX_NRHS)
      return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs_list[i], MRHS_MAX_NRHS);
  if (!ctx->have_gauge || !ctx->have_clover) return fail(ctx, MRHS_ERR_STATE, "fine operator not set");
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != ctx->device) (void)hipSetDevice(ctx->device);
  struct Restore {
    int p, d;
    ~Restore() {
      if (p >= 0 && p != d) (void)hipSetDevice(p);
    }
  } restore{prev, ctx->device};
  const std::string arch = arch_name(ctx->device);
  int nmax = *std::max_element(nrhs_list, nrhs_list + count);
  const size_t bytes = (size_t)ctx->g.V * 12 * nmax * 8;
  Buffer in, out;
  mrhs_status st = ensure(ctx, in, bytes);
  if (st == MRHS_OK) st = ensure(ctx, out, bytes);
  if (st != MRHS_OK) {
    release(in);
    release(out);
    return st;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(in.p, 0, bytes, ctx->stream);
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    const int n = nrhs_list[i];
    FineCfg best;
    if (cache_lookup(cache_path, arch, ctx->g, n, best)) {
      best.order = fine_order_table(ctx, best.T, best.curve);
      if (best.order) {
        ctx->fine_cfg[n] = best;
        continue;
      }
    }
    best.us = 1e30f;
    for (const Cand& c : candidates(ctx->g, n)) {
      FineCfg cfg;
      cfg.R = c.R;
      for (int m = 0; m < 4; ++m) cfg.T[m] = c.T[m];
      cfg.curve = c.curve;
      cfg.occ = c.occ;
      cfg.order = fine_order_table(ctx, c.T, c.curve);
      if (!cfg.order) {
        e = hipErrorOutOfMemory;
        break;
      }
      std::vector<float> t;
      for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, ctx->stream);
        if (e == hipSuccess)
          e = launch_fine_f32(ctx->g, ctx->t_bc, 0, (float)ctx->kappa, ctx->U32.p, ctx->A32.p, in.p, out.p, n,
                              ctx->stream, &cfg);
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) t.push_back(ms * 1000.f);  // the first launch is a warm-up
      }
      if (e != hipSuccess) break;
      std::sort(t.begin(), t.end());
      cfg.us = t[t.size() / 2];
      if (cfg.us < best.us) best = cfg;
    }
    if (e == hipSuccess) {
      ctx->fine_cfg[n] = best;
      cache_append(cache_path, arch, ctx->g, n, best);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t es = hipStreamSynchronize(ctx->stream);
  release(in);
  release(out);
  if (e != hipSuccess) return hip_fail(ctx, e, "autotuning");
  if (es != hipSuccess) return hip_fail(ctx, es, "autotuning");
  return MRHS_OK;
}

mrhs_status mrhs_get_tuning(mrhs_ctx ctx, int32_t nrhs, int32_t* rhs_per_thread, int32_t tile[4], int32_t* curve,
                            float* us) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  const FineCfg& c = ctx->fine_cfg[nrhs];
  if (rhs_per_thread) *rhs_per_thread = c.R;
  if (tile)
    for (int m = 0; m < 4; ++m) tile[m] = c.T[m];
  if (curve) *curve = c.curve + 2 * (c.occ == 4);
  if (us) *us = c.us;
  return MRHS_OK;
}

}  // extern "C"
