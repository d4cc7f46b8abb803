// Autotuner of the FP32 fine Wilson-clover kernel: for each requested Nrhs it
// times launch configurations -- traversal tile and tile order, or the t-walk
// kernel with its spatial block and time slices per thread, right-hand
// sides per thread (1, 2, 4), RHS chunks swept in turn (1, 2, 4; the tiles
// are scanned again if chunking wins), a cap on resident workgroups per CU,
// register budget, ordinary or non-temporal output stores -- on scratch
// fields of the context's lattice, by coordinate descent in that order, and
// keeps the fastest for all later FP32 applies of that Nrhs
// (the configurations compute bit-identical results: each output element
// sees the same operations in the same order).  Choices can be persisted in
// a plain text cache, one line per (device architecture, HIP runtime
// version, lattice, Nrhs):
//
//   <arch> <hip runtime version> <Lx> <Ly> <Lz> <Lt> <nrhs> <R> <Tx> <Ty> <Tz> <Tt> <curve> <occupancy> <nt>
//   <chunks> <cap> <microseconds>
//
// (curve 2 selects the t-walk kernel, Tx Ty Tz Tt then being its spatial
// block and time slices per thread)
// (one line each; a line tuned under another runtime or of another format is
// ignored, so a new ROCm retunes).
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace mrhs;

namespace {

// Tuning input: uniform values in [-1, 1) from an integer hash of the index
// (timing on zeros would understate the power draw, hence the clock drop, of
// real data).
__global__ void fill_hash(float* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(i >> 32);
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    p[i] = (float)(h >> 8) * (2.0f / 16777216.0f) - 1.0f;
  }
}

bool divides(const Geom& g, const int T[4]) {
  for (int m = 0; m < 4; ++m)
    if (T[m] < 1 || g.L[m] % T[m]) return false;
  return true;
}

// Tiles to try.  Those with a t-extent of Lt / 8 give every XCD its own slab
// of time slices; those with the full t-extent are columns swept along t, so
// that the +-t neighbours of a site are one small cross-section apart in the
// traversal and only the column faces are re-read from outside the L2.
std::vector<std::array<int, 4>> tile_candidates(const Geom& g) {
  std::vector<std::array<int, 4>> tiles = {{8, 4, 4, 4}, {4, 4, 4, 4}, {6, 6, 6, 6}, {8, 8, 2, 2},
                                           {2, 2, 2, 2}, {1, 1, 1, 1}};
  if (g.L[3] % 8 == 0) {
    const int st = g.L[3] / 8;
    for (auto t : {std::array<int, 4>{8, 4, 4, st}, {4, 4, 4, st}, {6, 6, 3, st}, {8, 8, 2, st}, {4, 4, 2, st},
                   {12, 4, 4, st}})
      tiles.push_back(t);
  }
  const int lt = g.L[3];
  for (auto t : {std::array<int, 4>{4, 4, 4, lt}, {6, 6, 4, lt}, {8, 4, 4, lt}, {6, 6, 6, lt}, {8, 8, 4, lt},
                 {8, 6, 6, lt}, {12, 6, 4, lt}, {12, 12, 4, lt}, {8, 8, 8, lt}})
    tiles.push_back(t);
  std::vector<std::array<int, 4>> out;
  for (auto& t : tiles) {
    const int T[4] = {t[0], t[1], t[2], t[3]};
    if (divides(g, T)) out.push_back(t);
  }
  return out;
}

// t-walk tiles (spatial block Bx x By x Bz, time slices per thread Ts): the
// block's sites x Nrhs / R threads should about fill what one XCD keeps
// resident, and Ts trades the two extra slices each run reads against the
// number of runs that balance the XCDs.
std::vector<std::array<int, 4>> walk_candidates(const Geom& g) {
  const std::array<int, 3> blocks[] = {{8, 8, 8}, {8, 8, 6}, {8, 8, 4}, {8, 8, 3},  {12, 8, 4}, {12, 12, 4},
                                       {6, 6, 6}, {8, 4, 4}, {4, 4, 4}, {12, 12, 2}, {24, 8, 2}, {24, 4, 4}};
  std::vector<std::array<int, 4>> out;
  for (const auto& b : blocks)
    for (int div : {1, 2, 4, 8}) {
      if (g.L[3] % div) continue;
      const int T[4] = {b[0], b[1], b[2], g.L[3] / div};
      if (divides(g, T)) out.push_back({T[0], T[1], T[2], T[3]});
    }
  return out;
}

int runtime_version() {
  int v = 0;
  return hipRuntimeGetVersion(&v) == hipSuccess ? v : 0;
}

std::string arch_name(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// Dynamic LDS per workgroup that leaves room for at most cap resident
// workgroups on one CU (0 if cap is 0 or the device cannot express it).
unsigned cap_lds(int dev, int cap) {
  if (cap <= 0) return 0;
  int per_cu = 0, per_block = 0;
  if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 0;
  const unsigned lds = (unsigned)(per_cu / (cap + 1) + 1024);
  if ((long)lds * cap > per_cu || (long)lds > per_block) return 0;
  return lds;
}

bool cache_lookup(const char* path, const std::string& arch, const Geom& g, int nrhs, FineCfg& out) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char a[64];
    int hv, L[4], n, R, T[4], curve, occ, nt, ch, cap;
    float us;
    if (std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %f", a, &hv, &L[0], &L[1], &L[2], &L[3],
                    &n, &R, &T[0], &T[1], &T[2], &T[3], &curve, &occ, &nt, &ch, &cap, &us) != 18)
      continue;  // lines of other formats are ignored
    if (arch == a && hv == runtime_version() && n == nrhs && L[0] == g.L[0] && L[1] == g.L[1] && L[2] == g.L[2] &&
        L[3] == g.L[3] &&
        (R == 1 || R == 2 || R == 4) && nrhs % R == 0 && divides(g, T) && (curve >= 0 && curve <= 2) &&
        (curve != 2 || R <= 2) &&
        (occ == 0 || occ == 4) && (nt == 0 || nt == 1) && (ch == 1 || ch == 2 || ch == 4) && nrhs % ch == 0 &&
        (nrhs / ch) % R == 0 && cap >= 0 && cap <= 3) {
      out.R = R;
      for (int m = 0; m < 4; ++m) out.T[m] = T[m];
      out.walk = curve == 2;  // 2 marks the t-walk kernel
      out.curve = curve == 2 ? 0 : curve;
      out.occ = occ;
      out.nt = nt;
      out.chunks = ch;
      out.cap = cap;
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
  std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.2f\n", arch.c_str(), runtime_version(), g.L[0],
               g.L[1], g.L[2], g.L[3], nrhs, c.R, c.T[0], c.T[1], c.T[2], c.T[3], c.walk ? 2 : c.curve, c.occ, c.nt, c.chunks,
               c.cap,
               c.us);
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
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fill_hash, dim3(2048), dim3(256), 0, ctx->stream, static_cast<float*>(in.p), bytes / 4);
    e = hipGetLastError();
  }
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    const int n = nrhs_list[i];
    FineCfg best;
    if (cache_lookup(cache_path, arch, ctx->g, n, best)) {
      best.order = best.walk ? ctx->g.order : fine_order_table(ctx, best.T, best.curve);
      best.lds = cap_lds(ctx->device, best.cap);
      if (best.cap && !best.lds) best.cap = 0;
      if (best.order) {
        ctx->fine_cfg[n] = best;
        continue;
      }
    }
    // coordinate descent: tile and tile order first (two RHS per thread for
    // even Nrhs), then RHS per thread, register budget and store kind
    auto time_cfg = [&](FineCfg& cfg) -> hipError_t {
      // a t-walk ignores the traversal table; the other modes keep the default
      cfg.order = cfg.walk ? ctx->g.order : fine_order_table(ctx, cfg.T, cfg.curve);
      if (!cfg.order) return hipErrorOutOfMemory;
      std::vector<float> t;
      hipError_t err = hipSuccess;
      for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
        err = hipEventRecord(e0, ctx->stream);
        if (err == hipSuccess)
          err = launch_fine_f32(ctx->g, ctx->t_bc, 0, (float)ctx->kappa, ctx->U32.p, ctx->A32.p, in.p, out.p, n,
                                ctx->stream, &cfg);
        if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) t.push_back(ms * 1000.f);  // the first launch is a warm-up
      }
      if (err != hipSuccess) return err;
      std::sort(t.begin(), t.end());
      cfg.us = t[t.size() / 2];
      return hipSuccess;
    };
    best.R = (n % 2 == 0) ? 2 : 1;
    best.us = 1e30f;
    auto scan_tiles = [&](const FineCfg& base) {
      for (const auto& t : tile_candidates(ctx->g)) {
        for (int curve : {0, 1}) {
          FineCfg cfg = base;
          for (int m = 0; m < 4; ++m) cfg.T[m] = t[m];
          cfg.curve = curve;
          e = time_cfg(cfg);
          if (e != hipSuccess) return;
          if (cfg.us < best.us) best = cfg;
        }
      }
    };
    // t-walk: one or two RHS per thread over every walk tile, at the current chunking
    auto scan_walks = [&](const FineCfg& base) {
      for (int R : {1, 2}) {
        if ((n / base.chunks) % R) continue;
        for (const auto& t : walk_candidates(ctx->g)) {
          FineCfg cfg = base;
          cfg.R = R;
          cfg.walk = 1;
          cfg.curve = 0;
          for (int m = 0; m < 4; ++m) cfg.T[m] = t[m];
          e = time_cfg(cfg);
          if (e != hipSuccess) return;
          if (cfg.us < best.us) best = cfg;
        }
      }
    };
    scan_tiles(best);
    if (e == hipSuccess) scan_walks(best);
    // stages: 0 RHS per thread, 1 RHS chunks, 2 workgroups per CU, 3 register budget, 4 store kind
    for (int stage = 0; stage < 5 && e == hipSuccess; ++stage) {
      const FineCfg cur = best;
      std::vector<int> opts;
      if (stage == 0) opts = {1, 2, 4};
      if (stage == 1) opts = {1, 2, 4};
      if (stage == 2) opts = {0, 1, 2, 3};
      if (stage == 3) opts = {0, 4};
      if (stage == 4) opts = {0, 1};
      for (int v : opts) {
        FineCfg cfg = cur;
        if (stage == 0) {
          if (n % v || v == cur.R || (n / cur.chunks) % v || (cur.walk && v > 2)) continue;
          cfg.R = v;
        } else if (stage == 1) {
          if (v == cur.chunks || n % v || (n / v) % cur.R) continue;
          cfg.chunks = v;
        } else if (stage == 2) {
          if (v == cur.cap) continue;
          cfg.cap = v;
          cfg.lds = cap_lds(ctx->device, v);
          if (v && !cfg.lds) continue;
        } else if (stage == 3) {
          if (v == cur.occ) continue;
          cfg.occ = v;
        } else {
          if (v == cur.nt) continue;
          cfg.nt = v;
        }
        e = time_cfg(cfg);
        if (e != hipSuccess) break;
        if (cfg.us < best.us) best = cfg;
      }
      // chunking changes the bytes per site a sweep keeps in L2: re-scan the tiles
      if (stage == 1 && e == hipSuccess && best.chunks != cur.chunks) {
        if (best.walk)
          scan_walks(best);
        else
          scan_tiles(best);
      }
    }
    if (e == hipSuccess) {
      ctx->fine_cfg[n] = best;
      cache_append(cache_path, arch, ctx->g, n, best);
    }
  }
  // The checkerboard hop of the even-odd smoother (lattices with even
  // extents): tiled kernel or t-walk, timed as one Schur step's pair of
  // launches (output parity 1 with a clover factor, output parity 0 with the
  // factor, the combination and the MR sums) on the same scratch fields; the
  // clover blocks stand in for their inverses (same layout and cost).  The
  // results are bit-identical either way (the MR sums up to their grouping),
  // so the choice is made afresh by every call and not cached.
  bool even = true;
  for (int m = 0; m < 4; ++m) even = even && ctx->g.L[m] % 2 == 0;
  if (even && e == hipSuccess) {
    mrhs_status est = ensure_eo_tables(ctx);
    Buffer part;
    const int nhalf = ctx->g.V / 2;
    if (est == MRHS_OK) est = ensure(ctx, part, hop_eo_dot_scratch_bytes(nhalf, nmax));
    if (est != MRHS_OK) {
      (void)hipStreamSynchronize(ctx->stream);
      release(in);
      release(out);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      return est;
    }
    const auto* te = static_cast<const int4*>(ctx->eo_tab[0].p);
    const auto* to = static_cast<const int4*>(ctx->eo_tab[1].p);
    const auto* oe = static_cast<const int*>(ctx->eo_order[0].p);
    const auto* oo = static_cast<const int*>(ctx->eo_order[1].p);
    char* half2 = static_cast<char*>(out.p) + (size_t)nhalf * 12 * nmax * 8;  // second half of out
    for (int i = 0; i < count && e == hipSuccess; ++i) {
      const int n = nrhs_list[i];
      auto time_eo = [&](const EoWalk& w, float& us) -> hipError_t {
        std::vector<float> t;
        hipError_t err = hipSuccess;
        for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
          int nb = 0;
          err = hipEventRecord(e0, ctx->stream);
          if (err == hipSuccess)
            err = launch_hop_eo(0, nhalf, to, oo, ctx->U32.p, in.p, out.p, n, ctx->stream, 1, ctx->A32.p, nullptr,
                                0.0, &ctx->g, 1, &w);
          if (err == hipSuccess)
            err = launch_hop_eo_dot(nhalf, te, oe, ctx->U32.p, out.p, half2, ctx->A32.p, in.p, -0.01, n, part.p, &nb,
                                    ctx->stream, &ctx->g, 0, &w);
          if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
          if (err == hipSuccess) err = hipEventSynchronize(e1);
          float ms = 0.f;
          if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) t.push_back(ms * 1000.f);
        }
        if (err != hipSuccess) return err;
        std::sort(t.begin(), t.end());
        us = t[t.size() / 2];
        return hipSuccess;
      };
      EoWalk best;  // tiled
      e = time_eo(best, best.us);
      const float tiled = best.us;
      // coordinate descent: spatial block at a short run, then the run length, then R
      const int Lh = ctx->g.L[3] / 2;
      const int ts0 = Lh % 4 == 0 ? 4 : (Lh % 2 == 0 ? 2 : 1);
      const std::array<int, 3> blocks[] = {{4, 4, 4}, {8, 4, 4}, {8, 8, 4}, {6, 6, 4}, {12, 4, 4},
                                           {24, 4, 4}, {4, 4, 2}, {8, 8, 8}, {6, 6, 6}};
      auto consider = [&](EoWalk w) {
        const int tile[4] = {w.B[0], w.B[1], w.B[2], w.Ts};
        if (e != hipSuccess || !eo_walk_fits(ctx->g, tile, n, w.R)) return;
        e = time_eo(w, w.us);
        if (e == hipSuccess && w.us < best.us) best = w;
      };
      for (const auto& b : blocks) {
        EoWalk w;
        w.on = 1;
        for (int m = 0; m < 3; ++m) w.B[m] = b[m];
        w.Ts = ts0;
        consider(w);
      }
      if (best.on) {
        const EoWalk base = best;
        for (int ts : {1, 2, 4, 8, 16, Lh}) {
          if (ts == base.Ts) continue;
          EoWalk w = base;
          w.Ts = ts;
          consider(w);
        }
        const EoWalk base2 = best;
        for (int R : {1, 2}) {
          const int r0 = base2.R ? base2.R : (n % 2 == 0 ? 2 : 1);
          if (R == r0) continue;
          EoWalk w = base2;
          w.R = R;
          consider(w);
        }
      }
      if (e == hipSuccess) {
        best.us_tiled = tiled;
        if (!best.on) best.us = tiled;
        ctx->eo_walk[n] = best;
      }
    }
    (void)hipStreamSynchronize(ctx->stream);
    release(part);
    ctx->op_gen++;  // captured V-cycles hold the hop's launch shape
  }
  // The FP64 operator (the outer solver's residuals): tiled kernel or t-walk
  // with one RHS per thread, timed per nrhs on FP64 scratch fields (the FP32
  // scratch input widened); every walk candidate of the FP32 tuning, then the
  // register budget and the store kind.  Bit-identical either way, so chosen
  // afresh by every call and not cached; skipped (tiled kernel) if the FP64
  // scratch fields do not fit.
  if (e == hipSuccess && ctx->U64.p && ctx->A64.p) {
    (void)hipStreamSynchronize(ctx->stream);
    release(out);
    Buffer in64, out64;
    mrhs_status fst = ensure(ctx, in64, 2 * bytes);
    if (fst == MRHS_OK) fst = ensure(ctx, out64, 2 * bytes);
    if (fst == MRHS_OK) {
      e = launch_convert_f32_to_f64(static_cast<const float*>(in.p), static_cast<double*>(in64.p), bytes / 4,
                                    ctx->stream);
      for (int i = 0; i < count && e == hipSuccess; ++i) {
        const int n = nrhs_list[i];
        auto time64 = [&](const F64Walk& w, float& us) -> hipError_t {
          std::vector<float> t;
          hipError_t err = hipSuccess;
          for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
            err = hipEventRecord(e0, ctx->stream);
            if (err == hipSuccess)
              err = launch_fine_f64(ctx->g, ctx->t_bc, 0, ctx->kappa, ctx->U64.p, ctx->A64.p, in64.p, out64.p, n,
                                    ctx->stream, &w);
            if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) t.push_back(ms * 1000.f);
          }
          if (err != hipSuccess) return err;
          std::sort(t.begin(), t.end());
          us = t[t.size() / 2];
          return hipSuccess;
        };
        F64Walk best;  // tiled
        e = time64(best, best.us);
        const float tiled = best.us;
        for (const auto& t : walk_candidates(ctx->g)) {
          if (e != hipSuccess) break;
          const int tile[4] = {t[0], t[1], t[2], t[3]};
          if (!f64_walk_fits(ctx->g, tile, n)) continue;
          F64Walk w;
          w.on = 1;
          for (int m = 0; m < 3; ++m) w.B[m] = t[m];
          w.Ts = t[3];
          e = time64(w, w.us);
          if (e == hipSuccess && w.us < best.us) best = w;
        }
        for (int stage = 0; stage < 2 && e == hipSuccess && best.on; ++stage) {
          F64Walk w = best;
          if (stage == 0)
            w.occ = 2;  // a register budget for two workgroups per CU
          else
            w.nt = 1;  // non-temporal output stores
          e = time64(w, w.us);
          if (e == hipSuccess && w.us < best.us) best = w;
        }
        if (e == hipSuccess) {
          best.us_tiled = tiled;
          if (!best.on) best.us = tiled;
          ctx->f64_walk[n] = best;
        }
      }
      ctx->op_gen++;
    }
    // without room for the FP64 scratch fields the tiled kernel stays
    (void)hipStreamSynchronize(ctx->stream);
    release(in64);
    release(out64);
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
  if (curve)
    *curve = c.curve + 2 * (c.occ == 4) + 4 * c.nt + 8 * (c.chunks == 4 ? 2 : c.chunks == 2 ? 1 : 0) + 32 * c.cap +
             128 * c.walk;
  if (us) *us = c.us;
  return MRHS_OK;
}

}  // extern "C"
