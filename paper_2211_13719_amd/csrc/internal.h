// Internal declarations shared by the libmrhs translation units: the context
// object, error plumbing and the kernel launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <array>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mrhs.h"

namespace mrhs {

// Lattice geometry passed by value to kernels.
struct Geom {
  int L[4];     // Lx, Ly, Lz, Lt
  int V;        // number of sites
  int stride[4];  // site-index step of +1 in each direction: 1, Lx, Lx*Ly, Lx*Ly*Lz
  int T[4] = {1, 1, 1, 1};  // default traversal tile of the fine kernels (divides L)
  // device tables of the fine lattice (null on coarse levels): traversal
  // order of the default tile, and per site the neighbours
  // (+x, -x, +y, -y) and (+z, -z, +t, -t)
  const int* order = nullptr;
  const int4* nbr = nullptr;
};

// Traversal tile: extent 8 (x) or 4 (others) where it divides the lattice,
// else the largest of 4, 2, 1 that does.
inline void set_tile(Geom& g) {
  for (int m = 0; m < 4; ++m) {
    const int pref[4] = {m == 0 ? 8 : 4, 4, 2, 1};
    g.T[m] = 1;
    for (int c : pref)
      if (g.L[m] % c == 0) {
        g.T[m] = c;
        break;
      }
  }
}

// Aggregation geometry of one coarsening step: fine lattice L, aggregate
// extent b, coarse lattice C = L / b.
struct AggGeom {
  int L[4];
  int b[4];
  int C[4];
  int V;   // fine sites
  int Vc;  // aggregates
};

// Selects the direction-resolved piece of an operator for the Galerkin
// construction: sign 2 = the whole operator; sign 0 = self term plus the hops
// that stay inside the next level's aggregate (extent b); sign +1 / -1 with
// direction mu = the hops leaving the aggregate through its +mu / -mu face.
// Launch configuration of the FP32 fine kernel: right-hand sides per thread
// (1, 2 or 4; 0 = untuned default) and traversal tile (T[0] = 0: the
// context's default tile).
struct FineCfg {
  int R = 0;
  int T[4] = {0, 0, 0, 0};
  int curve = 0;               // tile order: 0 lexicographic, 1 Morton in (x, y, z) per t-row of tiles
  int walk = 0;                // 1: t-walk kernel (MODE 0), T = spatial block and time slices per thread
  int occ = 0;                 // 0: compiler's register choice; 4: at least 4 wavefronts per SIMD
  int nt = 0;                  // 1: non-temporal output stores
  int chunks = 1;              // RHS chunks swept one after the other (1, 2, 4)
  int cap = 0;                 // 0: no limit; k: at most k workgroups per CU (via an LDS reservation)
  unsigned lds = 0;            // dynamic LDS bytes per workgroup that realise cap (0 when cap is 0)
  const int* order = nullptr;  // traversal table of tile T (device)
  float us = 0.f;              // measured time of the choice
};

// t-walk configuration of the checkerboard hop for one nrhs (FP32): spatial
// block B and Ts output sites per run; on = 0 runs the tiled kernel.
constexpr int kLowpCfgs = 6;        // launch shapes of the BF16/FP16 coarse stencil
constexpr int kEoWalkMinBlock = 16;  // smallest spatial block a walk may use
struct EoWalk {
  int on = 0;
  int R = 0;  // right-hand sides per thread (0: two for even nrhs, else one)
  int B[3] = {0, 0, 0};
  int Ts = 0;
  float us = 0.f;        // measured time of the choice (0 if set by hand)
  float us_tiled = 0.f;  // the tiled kernel's time in the same measurement
};

// The FP64 operator as a t-walk (one RHS per thread): spatial block B and
// time slices per thread Ts; off means the tiled kernel.
struct F64Walk {
  int on = 0;
  int B[3] = {0, 0, 0};
  int Ts = 0;
  int nt = 0;            // non-temporal output stores
  int occ = 0;           // register budget: 0 the compiler's, 2 for two workgroups per CU
  float us = 0.f;        // measured time of the choice (0 if set by hand)
  float us_tiled = 0.f;  // the tiled kernel's time in the same measurement
};

struct DirFilter {
  int sign = 2;
  int mu = 0;
  int b[4] = {1, 1, 1, 1};
  // sign 0 only: >= 0 restricts the output to the sites of the blocks of this
  // colour (X + Y + Z + T) mod 2 (Schwarz smoothing); the other sites are
  // neither read nor written
  int color = -1;
};

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace mrhs

struct mrhs_ctx_s {
  mrhs::Geom g{};
  int t_bc = -1;
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // library-owned device data
  mrhs::Buffer U64, U32;  // [V][4][3][3] complex
  mrhs::Buffer A64, A32;  // [V][2][36] real
  bool have_gauge = false;
  bool have_clover = false;
  double kappa = 0.0;
  // bumped whenever an operator of this context or of a hierarchy on it
  // changes (links, clover, kappa, basis, coarse blocks): captured V-cycle
  // graphs hold kappa by value and are replayed only while it is unchanged
  uint64_t op_gen = 0;

  // workspaces: reduction partials, small per-RHS scalar arrays
  mrhs::Buffer work;
  mrhs::Buffer scal;

  // autotuned launch configurations of the FP32 fine kernel, by nrhs
  mrhs::FineCfg fine_cfg[MRHS_MAX_NRHS + 1];
  mrhs::EoWalk eo_walk[MRHS_MAX_NRHS + 1];
  mrhs::F64Walk f64_walk[MRHS_MAX_NRHS + 1];

  // checkerboard tables (per parity, four int4 per site, and the traversal
  // order of its sites) and the inverse clover blocks, built on first use; an
  // odd-parity workspace field for the Schur operator
  mrhs::Buffer eo_tab[2], eo_order[2];
  mrhs::Buffer Ainv64, Ainv32;
  bool have_clover_inv = false;
  mrhs::Buffer eo_work;

  // fine-lattice index tables: neighbours, and one traversal order per tile
  mrhs::Buffer nbr;
  std::vector<std::pair<std::array<int, 5>, mrhs::Buffer>> orders;
};

namespace mrhs {

// Status helpers: record a message on the context and return the code.
mrhs_status fail(mrhs_ctx ctx, mrhs_status st, const char* fmt, ...);
mrhs_status hip_fail(mrhs_ctx ctx, hipError_t e, const char* what);

#define MRHS_HIP(ctx, call)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return mrhs::hip_fail(ctx, e_, #call); \
  } while (0)

// Checks after a kernel launch (launch-time errors only).
#define MRHS_LAUNCH_CHECK(ctx, name)                               \
  do {                                                             \
    hipError_t e_ = hipGetLastError();                             \
    if (e_ != hipSuccess) return mrhs::hip_fail(ctx, e_, name);    \
  } while (0)

mrhs_status ensure(mrhs_ctx ctx, Buffer& b, size_t bytes);
void release(Buffer& b);

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// ---- launchers (fine.hip) ---------------------------------------------------
// mode: 0 = A - kappa H, 1 = H, 2 = A
hipError_t launch_fine_f32(const Geom& g, int t_bc, int mode, float kappa, const void* U,
                           const void* A, const void* in, void* out, int nrhs, hipStream_t s,
                           const FineCfg* cfg = nullptr);
// r = b - D x (FP32) in one launch if the tuned configuration of nrhs allows
// it (the t-walk kernel): returns true and the launch status in *err, else
// false with nothing launched
bool launch_fine_residual_f32(const Geom& g, float kappa, const void* U, const void* A, const void* x, const void* b,
                              void* r, int nrhs, hipStream_t s, const FineCfg* cfg, hipError_t* err);
// fw (mode 0 only): the t-walk instead of the tiled kernel when fw->on
hipError_t launch_fine_f64(const Geom& g, int t_bc, int mode, double kappa, const void* U,
                           const void* A, const void* in, void* out, int nrhs, hipStream_t s,
                           const F64Walk* fw = nullptr);
// whether the FP64 walk's tile (B, Ts) divides the lattice
bool f64_walk_fits(const Geom& g, const int tile[4], int nrhs);
// D = A - kappa H in FP64 on an FP32 input field (widened exactly on load)
hipError_t launch_fine_f64_in32(const Geom& g, double kappa, const void* U, const void* A, const void* in, void* out,
                                int nrhs, hipStream_t s, const FineCfg* cfg = nullptr);

hipError_t launch_fine_dir_f64(const Geom& g, int t_bc, double kappa, const void* U, const void* A, const void* in,
                               void* out, int nrhs, const DirFilter& f, hipStream_t s);
// FP32 direction-resolved apply (the Schwarz smoother's block operator)
hipError_t launch_fine_dir_f32(const Geom& g, float kappa, const void* U, const void* A, const void* in, void* out,
                               int nrhs, const DirFilter& f, hipStream_t s);
// checkerboarded fine pieces (fine.hip): nhalf = V / 2 sites per parity,
// tab = that parity's table (four int4 per site)
// epi 0: out = H in; 1: out = Ablk (H in); 2: out = Ablk in2 + coef (H in)
// (Ablk: packed clover blocks or their inverses; in2 on the output parity);
// FP32 only: 3: out = in2 + coef (H in) and 4: out += Ablk (in2 + coef (H in)),
// both with in2 a full-lattice field and 4 adding into a full-lattice out
// whether tile = (Bx, By, Bz, Ts) with R right-hand sides per thread (0:
// the default) is a valid checkerboard walk for nrhs
bool eo_walk_fits(const Geom& g, const int tile[4], int nrhs, int R);
// With g, the output parity and an EoWalk that is on (FP32 only), the t-walk
// kernel runs instead of the tiled one (same results).
hipError_t launch_hop_eo(int prec64, int nhalf, const int4* tab, const int* order, const void* U, const void* in,
                         void* out, int nrhs, hipStream_t s, int epi = 0, const void* Ablk = nullptr,
                         const void* in2 = nullptr, double coef = 0.0, const Geom* g = nullptr, int parity = 0,
                         const EoWalk* ew = nullptr);
// epi 2 (FP32) that also writes the minimal-residual partial sums of
// <out, in2> and ||out||^2 per workgroup to part (*nblk rows of nrhs double4)
size_t hop_eo_dot_scratch_bytes(int nhalf, int nrhs);
hipError_t launch_hop_eo_dot(int nhalf, const int4* tab, const int* order, const void* U, const void* in, void* out,
                             const void* Ablk, const void* in2, double coef, int nrhs, void* part, int* nblk,
                             hipStream_t s, const Geom* g = nullptr, int parity = 0, const EoWalk* ew = nullptr);
// full_in: in is a full-lattice field (its parity rows are read)
hipError_t launch_clover_eo(int prec64, int nhalf, const int4* tab, const void* A, const void* in, const void* add,
                            double coef, void* out, int nrhs, hipStream_t s, bool full_in = false);
hipError_t launch_clover_invert(long nblk, const void* A64, void* Ai64, void* Ai32, int* flag, hipStream_t s);
// FP32 rows of one parity between a full-lattice field and a checkerboard one:
// half[i] = full[site(i)], or full[site(i)] += half[i]
hipError_t launch_eo_gather(int nhalf, const int4* tab, const void* full, void* half, int nrhs, hipStream_t s);
hipError_t launch_eo_scatter_add(int nhalf, const int4* tab, void* full, const void* half, int nrhs, hipStream_t s);

// ---- launchers (clover_build.hip) -------------------------------------------
hipError_t launch_clover_build(const Geom& g, double csw, double kappa, const void* U64,
                               void* F_scratch, void* A64, void* A32, hipStream_t s);
hipError_t launch_convert_f64_to_f32(const double* in, float* out, size_t n, hipStream_t s);
hipError_t launch_convert_f32_to_f64(const float* in, double* out, size_t n, hipStream_t s);

// ---- launchers (blas.hip) ---------------------------------------------------
constexpr int kMaxMultiDot = 16;
size_t blas_scratch_bytes(int nrhs, int m);
// mode 0: out (double2[nrhs]) = <a, b>; mode 1: out (double[nrhs]) = ||a||^2.  Device out.
hipError_t launch_dot(int prec64, int mode, const void* a, const void* b, long rows, int nrhs, void* out,
                      void* scratch, hipStream_t s);
// out (double2[m][nrhs]) = <v_j, w>
hipError_t launch_multi_dot(int prec64, const void* const* v, int m, const void* w, long rows, int nrhs,
                            void* out, void* scratch, hipStream_t s);
// y += alpha (double2[nrhs] on the device) * x
hipError_t launch_axpy(int prec64, void* y, const void* alpha_dev, const void* x, long rows, int nrhs,
                       hipStream_t s);

// ---- launchers (intergrid.hip) ------------------------------------------------
bool intergrid_supported(int nv, int h);
hipError_t launch_restrict(int prec64, const AggGeom& a, int h, int nv, int nrhs, const void* basis, const void* f,
                           void* y, hipStream_t s);
hipError_t launch_prolong(int prec64, const AggGeom& a, int h, int nv, int nrhs, const void* basis, const void* y,
                          void* f, hipStream_t s);
hipError_t launch_block_gs(const AggGeom& a, int h, int nv, void* basis64, int* flag_dev, hipStream_t s);
hipError_t launch_block_normalise(int prec64, const AggGeom& a, int h, int nrhs, void* f, double* norms,
                                  hipStream_t s);
hipError_t launch_basis_convert(const void* in, int in_prec64, void* out, int out_prec64, long nsite, int nv, int ncomp,
                                int to_internal, hipStream_t s);

// ---- launchers (coarse.hip) ----------------------------------------------------
hipError_t launch_coarse_valu(int prec64, const Geom& g, int nb, int nrhs, const void* BT, const void* in, void* out,
                              const DirFilter& f, hipStream_t s);
hipError_t launch_block_transpose(const void* in, int in64, void* out, int out64, long nblk, int nb, hipStream_t s);
hipError_t launch_basis_columns(int prec64, const void* basis, void* W, long nsite, int ncomp, int nv, hipStream_t s);

// Device address of the fixed scratch array of the allocation-free entry
// points on `device` (which must be current), looked up on first use per
// device (noalloc.hip).
hipError_t noalloc_scratch_init(int device, void** out);

// Traversal table of the fine lattice for tile T (built and cached on first
// use); null on failure.
const int* fine_order_table(mrhs_ctx ctx, const int T[4], int curve = 0);
// checkerboard tables and traversal orders, inverse clover blocks (api.hip)
mrhs_status ensure_eo_tables(mrhs_ctx ctx);
mrhs_status ensure_clover_inverse(mrhs_ctx ctx);
// Multiplies the t-links of the last time slice by t_bc (FP64 and FP32 copies).
hipError_t launch_fold_boundary_phase(const Geom& g, int t_bc, void* U64, void* U32, hipStream_t s);

}  // namespace mrhs
