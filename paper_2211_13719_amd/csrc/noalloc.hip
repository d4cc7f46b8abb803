// The multi-dot of one Gram-Schmidt step (the simultaneous inner products of
// paper Sec. 7) without any device allocation, for callers that cannot
// allocate: code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc.
//
// The per-workgroup partial sums and, for a host destination, the staged
// result live in one file-scope device array, `scratch`, of fixed size; each
// device that the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// that name is only a stand-in): its device address is looked up once per
// device with hipGetSymbolAddress when a context is created on that device,
// and that address is what the kernels receive.  Every call on one device
// shares the array and leaves the last call's partials in it; nothing has to
// start at zero (pass 1 writes every partial that pass 2 reads).  Calls that
// overlap in time on one device (two host threads, or two streams) race on
// the array.
#include <mutex>

#include "internal.h"

namespace mrhs {
namespace {

constexpr int kMaxDevices = 64;
// partials of the largest call (1024 workgroups x 16 vectors x 64 columns of
// complex FP64) plus the 16 x 64 complex FP64 results staged for a host copy
constexpr size_t kPartialBytes = (size_t)1024 * kMaxMultiDot * MRHS_MAX_NRHS * 16;
constexpr size_t kResultBytes = (size_t)kMaxMultiDot * MRHS_MAX_NRHS * 16;

__device__ __align__(256) char scratch[kPartialBytes + kResultBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the scratch array (the device must be
// current); later calls for the same device return the stored address.
hipError_t noalloc_scratch_init(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  if (out) *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace mrhs

using namespace mrhs;

extern "C" {

mrhs_status mrhs_multi_dot_noalloc(mrhs_ctx ctx, double* out, const void* const* v, int32_t m, const void* w,
                                   int64_t nsites, int32_t ncomp, int32_t nrhs, mrhs_prec prec,
                                   int32_t out_on_device) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (nsites < 1 || ncomp < 1 || nsites * (int64_t)ncomp > (int64_t(1) << 40))
    return fail(ctx, MRHS_ERR_SHAPE, "bad field shape nsites=%lld ncomp=%d", (long long)nsites, ncomp);
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return fail(ctx, MRHS_ERR_SHAPE, "nrhs = %d outside [1, %d]", nrhs, MRHS_MAX_NRHS);
  if (m < 1 || m > kMaxMultiDot) return fail(ctx, MRHS_ERR_SHAPE, "m = %d outside [1, %d]", m, kMaxMultiDot);
  if (prec != MRHS_F32 && prec != MRHS_F64)
    return fail(ctx, MRHS_ERR_UNSUPPORTED, "precision %d not supported for this call", (int)prec);
  if (!out || !v || !w) return fail(ctx, MRHS_ERR_INVALID_ARG, "null pointer");
  if (!aligned16(w)) return fail(ctx, MRHS_ERR_INVALID_ARG, "field pointers must be 16-byte aligned");
  for (int j = 0; j < m; ++j)
    if (!v[j] || !aligned16(v[j])) return fail(ctx, MRHS_ERR_INVALID_ARG, "v[%d] null or misaligned", j);
  // the partial sums the kernels write: at most blas_scratch_bytes(nrhs, m)
  const size_t need = blas_scratch_bytes(nrhs, m);
  if (need > kPartialBytes)
    return fail(ctx, MRHS_ERR_SHAPE, "multi-dot needs %zu scratch bytes, above the fixed %zu", need, kPartialBytes);
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != ctx->device) MRHS_HIP(ctx, hipSetDevice(ctx->device));
  struct Restore {
    int p, d;
    ~Restore() {
      if (p >= 0 && p != d) (void)hipSetDevice(p);
    }
  } restore{prev, ctx->device};
  void* base = nullptr;
  MRHS_HIP(ctx, noalloc_scratch_init(ctx->device, &base));
  char* part = static_cast<char*>(base);
  void* dst = out_on_device ? static_cast<void*>(out) : static_cast<void*>(part + kPartialBytes);
  const long rows = (long)nsites * ncomp;
  MRHS_HIP(ctx, launch_multi_dot(prec == MRHS_F64, v, m, w, rows, nrhs, dst, part, ctx->stream));
  if (!out_on_device) {
    MRHS_HIP(ctx, hipMemcpyAsync(out, dst, (size_t)m * nrhs * 16, hipMemcpyDeviceToHost, ctx->stream));
    MRHS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return MRHS_OK;
}

}  // extern "C"
