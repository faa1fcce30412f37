// pts_noalloc.hip -- pts_eval_noalloc: the plain evaluation (phi only) with its
// workspace in a file-scope device array instead of a caller buffer, for
// callers that cannot allocate device memory.
//
// The array `scratch` is a static device symbol: every device the library runs
// on holds its own copy, at its own address, until the process ends.  In host
// code the symbol's name is only a host-side stand-in, so its device address is
// looked up once per device with hipGetSymbolAddress (on that device's first
// call) and only that address is handed to kernels.  The kernels are those of
// pts_eval (farthest-point sweep, blend sweep, fixed-order combine); every byte
// of workspace they read was written earlier in the same call, so nothing needs
// clearing between calls.  Calls that overlap on one device share the array and
// race.
#include <mutex>

#include "pts_internal.h"

namespace pts {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device).
int scratch_address(void** out) {
  int dev = -1;
  if (int rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(PTS_EINVAL, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return rc;
    if (!p) return fail(PTS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PTS_OK;
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

int eval_noalloc(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, const pts_params& P,
                 const Plan& plan, hipStream_t st) {
  const size_t need = eval_ws_bytes(plan, Q);
  if (need > kScratchBytes)
    return fail(PTS_EINVAL, "pts_eval_noalloc: the evaluation needs " + std::to_string(need) +
                                " bytes of workspace, more than the static scratch of " +
                                std::to_string(kScratchBytes) + " bytes; use pts_eval with a workspace");
  void* ws = nullptr;
  if (int rc = scratch_address(&ws)) return rc;
  return launch_eval_plain(rec, N, x, Q, P.C, plan, ws_view(plan, Q, ws), sdf, st, P.offset);
}

}  // namespace pts
