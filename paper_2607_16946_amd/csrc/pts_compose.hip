// pts_compose.hip -- offsets and Booleans of signed distances (Sec. 5.2,
// "Offset surfaces and Booleans"): out = a - c, min(a, b), max(a, b) or
// max(a, -b), elementwise, NaN propagating.
#include "pts_internal.h"

namespace pts {
namespace {

__global__ __launch_bounds__(kBlock) void k_compose(const float* a, const float* b, int64_t n, int op, float c,
                                                    float* out) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const float x = a[i];
  if (op == PTS_OP_OFFSET) {
    out[i] = x - c;
    return;
  }
  const float y = op == PTS_OP_SUBTRACT ? -b[i] : b[i];
  float r;
  if (x != x || y != y)
    r = __builtin_nanf("");
  else if (op == PTS_OP_UNION)
    r = x < y ? x : y;
  else
    r = x > y ? x : y;
  out[i] = r;
}

}  // namespace

int launch_compose(const float* a, const float* b, int64_t n, int op, float c, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_compose, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a, b, n, op, c, out);
  return check_hip(hipGetLastError(), "compose kernel");
}

}  // namespace pts
