// pts_probe.hip -- gfx950 VALU issue-rate probes (libpts_probe.so).
//
// Measures, on the device the library runs on, the sustained throughput of the
// FP32 VALU instructions the SDF kernels are made of (v_fma_f32, v_exp_f32,
// v_sqrt_f32, v_rcp_f32, v_max_f32) and a mix, plus the shader clock during
// the run.  These fix the denominator of the VALU roofline the benchmark
// reports (transcendental issue cost relative to an FMA, sustained clock).
//
// Each lane runs 8 independent dependency chains so that the measurement is
// throughput, not latency.  Values stay finite or saturate to +-inf/0/1; the
// instruction rate does not depend on them.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;

__device__ __forceinline__ float op_apply(int op, float v, float a, float b) {
  switch (op) {
    case 0: return fmaf(v, a, b);
    case 1: return __builtin_amdgcn_exp2f(v);
    case 2: return __builtin_amdgcn_sqrtf(v);
    case 3: return __builtin_amdgcn_rcpf(v);
    case 4: return fmaxf(v, a);
    default: return v;
  }
}

template <int OP>
__global__ __launch_bounds__(256) void k_probe(float* out, int iters, float a, float b,
                                               unsigned long long* clk) {
  float v[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) v[c] = 0.5f + 1e-3f * float(threadIdx.x + c);
  const unsigned long long t0 = clock64();
  const unsigned long long w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if (OP == 5) {  // mix: 1 exp2 + 4 fma per chain step
          v[c] = __builtin_amdgcn_exp2f(v[c]);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
        } else if (OP == 6) {  // mix: 1 sqrt + 4 fma
          v[c] = __builtin_amdgcn_sqrtf(v[c]);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
        } else {
          v[c] = op_apply(OP, v[c], a, b);
        }
      }
    }
  }
  const unsigned long long t1 = clock64();
  const unsigned long long w1 = wall_clock64();
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk[0] = t1 - t0;
    clk[1] = w1 - w0;
  }
}

template <int OP>
void launch(int blocks, int iters, float* out, unsigned long long* clk, hipStream_t st) {
  hipLaunchKernelGGL(k_probe<OP>, dim3(blocks), dim3(256), 0, st, out, iters, 0.999f, 1e-3f, clk);
}

}  // namespace

extern "C" {

// Instructions of the probed kind per lane for `iters` iterations.
long long ptsprobe_instr_per_lane(int op, int iters) {
  const long long steps = (long long)iters * 4 * kChains;
  if (op == 5 || op == 6) return steps * 5;
  return steps;
}

// Run probe `op` (0 fma, 1 exp2, 2 sqrt, 3 rcp, 4 max, 5 exp2+4fma, 6 sqrt+4fma)
// on `blocks` workgroups of 256 threads.  out: device [blocks*256] floats,
// clk: device [2] (shader-clock ticks, 100 MHz wall ticks of workgroup 0).
// Returns 0, or the HIP error code.  *ms = kernel time (HIP events).
int ptsprobe_run(int op, int blocks, int iters, float* out, unsigned long long* clk, float* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
  hipStream_t st = nullptr;
  if (hipEventRecord(e0, st) != hipSuccess) return -1;
  switch (op) {
    case 0: launch<0>(blocks, iters, out, clk, st); break;
    case 1: launch<1>(blocks, iters, out, clk, st); break;
    case 2: launch<2>(blocks, iters, out, clk, st); break;
    case 3: launch<3>(blocks, iters, out, clk, st); break;
    case 4: launch<4>(blocks, iters, out, clk, st); break;
    case 5: launch<5>(blocks, iters, out, clk, st); break;
    case 6: launch<6>(blocks, iters, out, clk, st); break;
    default: return -2;
  }
  hipError_t err = hipEventRecord(e1, st);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  *ms = t;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return err == hipSuccess ? int(hipGetLastError()) : int(err);
}

}  // extern "C"
