// pts_probe.hip -- gfx950 VALU issue-rate probes (libpts_probe.so).
//
// Measures, on the device the library runs on, the sustained throughput of the
// FP32 VALU instruction forms the SDF kernels are made of, and of mixes of
// independent transcendental and FMA streams, plus the shader clock.  These
// fix the denominator of the VALU roofline the benchmark reports.
//
// Each lane runs kChains independent dependency chains so that the
// measurement is throughput, not latency.  Operands that must stay in VGPRs
// are per-lane values, so the compiler cannot fold them into scalar operands.
// Values stay finite or saturate; the instruction rate does not depend on them.
//
// Probe kinds (instructions per chain step):
//   0  v_fma_f32 with a scalar operand (VOP3)      6  v_fmac_f32 (VOP2, VGPR operands)
//   1  v_exp_f32                                   7  v_fma_f32 (VOP3, VGPR operands)
//   2  v_sqrt_f32                                  8  v_add_f32 (VOP2)
//   3  v_rcp_f32                                   9  v_mul_f32 (VOP2)
//   4  v_max3_f32                                  10 2 chains v_exp_f32 || 6 chains v_fmac_f32
//   5  1 v_exp_f32 then 4 dependent v_fma_f32     11 2 chains v_sqrt_f32 || 6 chains v_fmac_f32
//   12 v_max_f32 (VOP2)                            13 1 chain v_exp_f32 || 7 chains v_fmac_f32
//   14 1 chain v_exp_f32 || 7 chains 2x v_fmac_f32 15 v_sub_f32 (VOP2)
//   16 v_fmac_f32, two dependent steps back to back per chain
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;

template <int OP>
__global__ __launch_bounds__(256) void k_probe(float* out, int iters, float a, float b,
                                               unsigned long long* clk) {
  float v[kChains], w[kChains], u[kChains];
  const float t = float(threadIdx.x) * 1e-6f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    v[c] = 0.5f + 1e-3f * float(threadIdx.x + c);
    w[c] = 0.999f + t * float(c + 1);   // per-lane: stays in a VGPR
    u[c] = 1e-3f + t * float(c + 2);
  }
  const unsigned long long t0 = clock64();
  const unsigned long long w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if (OP == 0) v[c] = fmaf(v[c], a, b);
        if (OP == 1) v[c] = __builtin_amdgcn_exp2f(v[c]);
        if (OP == 2) v[c] = __builtin_amdgcn_sqrtf(v[c]);
        if (OP == 3) v[c] = __builtin_amdgcn_rcpf(v[c]);
        if (OP == 4) v[c] = fmaxf(v[c], fmaxf(w[c], u[c] + float(r)));
        if (OP == 5) {
          v[c] = __builtin_amdgcn_exp2f(v[c]);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
          v[c] = fmaf(v[c], a, b);
        }
        if (OP == 6) v[c] = fmaf(w[c], u[c], v[c]);
        if (OP == 7) v[c] = fmaf(v[c], w[c], u[c]);
        if (OP == 8) v[c] = v[c] + w[c];
        if (OP == 9) v[c] = v[c] * w[c];
        if (OP == 10) v[c] = (c < 2) ? __builtin_amdgcn_exp2f(v[c]) : fmaf(w[c], u[c], v[c]);
        if (OP == 11) v[c] = (c < 2) ? __builtin_amdgcn_sqrtf(v[c]) : fmaf(w[c], u[c], v[c]);
        if (OP == 12) v[c] = fmaxf(v[c], w[c]);
        if (OP == 13) v[c] = (c < 1) ? __builtin_amdgcn_exp2f(v[c]) : fmaf(w[c], u[c], v[c]);
        if (OP == 14) {
          if (c < 1) {
            v[c] = __builtin_amdgcn_exp2f(v[c]);
          } else {
            v[c] = fmaf(w[c], u[c], v[c]);
            v[c] = fmaf(u[c], w[c], v[c]);
          }
        }
        if (OP == 15) v[c] = v[c] - w[c];
        if (OP == 16)  // two dependent FMAs kept adjacent (register-only asm, no memory access)
          asm volatile("v_fmac_f32 %0, %1, %2\n\tv_fmac_f32 %0, %2, %1" : "+v"(v[c]) : "v"(w[c]), "v"(u[c]));
      }
    }
  }
  const unsigned long long t1 = clock64();
  const unsigned long long w1 = wall_clock64();
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c] + w[c] + u[c];
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

// Instructions per lane for `iters` iterations of probe `op` (for op 4 the
// compiler folds two max steps into one v_max3_f32).
long long ptsprobe_instr_per_lane(int op, int iters) {
  const long long steps = (long long)iters * 4 * kChains;
  if (op == 5) return steps * 5;
  if (op == 4 || op == 12) return steps / 2;   // folded max steps
  if (op == 16) return steps * 2;
  if (op == 14) return steps / kChains * (1 + 2 * (kChains - 1));
  return steps;
}

// Run probe `op` (kinds listed at the top of this file) on `blocks`
// workgroups of 256 threads.  out: device [blocks*256] floats, clk: device [2]
// (shader-clock ticks, 100 MHz wall ticks of workgroup 0).  Returns 0, or a
// negative code / the HIP error.  *ms = kernel time (HIP events).
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
    case 7: launch<7>(blocks, iters, out, clk, st); break;
    case 8: launch<8>(blocks, iters, out, clk, st); break;
    case 9: launch<9>(blocks, iters, out, clk, st); break;
    case 10: launch<10>(blocks, iters, out, clk, st); break;
    case 11: launch<11>(blocks, iters, out, clk, st); break;
    case 12: launch<12>(blocks, iters, out, clk, st); break;
    case 13: launch<13>(blocks, iters, out, clk, st); break;
    case 14: launch<14>(blocks, iters, out, clk, st); break;
    case 15: launch<15>(blocks, iters, out, clk, st); break;
    case 16: launch<16>(blocks, iters, out, clk, st); break;
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
