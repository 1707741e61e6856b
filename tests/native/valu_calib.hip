// Calibration of gfx950's FP32 issue rates and of the SQ instruction
// counters: kernels that run a known number of one FP32 instruction (16
// independent chains per lane, so dependences do not limit the issue), timed
// with HIP events.  Run under rocprofv3 --pmc, the counts per dispatch can be
// compared with the exact ones printed here.
//   valu_calib [blocks] [iters]
// prints, per kernel: the instruction, the time, the wave-level instruction
// count, wave instructions per SIMD per cycle at 2.4 GHz on 1,024 SIMDs, and
// lane operations per second.
//   valu_calib forms [iters]
// times four encodings (VOP3 fma with vector operands, VOP2 fmac with a
// scalar operand, VOP3 fma with a negated addend, VOP2 sub) at eight
// wavefronts per SIMD.
//   valu_calib sweep [iters]
// times v_fmac_f32_e32 with 1, 2, 4, 8 and 16 independent chains per lane at
// 1, 2, 4 and 8 resident wavefronts per SIMD (256, 512, 1024 and 2048
// four-wave workgroups on 256 compute units): the issue rate a kernel can
// reach with that much instruction-level parallelism and occupancy.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kChains = 16;

// v_fma_f32 (VOP3) with a scalar operand: x = x * a + b
__global__ void __launch_bounds__(256) k_fma_vop3(float *out, int iters, float a, float b) {
  float x[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) x[j] = (float)(threadIdx.x + j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = fmaf(x[j], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// v_fmac_f32_e32 (VOP2): x += y * z with vector operands
__global__ void __launch_bounds__(256) k_fmac_vop2(float *out, int iters, float a, float) {
  float x[kChains], y[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    x[j] = (float)(threadIdx.x + j);
    y[j] = a * (float)(j + 1);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = fmaf(y[j], y[(j + 1) % kChains], x[j]);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// v_mul_f32_e32
__global__ void __launch_bounds__(256) k_mul_vop2(float *out, int iters, float a, float) {
  float x[kChains], y[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    x[j] = (float)(threadIdx.x + j);
    y[j] = 1.f - a * (float)(j + 1);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = x[j] * y[j];
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// v_add_f32_e32
__global__ void __launch_bounds__(256) k_add_vop2(float *out, int iters, float a, float) {
  float x[kChains], y[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    x[j] = (float)(threadIdx.x + j);
    y[j] = a * (float)(j + 1);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = x[j] + y[j];
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// Encodings of the same operation: each kernel runs 16 independent chains
// of one instruction form, so the forms' issue rates can be compared.
enum Form { kFmaVvv, kFmacSgpr, kFmaNeg, kSub };

template <int F>
__global__ void __launch_bounds__(256) k_form(float *out, int iters, float a, float b) {
  float x[kChains], y[kChains], z[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    x[j] = (float)(threadIdx.x + j);
    y[j] = a * (float)(j + 1) * 0.01f;
    z[j] = b * (float)(j + 2);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      if (F == kFmaVvv) x[j] = fmaf(x[j], y[j], z[j]);         // v_fma_f32 v, v, v, v (VOP3)
      if (F == kFmacSgpr) x[j] = fmaf(a, y[j], x[j]);          // v_fmac_f32_e32 v, s, v
      if (F == kFmaNeg) x[j] = fmaf(y[j], z[j], -x[j]);        // v_fma_f32 v, v, v, -v (VOP3)
      if (F == kSub) x[j] = z[j] - x[j];                        // v_sub_f32_e32 v, v, v
    }
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

int forms(int iters) {
  typedef void (*K)(float *, int, float, float);
  const K ks[4] = {k_form<kFmaVvv>, k_form<kFmacSgpr>, k_form<kFmaNeg>, k_form<kSub>};
  const char *names[4] = {"v_fma_f32 v,v,v,v", "v_fmac_f32_e32 v,s,v", "v_fma_f32 v,v,v,-v", "v_sub_f32_e32 v,v,v"};
  const int blocks = 2048;
  float *out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  for (int k = 0; k < 4; ++k) {
    hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(256), 0, 0, out, 4, 0.999f, 1e-3f);
    if (hipDeviceSynchronize() != hipSuccess) return 3;
    if (hipEventRecord(e0, 0) != hipSuccess) return 3;
    hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f, 1e-3f);
    if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 3;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 3;
    const double wi = (double)blocks * 4 * iters * kChains;
    printf("%-22s ms %9.3f  per-SIMD-cycle %.3f\n", names[k], ms, wi / (1024.0 * 2.4e9 * ms * 1e-3));
  }
  (void)hipFree(out);
  return 0;
}

// v_fmac_f32_e32 in C independent chains per lane
template <int C>
__global__ void __launch_bounds__(256) k_fmac_chains(float *out, int iters, float a, float) {
  float x[C], y[C], z[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    x[j] = (float)(threadIdx.x + j);
    y[j] = a * (float)(j + 1);
    z[j] = a * (float)(j + 2);
  }
  // 16 instructions per loop body whatever C, so that the loop's scalar
  // instructions and branch weigh the same in every variant
  constexpr int kU = 16 / C;
  for (int i = 0; i < iters; i += kU) {
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int j = 0; j < C; ++j) x[j] = fmaf(y[j], z[j], x[j]);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < C; ++j) s += x[j];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

int sweep(int iters) {
  typedef void (*K)(float *, int, float, float);
  const K ks[5] = {k_fmac_chains<1>, k_fmac_chains<2>, k_fmac_chains<4>, k_fmac_chains<8>, k_fmac_chains<16>};
  const int chains[5] = {1, 2, 4, 8, 16};
  float *out = nullptr;
  if (hipMalloc(&out, (size_t)2048 * 256 * sizeof(float)) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  printf("v_fmac_f32_e32 wave instructions per SIMD per cycle (2.4 GHz, 1,024 SIMDs)\n");
  printf("%-8s", "chains");
  for (int w = 1; w <= 8; w *= 2) printf("  %d wave%s/SIMD", w, w > 1 ? "s" : " ");
  printf("\n");
  for (int k = 0; k < 5; ++k) {
    printf("%-8d", chains[k]);
    for (int w = 1; w <= 8; w *= 2) {
      const int blocks = 256 * w;
      // fewer iterations for more chains: about the same time per launch
      const int it = iters * 16 / chains[k];  // a multiple of 16 / chains
      hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(256), 0, 0, out, 4, 0.999f, 1e-3f);
      if (hipDeviceSynchronize() != hipSuccess) return 3;
      if (hipEventRecord(e0, 0) != hipSuccess) return 3;
      hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(256), 0, 0, out, it, 0.999f, 1e-3f);
      if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 3;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 3;
      const double wi = (double)blocks * 4 * it * chains[k];
      printf("  %12.3f", wi / (1024.0 * 2.4e9 * ms * 1e-3));
    }
    printf("\n");
  }
  (void)hipFree(out);
  return 0;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc > 1 && argv[1][0] == 's') return sweep(argc > 2 ? atoi(argv[2]) : 20000);
  if (argc > 1 && argv[1][0] == 'f') return forms(argc > 2 ? atoi(argv[2]) : 20000);
  const int blocks = argc > 1 ? atoi(argv[1]) : 8192;
  const int iters = argc > 2 ? atoi(argv[2]) : 25000;
  if (blocks < 1 || iters < 1) return 2;
  float *out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  typedef void (*K)(float *, int, float, float);
  const K ks[4] = {k_fma_vop3, k_fmac_vop2, k_mul_vop2, k_add_vop2};
  const char *names[4] = {"v_fma_f32(vop3,sgpr)", "v_fmac_f32_e32", "v_mul_f32_e32", "v_add_f32_e32"};
  for (int k = 0; k < 4; ++k) {
    hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(256), 0, 0, out, 4, 0.999f, 1e-3f);
    if (hipDeviceSynchronize() != hipSuccess) return 3;
    if (hipEventRecord(e0, 0) != hipSuccess) return 3;
    hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f, 1e-3f);
    if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 3;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 3;
    const double wi = (double)blocks * 4 * iters * kChains;
    printf("%-22s ms %9.3f  wave-instr %.4e  per-SIMD-cycle %.3f  lane-op/s %.3e\n", names[k], ms, wi,
           wi / (1024.0 * 2.4e9 * ms * 1e-3), wi * 64.0 / (ms * 1e-3));
  }
  (void)hipFree(out);
  return 0;
}
