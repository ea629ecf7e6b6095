// VALU issue-rate probe for gfx950: FP32 FMA and the v_exp_f32 / v_log_f32 /
// v_sqrt_f32 transcendentals, alone and mixed. The beamformer is bound by VALU
// issue, so these rates define the roofline bench.py reports against.
// Every kernel writes exactly one float per thread into out[gid] (gid < n).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>

#define CHAINS 8
#define ITERS 4096

__global__ void k_fma(float *out, float a, float b) {
  float v[CHAINS];
  for (int c = 0; c < CHAINS; ++c) v[c] = threadIdx.x * 1e-3f + c;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) v[c] = __builtin_fmaf(v[c], a, b);
  float s = 0; for (int c = 0; c < CHAINS; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_exp(float *out, float a, float b) {
  float v[CHAINS];
  for (int c = 0; c < CHAINS; ++c) v[c] = threadIdx.x * 1e-6f + c * 1e-3f;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) v[c] = __builtin_amdgcn_exp2f(v[c]);
  float s = 0; for (int c = 0; c < CHAINS; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_log(float *out, float a, float b) {
  float v[CHAINS];
  for (int c = 0; c < CHAINS; ++c) v[c] = 2.0f + threadIdx.x * 1e-6f + c;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) v[c] = __builtin_amdgcn_logf(v[c]) + 2.5f;
  float s = 0; for (int c = 0; c < CHAINS; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_sqrt(float *out, float a, float b) {
  float v[CHAINS];
  for (int c = 0; c < CHAINS; ++c) v[c] = 2.0f + threadIdx.x * 1e-6f + c;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) v[c] = __builtin_amdgcn_sqrtf(v[c]);
  float s = 0; for (int c = 0; c < CHAINS; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
// mixed: per chain step 1 exp + 4 fma (independent)
__global__ void k_mix(float *out, float a, float b) {
  float v[CHAINS], w[CHAINS];
  for (int c = 0; c < CHAINS; ++c) { v[c] = threadIdx.x * 1e-6f + c * 1e-3f; w[c] = c; }
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
      v[c] = __builtin_amdgcn_exp2f(v[c]);
      w[c] = __builtin_fmaf(w[c], a, b); w[c] = __builtin_fmaf(w[c], a, b);
      w[c] = __builtin_fmaf(w[c], a, b); w[c] = __builtin_fmaf(w[c], a, b);
    }
  float s = 0; for (int c = 0; c < CHAINS; ++c) s += v[c] + w[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));              \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

int main() {
  const int blocks = 256 * 16, threads = 256;
  const size_t n = (size_t)blocks * threads;
  float *out;
  CHECK(hipMalloc(&out, n * sizeof(float)));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  struct K { const char *name; void (*fn)(float *, float, float); double ops_per_step; } ks[] = {
    {"fma", k_fma, 1}, {"exp2", k_exp, 1}, {"log2", k_log, 2 /* log + add */}, {"sqrt", k_sqrt, 1},
    {"mix(1exp+4fma)", k_mix, 5}};
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  printf("device %s CUs %d clock %d kHz lds/block %zu\n", prop.gcnArchName, prop.multiProcessorCount,
         prop.clockRate, prop.sharedMemPerBlock);
  for (auto &k : ks) {
    hipLaunchKernelGGL(k.fn, dim3(blocks), dim3(threads), 0, 0, out, 0.999f, 0.001f);
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k.fn, dim3(blocks), dim3(threads), 0, 0, out, 0.999f, 0.001f);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    double instr = 5.0 * n * ITERS * CHAINS * k.ops_per_step;
    printf("%-16s %8.3f ms  %8.2f T lane-instr/s\n", k.name, ms / 5, instr / (ms * 1e-3) / 1e12);
  }
  std::vector<float> h(16);
  CHECK(hipMemcpy(h.data(), out, 16 * 4, hipMemcpyDeviceToHost));
  printf("sink %g\n", h[0]);
  CHECK(hipFree(out));
  return 0;
}
