// Matched filter (pulse compression), the pipeline step before the
// beamformer: out[i][t] = sum_{k<P} raw[i][t + k] * pulse[k], raw = 0 beyond
// the record. One workgroup = 256 consecutive outputs of one channel; the
// input window (256 + P - 1 samples) and the pulse are staged in LDS in
// pieces of at most 2048 taps, and every thread accumulates its output in
// FP32 in tap order.
#include <hip/hip_runtime.h>

#include "dmas_internal.hpp"

namespace dmas {

namespace {

constexpr int kMfOut = 256;      // outputs per workgroup (= threads)
constexpr int kMfTaps = 2048;    // taps staged per pass

__global__ void __launch_bounds__(kMfOut)
matched_filter_kernel(const float *__restrict__ raw, const float *__restrict__ pulse, int T, int P,
                      float *__restrict__ out)
{
    __shared__ float win[kMfOut + kMfTaps];
    __shared__ float taps[kMfTaps];
    const int t0 = blockIdx.x * kMfOut;
    const size_t chan = (size_t)blockIdx.y * (size_t)T;
    const int tid = threadIdx.x;
    float acc = 0.0f;
    for (int k0 = 0; k0 < P; k0 += kMfTaps) {
        const int np = min(kMfTaps, P - k0);
        __syncthreads();
        for (int i = tid; i < kMfOut + np - 1; i += kMfOut) {
            const int t = t0 + k0 + i;
            win[i] = t < T ? raw[chan + t] : 0.0f;
        }
        for (int i = tid; i < np; i += kMfOut) taps[i] = pulse[k0 + i];
        __syncthreads();
        for (int k = 0; k < np; ++k) acc = __builtin_fmaf(win[tid + k], taps[k], acc);
    }
    const int t = t0 + tid;
    if (t < T) out[chan + t] = acc;
}

}  // namespace

hipError_t launch_matched_filter(const float *raw, const float *pulse, int M, int T, int P, float *out,
                                 hipStream_t stream)
{
    const dim3 grid((unsigned)((T + kMfOut - 1) / kMfOut), (unsigned)M);
    hipLaunchKernelGGL(matched_filter_kernel, grid, dim3(kMfOut), 0, stream, raw, pulse, T, P, out);
    return hipGetLastError();
}

}  // namespace dmas
