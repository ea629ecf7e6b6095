// Matched filter (pulse compression), the pipeline step before the
// beamformer: out[i][t] = sum_{k<P} raw[i][t + k] * pulse[k], raw = 0 beyond
// the record.
//
// Per channel this is a correlation with a P-tap pulse, i.e. a dense Toeplitz
// product, so it runs on the matrix cores in FP32. A wave owns 256
// consecutive outputs t0 + o, o = 16j + i (i, j < 16), and computes
//   F[i][j] = sum_m G[i][m] R[m][j],  G[i][m] = pulse[m - i] (zero outside
//   [0, P)),  R[m][j] = raw[t0 + 16j + m],  m < P + 15,
// with v_mfma_f32_16x16x4f32 in K steps of 4: lane l supplies
// G[l % 16][4kk + l / 16] and R[4kk + l / 16][l % 16] and receives
// F[4 (l / 16) + v][l % 16], v < 4, the four consecutive outputs
// o = 16 (l % 16) + 4 (l / 16) + v (one 16-byte store). A workgroup of four
// waves covers 1024 outputs of one channel and shares one LDS window of the
// channel (index i stored at i + i / 16, so the 16 columns of an operand,
// 16 samples apart, fall on distinct banks) and a zero-padded copy of the
// pulse; pulses longer than kMfTaps run in pieces that add into the same
// accumulators.
#include <hip/hip_runtime.h>

#include "dmas_internal.hpp"

namespace dmas {

namespace {

constexpr int kMfWaves = 4;
constexpr int kMfBlock = 256;                    // outputs per wave
constexpr int kMfOut = kMfWaves * kMfBlock;      // outputs per workgroup
constexpr int kMfTaps = 2048;                    // pulse taps per piece
constexpr int kMfLead = 16;                      // zeros before the pulse (G at m < i)
// pulse table: kMfLead zeros, the piece's taps, zeros up to the last K step
constexpr int kMfTapTab = kMfLead + kMfTaps + 20;
// channel window: every index the last wave's last K step reads
constexpr int kMfWin = kMfOut + kMfTaps + 20;
constexpr int kMfWinSkewed = kMfWin + kMfWin / 16 + 1;

__global__ void __launch_bounds__(kMfWaves * kWaveSize)
matched_filter_kernel(const float *__restrict__ raw, const float *__restrict__ pulse, int T, int P,
                      float *__restrict__ out)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    __shared__ float win[kMfWinSkewed];
    __shared__ float tap[kMfTapTab];
    const int tid = threadIdx.x;
    const int lane = tid & (kWaveSize - 1);
    const int wave = tid / kWaveSize;
    const int t0 = blockIdx.x * kMfOut;
    const size_t chan = (size_t)blockIdx.y * (size_t)T;
    const int g = lane >> 4, c = lane & 15;

    v4f e0 = {0.0f, 0.0f, 0.0f, 0.0f}, e1 = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < P; k0 += kMfTaps) {
        const int np = min(kMfTaps, P - k0);
        const int ks = (np + 15 + 3) / 4;               // K steps: m < np + 15
        const int wlen = kMfOut + 4 * ks;               // window indices read: < 1008 + 4 ks
        __syncthreads();                                // previous piece's reads done
        for (int i = tid; i < wlen; i += kMfWaves * kWaveSize) {
            const int t = t0 + k0 + i;
            win[i + (i >> 4)] = t < T ? raw[chan + t] : 0.0f;
        }
        for (int i = tid; i < kMfLead + 4 * ks + 4; i += kMfWaves * kWaveSize) {
            const int k = i - kMfLead;
            tap[i] = (k >= 0 && k < np) ? pulse[k0 + k] : 0.0f;
        }
        __syncthreads();
        // G[c][4kk + g] = tap[4kk + g - c]; R[4kk + g][c] = window[256 wave + 16c + g + 4kk]
        const float *pa = tap + kMfLead + g - c;
        const float *rb = win + 272 * wave + 17 * c + g;   // skewed index of 256 wave + 16c + g
        // step kk = 4q + u: pa[4kk] = pq[4u] (pq = pa + 16q), rb[4kk + kk/4] = rq[4u]
        // (rq = rb + 17q); groups of four issue their eight reads together
        const float *pq = pa, *rq = rb;
        int kk = 0;
        for (; kk + 3 < ks; kk += 4, pq += 16, rq += 17) {
            const float a0 = pq[0], a1 = pq[4], a2 = pq[8], a3 = pq[12];
            const float b0 = rq[0], b1 = rq[4], b2 = rq[8], b3 = rq[12];
            e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, e1, 0, 0, 0);
            e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, b3, e1, 0, 0, 0);
        }
        for (; kk < ks; ++kk) {
            const float a = pa[4 * kk], b = rb[4 * kk + (kk >> 2)];
            if (kk & 1) e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, e1, 0, 0, 0);
            else e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, e0, 0, 0, 0);
        }
    }
    const v4f e = e0 + e1;
    const int t = t0 + kMfBlock * wave + 16 * c + 4 * g;   // a multiple of 4
    float *dst = out + chan + t;
    if (t + 3 < T && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        *reinterpret_cast<v4f *>(dst) = e;
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (t + v < T) dst[v] = e[v];
    }
}

}  // namespace

hipError_t launch_matched_filter(const float *raw, const float *pulse, int M, int T, int P, float *out,
                                 hipStream_t stream)
{
    const dim3 grid((unsigned)((T + kMfOut - 1) / kMfOut), (unsigned)M);
    hipLaunchKernelGGL(matched_filter_kernel, grid, dim3(kMfWaves * kWaveSize), 0, stream, raw, pulse, T, P, out);
    return hipGetLastError();
}

}  // namespace dmas
