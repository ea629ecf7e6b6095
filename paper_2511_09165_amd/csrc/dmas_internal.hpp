// Internal interface between the host API (dmas_api.hip) and the kernel
// instantiation units (dmas_order*.hip). Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmas {

constexpr int kWaveSize = 64;
constexpr int kMaxOrder = 8;
constexpr int kMaxMicBlock = 64;   // microphones staged in LDS at once (<= wave size)
// Microphones per block with kDelayTableBlocks (a block's offsets are read as
// one scalar block into SGPRs): 16 for every order (the order-3 kernels, which
// run eight waves per SIMD, hold them within their SGPR budget).
__host__ __device__ constexpr int table_block_max(int) { return 16; }
constexpr int kTableBlockMax = 16;  // the largest, for padding the tables

// Everything a beamforming launch needs, passed by value as the kernel argument.
struct KernelParams {
    const void *x;            // M x T channels (dtype below), device
    const float2 *roots;      // M x T (signed root, sample) pairs, device; used by
                              // plans that stage roots (whole-sample delays, n >= 2)
    float *out;               // D x T image, device
    const double *mic;        // M x 3, device
    const double *dirs;       // D x 3, device
    const int32_t *tile_dirs; // num_tiles x dirs_per_tile direction indices (-1 = empty), device
    const int32_t *tile_off;  // optional, num_tiles x dirs_per_tile x M: LDS element where
                              // each direction's window of each microphone starts,
                              // (mic % mic_block) * row + clamp(delay - reference + halo, 0, 2 halo)
    const int32_t *tile_dref; // optional, num_tiles x M: reference (first direction) delays
    const float *taps;        // fir_len envelope taps, device
    int32_t M, T, D;
    int32_t order;            // n
    int32_t fir_len;          // odd
    int32_t num_tiles;
    int32_t seg_len;          // output samples per direction per workgroup
    int32_t halo;             // bound on |delay - reference delay| within a tile
    int32_t row;              // LDS row length per microphone (floats)
    int32_t mic_block;        // microphones per LDS block, <= kMaxMicBlock
    int32_t dtype;            // dmas_dtype_t
    int32_t ng_fp64;          // evaluate Newton-Girard in FP64
    double fs, c;
    float cf_eps;
    float in_scale;
    int32_t env_decim;        // envelope keeps every env_decim-th sample
    int32_t out_T;            // output row length: T, or ceil(T / env_decim) for the envelope
};

// A batch of frames for the multi-frame kernel (device pointers).
struct BatchParams {
    const KernelParams *frames;   // num_frames entries
    const int32_t *starts;        // first workgroup of each frame, ascending, starts[0] = 0
    int32_t num_frames;
};

struct LaunchShape {
    int order;
    bool cf;
    bool env;
    bool nearfield;
    int delay;                // kDelayComputed, kDelayLinear or kDelayTable
    int accumulate;           // power-sum accumulation: 0 FP32, 1 Kahan FP32, 2 FP64
    unsigned grid;            // workgroups
    size_t lds_bytes;         // dynamic LDS
};

// How a kernel obtains its steering delays: evaluated on the device (whole
// samples), evaluated with linear interpolation, or from the plan's per-tile
// tables (whole samples). With kDelayTable the hot loop reads each
// microphone's offset through the scalar cache one ahead of use; with
// kDelayTableBlocks each wave reads its block's offsets and the reference
// delays of the rows it stages as scalars before the block's barrier, and the
// block's microphone loop is straight-line code (per-microphone scalar reads
// of a large table left their latency in the hot loop). The plan picks the
// block form for more than 64 microphones and for plain FP32 sums up to
// order 7.
// kDelayTableBlocksShared is kDelayTableBlocks with the envelope rings in the
// window region (below), which the plan picks when it raises the occupancy.
enum : int { kDelayComputed = 0, kDelayLinear = 1, kDelayTable = 2, kDelayTableBlocks = 3, kDelayTableBlocksShared = 4 };
__host__ __device__ constexpr bool block_tables(int delay)
{
    return delay == kDelayTableBlocks || delay == kDelayTableBlocksShared;
}

// Compile-time tiling shared by host and device: waves (= directions) per
// workgroup and output samples per lane per chunk.
constexpr int kDirsPerTile = 8;
constexpr int kSamplesPerLane = 4;
constexpr int kChunk = kWaveSize * kSamplesPerLane;

// Envelope chunk walk: the chunk of samples [tc, tc + kChunk) (tc a multiple
// of 32) yields the envelope outputs [tc - env_lead(H), ... + kChunk), where
// env_lead(H) is H rounded up to a multiple of 32, so every output block
// starts on a 128-byte line. The ring then keeps the env_prefix(H) values of
// |y| before the chunk.
__host__ __device__ constexpr int env_lead(int H) { return (H + 31) & ~31; }
__host__ __device__ constexpr int env_prefix(int H) { return H + env_lead(H); }

// Envelope LDS of a workgroup: after the channel windows come the reference
// delays (kMaxMicBlock ints, only in kernels that evaluate delays on the
// device: the table modes read them as scalars), a taps table of
// env_taps_len(H) floats (kTapLead
// zeros, the L = 2H + 1 taps in reverse order, zeros) and one ring per wave of
// ring_stride(H) floats. With per-block delay tables (more microphones than
// lanes: many blocks per chunk, where LDS decides the block size) the rings
// instead share the window region, which they need only in the epilogue after
// the chunk's last block:
// the region then holds max(windows, kDirsPerTile rings), and per wave
// carry_stride(H) floats after the taps keep the env_prefix(H) values of |y|
// carried from one chunk to the next while the windows occupy the region. A
// ring holds |y| for ring index i in [0, env_prefix(H) + kChunk) at float
// i + i / 16; the skew keeps the FIR's matrix-operand reads (16 indices 16
// apart) on distinct LDS banks. The FIR is a product with K = 2H + 16 in steps
// of 4 and reads ring indices up to 2H + kChunk + 2 (zero beyond the chunk).
constexpr int kTapLead = 20;
__host__ __device__ constexpr int env_ksteps(int H) { return (2 * H + 16 + 3) / 4; }
__host__ __device__ constexpr int env_taps_len(int H) { return (kTapLead + 2 * H + 24) & ~3; }
__host__ __device__ constexpr int ring_logical(int H)
{
    return kChunk + (env_prefix(H) > 2 * H + 8 ? env_prefix(H) : 2 * H + 8);
}
__host__ __device__ constexpr int ring_stride(int H) { return (ring_logical(H) + ring_logical(H) / 16 + 1 + 3) & ~3; }
__host__ __device__ constexpr int carry_stride(int H) { return (env_prefix(H) + 3) & ~3; }
// Whether the envelope rings share the window region: a property of the delay
// mode, so that the other kernels carry none of its address arithmetic.
__host__ __device__ constexpr bool rings_share_windows(int delay) { return delay == kDelayTableBlocksShared; }
// Floats of the window region: mic_block rows of `row` elements of elem_floats
// floats, or the rings if they share it and need more.
__host__ __device__ constexpr int window_region_floats(int mic_block, int row, int elem_floats, bool env, int H,
                                                       bool share)
{
    return env && share && kDirsPerTile * ring_stride(H) > mic_block * row * elem_floats
               ? kDirsPerTile * ring_stride(H)
               : mic_block * row * elem_floats;
}
// Ints of reference delays kept in LDS by a kernel of the given delay mode.
__host__ __device__ constexpr int dref_lds_ints(int delay)
{
    return delay == kDelayTable || block_tables(delay) ? 0 : kMaxMicBlock;
}
// Dynamic LDS bytes of a workgroup of the given delay mode.
__host__ __device__ constexpr int kernel_lds_bytes(int mic_block, int row, int elem_floats, bool env, int H, int delay)
{
    return 4 * (window_region_floats(mic_block, row, elem_floats, env, H, rings_share_windows(delay)) +
                dref_lds_ints(delay) +
                (env ? env_taps_len(H) + kDirsPerTile * (rings_share_windows(delay) ? carry_stride(H) : ring_stride(H))
                     : 0));
}
// Envelope taps on the device: fir_len taps, zero-padded to a multiple of 4.
__host__ __device__ constexpr int fir_taps_padded(int L) { return (L + 3) & ~3; }

// Batched launch over frames of order n with the given CF / envelope /
// geometry flags and whole-sample delay mode (kDelayComputed, kDelayTable or
// kDelayTableBlocks(Shared), the same for all frames; plain sums); grid = total
// workgroups.
hipError_t launch_batch(int order, const BatchParams &bp, bool cf, bool env, bool nearfield, int delay,
                        unsigned grid, size_t lds_bytes, hipStream_t stream);
hipError_t launch_batch_order1(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);
hipError_t launch_batch_order2(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);
hipError_t launch_batch_order3(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);
hipError_t launch_batch_order4(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);
hipError_t launch_batch_order5(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);
hipError_t launch_batch_order6(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);
hipError_t launch_batch_order7(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);
hipError_t launch_batch_order8(const BatchParams &, bool, bool, bool, int, unsigned, size_t, hipStream_t);

// Root plane of a frame: plane[e] = (sgn(x_e) |x_e|^(1/order), x_e) for the
// count = M * T channel samples of x (storage type dtype), in FP32.
hipError_t launch_roots(int order, int dtype, const void *x, float2 *plane, size_t count, hipStream_t stream);

// Matched filter: out[i*T + t] = sum_{k<P} raw[i*T + t + k] * pulse[k].
hipError_t launch_matched_filter(const float *raw, const float *pulse, int M, int T, int P, float *out,
                                 hipStream_t stream);

hipError_t launch_order1(const KernelParams *, const LaunchShape &, hipStream_t, int *);
hipError_t launch_order2(const KernelParams *, const LaunchShape &, hipStream_t, int *);
hipError_t launch_order3(const KernelParams *, const LaunchShape &, hipStream_t, int *);
hipError_t launch_order4(const KernelParams *, const LaunchShape &, hipStream_t, int *);
hipError_t launch_order5(const KernelParams *, const LaunchShape &, hipStream_t, int *);
hipError_t launch_order6(const KernelParams *, const LaunchShape &, hipStream_t, int *);
hipError_t launch_order7(const KernelParams *, const LaunchShape &, hipStream_t, int *);
hipError_t launch_order8(const KernelParams *, const LaunchShape &, hipStream_t, int *);

}  // namespace dmas
