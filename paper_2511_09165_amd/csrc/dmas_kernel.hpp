// DMAS-n + CF (+ envelope) beamforming kernel for gfx950 (CDNA4, wave64).
//
// Method (Jansen, Daems, Steckel, Section II):
//   x_i(t, p) = m_i(t + tau_{i,p})                      eq. (1)
//   s_i = sgn(x_i) |x_i|^(1/n)                          eq. (4)
//   S = E_n(s_1..s_M)                                   eqs. (5)/(6)
//     = Newton-Girard polynomial of P_k = sum_i s_i^k   eqs. (7)-(12)
//   y = S * CF,  CF = (sum x)^2 / (M sum x^2 + eps)     eqs. (13)/(14)
//   env = low-pass(|y|)                                 pipeline step 3
//
// Work decomposition (MI355X-first; not the paper's one-thread-per-pixel CUDA
// design):
//   * With whole-sample delays the root of a delayed sample is the root of a
//     channel sample, so a separate pass (root_plane_kernel) writes each
//     channel sample's (root, sample) pair once; the beamformer stages those.
//   * A workgroup owns one tile of kDirsPerTile nearby directions (one wave per
//     direction) and one time segment. Directions were grouped on the host so
//     that their steering delays stay within +-halo samples of the tile's first
//     (reference) direction.
//   * The segment is walked in chunks of kChunk samples. For each chunk the
//     workgroup stages, per microphone, one window
//     [t0 + d_ref - halo, t0 + d_ref - halo + row) into LDS (zero outside the
//     record); every wave then reads its own delayed samples from that window
//     with a wave-uniform offset, so one staged window serves all directions
//     of the tile. Microphones are staged in blocks of <= 64 when M is large.
//   * Window offsets come from per-tile tables built at plan creation (read
//     through the scalar cache when small) or are computed from the geometry.
//   * Each lane owns kSamplesPerLane output samples at stride 64 and keeps
//     their power sums in registers across all microphones; the LDS reads of a
//     wave are contiguous (conflict-free) and the per-microphone address update
//     is one scalar offset shared by all samples of the lane.
//   * The epilogue evaluates Newton-Girard, CF and either stores y, or writes
//     |y| into a per-wave LDS ring; the ring keeps the last L-1 values between
//     chunks so the envelope never round-trips through HBM and needs only L-1
//     samples of halo per segment.
//   * The microphone loop is a gather and sum, not a contraction, and runs on
//     the VALU (its bound); the envelope FIR of a chunk is a Toeplitz matrix
//     product and runs on the matrix cores in FP32.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <atomic>
#include <type_traits>

#include "dmas_internal.hpp"

namespace dmas {

// ---------------------------------------------------------------------------
// Steering delay, eq. (1), in samples (fs * tau). Written as a fixed sequence
// of IEEE double operations with contraction disabled, so that the whole-sample
// rounding is reproducible on any IEEE machine that evaluates the same steps.
// ---------------------------------------------------------------------------
// |v| of a near-field focal point (its distance from the origin, where the
// delays are referenced), by the same steps as the delay uses; 0 in the far
// field. A kernel evaluates it once per direction instead of once per delay.
template <bool NEAR>
__device__ __forceinline__ double steer_origin(const double *__restrict__ v)
{
#pragma clang fp contract(off)
    if constexpr (!NEAR) {
        return 0.0;
    } else {
        double q0 = v[0] * v[0];
        q0 = q0 + v[1] * v[1];
        q0 = q0 + v[2] * v[2];
        return __builtin_sqrt(q0);
    }
}

// vnorm = steer_origin<NEAR>(v).
template <bool NEAR>
__device__ __forceinline__ double steer_samples(const double *__restrict__ r, const double *__restrict__ v,
                                                double vnorm, double fs, double c)
{
#pragma clang fp contract(off)
    double tau;
    if constexpr (!NEAR) {
        // plane wave from unit vector v reaches r earlier by (r . v)/c
        double dot = r[0] * v[0];
        dot = dot + r[1] * v[1];
        dot = dot + r[2] * v[2];
        tau = -dot / c;
    } else {
        // spherical wave from point v, aligned to its arrival at the origin
        double dx = v[0] - r[0];
        double dy = v[1] - r[1];
        double dz = v[2] - r[2];
        double q = dx * dx;
        q = q + dy * dy;
        q = q + dz * dz;
        tau = (__builtin_sqrt(q) - vnorm) / c;
    }
    return fs * tau;
}

// Whole-sample part used to address the channel: nearest sample
// (floor(f + 1/2)) or, for linear interpolation, floor(f) plus the fraction.
// vnorm = steer_origin<NEAR>(v).
template <bool NEAR, bool LINEAR>
__device__ __forceinline__ int steer_whole(const double *r, const double *v, double vnorm, double fs, double c,
                                           float *frac)
{
    const double f = steer_samples<NEAR>(r, v, vnorm, fs, c);
    if constexpr (LINEAR) {
        const double q = __builtin_floor(f);
        *frac = (float)(f - q);
        return (int)q;
    } else {
        *frac = 0.0f;
        return (int)__builtin_floor(f + 0.5);
    }
}

template <bool NEAR, bool LINEAR>
__device__ __forceinline__ int steer_whole(const double *r, const double *v, double fs, double c, float *frac)
{
    return steer_whole<NEAR, LINEAR>(r, v, steer_origin<NEAR>(v), fs, c, frac);
}

// ---------------------------------------------------------------------------
// Channel sample conversion (storage type -> FP32).
// ---------------------------------------------------------------------------
template <int DT>
__device__ __forceinline__ float load_sample(const void *__restrict__ x, size_t idx)
{
    if constexpr (DT == 0) {
        return static_cast<const float *>(x)[idx];
    } else if constexpr (DT == 1) {
        return __half2float(static_cast<const __half *>(x)[idx]);
    } else {
        const uint32_t bits = static_cast<const uint16_t *>(x)[idx];
        return __uint_as_float(bits << 16);
    }
}

template <int DT>
struct StorageOf;
template <>
struct StorageOf<0> {
    using type = float;
};
template <>
struct StorageOf<1> {
    using type = __half;
};
template <>
struct StorageOf<2> {
    using type = uint16_t;
};

template <int DT>
__device__ __forceinline__ float to_f32(typename StorageOf<DT>::type v)
{
    if constexpr (DT == 0) return v;
    else if constexpr (DT == 1) return __half2float(v);
    else return __uint_as_float((uint32_t)v << 16);
}

// One microphone's window [base, base + row) of the channel starting at
// element chan, converted to FP32, zero outside [0, T); used where samples
// rather than roots are staged (n = 1, linear delays). Windows inside the
// record (all but the first and last chunks) take a path without per-element
// bounds checks; with FP32 storage that is the global-to-LDS copy of the
// root-plane windows below (four samples per lane; row is a multiple of 4),
// which the caller waits for before the barrier that publishes the windows
// (linear delays 4.7 % and order 1 20 % faster than through registers).
template <int DT>
__device__ __forceinline__ void stage_row(float *__restrict__ dst, const void *__restrict__ x, size_t chan,
                                          int base, int row, int T, int lane)
{
    using E = typename StorageOf<DT>::type;
    if (DT == 0 && base >= 0 && base + row <= T) {
        typedef __attribute__((address_space(3))) void lds_void;
        const char *src = reinterpret_cast<const char *>(static_cast<const float *>(x) + chan + (size_t)base);
        const int pieces = row >> 2;
        for (int q = 0; q < pieces; q += kWaveSize) {
            if (lane < pieces - q)
                __builtin_amdgcn_global_load_lds(src + (unsigned)(q + lane) * 16u, (lds_void *)(dst + 4 * q), 16, 0,
                                                 0);
        }
    } else if (base >= 0 && base + row <= T) {
        const E *src = static_cast<const E *>(x) + chan + (size_t)base + lane;
        float *d = dst + lane;
        for (int r = 0; r < row - lane; r += kWaveSize) d[r] = to_f32<DT>(src[r]);
    } else {
        for (int r = lane; r < row; r += kWaveSize) {
            const int t = base + r;
            dst[r] = (t >= 0 && t < T) ? load_sample<DT>(x, chan + (size_t)t) : 0.0f;
        }
    }
}

// Signed n-th root of one sample, eq. (4): sgn(x) |x|^(1/n) in FP32.
// |x|^(1/n) = 2^(log2|x| / n); log2(0) = -inf gives 0.
// The hardware log2 and square root take an input below the FP32 normal range
// (|x| < 2^-126) as zero. With SUBNORMAL such an input is first scaled by
// 2^32 (exact) and the scale is taken back out of the result, so the root
// follows eq. (4) for every finite input; normal inputs give the same bits
// either way. The root pass (once per channel sample) uses it; the linear-delay
// kernels, which take a root per microphone and pixel, do not.
template <int N, bool SUBNORMAL = false>
__device__ __forceinline__ float signed_root(float xv)
{
    const float ax = __builtin_fabsf(xv);
    float r;
    if constexpr (SUBNORMAL) {
        const bool tiny = ax < 0x1p-126f;
        const float as = tiny ? ax * 0x1p+32f : ax;
        if constexpr (N == 2) r = __builtin_amdgcn_sqrtf(as) * (tiny ? 0x1p-16f : 1.0f);
        else r = __builtin_amdgcn_exp2f((__builtin_amdgcn_logf(as) - (tiny ? 32.0f : 0.0f)) * (1.0f / (float)N));
    } else {
        if constexpr (N == 2) r = __builtin_amdgcn_sqrtf(ax);
        else r = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(ax) * (1.0f / (float)N));
    }
    return __builtin_copysignf(r, xv);
}

// With whole-sample delays the root of a delayed sample is the root of a
// channel sample: a separate pass takes it once per channel sample (the root
// plane of (s, x) pairs), and the beamformer stages windows of that plane.
template <int N, bool LINEAR>
constexpr bool kStagesRoots = N >= 2 && !LINEAR;

// Root plane: plane[e] = (signed_root(x_e), x_e) over count samples.
template <int N, int DT>
__global__ void __launch_bounds__(256) root_plane_kernel(const void *__restrict__ x, float2 *__restrict__ plane,
                                                         size_t count)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
        const float v = load_sample<DT>(x, e);
        plane[e] = make_float2(signed_root<N, true>(v), v);
    }
}

// One microphone's window [base, base + row) of the root plane starting at
// element chan, (0, 0) outside [0, T) (the pair of a zero sample). A window
// inside the record (all but the first and last chunks) is copied by the
// global-to-LDS loads: each lane moves 16 bytes (two pairs) straight into LDS
// at M0 + 16 * lane, a wave 1 KiB per load, with no vector registers and no
// vector ALU work; row is a multiple of 4 pairs, so the copy is whole 16-byte
// pieces into 32-byte aligned LDS rows. Those copies complete in the
// background (the wave's vmcnt): the caller waits for them before the barrier
// that publishes the windows. (Against loading into registers and writing
// them to LDS: 4.0-7.5 % faster across the kernels, bitwise the same.)
__device__ __forceinline__ void stage_row_roots(float2 *__restrict__ dst, const float2 *__restrict__ plane,
                                                size_t chan, int base, int row, int T, int lane)
{
    if (base >= 0 && base + row <= T) {
        typedef __attribute__((address_space(3))) void lds_void;
        const char *src = reinterpret_cast<const char *>(plane + chan + (size_t)base);
        const int pieces = row >> 1;
        for (int q = 0; q < pieces; q += kWaveSize) {   // wave-uniform
            if (lane < pieces - q)
                __builtin_amdgcn_global_load_lds(src + (unsigned)(q + lane) * 16u, (lds_void *)(dst + 2 * q), 16, 0,
                                                 0);
        }
    } else {
        for (int r = lane; r < row; r += kWaveSize) {
            const int t = base + r;
            dst[r] = (t >= 0 && t < T) ? plane[chan + (size_t)t] : make_float2(0.0f, 0.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// Power-sum accumulators for one output sample.
//   p[k], k = 1..N-1 : P_k = sum_i s_i^k                        eq. (7)
//   p[N]             : P_N = sum x (N odd) or sum |x| (N even), exact since
//                      s^N = x for odd N and |x| for even N
//   a                : sum x (only needed separately for even N with CF)
//   b                : sum x^2 (CF only)
// Accumulation modes: kAccF32 plain FP32 sums; kAccKahan FP32 sums with a
// Kahan compensation term each; kAccF64 powers and sums in FP64 from the FP32
// root (CDNA4 issues FP64 vector add/mul/FMA at the non-packed FP32 rate, so
// this costs only the conversions).
// ---------------------------------------------------------------------------
enum : int { kAccF32 = 0, kAccKahan = 1, kAccF64 = 2 };

template <int ACC>
using AccType = typename std::conditional<ACC == kAccF64, double, float>::type;

template <int N, bool CF, int ACC>
struct Acc {
    using T = AccType<ACC>;
    T p[N + 1];
    T a, b;
    float cp[ACC == kAccKahan ? N + 1 : 1];
    float ca, cb;

    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int k = 0; k <= N; ++k) p[k] = T(0);
        a = b = T(0);
#pragma unroll
        for (int k = 0; k < (ACC == kAccKahan ? N + 1 : 1); ++k) cp[k] = 0.0f;
        ca = cb = 0.0f;
    }
};

template <int ACC, typename T>
__device__ __forceinline__ void acc_add(T &sum, float &comp, T term)
{
    if constexpr (ACC == kAccKahan) {
#pragma clang fp contract(off)
        const T y = term - comp;
        const T t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    } else {
        sum += term;
    }
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T mul_rounded(T a, T b)
{
#pragma clang fp contract(off)
    return a * b;
}

// sum += a * b: one fused multiply-add for plain sums; for Kahan sums the
// product is rounded first and then added with compensation.
template <int ACC, typename T>
__device__ __forceinline__ void acc_fma(T &sum, float &comp, T a, T b)
{
    if constexpr (ACC == kAccKahan) acc_add<ACC>(sum, comp, mul_rounded(a, b));
    else sum = fma_t(a, b, sum);
}

// Factors of s^k used to form it: s^k = s^fa(k) * s^fb(k).
__host__ __device__ constexpr int pow_fa(int k) { return (k & 1) ? k - 1 : k / 2; }
__host__ __device__ constexpr int pow_fb(int k) { return (k & 1) ? 1 : k / 2; }

// Adds one microphone's terms given its signed root sv = sgn(x)|x|^(1/N) and
// its sample xv. The operations are written out rather than left to the
// compiler's contraction, so every kernel that calls this rounds alike:
// P_1 += s; P_k = fma(s^fa, s^fb, P_k) for 2 <= k < N, with the powers that
// later terms need formed by a rounded multiply; P_N += x (odd N) or |x|
// (s^N is x or |x|); with CF, B = fma(x, x, B) and, for even N, A += x.
template <int N, bool CF, int ACC>
__device__ __forceinline__ void accumulate_root(Acc<N, CF, ACC> &acc, float sv, float xv)
{
    using T = AccType<ACC>;
    constexpr bool KAHAN = ACC == kAccKahan;
    const T x = T(xv);
    if constexpr (N == 1) {
        acc_add<ACC>(acc.p[1], acc.cp[KAHAN ? 1 : 0], x);
    } else {
        T pw[N];                       // pw[k] = s^k (those a later term uses)
        pw[1] = T(sv);
        acc_add<ACC>(acc.p[1], acc.cp[KAHAN ? 1 : 0], pw[1]);
#pragma unroll
        for (int k = 2; k < N; ++k) {
            acc_fma<ACC>(acc.p[k], acc.cp[KAHAN ? k : 0], pw[pow_fa(k)], pw[pow_fb(k)]);
            pw[k] = mul_rounded(pw[pow_fa(k)], pw[pow_fb(k)]);
        }
        acc_add<ACC>(acc.p[N], acc.cp[KAHAN ? N : 0], (N & 1) ? x : T(__builtin_fabsf(xv)));
        if constexpr (CF && !(N & 1)) acc_add<ACC>(acc.a, acc.ca, x);
    }
    if constexpr (CF) acc_fma<ACC>(acc.b, acc.cb, x, x);
}

// The first microphone of a chunk (plain FP32 sums): the same operations
// applied to sums that are zero (literal zeros, so the sums need no clearing
// between chunks and the bits equal those of clearing first); P_2 takes s*s,
// which equals fma(s, s, +0). Compensated and FP64 sums are cleared after
// each epilogue instead (their kernels run at a register cap, and the peeled
// first microphone raised their spills).
template <int N, bool CF, int ACC>
__device__ __forceinline__ void accumulate_root_first(Acc<N, CF, ACC> &acc, float sv, float xv)
{
    static_assert(ACC == kAccF32, "only plain sums start from the first microphone");
    Acc<N, CF, ACC> z;
    z.zero();
    accumulate_root<N, CF, ACC>(z, sv, xv);
    if constexpr (N >= 3) z.p[2] = sv * sv;
    acc = z;
}

template <int N, bool CF, int ACC, bool FIRST = false>
__device__ __forceinline__ void accumulate(Acc<N, CF, ACC> &acc, float xv)
{
    const float sv = N == 1 ? xv : signed_root<N>(xv);
    if constexpr (FIRST) accumulate_root_first<N, CF, ACC>(acc, sv, xv);
    else accumulate_root<N, CF, ACC>(acc, sv, xv);
}

// ---------------------------------------------------------------------------
// Newton-Girard: E_n from P_1..P_n. Orders 2..5 use the paper's expansions,
// eqs. (9)-(12), multiplied by n! and nested in P_1 (Horner form: the same
// polynomial, with fewer operations); higher orders use the recursive form of
// the same identities (k e_k = sum_{i=1..k} (-1)^(i-1) e_{k-i} P_i),
// equivalent to eq. (8).
// ---------------------------------------------------------------------------
// newton_girard_scaled returns F with E_n = F * ng_scale(N): n! E_n for
// n <= 5 (so 1/n! can be folded into the output scale), E_n itself above.
// Written as explicit fused multiply-adds (and rounded products), so the
// rounding does not depend on the compiler's contraction choices in the
// surrounding kernel.
__host__ __device__ constexpr double ng_scale(int n)
{
    return n == 2 ? 1.0 / 2.0 : n == 3 ? 1.0 / 6.0 : n == 4 ? 1.0 / 24.0 : n == 5 ? 1.0 / 120.0 : 1.0;
}

template <int N, typename R>
__device__ __forceinline__ R newton_girard_scaled(const R *P)
{
    if constexpr (N == 1) {
        return P[1];
    } else if constexpr (N == 2) {
        // P1^2 - P2
        return fma_t(P[1], P[1], -P[2]);
    } else if constexpr (N == 3) {
        // P1^3 - 3 P1 P2 + 2 P3 = P1 (P1^2 - 3 P2) + 2 P3
        const R a = fma_t(P[1], P[1], mul_rounded(R(-3), P[2]));
        return fma_t(P[1], a, R(2) * P[3]);
    } else if constexpr (N == 4) {
        // P1^4 - 6 P1^2 P2 + 3 P2^2 + 8 P1 P3 - 6 P4
        //   = P1 (P1 (P1^2 - 6 P2) + 8 P3) + (3 P2^2 - 6 P4)
        const R a = fma_t(P[1], P[1], mul_rounded(R(-6), P[2]));
        const R b = fma_t(P[1], a, R(8) * P[3]);
        const R c = fma_t(mul_rounded(R(3), P[2]), P[2], mul_rounded(R(-6), P[4]));
        return fma_t(P[1], b, c);
    } else if constexpr (N == 5) {
        // P1^5 - 10 P1^3 P2 + 15 P1 P2^2 + 20 P1^2 P3 - 20 P2 P3 - 30 P1 P4 + 24 P5
        //   = P1 (P1 (P1 (P1^2 - 10 P2) + 20 P3) + (15 P2^2 - 30 P4)) + (24 P5 - 20 P2 P3)
        const R p3x20 = mul_rounded(R(20), P[3]);
        const R a = fma_t(P[1], P[1], mul_rounded(R(-10), P[2]));
        const R b = fma_t(P[1], a, p3x20);
        const R c = fma_t(mul_rounded(R(15), P[2]), P[2], mul_rounded(R(-30), P[4]));
        const R d = fma_t(P[1], b, c);
        const R f = fma_t(-P[2], p3x20, mul_rounded(R(24), P[5]));
        return fma_t(P[1], d, f);
    } else {
        R e[N + 1];
        e[0] = R(1);
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            R s = R(0);
#pragma unroll
            for (int i = 1; i <= k; ++i) s = fma_t((i & 1) ? e[k - i] : -e[k - i], P[i], s);
            e[k] = s * (R(1) / R(k));
        }
        return e[N];
    }
}

template <int N, typename R>
__device__ __forceinline__ R newton_girard(const R *P)
{
    return newton_girard_scaled<N, R>(P) * R(ng_scale(N));
}

// One output pixel from its sums: y = E_n * CF * in_scale, eqs. (13)/(14).
// In the FP32 form the 1/n! of the expansions is folded into `out_scale`
// (in_scale / n!, formed once per kernel by the caller).
// One output pixel from its sums: y = E_n * CF * in_scale, eqs. (13)/(14).
// Newton-Girard runs in FP64 for FP64 sums or with the plan's ng_fp64 flag
// (its result, n! E_n for n <= 5, is rounded to FP32 once the cancellation
// is done), else in FP32; either way the 1/n! of the expansions is folded
// into `out_scale` (in_scale / n!, formed once per kernel by the caller).
template <int N, bool CF, int ACC>
__device__ __forceinline__ float finish_pixel(const Acc<N, CF, ACC> &acc, const KernelParams &p,
                                              float out_scale)
{
    constexpr bool KAHAN = ACC == kAccKahan;
    float e;
    if (ACC == kAccF64 || p.ng_fp64) {
        double P[N + 1];
#pragma unroll
        for (int k = 1; k <= N; ++k) P[k] = (double)acc.p[k] - (KAHAN ? (double)acc.cp[KAHAN ? k : 0] : 0.0);
        e = (float)newton_girard_scaled<N, double>(P);
    } else {
        float P[N + 1];
#pragma unroll
        for (int k = 1; k <= N; ++k) P[k] = KAHAN ? (float)acc.p[k] - acc.cp[KAHAN ? k : 0] : (float)acc.p[k];
        e = newton_girard_scaled<N, float>(P);
    }
    if constexpr (CF) {
        float sx = (float)((N & 1) ? acc.p[N] : acc.a);
        float sb = (float)acc.b;
        if constexpr (KAHAN) {
            sx -= (N & 1) ? acc.cp[KAHAN ? N : 0] : acc.ca;
            sb -= acc.cb;
        }
        const float den = __builtin_fmaf((float)p.M, sb, p.cf_eps);
        e = e * (sx * sx) * __builtin_amdgcn_rcpf(den);
    }
    return e * out_scale;
}

// in_scale / n!: the output scale of the FP32 Newton-Girard form (wave-uniform,
// kept in a scalar register).
template <int N>
__device__ __forceinline__ float fp32_out_scale(const KernelParams &p)
{
    const float v = p.in_scale * (float)ng_scale(N);
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// ---------------------------------------------------------------------------
// The kernel.
// ---------------------------------------------------------------------------
// One workgroup's work: tile `tile` of directions over time segment `seg` of
// the frame described by p. Shared by the single-frame and the multi-frame
// (batched) kernels, so a pixel's arithmetic does not depend on how it was
// launched.
template <int N, bool CF, bool ENV, bool NEAR, int DM, int ACC>
// tx is the thread's index in the workgroup; a caller that runs the body in a
// loop passes a value the compiler cannot see through, so that nothing derived
// from it is kept live across iterations.
__device__ __forceinline__ void dmas_body(const KernelParams &p, const int tile, const int seg,
                                          float *__restrict__ smem, const int tx = (int)threadIdx.x)
{
    constexpr bool LINEAR = DM == kDelayLinear;
    constexpr bool TAB = DM == kDelayTable;          // tables through the scalar cache
    constexpr bool TAB_BLOCKS = block_tables(DM); // offsets and references per block, as scalars
    constexpr int W = kDirsPerTile;
    constexpr int K = kSamplesPerLane;
    constexpr int C = kChunk;

    const int lane = tx & (kWaveSize - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tx / kWaveSize);

    constexpr bool ROOTS = kStagesRoots<N, LINEAR>;
    using Elem = typename std::conditional<ROOTS, float2, float>::type;

    const int H = ENV ? (p.fir_len - 1) / 2 : 0;
    // LDS: the window region (mic_block x row windows; with `share` also the
    // per-wave rings in the envelope epilogue), reference delays, taps table,
    // then per wave either its ring or (share) the |y| it carries between chunks
    constexpr bool share = ENV && rings_share_windows(DM);
    const int region = window_region_floats(p.mic_block, p.row, ROOTS ? 2 : 1, ENV, H, share);
    Elem *xwin = reinterpret_cast<Elem *>(smem);                             // mic_block x row
    int *dref_lds = reinterpret_cast<int *>(smem + region);                  // dref_lds_ints(DM)
    float *tap_lds = reinterpret_cast<float *>(dref_lds + dref_lds_ints(DM)); // env_taps_len(H)
    float *side = tap_lds + env_taps_len(H);
    float *carry = side + wave * carry_stride(H);                            // share: |y| kept between chunks
    float *ring = share ? smem + wave * ring_stride(H)                       // |y| of index i at i + i/16
                        : side + wave * ring_stride(H);

    const int dir = __builtin_amdgcn_readfirstlane(p.tile_dirs[tile * W + wave]);
    const int dir0 = __builtin_amdgcn_readfirstlane(p.tile_dirs[tile * W]);
    const bool active = dir >= 0;
    const double *vdir = p.dirs + 3 * (active ? dir : dir0);
    // |v| of this wave's direction (near field), for the delays evaluated on
    // the device; wave-uniform, kept in scalar registers
    const double vnorm = [&] {
        const double v = steer_origin<NEAR>(vdir);
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
        return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    }();

    // The workgroup's outputs are [g0, g1) (g0 a multiple of 32). Pass ch
    // covers the samples [tc, tc + C), tc = ystart + ch * C, and outputs
    // [tc - lead, tc - lead + C), lead = 0 (RF) or H rounded up to a multiple
    // of 32 (envelope). |y| vanishes outside [0, T), so a walk that starts at
    // sample 0 begins on the zeroed ring, samples are computed only up to
    // min(g1 + H, T), and the outputs still missing after that come from
    // envelope-only passes (their own samples are unused: zeros).
    const int g0 = seg * p.seg_len;
    const int g1 = min(g0 + p.seg_len, p.T);
    const int lead = ENV ? env_lead(H) : 0;
    const int ystart = max(g0 - lead, 0);
    const int nchunks = (min(g1 + H, p.T) - ystart + C - 1) / C;
    const int npasses = (g1 - ystart + lead + C - 1) / C;   // >= nchunks
    const int nblocks = (p.M + p.mic_block - 1) / p.mic_block;
    const int two_halo = 2 * p.halo;

    // Steering delays, three ways:
    //  * plan-time tables (whole-sample delays): window offsets per (tile,
    //    direction, microphone) and reference delays per (tile, microphone),
    //    read through the scalar cache (constant address space: the tables
    //    do not change while a kernel runs), so the per-microphone LDS
    //    address of the hot loop costs one vector add. Either the hot loop
    //    reads each offset one microphone ahead (TAB), or (TAB_BLOCKS) a wave
    //    reads its block's offsets as one scalar block before the block's
    //    barrier, and the reference delays of the rows it stages;
    //  * M <= 64 without tables (linear delays): lane i of every wave computes
    //    its direction's delay for microphone i once, and wave 0 (the tile's
    //    reference direction) publishes its delays in LDS for the staging step;
    //  * otherwise the same per group of blocks (lane i holding microphone i
    //    of the group; the largest power of two of blocks that fits the
    //    lanes), once per group and chunk.
    // Without tables, after the barrier that publishes the reference delays
    // each lane turns (delay - reference delay) into its window's LDS offset,
    // and the hot loop reads microphone i's from lane (first lane of the
    // block) + i.
    typedef const __attribute__((address_space(4))) int32_t const_i32;
    constexpr bool table = TAB;   // p.tile_off and p.tile_dref are set (also with TAB_BLOCKS)
    const bool all_mics = !table && !TAB_BLOCKS && p.M <= kWaveSize;
    // groups of device-computed delays: 2^group_shift blocks (one group of
    // every block when each microphone has a lane)
    const int group_shift = all_mics ? 0 : 31 - __builtin_clz(max(1, kWaveSize / p.mic_block));
    // block blk's index within its group, and the lane of its microphone 0
    auto group_pos = [&](int blk) { return all_mics ? blk : blk & ((1 << group_shift) - 1); };
    auto group_lane = [&](int blk) { return group_pos(blk) * p.mic_block; };
    const_i32 *off_row = table ? reinterpret_cast<const_i32 *>(
                                     reinterpret_cast<uintptr_t>(p.tile_off + ((size_t)tile * W + wave) * p.M))
                               : nullptr;
    const_i32 *dref_row = (table || TAB_BLOCKS) ? reinterpret_cast<const_i32 *>(
                                                     reinterpret_cast<uintptr_t>(p.tile_dref + (size_t)tile * p.M))
                                               : nullptr;
    const int32_t *off_lanes = TAB_BLOCKS ? p.tile_off + ((size_t)tile * W + wave) * p.M : nullptr;
    // per-block tables: the block's window offsets of this wave's direction,
    // loaded as one scalar block before the block's barrier (mic_block <= 16;
    // the table is padded so that the 16-entry read stays inside it)
    const_i32 *off_srow = TAB_BLOCKS ? reinterpret_cast<const_i32 *>(reinterpret_cast<uintptr_t>(off_lanes)) : nullptr;
    constexpr int LB = table_block_max(N);
    int soff[LB];
    // TAB_BLOCKS: reference delays of the (at most two: mic_block <= 2 W) rows
    // this wave stages, wave and wave + W of the block
    int sdref0 = 0, sdref1 = 0;
    int mydw = 0;
    float myfrac = 0.0f;      // fraction of mydw's microphone (linear delays)
    int myoff = 0;            // LDS element where mydw's microphone's window starts
    auto block_geometry = [&](int blk) {
        if (table) return;
        const int mic = blk * p.mic_block + lane;
        if constexpr (TAB_BLOCKS) {
            // scalar loads issued before the block's barrier so they overlap the wait
            const_i32 *ob = off_srow + blk * p.mic_block;
#pragma unroll
            for (int k = 0; k < LB; ++k) soff[k] = ob[k];
            const int r0 = blk * p.mic_block + wave;
            sdref0 = (wave < p.mic_block && r0 < p.M) ? dref_row[r0] : 0;
            sdref1 = (wave + W < p.mic_block && r0 + W < p.M) ? dref_row[r0 + W] : 0;
            return;
        }
        // the first block of a group computes the group's delays
        if (group_pos(blk) != 0) return;
        const int nlanes = all_mics ? p.M : p.mic_block << group_shift;
        if (lane < nlanes) {
            if (mic < p.M) {
                mydw = steer_whole<NEAR, LINEAR>(p.mic + 3 * mic, vdir, vnorm, p.fs, p.c, &myfrac);
                if (wave == 0) dref_lds[lane] = mydw;
            } else if (wave == 0) {
                dref_lds[lane] = 0;
            }
        }
    };
    // Reference delay of microphone i (wave-uniform) of block blk, for staging.
    auto dref_of = [&](int blk, int i) {
        if constexpr (TAB_BLOCKS) return i == wave ? sdref0 : sdref1;
        return table ? dref_row[blk * p.mic_block + i] : dref_lds[group_lane(blk) + i];
    };
    // At a group's first block (after the barrier that publishes the reference
    // delays): each lane's microphone (row lane % mic_block of its block's
    // windows) gets the LDS element where its window starts.
    auto block_offsets = [&](int blk) {
        if (table || TAB_BLOCKS) return;
        if (group_pos(blk) != 0) return;
        const int mic = blk * p.mic_block + lane;
        const int nlanes = all_mics ? p.M : p.mic_block << group_shift;
        if (lane < nlanes && mic < p.M) {
            const int row = lane - (lane / p.mic_block) * p.mic_block;
            myoff = row * p.row + min(max(mydw - dref_lds[lane] + p.halo, 0), two_halo);  // the measured halo keeps this in range
        }
    };

    // Copy the taps' positions: the FIR reads them through the scalar cache.
    const float *__restrict__ taps = p.taps;

    if (all_mics) block_geometry(0);
    if constexpr (ENV) {
        if constexpr (share) {
            for (int i = lane; i < carry_stride(H); i += kWaveSize) carry[i] = 0.0f;
        } else {
            for (int i = lane; i < ring_stride(H); i += kWaveSize) ring[i] = 0.0f;
        }
        for (int j = tx; j < env_taps_len(H); j += W * kWaveSize) {
            const int k = j - kTapLead;   // reversed: entry kTapLead + k holds h[2H - k]
            tap_lds[j] = (k >= 0 && k <= 2 * H) ? taps[2 * H - k] : 0.0f;
        }
        // the first block's barrier makes the taps table visible before any epilogue
    }

    // Envelope of the outputs [tc - lead, tc - lead + C) from the ring, whose
    // indices [env_prefix(H), env_prefix(H) + C) hold |y| of the samples
    // [tc, tc + C); then keep the ring's last env_prefix(H) values.
    auto envelope_pass = [&](int tc, size_t orow) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // env[t] for t = tc - lead + o, o in [0, C): sum_k h[k] |y[t + H - k]|
        //   = sum_k h[k] r[2H + o - k], r = the ring (r[i] = |y[tc - H - lead + i]|).
        // With o = 16j + i (i, j < 16) this is the 16 x 16 matrix product
        //   F[i][j] = sum_m G[i][m] R[m][j],  G[i][m] = h[i + 2H - m] = hr[m - i]
        //   (hr = the taps reversed, zero outside),  R[m][j] = r[16j + m],
        //   m < 2H + 16,
        // done on the matrix cores in FP32, K = 4 per step: lane l holds
        // G[l % 16][4kk + l / 16] and R[4kk + l / 16][l % 16] and receives
        // F[4 (l / 16) + v][l % 16], v < 4, i.e. the four consecutive
        // outputs o = 16 (l % 16) + 4 (l / 16) + v: one 16-byte store per
        // lane, 1 KiB contiguous per wave.
        typedef float v4f __attribute__((ext_vector_type(4)));
        const int g = lane >> 4, c = lane & 15;
        const float *rb = ring + 17 * c + g;                  // r[16c + g], skewed
        const float *ha = tap_lds + kTapLead + g - c;         // hr[g - c]
        const int ks = env_ksteps(H);
        v4f e0 = {0.0f, 0.0f, 0.0f, 0.0f}, e1 = {0.0f, 0.0f, 0.0f, 0.0f};
        // K step kk = 4q + u reads the taps at ha[4kk] = hq[4u] (hq = ha + 16q) and
        // the ring at rb[4kk + kk/4] = rq[4u] (rq = rb + 17q): in groups of four
        // the eight reads use immediate offsets and are issued together. Even
        // steps go to e0, odd ones to e1.
        const float *hq = ha, *rq = rb;
        // the wave's matrix-core steps first, while the other waves fill the VALU
        // (raised wave priority: 1.3 % faster at order 5, no change at 3 or 7);
        // ks >= 4. Kernels without a register cap (plain sums, n <= 5) start
        // the first four steps from zero accumulators; in the others that
        // raised the spills.
        __builtin_amdgcn_s_setprio(3);
        int kk = 0;
        if constexpr (N <= 5 && ACC == kAccF32) {
            const float a0 = hq[0], a1 = hq[4], a2 = hq[8], a3 = hq[12];
            const float b0 = rq[0], b1 = rq[4], b2 = rq[8], b3 = rq[12];
            e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, e1, 0, 0, 0);
            e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, b3, e1, 0, 0, 0);
            kk = 4;
            hq += 16;
            rq += 17;
        }
        for (; kk + 3 < ks; kk += 4, hq += 16, rq += 17) {
            const float a0 = hq[0], a1 = hq[4], a2 = hq[8], a3 = hq[12];
            const float b0 = rq[0], b1 = rq[4], b2 = rq[8], b3 = rq[12];
            e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, e1, 0, 0, 0);
            e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, b3, e1, 0, 0, 0);
        }
        for (; kk < ks; ++kk) {
            const float a = ha[4 * kk], b = rb[4 * kk + (kk >> 2)];
            if (kk & 1) e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, e1, 0, 0, 0);
            else e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, e0, 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        const v4f e = e0 + e1;
        const int t0 = tc - lead + 16 * c + 4 * g;   // a multiple of 4 (tc - lead is one of 32)
        if (p.env_decim == 1) {
            float *dst = p.out + orow + t0;
            if (t0 >= g0 && t0 + 3 < g1 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                __builtin_nontemporal_store(e, reinterpret_cast<v4f *>(dst));
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (t0 + v >= g0 && t0 + v < g1) __builtin_nontemporal_store(e[v], dst + v);
            }
        } else if (t0 < g1 && t0 + 3 >= g0) {
            // Decimated envelope: keep the outputs at t = j * env_decim, each owned
            // by the segment that contains t (t0 >= g0 >= 0 here: both are
            // multiples of 4).
            const int dec = p.env_decim;
            const int tend = min(t0 + 4, g1);
            for (int j = (t0 + dec - 1) / dec; j * dec < tend; ++j) {
                const int v = j * dec - t0;
                const float ev = v == 0 ? e[0] : v == 1 ? e[1] : v == 2 ? e[2] : e[3];
                __builtin_nontemporal_store(ev, p.out + orow + j);
            }
        }
        // keep the last env_prefix(H) values of |y| for the next pass: in the
        // carry when the windows take the ring's region until then, else at the
        // ring's start (<= C: no overlap)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float *keep = share ? carry : ring;
        const int skew = share ? 0 : 1;
        for (int i = lane; i < env_prefix(H); i += kWaveSize)
            keep[i + skew * (i >> 4)] = ring[C + i + ((C + i) >> 4)];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };

    const float out_scale = fp32_out_scale<N>(p);

    // Power sums. Plain FP32 sums (PEEL): each chunk's first microphone starts
    // them, so they are the pass's own (nothing carried from one pass to the
    // next: sums kept live across the envelope's matrix-core steps cost 9-14
    // VGPRs and a workgroup per CU on some kernels) and envelope-only passes
    // do not read them. Other sums: cleared here and after each epilogue.
    constexpr bool PEEL = ACC == kAccF32;
    Acc<N, CF, ACC> acc_kept[K];
    if constexpr (!PEEL) {
#pragma unroll
        for (int j = 0; j < K; ++j) acc_kept[j].zero();
    }
    for (int ch = 0; ch < npasses; ++ch) {
        const int tc = ystart + ch * C;
        // Passes after the last computed chunk are envelope-only: their samples
        // lie past T (zero) or feed only outputs past g1, and enter the ring as zeros.
        const bool compute = ch < nchunks;
        Acc<N, CF, ACC> acc_pass[K];
        auto &acc = *(PEEL ? &acc_pass : &acc_kept);

        for (int blk = 0; blk < (compute ? nblocks : 0); ++blk) {
            if (!all_mics) block_geometry(blk);
            __syncthreads();  // reference delays visible; previous block's reads done
            block_offsets(blk);
            // ---- stage this block's channel windows into LDS ----
            // (issued at normal wave priority: raising it helped the loads
            // through registers by 0.9 % on the 1024-microphone frame, but costs
            // 0.5-0.9 % with the global-to-LDS copies)
            for (int i = wave; i < p.mic_block; i += W) {
                const int mic = blk * p.mic_block + i;
                Elem *dst = xwin + i * p.row;
                if (mic < p.M) {
                    const int base = tc + dref_of(blk, i) - p.halo;
                    const size_t chan = (size_t)mic * (size_t)p.T;
                    if constexpr (ROOTS) {
                        stage_row_roots(dst, p.roots, chan, base, p.row, p.T, lane);
                    } else {
                        if (p.dtype == 0) stage_row<0>(dst, p.x, chan, base, p.row, p.T, lane);
                        else if (p.dtype == 1) stage_row<1>(dst, p.x, chan, base, p.row, p.T, lane);
                        else stage_row<2>(dst, p.x, chan, base, p.row, p.T, lane);
                    }
                } else {
                    for (int r = lane; r < p.row; r += kWaveSize) dst[r] = Elem{};
                }
            }
            // this wave's global-to-LDS copies have landed (vmcnt(0), the other
            // counters untouched; FP16/BF16 samples are staged through registers)
            if (ROOTS || p.dtype == 0) __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
            // ---- hot loop: delayed samples -> roots -> power sums ----
            if (active) {
                const int nm = min(p.mic_block, p.M - blk * p.mic_block);
                // microphone i of the block: its window starts at LDS element off;
                // the chunk's first microphone starts the sums (no clearing)
                auto mic_step = [&](auto first, int i, int off) {
                    constexpr bool FIRST = decltype(first)::value;
                    const Elem *src = xwin + off + lane;
                    if constexpr (ROOTS) {
                        float2 v[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) v[j] = src[kWaveSize * j];
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            if constexpr (FIRST) accumulate_root_first<N, CF, ACC>(acc[j], v[j].x, v[j].y);
                            else accumulate_root<N, CF, ACC>(acc[j], v[j].x, v[j].y);
                        }
                    } else if constexpr (LINEAR) {
                        const float fr = __builtin_bit_cast(
                            float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, myfrac), group_lane(blk) + i));
                        float v0[K], v1[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            v0[j] = src[kWaveSize * j];
                            v1[j] = src[kWaveSize * j + 1];
                        }
#pragma unroll
                        for (int j = 0; j < K; ++j)
                            accumulate<N, CF, ACC, FIRST>(acc[j], __builtin_fmaf(fr, v1[j] - v0[j], v0[j]));
                    } else {
                        float v[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) v[j] = src[kWaveSize * j];
#pragma unroll
                        for (int j = 0; j < K; ++j) accumulate<N, CF, ACC, FIRST>(acc[j], v[j]);
                    }
                };
                using first_t = std::integral_constant<bool, PEEL>;
                using rest_t = std::false_type;
                // microphone 0 of block 0 starts the chunk's sums (block 0 has a
                // loop of its own from microphone 1: a start index chosen at run
                // time became a vector register and cost four VALU per microphone)
                if (table) {
                    // the next microphone's offset is loaded while this one is summed
                    const_i32 *ob = off_row + blk * p.mic_block;
                    int o_next = ob[0];
                    auto rest = [&](int i) {
                        const int o = o_next;
                        if (i + 1 < nm) o_next = ob[i + 1];
                        mic_step(rest_t{}, i, o);
                    };
                    if (PEEL && blk == 0) {
                        const int o = o_next;
                        if (nm > 1) o_next = ob[1];
                        mic_step(first_t{}, 0, o);
                        for (int i = 1; i < nm; ++i) rest(i);
                    } else {
                        for (int i = 0; i < nm; ++i) rest(i);
                    }
                } else if constexpr (TAB_BLOCKS) {
                    if (PEEL && blk == 0) mic_step(first_t{}, 0, soff[0]);
                    else mic_step(rest_t{}, 0, soff[0]);
#pragma unroll
                    for (int i = 1; i < LB; ++i)
                        if (i < nm) mic_step(rest_t{}, i, soff[i]);
                } else {
                    const int g0 = group_lane(blk);
                    auto off_of = [&](int i) { return __builtin_amdgcn_readlane(myoff, g0 + i); };
                    if (PEEL && blk == 0) {
                        mic_step(first_t{}, 0, off_of(0));
                        for (int i = 1; i < nm; ++i) mic_step(rest_t{}, i, off_of(i));
                    } else {
                        for (int i = 0; i < nm; ++i) mic_step(rest_t{}, i, off_of(i));
                    }
                }
            }
        }

        // rings in the window region: every wave (active or not) has read its
        // last window before any ring is written
        if constexpr (share) __syncthreads();
        if (!active) continue;
        // ---- epilogue: Newton-Girard, CF, store or envelope ----
        const size_t orow = (size_t)dir * (size_t)p.out_T;
        if constexpr (!ENV) {
            // (every pass computes: without the envelope there are no envelope-only passes)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int t = tc + lane + kWaveSize * j;
                const float y = finish_pixel<N, CF, ACC>(acc[j], p, out_scale);
                if constexpr (!PEEL) acc[j].zero();
                if (t < g1) __builtin_nontemporal_store(y, p.out + orow + t);
            }
        } else {
            // ring: the carried prefix, |y| of samples [tc, tc + C), zeros after
            // them. Samples at or past T (and every sample of an envelope-only
            // pass) enter as zeros; tc >= 0, so lane + 64 j < lim is the whole test.
            if constexpr (share) {
                for (int i = lane; i < env_prefix(H); i += kWaveSize) ring[i + (i >> 4)] = carry[i];
                for (int i = env_prefix(H) + C + lane; i < ring_logical(H); i += kWaveSize)
                    ring[i + (i >> 4)] = 0.0f;
            }
            const int lim = compute ? p.T - tc : 0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const float y = !PEEL || compute ? finish_pixel<N, CF, ACC>(acc[j], p, out_scale) : 0.0f;
                if constexpr (!PEEL) acc[j].zero();
                const int ri = env_prefix(H) + lane + kWaveSize * j;
                ring[ri + (ri >> 4)] = lane < lim - kWaveSize * j ? __builtin_fabsf(y) : 0.0f;
            }
            envelope_pass(tc, orow);
        }
    }
}

// Single-frame kernel: workgroup b covers tile b % num_tiles of segment
// b / num_tiles (tiles fastest, so workgroups resident at the same time share
// a time window of the channels). Consecutive workgroups land on different
// XCDs, so every XCD's L2 reads the whole root plane once per launch (8 x
// 4 MiB for the eRTIS-like frame); giving each XCD a contiguous range of
// segments instead cut those reads to 10 MB but measured 4-5 % slower.
//
// Register budget: the kernel is compiled for kMinWavesPerSimd waves per SIMD
// (512 / waves VGPRs; a workgroup puts two waves on each SIMD).
//  * 8 (64 VGPRs): orders up to 3 with FP32 sums and per-block tables fit it,
//    SGPRs included, which lets four workgroups share a CU where LDS allows
//    (measured 8 % faster on the 1024-microphone near-field frame, 2.0-2.7 %
//    at orders 2 and 3 on a 32-microphone frame with the rings in the window
//    region); so do the near-field kernels with delays computed on the device
//    (74 VGPRs unconstrained, 63 with no spill under the cap: 1.9 % faster on
//    the near-field frame; the far-field ones stay at 6, where the
//    32-microphone frame's LDS allows only three workgroups per CU anyway and
//    the cap cost 1.3-2.6 %).
//  * 6 (80 VGPRs, three workgroups per CU): orders 7 and 8 with FP32 sums
//    (83 and 95 VGPRs unconstrained) and Kahan / FP64 sums up to order 5 with
//    scalar-cache tables (87-89). The cap spills up to 56 bytes per lane, which
//    costs less than the third workgroup gains: 9-17 % faster on the
//    32-microphone frame, 10 % on the near-field frame at order 7. Also
//    delays computed on the device (whole-sample or linear) with FP32 sums:
//    the envelope kernels at orders 4 and 5 need 82-85 VGPRs unconstrained
//    and fit the cap with no spill (8 bytes for near-field linear delays).
//  * none otherwise: Kahan / FP64 sums at orders 6-8 spill 90-280 bytes under
//    the cap and ran 1.2-6x slower.
template <int N, int ACC, int DM, bool NEAR>
constexpr int kMinWavesPerSimd = (N <= 3 && ACC == kAccF32 && (block_tables(DM) || (NEAR && DM == kDelayComputed)))
                                     ? 8
                                 : ACC == kAccF32 ? (N >= 6 || DM == kDelayLinear || DM == kDelayComputed ? 6 : 1)
                                 : (N <= 5 && DM == kDelayTable) ? 6 : 1;

template <int N, bool CF, bool ENV, bool NEAR, int DM, int ACC>
__global__ void __launch_bounds__(kDirsPerTile * kWaveSize, (kMinWavesPerSimd<N, ACC, DM, NEAR>))
dmas_kernel(const KernelParams p)
{
    extern __shared__ float smem[];
    dmas_body<N, CF, ENV, NEAR, DM, ACC>(p, blockIdx.x % p.num_tiles, blockIdx.x / p.num_tiles, smem);
}

// Multi-frame kernel for the serving runtime: the batch lists the frames'
// parameters (all of order N) and the first workgroup index of each frame
// (ascending); each workgroup finds its frame by binary search.
template <int N, bool CF, bool ENV, bool NEAR, int DM>
__global__ void __launch_bounds__(kDirsPerTile * kWaveSize, (kMinWavesPerSimd<N, kAccF32, DM, NEAR>))
dmas_batch_kernel(const BatchParams bp)
{
    extern __shared__ float smem[];
    const int b = (int)blockIdx.x;
    int lo = 0, hi = bp.num_frames - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bp.starts[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const KernelParams p = bp.frames[lo];
    const int local = b - bp.starts[lo];
    dmas_body<N, CF, ENV, NEAR, DM, kAccF32>(p, local % p.num_tiles, local / p.num_tiles, smem);
}

// Dynamic LDS above 64 KiB must be allowed per kernel; the allowed size only
// grows. One counter per kernel instantiation, safe to share between host
// threads (a lost race only repeats the call).
// The batch kernels use the accumulation tag kBatchSlot, which no
// single-frame instantiation has.
constexpr int kBatchSlot = -1;

template <int N, bool CF, bool ENV, bool NEAR, int DM, int ACC>
std::atomic<size_t> &lds_limit_slot()
{
    static std::atomic<size_t> allowed{64 * 1024};
    return allowed;
}

inline hipError_t raise_lds_limit(const void *fn, size_t lds, std::atomic<size_t> &allowed)
{
    if (lds <= allowed.load(std::memory_order_relaxed)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    size_t cur = allowed.load(std::memory_order_relaxed);
    while (cur < lds && !allowed.compare_exchange_weak(cur, lds, std::memory_order_relaxed)) {
    }
    return hipSuccess;
}

// Host-side launcher for one order: picks the instantiation for the flags.
// Instantiated: every (CF, envelope, geometry) with whole-sample delays from
// tables or computed on the device; linear delays with CF; Kahan and FP64
// accumulation for the far field with CF.
template <int N, bool CF, bool ENV, bool NEAR, int DM, int ACC>
hipError_t launch_one(const KernelParams &p, const LaunchShape &s, hipStream_t stream)
{
    auto fn = dmas_kernel<N, CF, ENV, NEAR, DM, ACC>;
    hipError_t e = raise_lds_limit(reinterpret_cast<const void *>(fn), s.lds_bytes, lds_limit_slot<N, CF, ENV, NEAR, DM, ACC>());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(s.grid), dim3(kDirsPerTile * kWaveSize), s.lds_bytes, stream, p);
    return hipGetLastError();
}

// Resident workgroups per CU for this instantiation and LDS size.
template <int N, bool CF, bool ENV, bool NEAR, int DM, int ACC>
hipError_t occupancy_one(const LaunchShape &s, int *blocks)
{
    auto fn = dmas_kernel<N, CF, ENV, NEAR, DM, ACC>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, reinterpret_cast<const void *>(fn),
                                                        kDirsPerTile * kWaveSize, s.lds_bytes);
}

template <int N, bool CF, bool ENV, bool NEAR, int DM>
hipError_t launch_batch_one(const BatchParams &bp, unsigned grid, size_t lds, hipStream_t stream)
{
    auto fn = dmas_batch_kernel<N, CF, ENV, NEAR, DM>;
    hipError_t e = raise_lds_limit(reinterpret_cast<const void *>(fn), lds, lds_limit_slot<N, CF, ENV, NEAR, DM, kBatchSlot>());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kDirsPerTile * kWaveSize), lds, stream, bp);
    return hipGetLastError();
}

template <int N, int DM>
hipError_t launch_batch_dm(const BatchParams &bp, bool cf, bool env, bool nearfield, unsigned grid, size_t lds,
                           hipStream_t stream)
{
    if (cf) {
        if (env) return nearfield ? launch_batch_one<N, true, true, true, DM>(bp, grid, lds, stream)
                                  : launch_batch_one<N, true, true, false, DM>(bp, grid, lds, stream);
        return nearfield ? launch_batch_one<N, true, false, true, DM>(bp, grid, lds, stream)
                         : launch_batch_one<N, true, false, false, DM>(bp, grid, lds, stream);
    }
    if (env) return nearfield ? launch_batch_one<N, false, true, true, DM>(bp, grid, lds, stream)
                              : launch_batch_one<N, false, true, false, DM>(bp, grid, lds, stream);
    return nearfield ? launch_batch_one<N, false, false, true, DM>(bp, grid, lds, stream)
                     : launch_batch_one<N, false, false, false, DM>(bp, grid, lds, stream);
}

template <int N>
hipError_t launch_batch_order(const BatchParams &bp, bool cf, bool env, bool nearfield, int table, unsigned grid,
                              size_t lds, hipStream_t stream)
{
    if (table == kDelayTable) return launch_batch_dm<N, kDelayTable>(bp, cf, env, nearfield, grid, lds, stream);
    if (table == kDelayTableBlocks) return launch_batch_dm<N, kDelayTableBlocks>(bp, cf, env, nearfield, grid, lds, stream);
    if (table == kDelayTableBlocksShared)
        return launch_batch_dm<N, kDelayTableBlocksShared>(bp, cf, env, nearfield, grid, lds, stream);
    return launch_batch_dm<N, kDelayComputed>(bp, cf, env, nearfield, grid, lds, stream);
}

template <int N>
hipError_t launch_order(const KernelParams *p, const LaunchShape &s, hipStream_t stream, int *blocks)
{
#define DMAS_CASE(CF, ENV, NEAR, DM, ACC)                                                    \
    if (s.cf == CF && s.env == ENV && s.nearfield == NEAR && s.delay == DM &&             \
        s.accumulate == ACC)                                                              \
        return p ? launch_one<N, CF, ENV, NEAR, DM, ACC>(*p, s, stream)                   \
                 : occupancy_one<N, CF, ENV, NEAR, DM, ACC>(s, blocks);
#define DMAS_WHOLE(DM)                                          \
    DMAS_CASE(false, false, false, DM, kAccF32)                 \
    DMAS_CASE(false, true, false, DM, kAccF32)                  \
    DMAS_CASE(true, false, false, DM, kAccF32)                  \
    DMAS_CASE(true, true, false, DM, kAccF32)                   \
    DMAS_CASE(false, false, true, DM, kAccF32)                  \
    DMAS_CASE(false, true, true, DM, kAccF32)                   \
    DMAS_CASE(true, false, true, DM, kAccF32)                   \
    DMAS_CASE(true, true, true, DM, kAccF32)                    \
    DMAS_CASE(true, false, false, DM, kAccKahan)                \
    DMAS_CASE(true, true, false, DM, kAccKahan)                 \
    DMAS_CASE(true, false, false, DM, kAccF64)                  \
    DMAS_CASE(true, true, false, DM, kAccF64)
    DMAS_WHOLE(kDelayTable)
    DMAS_WHOLE(kDelayTableBlocks)
    DMAS_WHOLE(kDelayTableBlocksShared)
    DMAS_WHOLE(kDelayComputed)
    DMAS_CASE(true, false, false, kDelayLinear, kAccF32)
    DMAS_CASE(true, true, false, kDelayLinear, kAccF32)
    DMAS_CASE(true, false, true, kDelayLinear, kAccF32)
    DMAS_CASE(true, true, true, kDelayLinear, kAccF32)
#undef DMAS_WHOLE
#undef DMAS_CASE
    return hipErrorNotSupported;
}

}  // namespace dmas
