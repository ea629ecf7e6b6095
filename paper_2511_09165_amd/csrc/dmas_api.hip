// Host implementation of the C ABI declared in include/dmas.h, plus the two
// small device kernels it needs (steering-delay table and per-tile delay
// spread). The beamforming kernels live in dmas_kernel.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <map>
#include <vector>

#include "../../include/dmas.h"
#include "dmas_internal.hpp"
#include "dmas_kernel.hpp"
#include "dmas_plan.hpp"
#include "dmas_validate.hpp"

namespace {

thread_local std::string g_last_error;

// Largest per-tile delay table a plan builds (bytes); larger plans evaluate
// the delays per block of microphones instead.
constexpr size_t kMaxTileTableBytes = size_t(2) << 30;

dmas_status_t fail(dmas_status_t st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    if (std::getenv("DMAS_LOG")) fprintf(stderr, "[dmas] %s\n", buf);
    return st;
}

dmas_status_t hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? DMAS_ERR_OUT_OF_MEMORY : DMAS_ERR_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

// 10-bit-per-axis Morton key of a point scaled into [0, 1]^3.
uint32_t spread_bits(uint32_t v)
{
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

}  // namespace


namespace {

// Per-tile maximum |whole delay - reference whole delay| over all microphones.
template <bool NEAR, bool LINEAR>
__global__ void __launch_bounds__(dmas::kDirsPerTile * dmas::kWaveSize)
tile_spread_kernel(const double *__restrict__ mic, const double *__restrict__ dirs,
                   const int32_t *__restrict__ tiles, int M, double fs, double c,
                   int32_t *__restrict__ out)
{
    constexpr int W = dmas::kDirsPerTile;
    __shared__ int wave_max[W];
    const int lane = threadIdx.x % dmas::kWaveSize;
    const int wave = threadIdx.x / dmas::kWaveSize;
    const int dir = tiles[blockIdx.x * W + wave];
    const int dir0 = tiles[blockIdx.x * W];
    int m = 0;
    if (dir >= 0) {
        for (int i = lane; i < M; i += dmas::kWaveSize) {
            float f;
            const int d0 = dmas::steer_whole<NEAR, LINEAR>(mic + 3 * i, dirs + 3 * dir0, fs, c, &f);
            const int dw = dmas::steer_whole<NEAR, LINEAR>(mic + 3 * i, dirs + 3 * dir, fs, c, &f);
            m = max(m, abs(dw - d0));
        }
    }
    for (int s = dmas::kWaveSize / 2; s > 0; s >>= 1) m = max(m, __shfl_xor(m, s));
    if (lane == 0) wave_max[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int w = 0; w < W; ++w) r = max(r, wave_max[w]);
        out[blockIdx.x] = r;
    }
}

// Per-tile delay tables: the reference delays (the tile's first direction)
// and, per direction and microphone, the LDS element where the kernel finds
// that direction's window: (mic % mic_block) * row + clamp(delay - reference
// + halo, 0, 2 halo); empty direction slots get the row start.
template <bool NEAR>
__global__ void __launch_bounds__(dmas::kDirsPerTile * dmas::kWaveSize)
tile_table_kernel(const double *__restrict__ mic, const double *__restrict__ dirs,
                  const int32_t *__restrict__ tiles, int M, double fs, double c, int halo, int mic_block,
                  int row, int32_t *__restrict__ off, int32_t *__restrict__ dref)
{
    constexpr int W = dmas::kDirsPerTile;
    const int lane = threadIdx.x % dmas::kWaveSize;
    const int wave = threadIdx.x / dmas::kWaveSize;
    const int dir = tiles[blockIdx.x * W + wave];
    const int dir0 = tiles[blockIdx.x * W];
    int32_t *dst = off + ((size_t)blockIdx.x * W + wave) * M;
    for (int i = lane; i < M; i += dmas::kWaveSize) {
        float f;
        const int d0 = dmas::steer_whole<NEAR, false>(mic + 3 * i, dirs + 3 * dir0, fs, c, &f);
        if (wave == 0) dref[(size_t)blockIdx.x * M + i] = d0;
        int r = 0;
        if (dir >= 0) {
            const int dw = dmas::steer_whole<NEAR, false>(mic + 3 * i, dirs + 3 * dir, fs, c, &f);
            r = min(max(dw - d0 + halo, 0), 2 * halo);
        }
        dst[i] = (i % mic_block) * row + r;
    }
}

template <bool NEAR, bool LINEAR>
__global__ void delay_table_kernel(const double *__restrict__ mic, const double *__restrict__ dirs,
                                   int M, int D, double fs, double c, int32_t *__restrict__ whole,
                                   float *__restrict__ frac)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * D) return;
    const int p = (int)(idx / M);
    const int i = (int)(idx % M);
    float f;
    whole[idx] = dmas::steer_whole<NEAR, LINEAR>(mic + 3 * i, dirs + 3 * p, fs, c, &f);
    if (frac) frac[idx] = f;
}

void design_lowpass(int L, double fc, double fs, std::vector<double> &h)
{
    const double pi = 3.14159265358979323846;
    const int half = (L - 1) / 2;
    const double wc = 2.0 * fc / fs;
    h.assign(L, 0.0);
    double sum = 0.0;
    for (int k = 0; k < L; ++k) {
        const double m = k - half;
        const double ideal = (m == 0.0) ? wc : std::sin(pi * wc * m) / (pi * m);
        const double w = (L == 1) ? 1.0 : 0.54 - 0.46 * std::cos(2.0 * pi * k / (L - 1));
        h[k] = ideal * w;
        sum += h[k];
    }
    for (double &v : h) v /= sum;
}

void plan_free(dmas_plan_s *p)
{
    if (!p) return;
    int cur = 0;
    bool switched = false;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) switched = hipSetDevice(p->device) == hipSuccess;
    // teardown: a failed free has no caller to report to
    (void)hipFree(p->d_mic);
    (void)hipFree(p->d_dirs);
    (void)hipFree(p->d_tiles);
    (void)hipFree(p->d_tile_off);
    (void)hipFree(p->d_tile_dref);
    (void)hipFree(p->d_taps);
    (void)hipFree(p->d_pulse);
    if (switched) (void)hipSetDevice(cur);
    delete p;
}

// Launch time, in chunk-times, of segments of length s: workgroups go in
// launch order (tiles fastest, then segments) to whichever of the `slots`
// resident places frees first, and a workgroup of segment k takes its
// chunks plus kWorkgroupSetup. All workgroups of a segment take equally
// long, so the places' free times are kept as (time, count) pairs.
constexpr double kWorkgroupSetup = 0.5;   // fixed cost per workgroup, in chunk-times (measured fit)

double launch_makespan(int T, int H, int s, int num_tiles, int64_t slots, int64_t *total_chunks)
{
    const int C = dmas::kChunk, lead = dmas::env_lead(H);
    std::map<double, int64_t> free_at{{0.0, slots}};
    int64_t chunks = 0;
    for (int g0 = 0; g0 < T; g0 += s) {
        const int g1 = std::min(g0 + s, T);
        const int c = (std::min(g1 + H, T) - std::max(g0 - lead, 0) + C - 1) / C;
        chunks += c;
        const double d = c + kWorkgroupSetup;
        // the earliest free places take the next workgroups; a place whose
        // workgroup ends can take another of the same segment (d > 0)
        for (int64_t need = num_tiles; need > 0;) {
            const auto it = free_at.begin();
            const double t = it->first;
            const int64_t m = std::min(it->second, need);
            if ((it->second -= m) == 0) free_at.erase(it);
            free_at[t + d] += m;
            need -= m;
        }
    }
    *total_chunks = chunks * num_tiles;
    return free_at.rbegin()->first;
}

// Output samples per workgroup. Every segment is a multiple of 32 samples
// (aligned output lines); a segment away from the record's ends walks
// s + H + lead samples, and s is the longest that keeps that walk's chunk
// count. The count minimises the launch's makespan (above): long segments
// recompute little halo and pay the workgroup setup less often, but the last
// workgroups should not leave most of the device idle. Ties go to less work.
void choose_segments(int T, int num_tiles, int H, int64_t slots, int fixed, int *seg, int *nseg)
{
    const int C = dmas::kChunk;
    const int extra = H + dmas::env_lead(H);
    if (fixed > 0) {
        *seg = (fixed + 31) & ~31;
        *nseg = (T + *seg - 1) / *seg;
        return;
    }
    double best = 0;
    int64_t best_work = 0;
    int last_s = -1;
    const int max_seg = std::max(1, (T + 31) / 32);
    for (int want = 1; want <= max_seg; ++want) {
        int s = ((T + want - 1) / want + 31) & ~31;
        const int chunks = (s + extra + C - 1) / C;
        s = std::max(32, (chunks * C - extra) & ~31);
        if (s == last_s) continue;
        last_s = s;
        const int nsg = (T + s - 1) / s;
        int64_t work = 0;
        const double cost = launch_makespan(T, H, s, num_tiles, slots, &work);
        if (want == 1 || cost < best * (1.0 - 1e-9) || (cost <= best * (1.0 + 1e-9) && work < best_work)) {
            best = cost;
            best_work = work;
            *seg = s;
            *nseg = nsg;
        }
        if ((int64_t)num_tiles * nsg > 64 * slots) break;
    }
}

// Host estimate of fs*tau (tiling heuristics only; the kernels compute their own).
double host_steer(const double *r, const double *v, bool nearfield, double fs, double c)
{
    if (!nearfield) return -fs * (r[0] * v[0] + r[1] * v[1] + r[2] * v[2]) / c;
    const double dm = std::sqrt((v[0] - r[0]) * (v[0] - r[0]) + (v[1] - r[1]) * (v[1] - r[1]) +
                                (v[2] - r[2]) * (v[2] - r[2]));
    return fs * (dm - std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])) / c;
}

// Microphones that bound the delay spread: the extremes of the array along
// 13 axes, plus the one farthest from the centroid.
std::vector<int> probe_mics(const double *mic, int M)
{
    static const double axes[13][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {1, 1, 0},  {1, -1, 0},
                                       {1, 0, 1},  {1, 0, -1}, {0, 1, 1},  {0, 1, -1}, {1, 1, 1},
                                       {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};
    std::vector<int> out;
    auto add = [&](int i) {
        if (std::find(out.begin(), out.end(), i) == out.end()) out.push_back(i);
    };
    double cen[3] = {0, 0, 0};
    for (int i = 0; i < M; ++i)
        for (int a = 0; a < 3; ++a) cen[a] += mic[3 * i + a] / M;
    for (const auto &ax : axes) {
        int lo = 0, hi = 0;
        double vlo = INFINITY, vhi = -INFINITY;
        for (int i = 0; i < M; ++i) {
            const double d = mic[3 * i] * ax[0] + mic[3 * i + 1] * ax[1] + mic[3 * i + 2] * ax[2];
            if (d < vlo) vlo = d, lo = i;
            if (d > vhi) vhi = d, hi = i;
        }
        add(lo);
        add(hi);
    }
    int far = 0;
    double dfar = -1;
    for (int i = 0; i < M; ++i) {
        double d = 0;
        for (int a = 0; a < 3; ++a) d += (mic[3 * i + a] - cen[a]) * (mic[3 * i + a] - cen[a]);
        if (d > dfar) dfar = d, far = i;
    }
    add(far);
    return out;
}

// Group directions into tiles of up to kDirsPerTile whose steering delays stay
// close to the tile's first (reference) direction: walk the directions along a
// Morton curve and greedily add, from a short look-ahead window, those within
// a delay budget of the reference. The budget adapts to the grid (twice the
// median spread of plain consecutive groups); it only affects efficiency, the
// exact spread is measured on the device afterwards.
std::vector<int32_t> make_tiles(const dmas_plan_desc_t *d, bool nearfield, double c)
{
    constexpr int W = dmas::kDirsPerTile;
    const int D = d->num_dirs;
    std::vector<int> order(D);
    std::iota(order.begin(), order.end(), 0);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int q = 0; q < D; ++q)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], d->dirs[3 * q + a]);
            hi[a] = std::max(hi[a], d->dirs[3 * q + a]);
        }
    std::vector<uint32_t> key(D);
    for (int q = 0; q < D; ++q) {
        uint32_t k = 0;
        for (int a = 0; a < 3; ++a) {
            const double span = hi[a] - lo[a];
            const double u = span > 0 ? (d->dirs[3 * q + a] - lo[a]) / span : 0.0;
            k |= spread_bits((uint32_t)std::min(1023.0, std::floor(u * 1024.0))) << a;
        }
        key[q] = k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });

    const std::vector<int> probes = probe_mics(d->mic_pos, d->num_mics);
    const int P = (int)probes.size();
    std::vector<double> tau((size_t)D * P);
    for (int q = 0; q < D; ++q)
        for (int j = 0; j < P; ++j)
            tau[(size_t)q * P + j] = host_steer(d->mic_pos + 3 * probes[j], d->dirs + 3 * q, nearfield, d->fs, c);
    auto dist = [&](int a, int b) {
        double m = 0;
        for (int j = 0; j < P; ++j) m = std::max(m, std::fabs(tau[(size_t)a * P + j] - tau[(size_t)b * P + j]));
        return m;
    };
    std::vector<double> natural;
    for (int q = 0; q < D; q += W) {
        double m = 0;
        for (int w = 1; w < W && q + w < D; ++w) m = std::max(m, dist(order[q], order[q + w]));
        natural.push_back(m);
    }
    std::nth_element(natural.begin(), natural.begin() + natural.size() / 2, natural.end());
    const double budget = std::max(6.0, 2.0 * natural[natural.size() / 2] + 1.0);

    std::vector<int32_t> tiles;
    std::vector<char> used(D, 0);
    const int lookahead = 4 * W;
    for (int pos = 0; pos < D; ++pos) {
        if (used[pos]) continue;
        const int ref = order[pos];
        used[pos] = 1;
        int32_t tile[W];
        int cnt = 0;
        tile[cnt++] = ref;
        for (int j = pos + 1; j < D && j <= pos + lookahead && cnt < W; ++j) {
            if (used[j]) continue;
            if (dist(ref, order[j]) <= budget) {
                tile[cnt++] = order[j];
                used[j] = 1;
            }
        }
        for (int w = 0; w < W; ++w) tiles.push_back(w < cnt ? tile[w] : -1);
    }
    return tiles;
}



// Root planes live in a memory pool of the library's own on each device,
// allocated and freed in stream order around each launch, so that calls on
// several streams never share one plane and the pool keeps the memory for
// the next call instead of returning it to the device.
std::mutex g_pool_mutex;
std::vector<hipMemPool_t> g_pools;

hipError_t device_pool(int dev, hipMemPool_t *out)
{
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    if (g_pools.empty()) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess) return e;
        g_pools.assign((size_t)std::max(n, 1), nullptr);
    }
    if (dev < 0 || dev >= (int)g_pools.size()) return hipErrorInvalidDevice;
    if (!g_pools[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        hipError_t e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return e;
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return e;
        }
        g_pools[dev] = pool;
    }
    *out = g_pools[dev];
    return hipSuccess;
}

// Root plane of dmas_envelope_noalloc: one array per device for the
// library's lifetime, so that entry point allocates nothing. Host code uses
// the device address that hipGetSymbolAddress returns for the current device
// (the array's name on the host is only a stand-in for the symbol).
static __device__ __align__(256) float2 scratch[DMAS_NOALLOC_SCRATCH_BYTES / sizeof(float2)];

std::mutex g_scratch_mutex;
std::vector<float2 *> g_scratch;   // per device: address of `scratch`, null until looked up

// Address of `scratch` on device dev, which must be current: looked up on the
// first call for that device and kept.
hipError_t scratch_address(int dev, float2 **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch.empty()) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess) return e;
        g_scratch.assign((size_t)std::max(n, 1), nullptr);
    }
    if (dev < 0 || dev >= (int)g_scratch.size()) return hipErrorInvalidDevice;
    if (!g_scratch[dev]) {
        float2 *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// One beamforming launch. The root plane comes from the per-device pool
// (stream-ordered allocation around the launch), or with noalloc from the
// per-device `scratch` array.
dmas_status_t run(dmas_plan_t plan, const void *d_x, float *d_out, float in_scale, void *stream,
                  bool env, bool noalloc = false)
{
    if (!plan) return fail(DMAS_ERR_INVALID_ARG, "plan is NULL");
    if (!d_x || !d_out) return fail(DMAS_ERR_INVALID_ARG, "device pointer is NULL");
    if (!(in_scale > 0.0f) || !std::isfinite(in_scale))
        return fail(DMAS_ERR_INVALID_ARG, "in_scale must be finite and > 0 (got %g)", (double)in_scale);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != plan->device)
        return fail(DMAS_ERR_INVALID_ARG, "plan belongs to device %d but device %d is current", plan->device,
                    cur);
    hipStream_t st = static_cast<hipStream_t>(stream);
    float2 *plane = nullptr;
    hipError_t e = hipSuccess;
    if (plan->roots && noalloc) {
        const size_t need = dmas::plane_bytes(plan);
        if (need > DMAS_NOALLOC_SCRATCH_BYTES)
            return fail(DMAS_ERR_UNSUPPORTED,
                        "root plane of %zu bytes (M=%d x T=%d x 8) exceeds the %zu-byte fixed scratch of "
                        "dmas_envelope_noalloc",
                        need, plan->M, plan->T, (size_t)DMAS_NOALLOC_SCRATCH_BYTES);
        float2 *fixed = nullptr;
        e = scratch_address(plan->device, &fixed);
        if (e != hipSuccess) return hip_fail(e, "address of the fixed root-plane scratch");
        // every element the kernel reads is written here first: nothing needs clearing
        e = dmas::stage_roots(plan, d_x, fixed, st);
        if (e != hipSuccess) return hip_fail(e, "root-plane launch");
        const dmas::KernelParams kp = dmas::make_params(plan, d_x, fixed, d_out, in_scale, env);
        e = dmas::launch_plan(plan->order, &kp, dmas::shape_of(plan, env), st);
        if (e == hipErrorNotSupported)
            return fail(DMAS_ERR_UNSUPPORTED, "no kernel for order %d cf=%d env=%d near=%d accumulate=%d",
                        plan->order, (int)plan->cf, (int)env, (int)plan->nearfield, (int)plan->compensated);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return DMAS_OK;
    }
    if (plan->roots) {
        hipMemPool_t pool = nullptr;
        e = device_pool(plan->device, &pool);
        if (e != hipSuccess) return hip_fail(e, "root-plane memory pool");
        e = hipMallocFromPoolAsync(reinterpret_cast<void **>(&plane), dmas::plane_bytes(plan), pool, st);
        if (e != hipSuccess) return hip_fail(e, "root-plane allocation");
        e = dmas::stage_roots(plan, d_x, plane, st);
        if (e != hipSuccess) {
            (void)hipFreeAsync(plane, st);
            return hip_fail(e, "root-plane launch");
        }
    }
    const dmas::KernelParams kp = dmas::make_params(plan, d_x, plane, d_out, in_scale, env);
    const dmas::LaunchShape ls = dmas::shape_of(plan, env);
    e = dmas::launch_plan(plan->order, &kp, ls, st);
    if (plane) {
        const hipError_t ef = hipFreeAsync(plane, st);
        if (e == hipSuccess) e = ef;
    }
    if (e == hipErrorNotSupported)
        return fail(DMAS_ERR_UNSUPPORTED, "no kernel for order %d cf=%d env=%d near=%d linear=%d accumulate=%d",
                    plan->order, (int)plan->cf, (int)env, (int)plan->nearfield, (int)plan->linear,
                    (int)plan->compensated);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return DMAS_OK;
}

}  // namespace

void dmas::set_last_error(const char *msg)
{
    g_last_error = msg ? msg : "";
}

hipError_t dmas::launch_plan(int order, const dmas::KernelParams *kp, const dmas::LaunchShape &ls, hipStream_t st,
                             int *blocks)
{
    switch (order) {
    case 1: return dmas::launch_order1(kp, ls, st, blocks);
    case 2: return dmas::launch_order2(kp, ls, st, blocks);
    case 3: return dmas::launch_order3(kp, ls, st, blocks);
    case 4: return dmas::launch_order4(kp, ls, st, blocks);
    case 5: return dmas::launch_order5(kp, ls, st, blocks);
    case 6: return dmas::launch_order6(kp, ls, st, blocks);
    case 7: return dmas::launch_order7(kp, ls, st, blocks);
    case 8: return dmas::launch_order8(kp, ls, st, blocks);
    default: return hipErrorInvalidValue;
    }
}

extern "C" {

dmas_status_t dmas_plan_desc_init(dmas_plan_desc_t *d)
{
    if (!d) return fail(DMAS_ERR_INVALID_ARG, "desc is NULL");
    std::memset(d, 0, sizeof *d);
    d->order = 1;
    d->use_cf = 1;
    d->geometry = DMAS_FARFIELD;
    d->c = 343.0;
    d->cf_eps = 1e-20;
    d->fir_len = 63;
    d->fir_fc = 5000.0;
    d->in_dtype = DMAS_F32;
    d->delay_mode = DMAS_DELAY_NEAREST;
    d->env_decimation = 1;
    return DMAS_OK;
}

dmas_status_t dmas_plan_create(const dmas_plan_desc_t *d, dmas_plan_t *out)
{
    if (!d || !out) return fail(DMAS_ERR_INVALID_ARG, "desc or out is NULL");
    *out = nullptr;
    char msg[512];
    dmas::DescValues vals;
    const dmas_status_t vst = dmas::validate_desc(d, dmas::kChunk, msg, sizeof msg, &vals);
    if (vst != DMAS_OK) return fail(vst, "%s", msg);
    const int M = d->num_mics, T = d->num_samples, D = d->num_dirs, n = d->order;
    const double c = vals.c, eps = vals.cf_eps, fc = vals.fir_fc;
    const int L = vals.fir_len, decim = vals.env_decimation;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");

    dmas_plan_s *p = new (std::nothrow) dmas_plan_s();
    if (!p) return fail(DMAS_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->device = dev;
    p->M = M;
    p->T = T;
    p->D = D;
    p->order = n;
    p->cf = d->use_cf != 0;
    p->nearfield = d->geometry == DMAS_NEARFIELD;
    p->linear = d->delay_mode == DMAS_DELAY_LINEAR;
    p->roots = n >= 2 && !p->linear;
    p->compensated = d->compensated;
    p->ng_fp64 = d->ng_fp64;
    p->dtype = d->in_dtype;
    p->fs = d->fs;
    p->c = c;
    p->cf_eps = (float)eps;
    p->fir_len = L;
    p->env_decim = decim;
    p->mf_len = d->mf_pulse ? d->mf_len : 0;

    // ---- tiles of nearby directions (Morton order, greedy within a delay budget) ----
    constexpr int W = dmas::kDirsPerTile;
    std::vector<int32_t> tiles = make_tiles(d, p->nearfield, c);
    p->num_tiles = (int)(tiles.size() / W);

    std::vector<double> taps_d;
    // zero-padded to a multiple of 4: the envelope FIR reads taps in groups of 4
    std::vector<float> taps((size_t)dmas::fir_taps_padded(L), 0.0f);
    if (d->fir_taps) {
        std::copy(d->fir_taps, d->fir_taps + L, taps.begin());
    } else {
        design_lowpass(L, fc, d->fs, taps_d);
        for (int k = 0; k < L; ++k) taps[k] = (float)taps_d[k];
    }

    auto dev_copy = [&](void **dst, const void *src, size_t bytes, const char *what) -> dmas_status_t {
        hipError_t err = hipMalloc(dst, bytes);
        if (err != hipSuccess) return hip_fail(err, what);
        err = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        if (err != hipSuccess) return hip_fail(err, what);
        return DMAS_OK;
    };
    dmas_status_t st;
    if ((st = dev_copy((void **)&p->d_mic, d->mic_pos, sizeof(double) * 3 * M, "mic_pos")) != DMAS_OK ||
        (st = dev_copy((void **)&p->d_dirs, d->dirs, sizeof(double) * 3 * (size_t)D, "dirs")) != DMAS_OK ||
        (st = dev_copy((void **)&p->d_tiles, tiles.data(), sizeof(int32_t) * tiles.size(), "tiles")) != DMAS_OK ||
        (st = dev_copy((void **)&p->d_taps, taps.data(), sizeof(float) * taps.size(), "taps")) != DMAS_OK ||
        (p->mf_len && (st = dev_copy((void **)&p->d_pulse, d->mf_pulse, sizeof(float) * p->mf_len, "pulse")) != DMAS_OK)) {
        plan_free(p);
        return st;
    }

    // ---- delay spread per tile, measured with the kernels' own delay code ----
    {
        int32_t *d_spread = nullptr;
        e = hipMalloc(&d_spread, sizeof(int32_t) * p->num_tiles);
        if (e != hipSuccess) {
            plan_free(p);
            return hip_fail(e, "spread buffer");
        }
        auto kern = p->nearfield ? (p->linear ? tile_spread_kernel<true, true> : tile_spread_kernel<true, false>)
                                 : (p->linear ? tile_spread_kernel<false, true> : tile_spread_kernel<false, false>);
        hipLaunchKernelGGL(kern, dim3(p->num_tiles), dim3(W * dmas::kWaveSize), 0, nullptr, p->d_mic, p->d_dirs,
                           p->d_tiles, M, p->fs, p->c, d_spread);
        e = hipGetLastError();
        std::vector<int32_t> spread(p->num_tiles);
        if (e == hipSuccess)
            e = hipMemcpy(spread.data(), d_spread, sizeof(int32_t) * p->num_tiles, hipMemcpyDeviceToHost);
        (void)hipFree(d_spread);
        if (e != hipSuccess) {
            plan_free(p);
            return hip_fail(e, "tile spread");
        }
        p->halo = 0;
        for (int v : spread) p->halo = std::max(p->halo, v);
    }
    // ---- LDS layout: mic_block x row windows, reference delays, envelope rings ----
    // Per-tile delay tables for whole-sample delays, when of modest size (the
    // delay mode selects the kernel, so it is fixed before the LDS layout and
    // the occupancy queries below).
    const size_t table_bytes = (size_t)p->num_tiles * M * (W + 1) * sizeof(int32_t);
    p->tables = !p->linear && table_bytes <= kMaxTileTableBytes && !std::getenv("DMAS_NO_DELAY_TABLE");
    // Per-block tables (each wave reads its block's offsets and reference
    // delays as scalars before the block's barrier, and the block's microphone
    // loop is straight-line code): always with more microphones than lanes;
    // with fewer, for plain FP32 sums, where they measured 1-3 % faster on the
    // 32-microphone frame and 1.5-11 % on serving frames of 16-64 microphones
    // (bitwise identical; 1.8 % at order 8 once the windows are copied by
    // global-to-LDS loads). With Kahan or FP64 sums, whose register budgets
    // differ, the per-microphone reads one ahead stay (1.4-2.4 % faster
    // there). DMAS_BLOCK_TABLES=0/1 overrides the choice for M <= 64 (tuning).
    p->block_tables = M > dmas::kWaveSize || p->compensated == DMAS_ACCUM_F32;
    if (const char *bt = std::getenv("DMAS_BLOCK_TABLES"))
        p->block_tables = M > dmas::kWaveSize || std::atoi(bt) != 0;
    p->block_tables = p->block_tables && p->tables;
    const int C = dmas::kChunk;
    const int H = (L - 1) / 2;
    p->row = C + 2 * p->halo + (p->linear ? 1 : 0);
    p->row = (p->row + 3) & ~3;
    const size_t lds_cap = (size_t)prop.sharedMemPerBlock;
    // reference delays in LDS (kernels that evaluate delays on the device)
    const size_t fixed = sizeof(int) * dmas::dref_lds_ints(dmas::shape_of(p, true).delay);
    // Window elements: (root, sample) pairs when the kernel stages roots
    // (whole-sample delays, n >= 2), else samples.
    const size_t elem = p->roots ? 2 * sizeof(float) : sizeof(float);
    const size_t ring_bytes = sizeof(float) * (size_t)W * dmas::ring_stride(H);
    // LDS of a workgroup with m microphones per block. Envelope: taps, then
    // per-wave rings, or (share) per-wave carries while the rings take the
    // window region after a chunk's last block.
    auto lds_for = [&](int m, bool env, bool share) {
        const size_t win = elem * (size_t)m * p->row;
        const size_t side = sizeof(float) * (size_t)(dmas::env_taps_len(H) +
                                                     W * (share ? dmas::carry_stride(H) : dmas::ring_stride(H)));
        return fixed + (env ? (share ? std::max(win, ring_bytes) : win) + side : win);
    };
    // With per-block tables the kernel reads a block's offsets as one scalar
    // block of table_block_max(n) entries: that caps the block.
    const int mb_cap = p->block_tables ? dmas::table_block_max(n) : dmas::kMaxMicBlock;
    const int mb_max = std::min(M, mb_cap);
    // Microphones per LDS block, from the envelope kernel's occupancy (its
    // registers, LDS and the wave limit decide): with M <= 64 the largest
    // block that keeps three workgroups per CU (or as many as any block
    // reaches), since a whole array takes only a few blocks per chunk; with
    // more microphones the largest block that reaches the highest occupancy
    // (measured: 1024 microphones at order 3 run 7 % faster with 12-microphone
    // blocks at four workgroups per CU than with 16 at three, while 32
    // microphones run 5 % slower that way). Returns the block (0 if none
    // fits) and the workgroups per CU at that block.
    const int occ_target = M <= dmas::kWaveSize ? 3 : 1 << 30;
    auto choose_block = [&](bool share, int *mb_out, int *occ_out) -> hipError_t {
        p->share_rings = share;
        int best = 0, best_occ = 0, occ_at_best = 0;
        for (int cand : {mb_max, 48, 32, 24, 16, 12, 8, 4, 2, 1}) {
            if (cand > mb_max || lds_for(cand, true, share) > lds_cap) continue;
            dmas::LaunchShape ls = dmas::shape_of(p, true);
            ls.lds_bytes = lds_for(cand, true, share);
            int occ = 0;
            hipError_t q = dmas::launch_plan(n, nullptr, ls, nullptr, &occ);
            if (q == hipErrorNotSupported) {   // no kernel for these flags: reported at launch
                occ = (int)(lds_cap / lds_for(cand, true, share));
                q = hipSuccess;
            }
            if (q != hipSuccess) return q;
            if (std::min(occ, occ_target) > best_occ) {
                best_occ = std::min(occ, occ_target);
                best = cand;
                occ_at_best = occ;
            }
        }
        *mb_out = best;
        *occ_out = occ_at_best;
        return hipSuccess;
    };
    // The rings share the window region only where that buys occupancy or a
    // larger block (the 1024-microphone frame: 16-microphone blocks at four
    // workgroups per CU instead of 12; order-3 frames whose windows then fit
    // four workgroups per CU): elsewhere the carry between chunks and the
    // extra barrier cost 0.7-2.1 % on the 32-microphone frame.
    // DMAS_RING_SHARING=0/1 overrides the choice (tuning).
    int mb = 0, occ_mb = 0;
    e = choose_block(false, &mb, &occ_mb);
    if (e == hipSuccess && p->block_tables) {
        int mb_s = 0, occ_s = 0;
        e = choose_block(true, &mb_s, &occ_s);
        bool share = occ_s > occ_mb || (occ_s == occ_mb && mb_s > mb);
        if (const char *rs = std::getenv("DMAS_RING_SHARING")) share = std::atoi(rs) != 0;
        if (share) {
            mb = mb_s;
            occ_mb = occ_s;
        }
        p->share_rings = share;
    }
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "occupancy query");
    }
    const bool share = p->share_rings;
    if (const char *fixed_mb = std::getenv("DMAS_MIC_BLOCK")) mb = std::max(1, std::min(mb_max, std::atoi(fixed_mb)));
    if (mb == 0 || lds_for(mb, true, share) > lds_cap) {
        plan_free(p);
        return fail(DMAS_ERR_UNSUPPORTED,
                    "direction tiles spread over %d samples: the channel window does not fit in LDS", p->halo);
    }
    p->mic_block = mb;
    p->lds_rf = lds_for(mb, false, share);
    p->lds_env = lds_for(mb, true, share);
    // the kernel derives the same layout from (mic_block, row, H)
    const int delay_mode = dmas::shape_of(p, true).delay;
    if (p->lds_env != (size_t)dmas::kernel_lds_bytes(mb, p->row, (int)(elem / sizeof(float)), true, H, delay_mode) ||
        p->lds_rf != (size_t)dmas::kernel_lds_bytes(mb, p->row, (int)(elem / sizeof(float)), false, H, delay_mode)) {
        plan_free(p);
        return fail(DMAS_ERR_DEVICE, "internal: LDS layout mismatch");
    }

    // Build the delay tables: the kernel reads window offsets and reference
    // delays instead of evaluating eq. (1) on the device and moving the
    // results between lanes.
    if (p->tables) {
        const size_t n_off = (size_t)p->num_tiles * W * M, n_dref = (size_t)p->num_tiles * M;
        // kTableBlockMax spare entries: a scalar block read may run past the last row
        e = hipMalloc((void **)&p->d_tile_off, sizeof(int32_t) * (n_off + dmas::kTableBlockMax));
        if (e == hipSuccess) e = hipMemset(p->d_tile_off + n_off, 0, sizeof(int32_t) * dmas::kTableBlockMax);
        if (e == hipSuccess) e = hipMalloc((void **)&p->d_tile_dref, sizeof(int32_t) * n_dref);
        if (e == hipSuccess) {
            auto kern = p->nearfield ? tile_table_kernel<true> : tile_table_kernel<false>;
            hipLaunchKernelGGL(kern, dim3(p->num_tiles), dim3(W * dmas::kWaveSize), 0, nullptr, p->d_mic, p->d_dirs,
                               p->d_tiles, M, p->fs, p->c, p->halo, p->mic_block, p->row, p->d_tile_off,
                               p->d_tile_dref);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        }
        if (e != hipSuccess) {
            plan_free(p);
            return hip_fail(e, "tile delay table");
        }
    }

    p->device_bytes = sizeof(double) * 3 * ((size_t)M + (size_t)D) + sizeof(int32_t) * tiles.size() +
                      sizeof(float) * taps.size() + sizeof(float) * (size_t)p->mf_len +
                      (p->d_tile_off ? sizeof(int32_t) * ((size_t)p->num_tiles * W * M + dmas::kTableBlockMax +
                                                          (size_t)p->num_tiles * M)
                                     : 0);

    const char *fixed_seg = std::getenv("DMAS_SEGMENT");
    const int seg_override = fixed_seg ? std::atoi(fixed_seg) : 0;
    p->nseg_rf = p->nseg_env = 1;   // dmas::shape_of() needs a grid; the occupancy query ignores it
    for (int env = 0; env < 2; ++env) {
        int blocks = 0;
        e = dmas::launch_plan(n, nullptr, dmas::shape_of(p, env != 0), nullptr, &blocks);
        if (e != hipSuccess && e != hipErrorNotSupported) {
            plan_free(p);
            return hip_fail(e, "occupancy query");
        }
        const int64_t slots = (int64_t)prop.multiProcessorCount * std::max(1, blocks);
        if (env)
            choose_segments(T, p->num_tiles, H, slots, seg_override, &p->seg_env, &p->nseg_env);
        else
            choose_segments(T, p->num_tiles, 0, slots, seg_override, &p->seg_rf, &p->nseg_rf);
        if (env) p->occ_env = blocks; else p->occ_rf = blocks;
    }
    if ((int64_t)p->num_tiles * std::max(p->nseg_rf, p->nseg_env) > INT32_MAX) {
        plan_free(p);
        return fail(DMAS_ERR_UNSUPPORTED, "grid too large");
    }
    if (std::getenv("DMAS_LOG"))
        fprintf(stderr,
                "[dmas] plan M=%d T=%d D=%d n=%d tiles=%d halo=%d row=%d mb=%d seg=%d/%d nseg=%d/%d lds=%zu/%zu "
                "occupancy=%d/%d\n",
                M, T, D, n, p->num_tiles, p->halo, p->row, p->mic_block, p->seg_rf, p->seg_env, p->nseg_rf,
                p->nseg_env, p->lds_rf, p->lds_env, p->occ_rf, p->occ_env);
    *out = p;
    return DMAS_OK;
}

dmas_status_t dmas_plan_destroy(dmas_plan_t plan)
{
    plan_free(plan);
    return DMAS_OK;
}

dmas_status_t dmas_plan_query(dmas_plan_t p, dmas_plan_info_t *info)
{
    if (!p || !info) return fail(DMAS_ERR_INVALID_ARG, "plan or info is NULL");
    std::memset(info, 0, sizeof *info);
    info->num_mics = p->M;
    info->num_samples = p->T;
    info->num_dirs = p->D;
    info->order = p->order;
    info->dirs_per_tile = dmas::kDirsPerTile;
    info->num_tiles = p->num_tiles;
    info->samples_per_lane = dmas::kSamplesPerLane;
    info->chunk = dmas::kChunk;
    info->segment = p->seg_env;
    info->num_segments = p->nseg_env;
    info->window_halo = p->halo;
    info->mics_per_block = p->mic_block;
    info->lds_bytes = (int32_t)p->lds_env;
    info->fir_len = p->fir_len;
    info->workgroups = (int64_t)p->num_tiles * p->nseg_env;
    info->delay_table_bytes = p->d_tile_off ? (int64_t)p->num_tiles * p->M * (dmas::kDirsPerTile + 1) * 4 : 0;
    info->device_bytes = (int64_t)p->device_bytes;
    return DMAS_OK;
}

dmas_status_t dmas_beamform(dmas_plan_t plan, const void *d_x, float *d_y, float in_scale, void *stream)
{
    return run(plan, d_x, d_y, in_scale, stream, false);
}

dmas_status_t dmas_envelope(dmas_plan_t plan, const void *d_x, float *d_env, float in_scale, void *stream)
{
    return run(plan, d_x, d_env, in_scale, stream, true);
}

dmas_status_t dmas_envelope_noalloc(dmas_plan_t plan, const void *d_x, float *d_env, float in_scale,
                                    void *stream)
{
    return run(plan, d_x, d_env, in_scale, stream, true, true);
}

dmas_status_t dmas_matched_filter(dmas_plan_t p, const float *d_raw, float *d_x, void *stream)
{
    if (!p || !d_raw || !d_x) return fail(DMAS_ERR_INVALID_ARG, "plan or device pointer is NULL");
    if (!p->mf_len) return fail(DMAS_ERR_INVALID_ARG, "the plan has no matched-filter pulse");
    if (p->dtype != DMAS_F32) return fail(DMAS_ERR_UNSUPPORTED, "the matched filter writes FP32 channels");
    if (p->M > 65535) return fail(DMAS_ERR_UNSUPPORTED, "matched filter supports up to 65535 channels");
    if (d_raw == d_x) return fail(DMAS_ERR_INVALID_ARG, "the matched filter cannot run in place");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(DMAS_ERR_INVALID_ARG, "plan belongs to device %d but device %d is current", p->device, cur);
    hipError_t e = dmas::launch_matched_filter(d_raw, p->d_pulse, p->M, p->T, p->mf_len, d_x,
                                               static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "matched filter launch");
    return DMAS_OK;
}

dmas_status_t dmas_steering_delays(dmas_plan_t p, int32_t *d_whole, float *d_frac, void *stream)
{
    if (!p || !d_whole) return fail(DMAS_ERR_INVALID_ARG, "plan or d_whole is NULL");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(DMAS_ERR_INVALID_ARG, "plan belongs to device %d but device %d is current", p->device, cur);
    const int64_t n = (int64_t)p->M * p->D;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    if (blocks > INT32_MAX) return fail(DMAS_ERR_UNSUPPORTED, "delay table too large");
    auto kern = p->nearfield ? (p->linear ? delay_table_kernel<true, true> : delay_table_kernel<true, false>)
                             : (p->linear ? delay_table_kernel<false, true> : delay_table_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), 0, static_cast<hipStream_t>(stream), p->d_mic,
                       p->d_dirs, p->M, p->D, p->fs, p->c, d_whole, d_frac);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "delay table launch");
    return DMAS_OK;
}

dmas_status_t dmas_design_lowpass(int32_t L, double fc, double fs, float *taps)
{
    if (!taps) return fail(DMAS_ERR_INVALID_ARG, "taps is NULL");
    if (L < 1 || L > DMAS_MAX_FIR_LEN || (L % 2) == 0)
        return fail(DMAS_ERR_INVALID_ARG, "fir_len %d must be odd in 1..%d", L, DMAS_MAX_FIR_LEN);
    if (!(fs > 0.0) || !(fc > 0.0) || !(fc < 0.5 * fs))
        return fail(DMAS_ERR_INVALID_ARG, "need 0 < fc < fs/2");
    std::vector<double> h;
    design_lowpass(L, fc, fs, h);
    for (int k = 0; k < L; ++k) taps[k] = (float)h[k];
    return DMAS_OK;
}

const char *dmas_last_error(void)
{
    return g_last_error.c_str();
}

const char *dmas_version(void)
{
    return "dmas-mi355x 0.1 (gfx950)";
}

}  // extern "C"
