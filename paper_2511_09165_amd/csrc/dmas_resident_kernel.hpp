// Resident worker kernel (device code), one instantiation per kernel class;
// included by the per-order units dmas_resident<n>.hip. Queue layout and
// memory ordering are described in dmas_resident.hpp.
#pragma once

#include <cstring>

#include "dmas_kernel.hpp"
#include "dmas_resident.hpp"

namespace dmas {

constexpr int32_t kClaimIdle = -1;   // nothing to claim now
constexpr int32_t kClaimExit = -2;   // nothing to claim and the host asked the workers to stop
constexpr int kClaimTries = 64;      // jobs passed over per claim before reporting idle
constexpr int kHostPollEvery = 16;   // idle polls of the device mirrors per read of host memory

template <typename T>
__device__ __forceinline__ T load_relaxed_sys(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Thread 0 of a workgroup: the next (job, item), or (kClaimIdle | kClaimExit, 0).
// pub_seen caches the last published count this workgroup knows of; jobs below
// it are complete in host memory. Items are handed out in job order: a job's
// counter is raised until it passes the job's item count, then cur_job moves on.
// The published count and the stop request are read from host memory only on
// every kHostPollEvery-th idle poll of a workgroup (poll_host) and are mirrored
// in device memory for the others. No poll is an acquire (memory epochs order
// the jobs' device memory).
__device__ __forceinline__ int2 claim_item(const ResidentArgs &a, int &pub_seen, int &c_job, int &c_items,
                                           bool poll_host)
{
    ResidentDevice *dv = a.dev;
    int j = __hip_atomic_load(&dv->cur_job, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int tries = 0; tries < kClaimTries; ++tries) {
        if (j >= pub_seen) {
            pub_seen = max(pub_seen, __hip_atomic_load(&dv->pub_mirror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (j >= pub_seen) {
                int stop = __hip_atomic_load(&dv->stop_mirror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (poll_host || stop) {
                    stop |= load_relaxed_sys(&a.host->stop);
                    // a stop seen first orders the count after it: the count is final
                    if (stop) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                    const int pub = load_relaxed_sys(&a.host->published);
                    __hip_atomic_fetch_max(&dv->pub_mirror, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (stop) __hip_atomic_store(&dv->stop_mirror, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    pub_seen = max(pub_seen, pub);
                }
                if (j >= pub_seen) return make_int2(stop ? kClaimExit : kClaimIdle, 0);
            }
        }
        if (j != c_job) {
            c_job = j;
            c_items = load_relaxed_sys(&a.host->jobs[j].items);
        }
        const int i = __hip_atomic_fetch_add(&dv->claimed[j], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (i < c_items) return make_int2(j, i);
        int expected = j;
        __hip_atomic_compare_exchange_strong(&dv->cur_job, &expected, j + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        j = expected == j ? j + 1 : expected;   // cur_job only grows: expected > j on failure
    }
    return make_int2(kClaimIdle, 0);
}

// Root-plane chunk [item * kRootItem, ...) of a frame whose input x is in host
// memory: every thread issues its kRootLoads loads before it stores, so the
// host-memory latency is paid once per item.
constexpr int kRootLoads = kRootItem / (kDirsPerTile * kWaveSize);

template <int N>
__device__ __forceinline__ void roots_item(const ResidentJob &jd, int item)
{
    float2 *plane = const_cast<float2 *>(jd.kp.roots);
    const int64_t e0 = (int64_t)item * kRootItem + threadIdx.x;
    float v[kRootLoads];
#pragma unroll
    for (int k = 0; k < kRootLoads; ++k) {
        const int64_t e = e0 + (int64_t)k * (kDirsPerTile * kWaveSize);
        v[k] = e >= jd.count       ? 0.0f
               : jd.kp.dtype == 0 ? load_sample<0>(jd.kp.x, (size_t)e)
               : jd.kp.dtype == 1 ? load_sample<1>(jd.kp.x, (size_t)e)
                                  : load_sample<2>(jd.kp.x, (size_t)e);
    }
#pragma unroll
    for (int k = 0; k < kRootLoads; ++k) {
        const int64_t e = e0 + (int64_t)k * (kDirsPerTile * kWaveSize);
        if (e < jd.count) plane[e] = make_float2(signed_root<N, true>(v[k]), v[k]);
    }
}

template <int N, bool CF, bool ENV, bool NEAR, int DM>
__global__ void __launch_bounds__(kDirsPerTile * kWaveSize, (kMinWavesPerSimd<N, kAccF32, DM, NEAR>))
dmas_resident_kernel(const ResidentArgs a)
{
    extern __shared__ float smem[];
    __shared__ int32_t s_cmd[2];
    __shared__ uint32_t s_job[kJobWords];
    const int tid = threadIdx.x;
    int pub_seen = 0, c_job = -1, c_items = 0;   // thread 0 only
    int have = -1;          // job whose descriptor is in s_job (the same in every thread)
    int dep_ready = -1;     // roots job known complete by this workgroup
    int seen_epoch = a.epoch0;
    int idle = 0;
    // items of one job completed here and not yet counted (the same in every thread)
    int cnt_job = -1, cnt_n = 0, cnt_items = 0;
    // Count them: their stores have reached the L2 (each item waits for its own),
    // one system-scope release writes the L2 back ahead of the count, and the
    // workgroup that completes the job raises its done flag.
    auto flush_count = [&]() {
        if (cnt_n == 0) return;
        if (tid == 0) {
            const int prev =
                __hip_atomic_fetch_add(&a.dev->finished[cnt_job], cnt_n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            if (prev + cnt_n == cnt_items)
                __hip_atomic_store(&a.host->done[cnt_job], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        cnt_n = 0;
    };
    for (;;) {
        if (tid == 0) {
            const int2 c = claim_item(a, pub_seen, c_job, c_items, idle % kHostPollEvery == 0);
            s_cmd[0] = c.x;
            s_cmd[1] = c.y;
        }
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_cmd[0]);
        const int item = __builtin_amdgcn_readfirstlane(s_cmd[1]);
        __syncthreads();   // every thread has read s_cmd before thread 0 writes it again
        // a workgroup moving on from a job (or going idle) counts what it did there
        // first, so no wait on a job's completion can depend on an uncounted item
        if (job != cnt_job) flush_count();
        if (job == kClaimExit) break;
        if (job == kClaimIdle) {
            if (++idle > a.idle_limit) break;
            __builtin_amdgcn_s_sleep(127);
            continue;
        }
        idle = 0;
        if (job != have) {
            // first item of this job here: read its descriptor
            const int32_t *src = reinterpret_cast<const int32_t *>(&a.host->jobs[job]);
            for (int w = tid; w < kJobWords; w += blockDim.x)
                s_job[w] = (uint32_t)__hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __syncthreads();
            have = job;
        }
        uint32_t words[kJobWords];
#pragma unroll
        for (int w = 0; w < kJobWords; ++w) words[w] = __builtin_amdgcn_readfirstlane(s_job[w]);
        ResidentJob jd;
        __builtin_memcpy(&jd, words, sizeof jd);
        if (jd.epoch > seen_epoch) {
            // the job's device memory was returned after this workgroup last dropped its caches
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            seen_epoch = jd.epoch;
        }
        if (jd.kind == kJobRoots) {
            roots_item<N>(jd, item);
        } else {
            if (jd.dep >= 0 && jd.dep != dep_ready) {
                if (tid == 0) {
                    int k = 0;
                    while (__hip_atomic_load(&a.dev->finished[jd.dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                           jd.dep_items) {
                        if (++k > a.dep_limit) {
                            __hip_atomic_store(&a.host->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
                __syncthreads();
                dep_ready = jd.dep;
            }
            // the thread index through an empty asm: per-lane values of the body are
            // then computed per item instead of held across the loop (96 -> 79 VGPRs)
            int tx = tid;
            asm volatile("" : "+v"(tx));
            dmas_body<N, CF, ENV, NEAR, DM, kAccF32>(jd.kp, item % jd.kp.num_tiles, item / jd.kp.num_tiles, smem, tx);
        }
        // every wave waits for this item's stores to reach the L2; the item is
        // counted when the workgroup leaves the job
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __syncthreads();
        cnt_job = job;
        cnt_items = jd.items;
        ++cnt_n;
    }
}

template <int N, bool CF, bool ENV, bool NEAR, int DM>
hipError_t resident_one(const ResidentArgs &a, unsigned grid, size_t lds, hipStream_t stream, int *blocks)
{
    auto fn = dmas_resident_kernel<N, CF, ENV, NEAR, DM>;
    if (blocks)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, reinterpret_cast<const void *>(fn),
                                                            kDirsPerTile * kWaveSize, lds);
    static std::atomic<size_t> allowed{64 * 1024};
    hipError_t e = raise_lds_limit(reinterpret_cast<const void *>(fn), lds, allowed);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kDirsPerTile * kWaveSize), lds, stream, a);
    return hipGetLastError();
}

// Classes with a worker: CF or not, envelope or not, either geometry; delays
// from the per-tile tables (either table mode).
template <int N>
hipError_t launch_resident_order(bool cf, bool env, bool nearfield, int delay, const ResidentArgs &a, unsigned grid,
                                 size_t lds, hipStream_t stream, int *blocks)
{
#define DMAS_RES(CF, ENV, NEAR, DM)                                                   \
    if (cf == CF && env == ENV && nearfield == NEAR && delay == DM)                   \
        return resident_one<N, CF, ENV, NEAR, DM>(a, grid, lds, stream, blocks);
#define DMAS_RES_DM(DM)                                                                \
    DMAS_RES(true, true, false, DM) DMAS_RES(true, false, false, DM)                  \
    DMAS_RES(true, true, true, DM) DMAS_RES(true, false, true, DM)                    \
    DMAS_RES(false, true, false, DM) DMAS_RES(false, false, false, DM)                \
    DMAS_RES(false, true, true, DM) DMAS_RES(false, false, true, DM)
    DMAS_RES_DM(kDelayTable)
    DMAS_RES_DM(kDelayTableBlocks)
    DMAS_RES_DM(kDelayTableBlocksShared)
#undef DMAS_RES_DM
#undef DMAS_RES
    return hipErrorNotSupported;
}

}  // namespace dmas
