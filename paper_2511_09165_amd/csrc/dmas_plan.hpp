// Internal: the plan object behind dmas_plan_t, and helpers shared by the
// host API (dmas_api.hip) and the serving runtime (dmas_server.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>

#include "dmas_internal.hpp"

namespace dmas {
// Source of plan serial numbers, in creation order.
inline std::atomic<uint64_t> &plan_serials()
{
    static std::atomic<uint64_t> next{1};
    return next;
}
}  // namespace dmas

struct dmas_plan_s {
    uint64_t serial = dmas::plan_serials().fetch_add(1);   // creation order
    int device = 0;
    int M = 0, T = 0, D = 0, order = 0;
    bool cf = true, nearfield = false, linear = false;
    bool roots = false;    // kernel reads a root plane (whole-sample delays, n >= 2)
    bool tables = false;   // per-tile delay tables (whole-sample delays, <= 2 GiB)
    bool block_tables = false;   // tables read a block of offsets at a time (kDelayTableBlocks)
    bool share_rings = false;    // with them, the envelope rings in the window region (...Shared)
    int compensated = 0;   // 0 FP32 sums, 1 Kahan FP32, 2 FP64
    int ng_fp64 = 0;
    int dtype = DMAS_F32;
    double fs = 0, c = 0;
    float cf_eps = 0;
    int fir_len = 0;
    int num_tiles = 0;
    int halo = 0;
    int mic_block = 0;
    int row = 0;
    int seg_rf = 0, seg_env = 0;
    int nseg_rf = 0, nseg_env = 0;
    size_t lds_rf = 0, lds_env = 0;
    int occ_rf = 0, occ_env = 0;
    double *d_mic = nullptr;
    double *d_dirs = nullptr;
    int32_t *d_tiles = nullptr;
    int32_t *d_tile_off = nullptr;    // per-tile delay tables (whole-sample delays), or null
    int32_t *d_tile_dref = nullptr;
    float *d_taps = nullptr;
    int env_decim = 1;
    int mf_len = 0;
    float *d_pulse = nullptr;
    size_t device_bytes = 0;   // all device memory the plan holds (geometry, taps, tiles, tables)
};

namespace dmas {

// Device bytes of a frame's root plane (zero when the plan does not use one).
inline size_t plane_bytes(const dmas_plan_s *plan)
{
    return plan->roots ? (size_t)plan->M * (size_t)plan->T * sizeof(float2) : 0;
}

// Fill the root plane of input d_x (plans with roots only).
inline hipError_t stage_roots(const dmas_plan_s *plan, const void *d_x, float2 *d_plane, hipStream_t stream)
{
    return launch_roots(plan->order, plan->dtype, d_x, d_plane, (size_t)plan->M * (size_t)plan->T, stream);
}

// Kernel arguments for one launch of `plan` on input d_x (and its root plane
// d_plane when the plan uses one) / output d_out.
inline KernelParams make_params(const dmas_plan_s *plan, const void *d_x, const float2 *d_plane, float *d_out,
                                float in_scale, bool env)
{
    KernelParams kp{};
    kp.x = d_x;
    kp.roots = d_plane;
    kp.out = d_out;
    kp.mic = plan->d_mic;
    kp.dirs = plan->d_dirs;
    kp.tile_dirs = plan->d_tiles;
    kp.tile_off = plan->d_tile_off;
    kp.tile_dref = plan->d_tile_dref;
    kp.taps = plan->d_taps;
    kp.M = plan->M;
    kp.T = plan->T;
    kp.D = plan->D;
    kp.order = plan->order;
    kp.fir_len = env ? plan->fir_len : 1;
    kp.num_tiles = plan->num_tiles;
    kp.seg_len = env ? plan->seg_env : plan->seg_rf;
    kp.halo = plan->halo;
    kp.row = plan->row;
    kp.mic_block = plan->mic_block;
    kp.dtype = plan->dtype;
    kp.ng_fp64 = plan->ng_fp64;
    kp.fs = plan->fs;
    kp.c = plan->c;
    kp.cf_eps = plan->cf_eps;
    kp.in_scale = in_scale;
    kp.env_decim = env ? plan->env_decim : 1;
    kp.out_T = env ? (plan->T + plan->env_decim - 1) / plan->env_decim : plan->T;
    return kp;
}

inline LaunchShape shape_of(const dmas_plan_s *p, bool env)
{
    LaunchShape ls{};
    ls.order = p->order;
    ls.cf = p->cf;
    ls.env = env;
    ls.nearfield = p->nearfield;
    ls.delay = p->linear ? kDelayLinear
               : !p->tables ? kDelayComputed
               : !p->block_tables ? kDelayTable
               : p->share_rings   ? kDelayTableBlocksShared
                                  : kDelayTableBlocks;
    ls.accumulate = p->compensated;
    ls.grid = (unsigned)((int64_t)p->num_tiles * (env ? p->nseg_env : p->nseg_rf));
    ls.lds_bytes = env ? p->lds_env : p->lds_rf;
    return ls;
}

// Workgroups of one launch of the plan.
inline int64_t plan_workgroups(const dmas_plan_s *p, bool env)
{
    return (int64_t)p->num_tiles * (env ? p->nseg_env : p->nseg_rf);
}

// Record the calling thread's last error message (returned by dmas_last_error).
void set_last_error(const char *msg);

// Launch one plan (order dispatch); with kp == nullptr, report occupancy in *blocks.
hipError_t launch_plan(int order, const KernelParams *kp, const LaunchShape &ls, hipStream_t st,
                       int *blocks = nullptr);

}  // namespace dmas
