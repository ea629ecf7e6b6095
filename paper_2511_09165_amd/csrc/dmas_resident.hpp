// Internal: resident workers for the serving runtime. A worker is one
// persistent launch of a kernel class (order, CF, envelope, geometry, delay
// table mode) whose workgroups take work items from a queue of jobs that the
// host publishes in pinned memory while the launch runs, instead of one launch
// per batch of frames.
//
// Jobs: a frame whose plan stages roots publishes a roots job (chunks of its
// root plane) and then a pixels job (its (tile, segment) workgroups of the
// single-frame launch, computed by the same dmas_body); other frames publish
// the pixels job only. A pixels job names the roots job it needs; its items
// wait for that job on a device counter. Roots items wait for nothing, and
// every item is claimed in job order by a running workgroup, so such waits
// always end.
//
// Memory ordering: the host writes a job, then raises `published` (release);
// workgroups read job words and the count with system-scope loads, which
// bypass the caches; a job's input is read from coherent pinned memory. Device
// memory freed while a worker runs (root planes, outputs) is held back by the
// host and returned in epochs; a job carries the epoch of its memory, and a
// workgroup performs one system-scope acquire (dropping stale cache lines) when
// it first meets a job of a newer epoch than it has seen. Stale lines of a
// returned range can only predate its return, since no one reads a range while
// it is free; a launch starts with clean caches. After each item the
// workgroup's stores reach the L2; when the workgroup leaves a job, one
// system-scope release writes the L2 back before its items of that job are
// counted. The workgroup that completes a job stores its `done` flag with
// system-scope release, so the host can read the job's outputs once it sees
// the flag.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dmas_internal.hpp"

namespace dmas {

constexpr int kResidentJobs = 4096;           // jobs per queue generation
constexpr int kRootItem = 8 * kWaveSize * 16; // root-plane samples per roots item
enum : int32_t { kJobPixels = 0, kJobRoots = 1 };

struct ResidentJob {
    KernelParams kp;         // the frame's launch parameters (kp.roots: its plane)
    int32_t kind;            // kJobPixels or kJobRoots
    int32_t items;           // work items
    int32_t dep;             // roots job this pixels job needs, or -1
    int32_t dep_items;       // items of that roots job
    int32_t epoch;           // memory epoch of the job's device memory
    int32_t pad;
    int64_t count;           // roots: samples in the plane
};
constexpr int kJobWords = (int)(sizeof(ResidentJob) / 4);
static_assert(sizeof(ResidentJob) % 4 == 0, "job words");

// Pinned host memory, written by the host (jobs, published, stop) and by the
// device (done, error).
struct ResidentHost {
    int32_t published;                 // jobs [0, published) are complete in `jobs`
    int32_t stop;                      // exit once every published item is claimed
    int32_t error;                     // a dependency wait gave up (outputs unreliable)
    int32_t pad;
    int32_t done[kResidentJobs];       // 1 once every item of the job is complete
    ResidentJob jobs[kResidentJobs];
};

// Device memory, zeroed at the start of a queue generation.
struct ResidentDevice {
    int32_t cur_job;                   // first job that may have unclaimed items
    int32_t pub_mirror;                // largest published count read from host memory
    int32_t stop_mirror;               // 1 once a workgroup has read the stop request
    int32_t pad[61];
    int32_t claimed[kResidentJobs];    // items handed out per job (may exceed items)
    int32_t finished[kResidentJobs];   // items completed per job
};

struct ResidentArgs {
    ResidentHost *host;
    ResidentDevice *dev;
    int32_t idle_limit;                // empty polls before a workgroup exits
    int32_t dep_limit;                 // polls of a dependency before giving up
    int32_t epoch0;                    // memory epoch at launch
};

// Resident worker for one kernel class (nearest delays from tables, plain
// sums); hipErrorNotSupported for classes without a worker. With blocks !=
// nullptr nothing is launched and *blocks receives the resident workgroups per
// CU at `lds` bytes of dynamic LDS.
hipError_t launch_resident(int order, bool cf, bool env, bool nearfield, int delay, const ResidentArgs &a,
                           unsigned grid, size_t lds, hipStream_t stream, int *blocks = nullptr);
hipError_t launch_resident_order3(bool, bool, bool, int, const ResidentArgs &, unsigned, size_t, hipStream_t, int *);
hipError_t launch_resident_order5(bool, bool, bool, int, const ResidentArgs &, unsigned, size_t, hipStream_t, int *);

}  // namespace dmas
