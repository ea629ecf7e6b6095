// Serving runtime behind the dmas_server_* entry points of include/dmas.h:
// admission by an HBM budget, pinned staging, asynchronous input copies and
// continuous batching of heterogeneous frames into multi-frame launches on
// several streams. Host C++ only; the device work is dmas_batch_kernel /
// dmas_kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dmas.h"
#include "dmas_internal.hpp"
#include "dmas_plan.hpp"
#include "dmas_resident.hpp"
#include "dmas_sched.hpp"

namespace {

constexpr int kMaxBatchFrames = 1024;

using dmas::sched::Arena;
using dmas::sched::align_up;
using dmas::sched::kAlign;

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Deadline `timeout` seconds from now on the steady clock. Waits are capped at
// kMaxWait seconds (infinity included) so the deadline stays representable.
constexpr double kMaxWait = 1.0e9;
std::chrono::steady_clock::time_point deadline_after(double timeout)
{
    using namespace std::chrono;
    const double t = std::min(timeout, kMaxWait);
    return steady_clock::now() + duration_cast<steady_clock::duration>(duration<double>(t));
}

enum FrameState { kQueued = 0, kAdmitted = 1, kLaunched = 2, kDone = 3, kFailed = -1 };

struct Frame {
    uint64_t ticket = 0;
    dmas_plan_s *plan = nullptr;
    float in_scale = 1.0f;
    bool env = false, auto_release = false;
    size_t in_bytes = 0, out_bytes = 0;
    size_t stage_off = 0;
    bool staged = false;
    size_t in_off = 0, out_off = 0;
    size_t in_dev_bytes = 0;                 // device copy of the input (none for resident frames)
    size_t plane_bytes = 0, plane_off = 0;   // root plane (plans that stage roots)
    bool on_device = false;
    bool resident = false;   // served by a resident worker
    int res_roots_job = -1, res_roots_items = 0;   // its roots job in the worker's queue
    hipEvent_t copied = nullptr;
    int state = kQueued;
    int batch_frames = 0;
    double t_arrival = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

struct Launch {
    std::vector<Frame *> frames;
    hipEvent_t done = nullptr;
    bool busy = false;
    double t_launch = 0;      // issue time
    double t_start = 0;       // when it had the device to itself (previous launch done, or issue)
    double work = 0;          // modelled VALU work (lane-op slots)
    int64_t workgroups = 0;
    double tail_start = 0;    // predicted start of its last device round
};

// Modelled VALU issue slots of one frame (per-microphone power sums,
// Newton-Girard, CF and envelope per pixel; roots are taken once per channel
// sample); used only to predict durations.
double frame_work(const dmas_plan_s *p, bool env)
{
    const double per_mic = p->order == 1 ? 2.0 : p->roots ? 3.0 + p->order : 8.0 + p->order;
    return (double)p->D * p->T * (p->M * per_mic + 30.0 + (env ? p->fir_len : 0));
}

size_t elem_size(int dtype)
{
    return dtype == DMAS_F32 ? 4 : 2;
}

// Frames that the multi-frame kernel serves (nearest delays, plain sums).
bool batchable(const dmas_plan_s *p)
{
    return !p->linear && !p->compensated;
}

// Kernel class of a frame: frames of one class can share a multi-frame
// launch (same kernel instantiation).
int64_t kernel_class(const Frame *f)
{
    return (int64_t)f->env | (int64_t)f->plan->cf << 1 | (int64_t)f->plan->nearfield << 2 |
           (int64_t)dmas::shape_of(f->plan, f->env).delay << 3 | (int64_t)f->plan->order << 8;
}

dmas_status_t srv_fail(dmas_status_t st, const char *msg)
{
    dmas::set_last_error(msg);
    return st;
}

// Resident workers: polls (about 3.4 us each at 2.4 GHz) before an idle
// workgroup exits; polls (about 0.2 us each) of a root plane before a
// workgroup gives up on it; how long a worker takes new jobs; how long a frame
// of another class waits before the worker is asked to exit.
constexpr int32_t kResidentIdlePolls = 2000;
constexpr int32_t kResidentDepPolls = 1 << 22;
constexpr double kResidentLife = 0.100;
constexpr double kResidentSwitchWait = 0.001;   // DMAS_RESIDENT_SWITCH_US overrides
constexpr double kEpochMin = 0.002;             // shortest memory epoch

// Frames that a resident worker serves: nearest delays from the per-tile
// tables, plain sums, orders 3 and 5.
bool resident_capable(const dmas_plan_s *p, bool env)
{
    if (!batchable(p) || (p->order != 3 && p->order != 5)) return false;
    const int dm = dmas::shape_of(p, env).delay;
    return dm == dmas::kDelayTable || dmas::block_tables(dm);
}

}  // namespace

hipError_t dmas::launch_resident(int order, bool cf, bool env, bool nearfield, int delay, const ResidentArgs &a,
                                 unsigned grid, size_t lds, hipStream_t stream, int *blocks)
{
    switch (order) {
    case 3: return launch_resident_order3(cf, env, nearfield, delay, a, grid, lds, stream, blocks);
    case 5: return launch_resident_order5(cf, env, nearfield, delay, a, grid, lds, stream, blocks);
    default: return hipErrorNotSupported;
    }
}

struct dmas_server_s {
    int device = 0;
    size_t budget = 0, staging = 0;
    int nstreams = 2, max_batch = 64;
    int64_t batch_wg_cap = 0;   // workgroups per multi-frame launch (about two device rounds)
    int64_t resident_wgs = 0;   // workgroups the device holds at once (typical occupancy)
    int64_t small_wg_cap = 0;   // groups this small may start while the gate is closed (four device rounds)
    double rate = 3.0e13;       // learned work rate (modelled slots per second)
    double rate_cap = 3.6e13;   // about 92% of the VALU issue peak of the device
    char *d_arena = nullptr;
    char *h_staging = nullptr;
    const char *d_staging = nullptr;   // device view of h_staging (resident mode)
    Arena arena, stage_arena;
    size_t hbm_peak = 0;
    hipStream_t copy_stream = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<Launch> launches;
    std::vector<char *> d_tables, h_tables;
    size_t table_bytes = 0;
    std::vector<hipEvent_t> event_pool;

    std::deque<Frame *> queued, admitted;
    // Plans with frames holding device memory: the plan's own device memory is
    // counted in the budget (an arena range) while any of its frames is.
    struct PlanUse {
        size_t off, bytes;
        int frames;
    };
    std::unordered_map<uint64_t, PlanUse> plan_use;   // by plan serial
    std::unordered_map<uint64_t, Frame *> frames;
    std::deque<dmas_frame_info_t> finished;   // records of auto-released frames
    uint64_t next_ticket = 1;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_launches = 0, n_batched = 0;

    // ---- resident workers (one at a time, one kernel class each) ----
    bool res_on = false;
    dmas::ResidentHost *res_h = nullptr;    // pinned job queue, host view
    dmas::ResidentHost *res_hd = nullptr;   // the same memory, device view
    dmas::ResidentDevice *res_d = nullptr;
    hipStream_t res_stream = nullptr;
    hipEvent_t res_end = nullptr;
    bool res_running = false, res_stopping = false;
    int res_order = 0, res_delay = 0;
    bool res_cf = false, res_env = false, res_near = false;
    size_t res_lds = 0;
    uint64_t res_serial = 0;                // the worker serves plans with smaller serials
    double res_t_launch = 0;
    int res_published = 0, res_checked = 0; // jobs written / jobs seen done
    std::vector<Frame *> res_job_frame;     // per job: its frame for a pixels job, else null
    std::deque<Frame *> res_admitted;       // admitted frames for the resident workers
    std::vector<std::pair<size_t, size_t>> res_held;   // arena ranges freed while the worker runs
    int64_t res_queued_items = 0;           // pixels items published and not yet done
    int drain_waiters = 0;                  // threads inside dmas_server_drain
    int32_t res_epoch = 0;                  // memory epoch (see release_held)
    double res_t_epoch = 0;
    double res_switch_wait = kResidentSwitchWait;
    int64_t res_items_cap = 0;              // bound on res_queued_items (about sixteen device rounds)
    int res_cus = 256;
    int64_t n_res_launches = 0, n_res_frames = 0;

    std::mutex mu;
    std::condition_variable cv_done;     // frame completions, for waiters
    std::condition_variable cv_work;     // new submissions, for the scheduler
    std::thread worker;
    std::atomic<bool> stop{false};
    std::string worker_error;

    hipEvent_t get_event()
    {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    void fill_info(const Frame *f, dmas_frame_info_t *info) const
    {
        info->ticket = f->ticket;
        info->state = f->state;
        info->batch_frames = f->batch_frames;
        info->t_arrival = f->t_arrival;
        info->t_admit = f->t_admit;
        info->t_launch = f->t_launch;
        info->t_done = f->t_done;
        info->d_out = (f->on_device && f->state == kDone) ? reinterpret_cast<float *>(d_arena + f->out_off) : nullptr;
        info->pixels = (int64_t)f->plan->D * f->plan->T;   // beamformed pixels (before decimation)
    }

    float2 *plane_of(const Frame *f) const
    {
        return f->plane_bytes ? reinterpret_cast<float2 *>(d_arena + f->plane_off) : nullptr;
    }

    // Return a frame's device memory. While a resident worker runs, the ranges
    // are held back and returned in epochs (release_held): the worker drops its
    // caches once per epoch, not per job.
    void free_device(Frame *f)
    {
        if (!f->on_device) return;
        if (f->in_dev_bytes) arena_free(f->in_off, f->in_dev_bytes);
        arena_free(f->out_off, f->out_bytes);
        if (f->plane_bytes) arena_free(f->plane_off, f->plane_bytes);
        auto pu = plan_use.find(f->plan->serial);
        if (pu != plan_use.end() && --pu->second.frames == 0) {
            if (pu->second.bytes) arena_free(pu->second.off, pu->second.bytes);
            plan_use.erase(pu);
        }
        f->on_device = false;
    }

    void arena_free(size_t off, size_t bytes)
    {
        if (res_running) res_held.emplace_back(off, bytes);
        else arena.release(off, bytes);
    }

    void release_held()
    {
        if (res_held.empty()) return;
        for (auto &r : res_held) arena.release(r.first, r.second);
        res_held.clear();
        ++res_epoch;   // jobs published from now on may use the returned memory
        res_t_epoch = now_s();
    }

    void free_staging(Frame *f)
    {
        if (!f->staged) return;
        stage_arena.release(f->stage_off, f->in_bytes);
        f->staged = false;
    }

    // A frame that failed before its launch completed (input copy or launch
    // call): memory and event returned, and an auto-released frame reported
    // through the completed records, as a frame whose launch failed on the
    // device is. The caller has made the frame's streams idle.
    void fail_unlaunched(Frame *f)
    {
        f->state = kFailed;
        f->t_done = now_s();
        ++n_failed;
        free_staging(f);
        free_device(f);
        if (f->copied) event_pool.push_back(f->copied), f->copied = nullptr;
        if (f->auto_release) {
            dmas_frame_info_t info;
            fill_info(f, &info);
            finished.push_back(info);
            frames.erase(f->ticket);
            delete f;
        }
    }

    // ---- scheduler steps (called with mu held) ----
    bool collect_completions()
    {
        bool progress = false;
        for (auto &l : launches) {
            if (!l.busy) continue;
            hipError_t q = hipEventQuery(l.done);
            if (q == hipErrorNotReady) continue;
            const double t = now_s();
            for (Frame *f : l.frames) {
                f->t_done = t;
                f->state = (q == hipSuccess) ? kDone : kFailed;
                free_staging(f);
                if (f->copied) event_pool.push_back(f->copied), f->copied = nullptr;
                if (q == hipSuccess) ++n_completed; else ++n_failed;
                if (f->auto_release || q != hipSuccess) {
                    free_device(f);
                    if (f->auto_release) {
                        dmas_frame_info_t info;
                        fill_info(f, &info);
                        finished.push_back(info);
                        frames.erase(f->ticket);
                        delete f;
                    }
                }
            }
            if (q != hipSuccess) worker_error = hipGetErrorString(q);
            if (q == hipSuccess && t > l.t_start && l.work > 0) {
                // the modelled work cannot run faster than the device's issue rate
                const double measured = std::min(std::max(l.work / (t - l.t_start), 0.25 * rate_cap), rate_cap);
                rate = 0.8 * rate + 0.2 * measured;
            }
            for (auto &other : launches)
                if (other.busy && &other != &l) other.t_start = std::max(other.t_start, t);
            l.frames.clear();
            l.busy = false;
            progress = true;
        }
        if (progress) cv_done.notify_all();
        return progress;
    }

    bool admit()
    {
        bool progress = false;
        while (!queued.empty()) {
            Frame *f = queued.front();
            // A resident worker reads the input from the pinned staging memory (in its
            // roots job), so a resident frame takes device memory for its root plane
            // and output only, and needs no copy.
            const bool resident = res_on && resident_capable(f->plan, f->env);
            const size_t in_dev = resident ? 0 : f->in_bytes;
            // arrival order: the first frame that does not fit stops admission; a
            // frame whose plan has no other frame holding device memory also
            // reserves the plan's device memory
            auto pu = plan_use.find(f->plan->serial);
            const bool new_plan = pu == plan_use.end();
            dmas::sched::Grant g;
            if (!dmas::sched::grant(arena, in_dev, f->out_bytes, f->plane_bytes,
                                    new_plan ? f->plan->device_bytes : 0, &g))
                break;
            if (new_plan) pu = plan_use.emplace(f->plan->serial, PlanUse{g.plan_off, f->plan->device_bytes, 0}).first;
            ++pu->second.frames;
            f->resident = resident;
            f->in_dev_bytes = in_dev;
            f->in_off = g.in_off;
            f->out_off = g.out_off;
            f->plane_off = g.plane_off;
            f->on_device = true;
            hbm_peak = std::max(hbm_peak, arena.used());
            f->t_admit = now_s();
            queued.pop_front();
            if (resident) {
                f->state = kAdmitted;
                res_admitted.push_back(f);
                progress = true;
                continue;
            }
            f->copied = get_event();
            // input copy, then the root plane, on the copy stream
            hipError_t e = hipMemcpyAsync(d_arena + f->in_off, h_staging + f->stage_off, f->in_bytes,
                                          hipMemcpyHostToDevice, copy_stream);
            if (e == hipSuccess && f->plane_bytes) e = dmas::stage_roots(f->plan, d_arena + f->in_off, plane_of(f), copy_stream);
            if (e == hipSuccess && f->copied) e = hipEventRecord(f->copied, copy_stream);
            if (e != hipSuccess || !f->copied) {
                (void)hipStreamSynchronize(copy_stream);   // done with the staging and arena ranges
                fail_unlaunched(f);
                worker_error = "input copy failed";
                cv_done.notify_all();
            } else {
                f->state = kAdmitted;
                admitted.push_back(f);
            }
            progress = true;
        }
        return progress;
    }

    bool launch()
    {
        bool progress = false;
        while (!admitted.empty()) {
            // A new launch may overlap running ones only in their predicted last
            // device round (overlapping their main body would only slow them
            // down), except a group of at most small_wg_cap workgroups: it starts
            // on an idle stream at once, so a shorter frame does not wait for a
            // long frame's main body. Frames that fill the device by themselves go
            // alone; smaller frames of the same kernel class are packed, in arrival
            // order, up to about two device rounds of workgroups.
            std::vector<dmas::sched::StreamState> ss(nstreams);
            for (int i = 0; i < nstreams; ++i) ss[i] = {launches[i].busy, launches[i].tail_start};
            std::vector<dmas::sched::Candidate> cand;
            cand.reserve(admitted.size());
            for (Frame *f : admitted)
                cand.push_back({kernel_class(f), batchable(f->plan), dmas::plan_workgroups(f->plan, f->env)});
            const dmas::sched::LaunchPick lp =
                dmas::sched::pick_launch(ss, now_s(), cand, max_batch, batch_wg_cap, small_wg_cap);
            if (lp.stream < 0) break;
            const int s = lp.stream;
            const std::vector<size_t> &pick = lp.frames;
            Launch &l = launches[s];
            hipStream_t st = streams[s];
            std::vector<Frame *> group;
            for (size_t k = pick.size(); k-- > 0;) {   // erase from the back so indices stay valid
                group.insert(group.begin(), admitted[pick[k]]);
                admitted.erase(admitted.begin() + (std::ptrdiff_t)pick[k]);
            }
            Frame *head = group.front();
            hipError_t e = hipSuccess;
            for (Frame *f : group)
                if (e == hipSuccess) e = hipStreamWaitEvent(st, f->copied, 0);
            if (e == hipSuccess) {
                if (group.size() == 1) {
                    Frame *f = group[0];
                    const dmas::KernelParams kp = dmas::make_params(
                        f->plan, d_arena + f->in_off, plane_of(f), reinterpret_cast<float *>(d_arena + f->out_off),
                        f->in_scale, f->env);
                    e = dmas::launch_plan(f->plan->order, &kp, dmas::shape_of(f->plan, f->env), st);
                } else {
                    // Table layout: nf KernelParams, then nf int32 first-workgroup indices.
                    const int nf = (int)group.size();
                    auto *kp = reinterpret_cast<dmas::KernelParams *>(h_tables[s]);
                    auto *starts = reinterpret_cast<int32_t *>(h_tables[s] + sizeof(dmas::KernelParams) * nf);
                    int64_t total = 0;
                    size_t lds = 0;
                    for (int i = 0; i < nf; ++i) {
                        Frame *f = group[i];
                        kp[i] = dmas::make_params(f->plan, d_arena + f->in_off, plane_of(f),
                                                  reinterpret_cast<float *>(d_arena + f->out_off), f->in_scale, f->env);
                        starts[i] = (int32_t)total;
                        total += dmas::plan_workgroups(f->plan, f->env);
                        lds = std::max(lds, f->env ? f->plan->lds_env : f->plan->lds_rf);
                    }
                    if (total > INT32_MAX) {
                        e = hipErrorInvalidValue;
                    } else {
                        const size_t used = (sizeof(dmas::KernelParams) + sizeof(int32_t)) * nf;
                        e = hipMemcpyAsync(d_tables[s], h_tables[s], used, hipMemcpyHostToDevice, st);
                        if (e == hipSuccess) {
                            dmas::BatchParams bp;
                            bp.frames = reinterpret_cast<const dmas::KernelParams *>(d_tables[s]);
                            bp.starts = reinterpret_cast<const int32_t *>(d_tables[s] + sizeof(dmas::KernelParams) * nf);
                            bp.num_frames = nf;
                            e = dmas::launch_batch(head->plan->order, bp, head->plan->cf, head->env,
                                                   head->plan->nearfield, dmas::shape_of(head->plan, head->env).delay,
                                                   (unsigned)total, lds, st);
                        }
                    }
                }
            }
            if (e == hipSuccess) e = hipEventRecord(l.done, st);
            const double t = now_s();
            {
                double work = 0;
                int64_t wgs = 0;
                for (Frame *f : group) {
                    work += frame_work(f->plan, f->env);
                    wgs += dmas::plan_workgroups(f->plan, f->env);
                }
                bool alone = true;
                for (auto &other : launches)
                    if (other.busy) alone = false;
                const double dur = work / rate;
                l.t_launch = t;
                l.t_start = t;
                if (!alone) {
                    // starts on the leftover CUs of the running launches
                    for (auto &other : launches)
                        if (other.busy) l.t_start = std::max(l.t_start, other.t_start + other.work / rate);
                }
                l.work = work;
                l.workgroups = wgs;
                const double body = wgs > resident_wgs ? 1.0 - (double)resident_wgs / (double)wgs : 0.0;
                // a small group started beside a running launch does not hold the gate
                l.tail_start = lp.small ? t : l.t_start + dur * body;
            }
            ++n_launches;
            if (group.size() > 1) n_batched += (int64_t)group.size();
            for (Frame *f : group) {
                f->t_launch = t;
                f->batch_frames = (int)group.size();
                f->state = kLaunched;
            }
            l.frames = group;
            l.busy = true;
            if (e != hipSuccess) {
                // The launch did not happen: fail its frames now (their event may never fire).
                worker_error = hipGetErrorString(e);
                (void)hipStreamSynchronize(st);
                for (Frame *f : group) fail_unlaunched(f);
                l.frames.clear();
                l.busy = false;
                cv_done.notify_all();
            }
            progress = true;
        }
        return progress;
    }

    // ---- resident workers (called with mu held) ----
    // A frame whose pixels job is done.
    void res_finish(Frame *f)
    {
        res_queued_items -= dmas::plan_workgroups(f->plan, f->env);
        const bool ok = __atomic_load_n(&res_h->error, __ATOMIC_ACQUIRE) == 0;
        f->t_done = now_s();
        f->state = ok ? kDone : kFailed;
        free_staging(f);
        if (f->copied) event_pool.push_back(f->copied), f->copied = nullptr;
        if (ok) ++n_completed; else ++n_failed;
        if (!ok) worker_error = "a resident worker gave up waiting for a root plane";
        if (f->auto_release || !ok) {
            free_device(f);
            if (f->auto_release) {
                dmas_frame_info_t info;
                fill_info(f, &info);
                finished.push_back(info);
                frames.erase(f->ticket);
                delete f;
            }
        }
    }

    // Fail the frames of every job not seen done and empty the queue (after a
    // worker launch failed or a worker ended with an error; the worker stream is idle).
    void res_fail_outstanding(const char *why)
    {
        worker_error = why;
        for (int j = res_checked; j < res_published; ++j)
            if (Frame *f = res_job_frame[j]) fail_unlaunched(f);
        res_checked = res_published;
        res_queued_items = 0;
    }

    // Launch a worker for the current class; reset starts a new queue
    // generation (every published job done), else the worker continues the
    // queue as it stands.
    bool res_launch(bool reset)
    {
        hipError_t e = hipSuccess;
        if (reset) {
            e = hipMemsetAsync(res_d, 0, sizeof(dmas::ResidentDevice), res_stream);
            std::memset(res_h->done, 0, sizeof(int32_t) * (size_t)res_published);
            __atomic_store_n(&res_h->error, 0, __ATOMIC_RELAXED);
            __atomic_store_n(&res_h->published, 0, __ATOMIC_RELEASE);
            res_published = res_checked = 0;
            res_job_frame.clear();
        }
        __atomic_store_n(&res_h->stop, 0, __ATOMIC_RELEASE);
        if (!reset && e == hipSuccess)
            e = hipMemsetAsync(&res_d->stop_mirror, 0, sizeof(int32_t), res_stream);
        res_serial = dmas::plan_serials().load();
        const dmas::ResidentArgs a{res_hd, res_d, kResidentIdlePolls, kResidentDepPolls, res_epoch};
        int blocks = 0;
        if (e == hipSuccess)
            e = dmas::launch_resident(res_order, res_cf, res_env, res_near, res_delay, a, 0, res_lds, res_stream, &blocks);
        if (e == hipSuccess && blocks < 1) e = hipErrorInvalidConfiguration;
        res_items_cap = (int64_t)16 * blocks * res_cus;
        if (e == hipSuccess)
            e = dmas::launch_resident(res_order, res_cf, res_env, res_near, res_delay, a, (unsigned)(blocks * res_cus),
                                      res_lds, res_stream, nullptr);
        if (e == hipSuccess) e = hipEventRecord(res_end, res_stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(res_stream);
            res_fail_outstanding(hipGetErrorString(e));
            return false;
        }
        res_running = true;
        res_stopping = false;
        res_t_launch = now_s();
        ++n_res_launches;
        return true;
    }

    // Write and publish a frame's roots job (frames with a root plane); its
    // pixels job follows in res_publish_pixels, after the next frame's roots job
    // when several frames are published together, so that a root plane is being
    // filled while the previous frame's pixels run.
    void res_publish_roots(Frame *f)
    {
        f->res_roots_job = -1;
        f->res_roots_items = 0;
        f->state = kLaunched;
        f->t_launch = now_s();
        f->batch_frames = 1;
        ++n_res_frames;
        if (!f->plane_bytes) return;
        dmas::ResidentJob &r = res_h->jobs[res_published];
        r.kp = res_params(f);
        r.kind = dmas::kJobRoots;
        r.count = (int64_t)f->plan->M * f->plan->T;
        r.items = (int32_t)((r.count + dmas::kRootItem - 1) / dmas::kRootItem);
        r.dep = -1;
        r.dep_items = 0;
        r.epoch = res_epoch;
        r.pad = 0;
        f->res_roots_job = res_published;
        f->res_roots_items = r.items;
        res_job_frame.push_back(nullptr);
        ++res_published;
        __atomic_store_n(&res_h->published, res_published, __ATOMIC_RELEASE);
    }

    void res_publish_pixels(Frame *f)
    {
        dmas::ResidentJob &j = res_h->jobs[res_published];
        j.kp = res_params(f);
        j.kind = dmas::kJobPixels;
        j.count = 0;
        j.items = (int32_t)dmas::plan_workgroups(f->plan, f->env);
        j.dep = f->res_roots_job;
        j.dep_items = f->res_roots_items;
        j.epoch = res_epoch;
        j.pad = 0;
        res_job_frame.push_back(f);
        ++res_published;
        res_queued_items += j.items;
        __atomic_store_n(&res_h->published, res_published, __ATOMIC_RELEASE);
    }

    dmas::KernelParams res_params(const Frame *f) const
    {
        return dmas::make_params(f->plan, d_staging + f->stage_off, plane_of(f),
                                 reinterpret_cast<float *>(d_arena + f->out_off), f->in_scale, f->env);
    }

    bool res_same_class(const Frame *f) const
    {
        return f->plan->order == res_order && f->plan->cf == res_cf && f->env == res_env &&
               f->plan->nearfield == res_near && dmas::shape_of(f->plan, f->env).delay == res_delay;
    }

    bool resident_step()
    {
        if (!res_on) return false;
        bool progress = false;
        // jobs done, in queue order
        while (res_checked < res_published && __atomic_load_n(&res_h->done[res_checked], __ATOMIC_ACQUIRE)) {
            if (Frame *f = res_job_frame[res_checked]) res_finish(f);
            ++res_checked;
            progress = true;
        }
        if (res_running) {
            const hipError_t q = hipEventQuery(res_end);
            if (q != hipErrorNotReady) {
                res_running = false;
                res_stopping = false;
                release_held();
                progress = true;
                if (q != hipSuccess) res_fail_outstanding(hipGetErrorString(q));
                // a worker that ended has completed every job it claimed: read the flags again
                while (res_checked < res_published && __atomic_load_n(&res_h->done[res_checked], __ATOMIC_ACQUIRE)) {
                    if (Frame *f = res_job_frame[res_checked]) res_finish(f);
                    ++res_checked;
                }
            }
        }
        // jobs published after the last workgroup went idle: continue the queue
        if (!res_running && res_checked < res_published) {
            res_launch(false);
            return true;
        }
        const double t_now = now_s();
        const bool can_take = res_running && !res_stopping && t_now - res_t_launch < kResidentLife;
        double oldest_other = -1;   // admission time of the oldest frame the worker cannot take
        Frame *pending = nullptr;   // roots published, pixels not yet
        for (auto it = res_admitted.begin(); it != res_admitted.end();) {
            Frame *f = *it;
            if (!res_running && !res_stopping && res_checked == res_published) {
                // no worker: launch one for this frame's class with the largest LDS that the
                // class's admitted frames need
                res_order = f->plan->order;
                res_cf = f->plan->cf;
                res_env = f->env;
                res_near = f->plan->nearfield;
                res_delay = dmas::shape_of(f->plan, f->env).delay;
                res_lds = 0;
                for (Frame *g : res_admitted)
                    if (res_same_class(g)) res_lds = std::max(res_lds, g->env ? g->plan->lds_env : g->plan->lds_rf);
                if (!res_launch(true)) {
                    it = res_admitted.erase(it);
                    fail_unlaunched(f);
                    progress = true;
                    continue;
                }
                progress = true;
            }
            const size_t lds = f->env ? f->plan->lds_env : f->plan->lds_rf;
            const bool fits = (can_take || (res_running && !res_stopping && t_now - res_t_launch < kResidentLife)) &&
                              res_same_class(f) && lds <= res_lds && f->plan->serial < res_serial &&
                              res_published + 3 <= dmas::kResidentJobs;
            if (fits && res_queued_items >= res_items_cap) break;   // queue deep enough: keep arrival order
            if (fits) {
                it = res_admitted.erase(it);
                res_publish_roots(f);
                if (pending) res_publish_pixels(pending);
                pending = f;
                progress = true;
            } else {
                if (oldest_other < 0) oldest_other = f->t_admit;
                ++it;
            }
        }
        if (pending) res_publish_pixels(pending);
        // held memory goes back when frames wait for memory or a drain waits for it
        if (res_running && !res_held.empty() && (!queued.empty() || drain_waiters > 0) &&
            t_now - res_t_epoch >= kEpochMin) {
            release_held();
            progress = true;
        }
        // let the worker finish its queue and exit when a frame it cannot take has waited,
        // when it has nothing left, when it has run its time, or when launches wait for the device
        if (res_running && !res_stopping) {
            const bool idle = res_checked == res_published;
            bool launches_wait = !admitted.empty();
            for (auto &l : launches) launches_wait |= l.busy;

            if ((oldest_other >= 0 && (idle || t_now - oldest_other > res_switch_wait)) ||
                t_now - res_t_launch >= kResidentLife || launches_wait || res_published + 2 > dmas::kResidentJobs) {
                __atomic_store_n(&res_h->stop, 1, __ATOMIC_RELEASE);
                res_stopping = true;
                progress = true;
            }
        }
        if (progress) cv_done.notify_all();
        return progress;
    }

    void run()
    {
        std::unique_lock<std::mutex> lk(mu);
        // a failure here makes every later device call of this thread fail too,
        // and those mark their frames failed
        if (hipSetDevice(device) != hipSuccess) worker_error = "cannot select the server's device";
        while (!stop.load()) {
            bool progress = collect_completions();
            progress |= admit();
            progress |= resident_step();
            progress |= launch();
            bool busy = res_running;
            for (auto &l : launches) busy |= l.busy;
            if (!progress) {
                if (!busy && queued.empty() && admitted.empty() && res_admitted.empty()) {
                    cv_work.wait_for(lk, std::chrono::milliseconds(5));
                } else {
                    lk.unlock();
                    // a resident worker waits on this loop for new jobs: poll faster
                    std::this_thread::sleep_for(std::chrono::microseconds(res_running ? 5 : 20));
                    lk.lock();
                }
            }
        }
    }
};

extern "C" {

double dmas_server_clock(void)
{
    return now_s();
}

dmas_status_t dmas_server_create(const dmas_server_desc_t *d, dmas_server_t *out)
{
    if (!d || !out) return srv_fail(DMAS_ERR_INVALID_ARG, "desc or out is NULL");
    *out = nullptr;
    if (d->hbm_budget_bytes <= 0) return srv_fail(DMAS_ERR_INVALID_ARG, "hbm_budget_bytes must be > 0");
    if (d->staging_bytes < 0 || d->num_streams < 0 || d->max_batch_frames < 0)
        return srv_fail(DMAS_ERR_INVALID_ARG, "negative server parameter");
    if (d->max_batch_frames > kMaxBatchFrames) return srv_fail(DMAS_ERR_INVALID_ARG, "max_batch_frames > 1024");
    if (d->num_streams > 16) return srv_fail(DMAS_ERR_INVALID_ARG, "num_streams > 16");
    if ((d->resident != 0 && d->resident != 1) || d->reserved != 0)
        return srv_fail(DMAS_ERR_INVALID_ARG, "resident must be 0 or 1 and reserved 0");
    auto *s = new (std::nothrow) dmas_server_s();
    if (!s) return srv_fail(DMAS_ERR_OUT_OF_MEMORY, "host allocation failed");
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return srv_fail(DMAS_ERR_DEVICE, "no current device");
    }
    s->budget = align_up((size_t)d->hbm_budget_bytes);
    s->staging = align_up(d->staging_bytes ? (size_t)d->staging_bytes : (size_t)256 << 20);
    s->nstreams = d->num_streams ? d->num_streams : 2;
    s->max_batch = d->max_batch_frames ? d->max_batch_frames : 64;
    {
        hipDeviceProp_t prop;
        int cus = 256;
        double clk = 2.4e9;   // peak clock; clockRate is in kHz
        if (hipGetDeviceProperties(&prop, s->device) == hipSuccess) {
            cus = prop.multiProcessorCount;
            if (prop.clockRate > 0) clk = prop.clockRate * 1e3;
        }
        s->res_cus = cus;
        s->resident_wgs = (int64_t)3 * cus;
        // 4 SIMDs x 16 lanes per CU issue one lane-instruction each per clock
        s->rate_cap = 0.92 * cus * 64.0 * clk;
        s->rate = std::min(s->rate, s->rate_cap);
        s->batch_wg_cap = 2 * s->resident_wgs;
        // Groups of up to four device rounds start beside a running launch's main
        // body. Measured on the serving mix against none: p50 at 2000 frames/s
        // 1.42 -> 1.07 ms, p99 9.97 -> 7.19 ms, capacity 2673 -> 2888 frames/s;
        // one or two rounds gained less, six or more or no limit lost again.
        s->small_wg_cap = 4 * s->resident_wgs;
        if (const char *sc = std::getenv("DMAS_SMALL_LAUNCH_WGS")) s->small_wg_cap = std::max(0L, std::atol(sc));
    }
    auto fail_all = [&](hipError_t e, const char *what) {
        dmas_server_destroy(s);
        dmas::set_last_error((std::string(what) + ": " + hipGetErrorString(e)).c_str());
        return e == hipErrorOutOfMemory ? DMAS_ERR_OUT_OF_MEMORY : DMAS_ERR_DEVICE;
    };
    hipError_t e = hipMalloc(&s->d_arena, s->budget);
    if (e != hipSuccess) return fail_all(e, "HBM arena");
    // resident workers read frames' inputs from the staging memory itself: coherent there
    e = hipHostMalloc(&s->h_staging, s->staging,
                      d->resident ? (hipHostMallocCoherent | hipHostMallocMapped) : hipHostMallocDefault);
    if (e != hipSuccess) return fail_all(e, "pinned staging");
    if (d->resident) {
        void *dv = nullptr;
        if ((e = hipHostGetDevicePointer(&dv, s->h_staging, 0)) != hipSuccess)
            return fail_all(e, "pinned staging (device view)");
        s->d_staging = static_cast<const char *>(dv);
    }
    s->arena.reset(s->budget);
    s->stage_arena.reset(s->staging);
    e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail_all(e, "copy stream");
    s->table_bytes = align_up((sizeof(dmas::KernelParams) + sizeof(int32_t)) * kMaxBatchFrames);
    s->streams.resize(s->nstreams, nullptr);
    s->launches.resize(s->nstreams);
    s->d_tables.resize(s->nstreams, nullptr);
    s->h_tables.resize(s->nstreams, nullptr);
    for (int i = 0; i < s->nstreams; ++i) {
        if ((e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking)) != hipSuccess)
            return fail_all(e, "compute stream");
        if ((e = hipEventCreateWithFlags(&s->launches[i].done, hipEventDisableTiming)) != hipSuccess)
            return fail_all(e, "event");
        if ((e = hipMalloc(&s->d_tables[i], s->table_bytes)) != hipSuccess) return fail_all(e, "batch table");
        if ((e = hipHostMalloc(&s->h_tables[i], s->table_bytes, hipHostMallocDefault)) != hipSuccess)
            return fail_all(e, "batch table (host)");
    }
    // Touch every stream once so that their hardware queues exist before the
    // first frame arrives (created lazily otherwise, stalling the scheduler).
    for (int i = 0; i < s->nstreams; ++i) {
        if ((e = hipMemsetAsync(s->d_tables[i], 0, kAlign, s->streams[i])) != hipSuccess) return fail_all(e, "stream warm-up");
        if ((e = hipEventRecord(s->launches[i].done, s->streams[i])) != hipSuccess) return fail_all(e, "stream warm-up");
    }
    if ((e = hipMemcpyAsync(s->d_tables[0], s->h_tables[0], kAlign, hipMemcpyHostToDevice, s->copy_stream)) != hipSuccess)
        return fail_all(e, "copy stream warm-up");
    if (d->resident) {
        if (const char *sw = std::getenv("DMAS_RESIDENT_SWITCH_US")) s->res_switch_wait = std::max(0.0, std::atof(sw)) * 1e-6;
        // the job queue in coherent pinned memory (polled by the device), the claim
        // counters on the device
        s->res_on = true;
        if ((e = hipHostMalloc((void **)&s->res_h, sizeof(dmas::ResidentHost), hipHostMallocCoherent | hipHostMallocMapped)) !=
            hipSuccess)
            return fail_all(e, "resident job queue");
        std::memset(s->res_h, 0, sizeof(dmas::ResidentHost));
        if ((e = hipHostGetDevicePointer((void **)&s->res_hd, s->res_h, 0)) != hipSuccess)
            return fail_all(e, "resident job queue (device view)");
        if ((e = hipMalloc((void **)&s->res_d, sizeof(dmas::ResidentDevice))) != hipSuccess)
            return fail_all(e, "resident counters");
        if ((e = hipStreamCreateWithFlags(&s->res_stream, hipStreamNonBlocking)) != hipSuccess)
            return fail_all(e, "resident stream");
        if ((e = hipEventCreateWithFlags(&s->res_end, hipEventDisableTiming)) != hipSuccess)
            return fail_all(e, "resident event");
        if ((e = hipMemsetAsync(s->res_d, 0, sizeof(dmas::ResidentDevice), s->res_stream)) != hipSuccess ||
            (e = hipEventRecord(s->res_end, s->res_stream)) != hipSuccess ||
            (e = hipStreamSynchronize(s->res_stream)) != hipSuccess)
            return fail_all(e, "resident stream warm-up");
    }
    for (hipStream_t st : s->streams)
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail_all(e, "stream warm-up");
    if ((e = hipStreamSynchronize(s->copy_stream)) != hipSuccess) return fail_all(e, "copy stream warm-up");
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return DMAS_OK;
}

dmas_status_t dmas_server_submit(dmas_server_t s, dmas_plan_t plan, const void *h_x, float in_scale, int32_t flags,
                                 double arrival, uint64_t *ticket)
{
    if (!s || !plan || !h_x || !ticket) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL argument");
    if (!(in_scale > 0.0f) || !std::isfinite(in_scale)) return srv_fail(DMAS_ERR_INVALID_ARG, "in_scale must be > 0");
    if (flags & ~(DMAS_SUBMIT_ENVELOPE | DMAS_SUBMIT_AUTO_RELEASE)) return srv_fail(DMAS_ERR_INVALID_ARG, "unknown flags");
    if (plan->device != s->device) return srv_fail(DMAS_ERR_INVALID_ARG, "plan and server are on different devices");
    auto *f = new (std::nothrow) Frame();
    if (!f) return srv_fail(DMAS_ERR_OUT_OF_MEMORY, "host allocation failed");
    f->plan = plan;
    f->in_scale = in_scale;
    f->env = (flags & DMAS_SUBMIT_ENVELOPE) != 0;
    f->auto_release = (flags & DMAS_SUBMIT_AUTO_RELEASE) != 0;
    f->in_bytes = (size_t)plan->M * plan->T * elem_size(plan->dtype);
    const size_t out_T = f->env ? (size_t)(plan->T + plan->env_decim - 1) / plan->env_decim : (size_t)plan->T;
    f->out_bytes = (size_t)plan->D * out_T * sizeof(float);
    f->plane_bytes = dmas::plane_bytes(plan);
    if (!dmas::sched::admissible(f->in_bytes, f->out_bytes, f->plane_bytes, plan->device_bytes, s->budget)) {
        delete f;
        return srv_fail(DMAS_ERR_INVALID_ARG,
                        "frame input, root plane and output with the plan's device memory exceed the server's HBM "
                        "budget");
    }
    if (align_up(f->in_bytes) > s->staging) {
        delete f;
        return srv_fail(DMAS_ERR_INVALID_ARG, "frame input exceeds the server's staging memory");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->stage_arena.alloc(f->in_bytes, &f->stage_off)) {
            delete f;
            return srv_fail(DMAS_ERR_BUSY, "staging memory full");
        }
        f->staged = true;
    }
    // The staging range is reserved for this frame: copy outside the lock.
    std::memcpy(s->h_staging + f->stage_off, h_x, f->in_bytes);
    const double t = now_s();
    f->t_arrival = arrival >= 0 ? arrival : t;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        f->ticket = s->next_ticket++;
        s->frames[f->ticket] = f;
        s->queued.push_back(f);
        ++s->n_submitted;
        *ticket = f->ticket;
    }
    s->cv_work.notify_one();
    return DMAS_OK;
}

dmas_status_t dmas_server_query(dmas_server_t s, uint64_t ticket, dmas_frame_info_t *info)
{
    if (!s || !info) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->frames.find(ticket);
    if (it == s->frames.end()) return srv_fail(DMAS_ERR_INVALID_ARG, "unknown ticket");
    s->fill_info(it->second, info);
    return DMAS_OK;
}

dmas_status_t dmas_server_wait(dmas_server_t s, uint64_t ticket, double timeout, dmas_frame_info_t *info)
{
    if (!s) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL server");
    if (!(timeout >= 0.0)) return srv_fail(DMAS_ERR_INVALID_ARG, "timeout must be >= 0");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = deadline_after(timeout);
    while (true) {
        auto it = s->frames.find(ticket);
        if (it == s->frames.end()) return srv_fail(DMAS_ERR_INVALID_ARG, "unknown ticket");
        Frame *f = it->second;
        if (f->state == kDone || f->state == kFailed) {
            if (info) s->fill_info(f, info);
            return f->state == kDone ? DMAS_OK : srv_fail(DMAS_ERR_DEVICE, "frame failed");
        }
        if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            auto it2 = s->frames.find(ticket);
            if (it2 != s->frames.end() && (it2->second->state == kDone || it2->second->state == kFailed)) continue;
            return srv_fail(DMAS_ERR_TIMEOUT, "timed out waiting for the frame");
        }
    }
}

dmas_status_t dmas_server_release(dmas_server_t s, uint64_t ticket)
{
    if (!s) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->frames.find(ticket);
    if (it == s->frames.end()) return srv_fail(DMAS_ERR_INVALID_ARG, "unknown ticket");
    Frame *f = it->second;
    if (f->state != kDone && f->state != kFailed)
        return srv_fail(DMAS_ERR_INVALID_ARG, "frame is not finished; wait for it before releasing");
    s->free_device(f);
    s->free_staging(f);
    s->frames.erase(it);
    delete f;
    return DMAS_OK;
}

dmas_status_t dmas_server_fetch(dmas_server_t s, uint64_t ticket, float *h_out)
{
    if (!s || !h_out) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL argument");
    const float *src = nullptr;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->frames.find(ticket);
        if (it == s->frames.end()) return srv_fail(DMAS_ERR_INVALID_ARG, "unknown ticket");
        Frame *f = it->second;
        if (f->state != kDone || !f->on_device) return srv_fail(DMAS_ERR_INVALID_ARG, "frame has no result");
        src = reinterpret_cast<const float *>(s->d_arena + f->out_off);
        bytes = f->out_bytes;
    }
    // The result stays allocated until the caller releases the ticket.
    hipError_t e = hipMemcpy(h_out, src, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return srv_fail(DMAS_ERR_DEVICE, hipGetErrorString(e));
    return DMAS_OK;
}

dmas_status_t dmas_server_completed(dmas_server_t s, dmas_frame_info_t *out, int32_t max, int32_t *count)
{
    if (!s || !count || (max > 0 && !out)) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t n = 0;
    while (n < max && !s->finished.empty()) {
        out[n++] = s->finished.front();
        s->finished.pop_front();
    }
    *count = n;
    return DMAS_OK;
}

dmas_status_t dmas_server_drain(dmas_server_t s, double timeout)
{
    if (!s) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL server");
    if (!(timeout >= 0.0)) return srv_fail(DMAS_ERR_INVALID_ARG, "timeout must be >= 0");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = deadline_after(timeout);
    auto busy_now = [s] {
        bool busy = !s->queued.empty() || !s->admitted.empty() || !s->res_admitted.empty() ||
                    s->res_checked < s->res_published || !s->res_held.empty();
        for (auto &l : s->launches) busy |= l.busy;
        return busy;
    };
    struct Waiter {   // counted while waiting (under mu): an idle worker exits for a drain
        int &n;
        explicit Waiter(int &c) : n(c) { ++n; }
        ~Waiter() { --n; }
    } waiter(s->drain_waiters);
    while (true) {
        bool busy = busy_now();
        if (!busy) return DMAS_OK;
        if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            busy = busy_now();
            if (!busy) return DMAS_OK;
            return srv_fail(DMAS_ERR_TIMEOUT, "timed out draining the server");
        }
    }
}

dmas_status_t dmas_server_stats(dmas_server_t s, dmas_server_stats_t *st)
{
    if (!s || !st) return srv_fail(DMAS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->n_submitted;
    st->completed = s->n_completed;
    st->failed = s->n_failed;
    st->launches = s->n_launches;
    st->batched_frames = s->n_batched;
    st->queued = (int64_t)s->queued.size();
    st->admitted_not_launched = (int64_t)(s->admitted.size() + s->res_admitted.size());
    int64_t inflight = 0;
    for (auto &l : s->launches) inflight += (int64_t)l.frames.size();
    for (int j = s->res_checked; j < s->res_published; ++j) inflight += s->res_job_frame[j] != nullptr;
    st->in_flight = inflight;
    st->hbm_in_use = (int64_t)s->arena.used();
    st->hbm_peak = (int64_t)s->hbm_peak;
    st->hbm_budget = (int64_t)s->budget;
    st->resident_launches = s->n_res_launches;
    st->resident_frames = s->n_res_frames;
    return DMAS_OK;
}

dmas_status_t dmas_server_destroy(dmas_server_t s)
{
    if (!s) return DMAS_OK;
    if (s->worker.joinable()) {
        s->stop.store(true);
        s->cv_work.notify_all();
        s->worker.join();
    }
    // teardown: failures here have no caller to report to
    if (s->res_h) __atomic_store_n(&s->res_h->stop, 1, __ATOMIC_RELEASE);   // a running worker exits
    if (s->res_stream) (void)hipStreamSynchronize(s->res_stream);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamSynchronize(st);
    if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
    for (auto &kv : s->frames) {
        if (kv.second->copied) (void)hipEventDestroy(kv.second->copied);
        delete kv.second;
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (auto &l : s->launches)
        if (l.done) (void)hipEventDestroy(l.done);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    if (s->res_end) (void)hipEventDestroy(s->res_end);
    if (s->res_stream) (void)hipStreamDestroy(s->res_stream);
    if (s->res_d) (void)hipFree(s->res_d);
    if (s->res_h) (void)hipHostFree(s->res_h);
    for (char *p : s->d_tables) (void)hipFree(p);
    for (char *p : s->h_tables) (void)hipHostFree(p);
    (void)hipFree(s->d_arena);
    (void)hipHostFree(s->h_staging);
    delete s;
    return DMAS_OK;
}

}  // extern "C"
