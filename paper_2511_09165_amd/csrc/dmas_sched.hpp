// Scheduling policy of the serving runtime (dmas_server.hip), kept free of
// device calls so that a CPU executor can drive the same code in tests:
//   * Arena: first-fit allocator of the HBM budget with coalescing;
//   * admissible / grant: a frame's device memory (input copy, output, root
//     plane, and its plan's own memory while no other frame of the plan holds
//     any), all of it or none;
//   * pick_stream: the stream for the next launch, or none while a running
//     launch is still in its main body;
//   * pick_group: the admitted frames that share the next launch;
//   * pick_launch: both, and while the gate is closed a small group (a few
//     device rounds of workgroups at most) on an idle stream.
// Admission is in arrival order and stops at the first frame that does not
// fit (no frame overtakes an earlier one); the server applies that rule around
// grant(). Launches follow arrival order too, with one exception: while the
// head waits for the gate, a small group may start (pick_launch).
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace dmas {
namespace sched {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v)
{
    return (v + kAlign - 1) & ~(kAlign - 1);
}

// First-fit allocator over [0, size) with coalescing of free ranges; sizes are
// rounded up to kAlign.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t free_ranges() const { return free_.size(); }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

// Whether a frame can ever be admitted: its input, output, root plane and
// the device memory of its plan (plan_bytes, 0 if already counted) within the
// budget.
inline bool admissible(size_t in_bytes, size_t out_bytes, size_t plane_bytes, size_t plan_bytes, size_t budget)
{
    return align_up(in_bytes) + align_up(out_bytes) + align_up(plane_bytes) + align_up(plan_bytes) <= budget;
}

// Offsets of a frame's device memory in the arena.
struct Grant {
    size_t in_off = 0, out_off = 0, plane_off = 0, plan_off = 0;
};

// The frame's input copy (in_bytes, 0 for none), output, root plane
// (plane_bytes, 0 for none) and, when no other frame of its plan holds
// device memory, the plan's own device memory (plan_bytes, 0 otherwise; held
// while frames of the plan are) from the arena, all or nothing.
inline bool grant(Arena &a, size_t in_bytes, size_t out_bytes, size_t plane_bytes, size_t plan_bytes, Grant *g)
{
    Grant r;
    const size_t want[4] = {in_bytes, out_bytes, plane_bytes, plan_bytes};
    size_t *off[4] = {&r.in_off, &r.out_off, &r.plane_off, &r.plan_off};
    for (int k = 0; k < 4; ++k) {
        if (want[k] && !a.alloc(want[k], off[k])) {
            for (int j = 0; j < k; ++j)
                if (want[j]) a.release(*off[j], want[j]);
            return false;
        }
    }
    *g = r;
    return true;
}

// A launch in flight as the launcher sees it.
struct StreamState {
    bool busy = false;
    double tail_start = 0;   // predicted start of its last device round
};

// The first idle stream, or -1 if none is idle or a busy launch has not yet
// reached its last device round at time t (overlapping a launch's main body
// would only slow it down).
inline int pick_stream(const std::vector<StreamState> &streams, double t)
{
    int s = -1;
    for (int i = 0; i < (int)streams.size(); ++i) {
        if (streams[i].busy) {
            if (t < streams[i].tail_start) return -1;
        } else if (s < 0) {
            s = i;
        }
    }
    return s;
}

// The first idle stream, or -1.
inline int idle_stream(const std::vector<StreamState> &streams)
{
    for (int i = 0; i < (int)streams.size(); ++i)
        if (!streams[i].busy) return i;
    return -1;
}

// What the grouping needs to know of an admitted frame.
struct Candidate {
    int64_t cls = 0;          // kernel class: frames of one class share an instantiation
    bool batchable = false;   // the multi-frame kernel serves it
    int64_t workgroups = 0;
};

// Indices (into the admitted queue, arrival order, 0 = head) of the frames
// of the next launch. A head that fills the device by itself (wg_cap or more
// workgroups), is not batchable or is limited to one frame per launch goes
// alone; otherwise frames of the head's class join in arrival order while the
// launch stays within max_batch frames and wg_cap workgroups.
inline std::vector<size_t> pick_group(const std::vector<Candidate> &q, int max_batch, int64_t wg_cap)
{
    std::vector<size_t> group;
    if (q.empty()) return group;
    const Candidate &head = q[0];
    if (max_batch <= 1 || !head.batchable || head.workgroups >= wg_cap) {
        group.push_back(0);
        return group;
    }
    int64_t wgs = 0;
    for (size_t i = 0; i < q.size() && (int)group.size() < max_batch; ++i) {
        const Candidate &f = q[i];
        if (f.batchable && f.cls == head.cls && (group.empty() || wgs + f.workgroups <= wg_cap)) {
            group.push_back(i);
            wgs += f.workgroups;
        }
    }
    return group;
}

// The frames of a small launch: the first admitted frame (arrival order) of
// at most small_cap workgroups, with frames of its class behind it while the
// launch stays within small_cap workgroups (the rules of pick_group, with
// small_cap as the cap); empty if no frame is that small.
inline std::vector<size_t> pick_small(const std::vector<Candidate> &q, int max_batch, int64_t small_cap)
{
    for (size_t i = 0; i < q.size(); ++i) {
        if (q[i].workgroups > small_cap) continue;
        const std::vector<Candidate> rest(q.begin() + (std::ptrdiff_t)i, q.end());
        std::vector<size_t> g = pick_group(rest, max_batch, small_cap);
        for (size_t &k : g) k += i;
        return g;
    }
    return {};
}

// The next launch: a stream and the frames (indices into the admitted queue,
// arrival order), or stream -1 when nothing may start at time t.
//   * The gate is open (pick_stream): the head and the frames grouped with it.
//   * The gate is closed but a stream is idle: a small group (pick_small, at
//     most small_cap workgroups). A small launch does not hold the gate, so
//     the head starts as soon as the gate opens and a stream is free: it waits
//     at most for one small launch. The small launch shares the compute units
//     with the running one, which lets a shorter frame finish without waiting
//     for a long frame's main body.
struct LaunchPick {
    int stream = -1;
    std::vector<size_t> frames;
    bool small = false;   // started while the gate was closed
};

inline LaunchPick pick_launch(const std::vector<StreamState> &streams, double t, const std::vector<Candidate> &q,
                              int max_batch, int64_t wg_cap, int64_t small_cap)
{
    LaunchPick r;
    if (q.empty()) return r;
    const int s = pick_stream(streams, t);
    if (s >= 0) {
        r.stream = s;
        r.frames = pick_group(q, max_batch, wg_cap);
        return r;
    }
    const int idle = idle_stream(streams);
    if (idle < 0 || small_cap <= 0) return r;
    r.frames = pick_small(q, max_batch, small_cap);
    if (!r.frames.empty()) {
        r.stream = idle;
        r.small = true;
    }
    return r;
}

}  // namespace sched
}  // namespace dmas
