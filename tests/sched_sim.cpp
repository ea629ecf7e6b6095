// CPU executor for the serving runtime's scheduling policy
// (paper_2511_09165_amd/csrc/dmas_sched.hpp): simulated arrivals, a simulated
// device whose streams finish their launches after modelled durations (in any
// order), and the server's rules around the policy (arrival-order admission
// that stops at the first frame that does not fit, plan memory counted while
// frames of the plan hold memory, one launch per idle stream). It checks
// invariants after every step and prints a JSON summary; a broken invariant
// prints a message and exits with status 1.
//
// usage: sched_sim SCENARIO SEED   (SCENARIO: mix, tight, oversize, single)
// Built with -DSCHED_SIM_PLANT_OVERTAKE the harness breaks the arrival-order
// rule on purpose, to show that the checks catch it.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "../paper_2511_09165_amd/csrc/dmas_sched.hpp"

namespace sched = dmas::sched;

namespace {

#define CHECK(cond, ...)                                                                   \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            std::fprintf(stderr, "invariant broken: %s: ", #cond);                         \
            std::fprintf(stderr, __VA_ARGS__);                                             \
            std::fprintf(stderr, "\n");                                                    \
            std::exit(1);                                                                  \
        }                                                                                  \
    } while (0)

struct Plan {
    size_t bytes;
    int64_t cls;
    int64_t workgroups;
    bool batchable;
};

struct Frame {
    int id;
    int plan;
    double arrival;
    size_t in, out, plane;
    double work;   // seconds alone on the device
    int state = 0; // 0 queued, 1 admitted, 2 launched, 3 done, -1 rejected
    sched::Grant g;
    double t_admit = -1, t_launch = -1, t_done = -1;
    int launch_seq = -1, done_seq = -1;
};

struct Launch {
    bool busy = false;
    double end = 0, tail_start = 0;
    std::vector<int> frames;
};

struct Scenario {
    int n_frames = 400;
    double rate = 2000.0;       // arrivals per second
    size_t budget = 64u << 20;
    int nstreams = 2;
    int max_batch = 16;
    int64_t wg_cap = 1536;      // about two device rounds
    int64_t small_cap = 3072;   // four device rounds: such a group may start while the gate is closed
    int n_plans = 8;
    bool oversize = false;      // some frames larger than the budget
};

Scenario scenario(const std::string &name)
{
    Scenario s;
    if (name == "tight") {
        s.budget = 20u << 20;   // about two frames: admission waits for memory
        s.rate = 4000.0;
    } else if (name == "oversize") {
        s.oversize = true;
    } else if (name == "single") {
        s.nstreams = 1;
        s.max_batch = 1;
    } else if (name != "mix") {
        std::fprintf(stderr, "unknown scenario %s\n", name.c_str());
        std::exit(2);
    }
    return s;
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc < 3) {
        std::fprintf(stderr, "usage: sched_sim SCENARIO SEED\n");
        return 2;
    }
    const std::string name = argv[1];
    const Scenario sc = scenario(name);
    std::mt19937_64 rng(std::strtoull(argv[2], nullptr, 10));
    std::uniform_real_distribution<double> U(0.0, 1.0);

    // plans: kernel class, workgroups (some fill the device alone), own memory
    std::vector<Plan> plans;
    for (int p = 0; p < sc.n_plans; ++p) {
        Plan pl;
        pl.bytes = (size_t)(U(rng) * (1u << 20)) + 4096;
        pl.cls = p % 3;
        pl.workgroups = (p % 2) ? 256 + (int64_t)(U(rng) * 512) : 2000 + (int64_t)(U(rng) * 4000);
        pl.batchable = p != 5;
        plans.push_back(pl);
    }
    std::vector<Frame> frames;
    double t = 0;
    for (int i = 0; i < sc.n_frames; ++i) {
        t += -std::log(1.0 - U(rng)) / sc.rate;
        Frame f;
        f.id = i;
        f.plan = (int)(U(rng) * sc.n_plans);
        f.arrival = t;
        f.in = (size_t)(U(rng) * (2u << 20)) + 1;
        f.out = (size_t)(U(rng) * (6u << 20)) + 1;
        f.plane = (i % 3) ? (size_t)(U(rng) * (2u << 20)) : 0;
        if (sc.oversize && i % 17 == 5) f.out = sc.budget;   // never admissible
        f.work = 0.2e-3 + U(rng) * 0.6e-3;
        frames.push_back(f);
    }

    sched::Arena arena;
    arena.reset(sc.budget);
    std::map<int, std::pair<size_t, int>> plan_use;   // plan -> (offset, frames holding memory)
    std::map<size_t, size_t> live;                    // offset -> bytes of every granted range
    std::deque<int> queued, admitted;
    std::vector<Launch> launches(sc.nstreams);
    int next_arrival = 0, launch_seq = 0, done_seq = 0, admit_seq = 0;
    int64_t rejected = 0, waits_for_memory = 0, n_launches = 0, batched = 0, max_group = 0, n_small = 0;
    size_t max_used = 0;
    std::vector<int> admit_order;

    auto take = [&](size_t off, size_t bytes) {
        if (!bytes) return;
        bytes = sched::align_up(bytes);
        CHECK(off + bytes <= sc.budget, "range [%zu, %zu) outside the budget", off, off + bytes);
        auto it = live.lower_bound(off);
        CHECK(it == live.end() || it->first >= off + bytes, "range at %zu overlaps a live one", off);
        if (it != live.begin()) {
            auto pr = std::prev(it);
            CHECK(pr->first + pr->second <= off, "range at %zu overlaps a live one", off);
        }
        live[off] = bytes;
    };
    auto give = [&](size_t off, size_t bytes) {
        if (!bytes) return;
        auto it = live.find(off);
        CHECK(it != live.end() && it->second == sched::align_up(bytes), "release of a range not granted");
        live.erase(it);
        arena.release(off, bytes);
    };
    auto check_used = [&]() {
        size_t sum = 0;
        for (auto &r : live) sum += r.second;
        CHECK(sum == arena.used(), "arena reports %zu bytes used, live ranges hold %zu", arena.used(), sum);
        CHECK(arena.used() <= sc.budget, "%zu bytes used > budget %zu", arena.used(), sc.budget);
        max_used = std::max(max_used, arena.used());
    };

    double now = 0;
    int done = 0;
    const int total = (int)frames.size();
    for (int step = 0; step < 10000000 && done + rejected < total; ++step) {
        // next event: an arrival, a launch ending, or a gate opening
        double t_next = 1e300;
        if (next_arrival < total) t_next = frames[next_arrival].arrival;
        for (auto &l : launches)
            if (l.busy) t_next = std::min(t_next, l.end);
        if (!admitted.empty())
            for (auto &l : launches)
                if (l.busy && l.tail_start > now) t_next = std::min(t_next, l.tail_start);
        CHECK(t_next < 1e300, "nothing left to happen with %d frames unfinished", total - done - (int)rejected);
        now = std::max(now, t_next);

        // arrivals (submit: never-admissible frames are refused at once)
        while (next_arrival < total && frames[next_arrival].arrival <= now) {
            Frame &f = frames[next_arrival++];
            if (!sched::admissible(f.in, f.out, f.plane, plans[f.plan].bytes, sc.budget)) {
                f.state = -1;
                ++rejected;
            } else {
                queued.push_back(f.id);
            }
        }
        // completions, in random order among the streams that have ended
        std::vector<int> ended;
        for (int s = 0; s < sc.nstreams; ++s)
            if (launches[s].busy && launches[s].end <= now) ended.push_back(s);
        std::shuffle(ended.begin(), ended.end(), rng);
        for (int s : ended) {
            for (int id : launches[s].frames) {
                Frame &f = frames[id];
                CHECK(f.state == 2, "frame %d completes without a launch", id);
                f.state = 3;
                f.t_done = now;
                f.done_seq = done_seq++;
                give(f.g.in_off, f.in);
                give(f.g.out_off, f.out);
                give(f.g.plane_off, f.plane);
                auto &pu = plan_use.at(f.plan);
                if (--pu.second == 0) {
                    give(pu.first, plans[f.plan].bytes);
                    plan_use.erase(f.plan);
                }
                ++done;
            }
            launches[s].busy = false;
            launches[s].frames.clear();
            check_used();
        }
        // admission: arrival order, stop at the first frame that does not fit
        bool overtook = false;
        (void)overtook;
        while (!queued.empty()) {
            Frame &f = frames[queued.front()];
            const bool new_plan = plan_use.count(f.plan) == 0;
            sched::Grant g;
            if (!sched::grant(arena, f.in, f.out, f.plane, new_plan ? plans[f.plan].bytes : 0, &g)) {
#ifdef SCHED_SIM_PLANT_OVERTAKE
                // planted mistake (harness only): once per pass, let the next frame
                // overtake one that does not fit
                if (queued.size() > 1 && !overtook) {
                    std::swap(queued[0], queued[1]);
                    overtook = true;
                    continue;
                }
#endif
                bool busy = false;
                for (auto &l : launches) busy |= l.busy;
                // a frame that does not fit waits only while others hold memory
                CHECK(busy || !admitted.empty(), "frame %d does not fit an idle device", f.id);
                ++waits_for_memory;
                break;
            }
            take(g.in_off, f.in);
            take(g.out_off, f.out);
            take(g.plane_off, f.plane);
            if (new_plan) {
                take(g.plan_off, plans[f.plan].bytes);
                plan_use[f.plan] = {g.plan_off, 0};
            }
            ++plan_use[f.plan].second;
            f.g = g;
            f.state = 1;
            f.t_admit = now;
            admit_order.push_back(f.id);
            ++admit_seq;
            queued.pop_front();
            admitted.push_back(f.id);
            check_used();
        }
        // launches
        while (!admitted.empty()) {
            std::vector<sched::StreamState> ss;
            for (auto &l : launches) ss.push_back({l.busy, l.tail_start});
            std::vector<sched::Candidate> cand;
            for (int id : admitted) {
                const Plan &pl = plans[frames[id].plan];
                cand.push_back({pl.cls, pl.batchable, pl.workgroups});
            }
            const sched::LaunchPick lp = sched::pick_launch(ss, now, cand, sc.max_batch, sc.wg_cap, sc.small_cap);
            if (lp.stream < 0) break;
            const int s = lp.stream;
            const std::vector<size_t> &pick = lp.frames;
            CHECK(!launches[s].busy, "picked a busy stream");
            CHECK(!pick.empty(), "a launch without frames");
            bool gate_closed = false;
            for (auto &l : launches) gate_closed = gate_closed || (l.busy && l.tail_start > now);
            if (!lp.small) {
                CHECK(!gate_closed, "launch overlaps a running main body");
                CHECK(pick[0] == 0, "the head of the queue must lead its launch");
            } else {
                // only while the gate is closed, led by the first frame that small
                CHECK(gate_closed, "a small launch while the gate is open");
                for (size_t k = 0; k < pick[0]; ++k)
                    CHECK(cand[k].workgroups > sc.small_cap, "a small launch skipped an earlier small frame");
                ++n_small;
            }
            int64_t wgs = 0;
            for (size_t k = 0; k < pick.size(); ++k) {
                CHECK(k == 0 || pick[k] > pick[k - 1], "group out of arrival order");
                const sched::Candidate &c = cand[pick[k]];
                CHECK(c.cls == cand[pick[0]].cls, "frames of two kernel classes in one launch");
                wgs += c.workgroups;
            }
            if (lp.small) CHECK(wgs <= sc.small_cap, "small launch of %lld workgroups", (long long)wgs);
            if (pick.size() > 1) {
                CHECK((int)pick.size() <= sc.max_batch, "more than max_batch frames");
                // a small launch packs up to its own cap (checked above)
                CHECK(lp.small || wgs <= sc.wg_cap, "batch of %lld workgroups over the cap", (long long)wgs);
                for (size_t k : pick) CHECK(cand[k].batchable, "a frame the multi-frame kernel does not serve");
            }
            double work = 0;
            Launch &l = launches[s];
            for (size_t k = pick.size(); k-- > 0;) {
                const int id = admitted[pick[k]];
                admitted.erase(admitted.begin() + (std::ptrdiff_t)pick[k]);
                Frame &f = frames[id];
                f.state = 2;
                f.t_launch = now;
                f.launch_seq = launch_seq;
                work += f.work;
                l.frames.push_back(id);
            }
            ++launch_seq;
            ++n_launches;
            if (pick.size() > 1) batched += (int64_t)pick.size();
            max_group = std::max<int64_t>(max_group, (int64_t)pick.size());
            const double dur = work * (0.7 + 0.6 * U(rng));   // durations vary: completions reorder
            l.busy = true;
            l.end = now + dur;
            l.tail_start = lp.small ? now : now + 0.8 * dur;   // a small launch does not hold the gate
        }
    }

    CHECK(done + rejected == total, "%d of %d frames finished", done + (int)rejected, total);
    CHECK(arena.used() == 0 && live.empty() && plan_use.empty(), "memory left after every frame finished");
    CHECK(arena.free_ranges() == 1, "free ranges did not coalesce (%zu left)", arena.free_ranges());
    // admission in arrival order
    for (size_t k = 1; k < admit_order.size(); ++k)
        CHECK(admit_order[k] > admit_order[k - 1], "frame %d admitted before frame %d", admit_order[k],
              admit_order[k - 1]);
    // completions out of launch order happen (several streams, varying durations)
    int64_t reordered = 0;
    for (auto &a : frames)
        for (auto &b : frames)
            if (a.state == 3 && b.state == 3 && a.launch_seq < b.launch_seq && a.done_seq > b.done_seq) {
                ++reordered;
                break;
            }
    std::printf("{\"scenario\": \"%s\", \"frames\": %d, \"done\": %d, \"rejected\": %lld, \"launches\": %lld, "
                "\"batched_frames\": %lld, \"max_group\": %lld, \"waits_for_memory\": %lld, "
                "\"completed_out_of_launch_order\": %lld, \"max_used\": %zu, \"budget\": %zu, "
                "\"small_launches\": %lld}\n",
                name.c_str(), total, done, (long long)rejected, (long long)n_launches, (long long)batched,
                (long long)max_group, (long long)waits_for_memory, (long long)reordered, max_used, sc.budget,
                (long long)n_small);
    return 0;
}
