// The serving scheduler's admission policy (admission.h, the code the library
// runs) over a simulated pool: a mock executor with four workers whose
// workspaces grow to each job's per-buffer needs and are kept between jobs,
// seeded random job streams, jobs that finish while the policy frees idle
// workspaces, and queued jobs withdrawn meanwhile.  Host code only (no HIP).
// Exit status 0 when every invariant holds, 1 otherwise.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <array>
#include <deque>
#include <random>
#include <vector>

#include "admission.h"

namespace {

constexpr int kBuf = 3;        // buffers per workspace
constexpr int kWorkers = 4;
using Need = std::array<size_t, kBuf>;

int fails = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            if (fails < 20) {                          \
                fprintf(stderr, "violated: %s: ", #c); \
                fprintf(stderr, __VA_ARGS__);          \
                fprintf(stderr, "\n");                 \
            }                                          \
            ++fails;                                   \
        }                                              \
    } while (0)

size_t sum(const Need &a)
{
    size_t t = 0;
    for (size_t v : a) t += v;
    return t;
}

struct Job {
    Need need{};
    int duration = 1;    // steps it runs once dispatched
    int arrival = 0;
    int dispatched = -1; // step, or -1
    bool withdrawn = false;
};

struct Worker {
    bool busy = false;
    Need cap{};          // per-buffer capacity of its workspace
    size_t held = 0;     // reservation recorded at dispatch
    int job = -1, finish = 0;
    size_t bytes() const { return sum(cap); }
};

struct Sim {
    size_t budget;
    std::vector<Job> jobs;
    std::deque<int> queue;
    std::vector<Worker> w = std::vector<Worker>(kWorkers);
    int now = 0;
    bool starving = false;
    std::mt19937_64 rng;
    double p_finish_in_release = 0.0, p_withdraw_in_release = 0.0;
    int dispatches = 0, releases = 0, rescans = 0;

    // ---- the Pool interface of admit_one ----
    size_t queue_size() const { return queue.size(); }
    int first_idle() const
    {
        for (int i = 0; i < kWorkers; ++i)
            if (!w[i].busy) return i;
        return -1;
    }
    size_t others(int x) const
    {
        size_t t = 0;
        for (int i = 0; i < kWorkers; ++i)
            if (i != x) t += w[i].busy ? std::max(w[i].held, w[i].bytes()) : w[i].bytes();
        return t;
    }
    size_t grown(int x, size_t qi) const
    {
        size_t t = 0;
        for (int b = 0; b < kBuf; ++b) t += std::max(w[x].cap[b], jobs[queue[qi]].need[b]);
        return t;
    }
    bool release_idle(size_t qi)
    {
        ++releases;
        const int j = queue[qi];
        for (auto &c : w)
            if (!c.busy) c.cap = Need{};
        // while the lock is given up: a busy worker may finish (and is then
        // idle with its last job's workspace), a queued job may be withdrawn
        std::uniform_real_distribution<double> U(0.0, 1.0);
        if (U(rng) < p_finish_in_release) {
            for (int i = 0; i < kWorkers; ++i)
                if (w[i].busy) {
                    finish(i);
                    break;
                }
        }
        if (U(rng) < p_withdraw_in_release && !queue.empty()) {
            const size_t k = (size_t)(U(rng) * queue.size());
            jobs[queue[k]].withdrawn = true;
            queue.erase(queue.begin() + k);
        }
        const bool same = queue.size() > qi && queue[qi] == j;
        rescans += !same;
        return same;
    }
    void dispatch(size_t qi, int x, size_t mine, size_t total)
    {
        const int j = queue[qi];
        CHECK(!w[x].busy, "worker %d dispatched while busy", x);
        CHECK(!(starving && qi > 0), "job at position %zu passed a starving head", qi);
        CHECK(total <= budget, "admitted total %zu over budget %zu", total, budget);
        CHECK(mine == grown(x, qi), "reservation %zu is not the grown workspace", mine);
        queue.erase(queue.begin() + qi);
        w[x].busy = true;
        w[x].held = mine;
        w[x].job = j;
        w[x].finish = now + jobs[j].duration;
        jobs[j].dispatched = now;
        ++dispatches;
        // what the device may hold from now on: every busy workspace at its
        // grown size, every idle one as it is
        size_t dev = 0;
        for (int i = 0; i < kWorkers; ++i) {
            if (w[i].busy) {
                size_t g = 0;
                for (int b = 0; b < kBuf; ++b) g += std::max(w[i].cap[b], jobs[w[i].job].need[b]);
                dev += g;
            } else {
                dev += w[i].bytes();
            }
        }
        CHECK(dev <= budget, "device bytes %zu over budget %zu after dispatching job %d", dev, budget, j);
    }

    // ---- the executor ----
    void finish(int i)
    {
        Worker &c = w[i];
        for (int b = 0; b < kBuf; ++b) c.cap[b] = std::max(c.cap[b], jobs[c.job].need[b]);
        c.busy = false;
        c.held = 0;
        c.job = -1;
    }
};

// Runs a stream to completion; head_wait: steps after which a blocked head
// is starving.  Returns the dispatch order.
std::vector<int> run(Sim &s, int head_wait, int max_steps)
{
    std::vector<int> order;
    size_t next = 0;
    int head = -1, head_since = 0;
    for (s.now = 0; s.now < max_steps; ++s.now) {
        for (int i = 0; i < kWorkers; ++i)
            if (s.w[i].busy && s.w[i].finish <= s.now) s.finish(i);
        while (next < s.jobs.size() && s.jobs[next].arrival <= s.now) s.queue.push_back((int)next++);
        for (;;) {
            if (s.queue.empty()) break;
            if (s.queue.front() != head) {
                head = s.queue.front();
                head_since = s.now;
            }
            s.starving = s.now - head_since > head_wait;
            std::vector<int> q(s.queue.begin(), s.queue.end());
            if (!gbem::admit_one(s, s.budget, s.starving)) break;
            // the dispatched job: the one that left the queue (withdrawals
            // during a release are not dispatches)
            for (int j : q)
                if (s.jobs[j].dispatched == s.now && std::find(order.begin(), order.end(), j) == order.end()) {
                    order.push_back(j);
                    break;
                }
        }
        bool all = next == s.jobs.size() && s.queue.empty();
        for (auto &c : s.w) all = all && !c.busy;
        if (all) break;
    }
    return order;
}

}  // namespace

int main(int argc, char **argv)
{
    const int streams = argc > 1 ? atoi(argv[1]) : 200;
    std::mt19937_64 rng(20221203);
    std::uniform_real_distribution<double> U(0.0, 1.0);

    // 1. everything fits: first come, first served
    {
        Sim s{1000};
        for (int j = 0; j < 12; ++j) s.jobs.push_back({Need{5, 5, 5}, 3, 0});
        const auto order = run(s, 10, 1000);
        CHECK((int)order.size() == 12, "%zu of 12 jobs dispatched", order.size());
        for (size_t k = 0; k < order.size(); ++k) CHECK(order[k] == (int)k, "job %d dispatched at place %zu", order[k], k);
    }
    // 2. a large head that does not fit beside a running job is passed by a
    //    small one, then runs once the budget frees up
    {
        Sim s{100};
        s.jobs.push_back({Need{30, 30, 0}, 50, 0});   // runs first
        s.jobs.push_back({Need{40, 40, 0}, 5, 1});    // head: 60 + 80 > 100
        s.jobs.push_back({Need{5, 5, 0}, 5, 1});      // fits beside the first
        const auto order = run(s, 1000, 1000);
        CHECK(order.size() == 3 && order[0] == 0 && order[1] == 2 && order[2] == 1, "order %d %d %d",
              order.size() > 0 ? order[0] : -1, order.size() > 1 ? order[1] : -1, order.size() > 2 ? order[2] : -1);
        CHECK(s.jobs[1].dispatched >= 50, "the head ran at step %d, before the first job ended", s.jobs[1].dispatched);
    }
    // 3. the same with a short wait: once the head starves nobody passes it
    {
        Sim s{100};
        s.jobs.push_back({Need{30, 30, 0}, 50, 0});
        s.jobs.push_back({Need{40, 40, 0}, 5, 1});
        for (int j = 0; j < 5; ++j) s.jobs.push_back({Need{5, 5, 0}, 5, 10 + j});   // arrive after the wait
        const auto order = run(s, 3, 1000);
        CHECK(order.size() == 7 && order[1] == 1, "a starving head was passed (second dispatch: job %d)",
              order.size() > 1 ? order[1] : -1);
    }
    // 4. idle workspaces are released when they are in the way
    {
        Sim s{100};
        for (int j = 0; j < 4; ++j) s.jobs.push_back({Need{20, 0, 0}, 2, 0});   // four workspaces of 20
        s.jobs.push_back({Need{0, 90, 0}, 2, 10});                               // needs them gone
        const auto order = run(s, 1000, 1000);
        CHECK(order.size() == 5 && s.releases >= 1, "%zu dispatched, %d releases", order.size(), s.releases);
    }
    // 5. seeded random streams: budget, starvation bound and completion
    int total = 0;
    for (int it = 0; it < streams; ++it) {
        const size_t budget = 200 + (size_t)(U(rng) * 800);
        Sim s{budget};
        s.rng.seed(it + 1);
        s.p_finish_in_release = U(rng) * 0.5;
        s.p_withdraw_in_release = U(rng) * 0.2;
        const int n = 20 + (int)(U(rng) * 60);
        int t = 0;
        for (int j = 0; j < n; ++j) {
            Job jb;
            const double big = U(rng) < 0.15 ? 0.9 : 0.3;   // some jobs need most of the budget
            for (int b = 0; b < kBuf; ++b) jb.need[b] = (size_t)(U(rng) * big * budget / kBuf);
            jb.duration = 1 + (int)(U(rng) * 20);
            t += (int)(U(rng) * 4);
            jb.arrival = t;
            s.jobs.push_back(jb);
        }
        const int head_wait = 1 + (int)(U(rng) * 30);
        run(s, head_wait, 100000);
        for (size_t j = 0; j < s.jobs.size(); ++j) {
            const Job &jb = s.jobs[j];
            CHECK(jb.withdrawn || jb.dispatched >= 0, "stream %d: job %zu (needs %zu of %zu) never ran", it, j,
                  sum(jb.need), budget);
            CHECK(jb.dispatched < 0 || jb.dispatched >= jb.arrival, "stream %d: job %zu ran before it arrived", it, j);
        }
        total += s.dispatches;
    }
    printf("scheduler policy: %d random streams, %d dispatches, %d violations\n", streams, total, fails);
    return fails ? 1 : 0;
}
