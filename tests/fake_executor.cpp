// A simulated executor for the server's admission control (fpo_sched.h),
// with no GPU: requests arrive at given times with a workspace size, a build
// duration and a hold time (how long the client keeps the result, and so the
// memory, after the build ends); some are cancelled while they wait.  The
// simulation admits through fpo::Admission exactly as the server does, checks
// its invariants after every event, and prints one line per event:
//
//   submit <id> <t>          admit <id> <t> <offset> <bytes>
//   finish <id> <t>          release <id> <t>          cancel <id> <t> <0|1>
//   summary <admitted> <cancelled> <max_running> <max_used> <end_time>
//
// Usage: fake_executor <seed> <requests> <slots> <budget> [cancel_every]
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <cmath>
#include <queue>
#include <random>
#include <vector>

#include "../paper_2302_05002_amd/csrc/fpo_sched.h"

namespace {

struct Req {
    double arrival, duration, hold;
    uint64_t bytes;
    bool cancel;          // cancelled 0.3 time units after its arrival, if it is still waiting then
    uint64_t off = 0;
    bool admitted = false, done = false;
};

enum Kind { SUBMIT, FINISH, RELEASE, CANCEL };

struct Ev {
    double t;
    int kind, id;
    uint64_t seq;
    bool operator>(const Ev &o) const { return t != o.t ? t > o.t : seq > o.seq; }
};

void check(const fpo::Admission<int> &adm, uint64_t budget)
{
    const auto &A = adm.arena();
    uint64_t free_sum = 0, last_end = 0;
    bool first = true;
    for (auto &b : A.free_blocks()) {
        if (b.second == 0) { fprintf(stderr, "empty free block\n"); abort(); }
        if (!first && b.first <= last_end) { fprintf(stderr, "free blocks overlap or touch\n"); abort(); }
        if (b.first + b.second > budget) { fprintf(stderr, "free block beyond the arena\n"); abort(); }
        last_end = b.first + b.second;
        first = false;
        free_sum += b.second;
    }
    if (free_sum + A.used() != budget) { fprintf(stderr, "free + used != budget\n"); abort(); }
    if (adm.running() > adm.slots()) { fprintf(stderr, "more builds than slots\n"); abort(); }
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc < 5) {
        fprintf(stderr, "usage: %s seed requests slots budget [cancel_every]\n", argv[0]);
        return 2;
    }
    const uint64_t seed = strtoull(argv[1], nullptr, 10);
    const int nreq = atoi(argv[2]);
    const uint32_t slots = (uint32_t)atoi(argv[3]);
    const uint64_t budget = strtoull(argv[4], nullptr, 10);
    const int cancel_every = argc > 5 ? atoi(argv[5]) : 0;
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    std::vector<Req> R(nreq);
    double t = 0.0;
    for (int i = 0; i < nreq; ++i) {
        t += -std::log(1.0 - u01(rng)) * 1.0;                        // Poisson arrivals, mean gap 1
        R[i].arrival = t;
        // sizes log-uniform from budget/1000 to the whole budget
        const double lo = std::log((double)budget / 1000.0), hi = std::log((double)budget);
        R[i].bytes = (uint64_t)std::exp(lo + (hi - lo) * u01(rng));
        if (R[i].bytes == 0) R[i].bytes = 1;
        if (R[i].bytes > budget) R[i].bytes = budget;
        R[i].duration = 0.5 + 4.0 * u01(rng);
        R[i].hold = u01(rng) < 0.3 ? 10.0 * u01(rng) : 0.0;
        R[i].cancel = cancel_every > 0 && i % cancel_every == cancel_every - 1;
    }
    fpo::Admission<int> adm(budget, slots);
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> q;
    uint64_t seq = 0;
    for (int i = 0; i < nreq; ++i) q.push({R[i].arrival, SUBMIT, i, seq++});
    int admitted = 0, cancelled = 0;
    uint32_t max_running = 0;
    uint64_t max_used = 0;
    double now = 0.0;
    auto start = [&](int id, uint64_t off) {
        R[id].off = off;
        R[id].admitted = true;
        ++admitted;
        printf("admit %d %.6f %llu %llu\n", id, now, (unsigned long long)off, (unsigned long long)R[id].bytes);
        q.push({now + R[id].duration, FINISH, id, seq++});
    };
    while (!q.empty()) {
        const Ev e = q.top();
        q.pop();
        now = e.t;
        Req &r = R[e.id];
        switch (e.kind) {
        case SUBMIT:
            printf("submit %d %.6f\n", e.id, now);
            adm.submit(e.id, r.bytes);
            if (r.cancel) q.push({now + 0.3, CANCEL, e.id, seq++});
            break;
        case CANCEL: {
            const bool removed = adm.remove_waiting(e.id);
            if (removed) ++cancelled;
            if (removed == r.admitted) { fprintf(stderr, "cancel of %d disagrees with admission\n", e.id); abort(); }
            printf("cancel %d %.6f %d\n", e.id, now, removed ? 1 : 0);
            break;
        }
        case FINISH:
            printf("finish %d %.6f\n", e.id, now);
            adm.finished();
            q.push({now + r.hold, RELEASE, e.id, seq++});
            break;
        case RELEASE:
            printf("release %d %.6f\n", e.id, now);
            adm.release(r.off, r.bytes);
            r.done = true;
            break;
        }
        adm.admit(start);
        check(adm, budget);
        if (adm.running() > max_running) max_running = adm.running();
        if (adm.arena().used() > max_used) max_used = adm.arena().used();
    }
    if (adm.waiting() != 0 || adm.running() != 0 || adm.arena().used() != 0) {
        fprintf(stderr, "the simulation ended with work left\n");
        abort();
    }
    printf("summary %d %d %u %llu %.6f\n", admitted, cancelled, max_running, (unsigned long long)max_used, now);
    return 0;
}
