// CPU mock device for the serving scheduler core (serve.h): a simulated clock
// and slots whose batches finish after a modelled service time. Replays a
// seeded Poisson trace and prints one JSON object with every completion and
// every batch the scheduler formed, for tests/test_serve_sched.py to check.
//
// usage: serve_mock seed rate_per_s n_requests slots max_batch capacity
//                   p_decompress oversize_every
#include "serve.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using hiz::serve::Done;
using hiz::serve::Req;

struct MockDevice {
    double clock = 0.0;
    struct Slot {
        bool busy = false;
        double t_end = 0.0;
        std::vector<uint64_t> ids;
        std::vector<uint64_t> need;
        int op = 0;
        bool rejected = false;
    };
    std::vector<Slot> slots;
    uint64_t capacity = 0;
    struct BatchLog {
        int slot, op;
        double t_start, t_end;
        uint64_t need;
        std::vector<uint64_t> ids;
    };
    std::vector<BatchLog> log;

    double now() { return clock; }

    bool submit(int s, const std::vector<const Req *> &b)
    {
        Slot &sl = slots[s];
        sl.ids.clear();
        sl.need.clear();
        uint64_t need = 0;
        for (const Req *r : b) {
            sl.ids.push_back(r->id);
            sl.need.push_back(r->need);
            need += r->need;
        }
        sl.op = b[0]->op;
        if (need > capacity) {
            sl.rejected = true;
            return false;
        }
        sl.rejected = false;
        sl.busy = true;
        // service model: launch overhead plus bytes at a fixed rate
        sl.t_end = clock + 2e-4 + (double)need / 1e11;
        log.push_back({s, sl.op, clock, sl.t_end, need, sl.ids});
        return true;
    }
    bool ready(int s) { return slots[s].busy && clock >= slots[s].t_end; }
    void finish(int s, std::vector<Done> &out)
    {
        Slot &sl = slots[s];
        out.assign(sl.ids.size(), Done());
        for (size_t i = 0; i < sl.ids.size(); i++) {
            out[i].status = sl.rejected ? 5 : 0;
            out[i].size = sl.need[i];
        }
        sl.busy = false;
    }
    double next_event() const
    {
        double t = INFINITY;
        for (const Slot &sl : slots)
            if (sl.busy && sl.t_end < t)
                t = sl.t_end;
        return t;
    }
};

int main(int argc, char **argv)
{
    if (argc != 9) {
        fprintf(stderr, "usage: serve_mock seed rate n slots max_batch capacity p_dec oversize\n");
        return 2;
    }
    const unsigned seed = (unsigned)atoi(argv[1]);
    const double rate = atof(argv[2]);
    const int n = atoi(argv[3]);
    const int slots = atoi(argv[4]);
    hiz::serve::Policy pol;
    pol.max_batch = atoi(argv[5]);
    pol.slot_capacity = strtoull(argv[6], nullptr, 10);
    const double p_dec = atof(argv[7]);
    const int oversize_every = atoi(argv[8]);

    MockDevice dev;
    dev.slots.resize(slots);
    dev.capacity = pol.slot_capacity;
    hiz::serve::Scheduler<MockDevice> sched(dev, slots, pol);

    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(rate);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    std::vector<double> arrive(n);
    std::vector<Req> reqs(n);
    double t = 0.0;
    for (int i = 0; i < n; i++) {
        t += gap(rng);
        arrive[i] = t;
        Req r;
        r.id = (uint64_t)i;
        r.op = u01(rng) < p_dec ? 1 : 0;
        // sizes log-uniform between 64^3 and 512^3 points
        const double lo = std::log(262144.0), hi = std::log(134217728.0);
        r.need = (uint64_t)std::exp(lo + (hi - lo) * u01(rng));
        if (oversize_every > 0 && i % oversize_every == oversize_every - 1)
            r.need = pol.slot_capacity + 1;
        r.t_submit = t;
        reqs[i] = r;
    }
    int next = 0;
    std::vector<Done> done;
    while ((int)done.size() < n) {
        // deliver due arrivals, then run the loop until it makes no progress
        while (next < n && arrive[next] <= dev.clock)
            sched.submit(reqs[next++]);
        sched.step();
        Done buf[64];
        size_t k;
        while ((k = sched.poll(buf, 64)) > 0)
            for (size_t i = 0; i < k; i++)
                done.push_back(buf[i]);
        // advance the simulated clock to the next event
        double tn = dev.next_event();
        if (next < n && arrive[next] < tn)
            tn = arrive[next];
        if (tn == INFINITY)
            break;
        if (tn > dev.clock)
            dev.clock = tn;
    }
    printf("{\"completions\": [");
    for (size_t i = 0; i < done.size(); i++)
        printf("%s[%llu, %d, %llu, %.9f, %.9f, %.9f, %d, %d]", i ? ", " : "",
               (unsigned long long)done[i].id, done[i].status, (unsigned long long)done[i].size,
               done[i].t_submit, done[i].t_start, done[i].t_done, done[i].batch_size,
               done[i].slot);
    printf("], \"ops\": [");
    for (int i = 0; i < n; i++)
        printf("%s%d", i ? ", " : "", reqs[i].op);
    printf("], \"batches\": [");
    for (size_t i = 0; i < dev.log.size(); i++) {
        const MockDevice::BatchLog &b = dev.log[i];
        printf("%s{\"slot\": %d, \"op\": %d, \"t0\": %.9f, \"t1\": %.9f, \"need\": %llu, \"ids\": [",
               i ? ", " : "", b.slot, b.op, b.t_start, b.t_end, (unsigned long long)b.need);
        for (size_t j = 0; j < b.ids.size(); j++)
            printf("%s%llu", j ? ", " : "", (unsigned long long)b.ids[j]);
        printf("]}");
    }
    printf("], \"max_running\": %d, \"submitted\": %llu, \"n\": %d}\n", sched.max_running(),
           (unsigned long long)sched.submitted(), n);
    return 0;
}
