// Threaded stress driver of the serving scheduler core (serve.h), for the
// thread sanitizer: several submitter threads queue requests while one thread
// runs the scheduling loop against a device whose slots finish after a short
// real-time delay, and another thread polls completions, as the library's
// server does. Prints "ok <completions>" and exits 0 when every request
// completed exactly once.
//
// usage: serve_threads submitters requests_per_submitter slots max_batch
#include "serve.h"

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

using hiz::serve::Done;
using hiz::serve::Req;

struct TimedDevice {
    struct Slot {
        double t_end = 0;
        size_t n = 0;
    };
    std::vector<Slot> slots;
    uint64_t capacity;
    explicit TimedDevice(int n, uint64_t cap) : slots(n), capacity(cap) {}
    double now()
    {
        using namespace std::chrono;
        return duration<double>(steady_clock::now().time_since_epoch()).count();
    }
    bool submit(int s, const std::vector<const Req *> &b)
    {
        uint64_t need = 0;
        for (const Req *r : b)
            need += r->need;
        slots[s].n = b.size();
        if (need > capacity)
            return false;
        slots[s].t_end = now() + 20e-6 * (double)b.size();
        return true;
    }
    bool ready(int s) { return now() >= slots[s].t_end; }
    void finish(int s, std::vector<Done> &out)
    {
        out.assign(slots[s].n, Done());
        for (Done &d : out)
            d.status = 0;
    }
};

int main(int argc, char **argv)
{
    const int nsub = argc > 1 ? atoi(argv[1]) : 4;
    const int per = argc > 2 ? atoi(argv[2]) : 200;
    const int slots = argc > 3 ? atoi(argv[3]) : 4;
    const int max_batch = argc > 4 ? atoi(argv[4]) : 8;
    TimedDevice dev(slots, 1000);
    hiz::serve::Policy pol;
    pol.max_batch = max_batch;
    pol.slot_capacity = 1000;
    hiz::serve::Scheduler<TimedDevice> sched(dev, slots, pol);
    const int total = nsub * per;
    std::atomic<int> submitted{0};
    std::vector<std::thread> subs;
    for (int t = 0; t < nsub; t++)
        subs.emplace_back([&, t]() {
            for (int i = 0; i < per; i++) {
                Req r;
                r.id = (uint64_t)(t * per + i);
                r.op = (i % 5 == 0) ? 1 : 0;
                r.need = (uint64_t)(10 + (i * 37 + t) % 200);
                sched.submit(r);
                submitted++;
                if (i % 16 == 0)
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
        });
    std::vector<int> seen(total, 0);
    std::atomic<bool> stop{false};
    std::thread poller([&]() {
        Done buf[64];
        int got = 0;
        while (got < total) {
            const size_t n = sched.poll(buf, 64);
            for (size_t k = 0; k < n; k++)
                seen[buf[k].id]++;
            got += (int)n;
            if (!n)
                std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        stop = true;
    });
    while (!stop) {
        if (!sched.step())
            std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
    for (std::thread &t : subs)
        t.join();
    poller.join();
    for (int i = 0; i < total; i++)
        if (seen[i] != 1) {
            printf("request %d completed %d times\n", i, seen[i]);
            return 1;
        }
    printf("ok %d\n", total);
    return 0;
}
