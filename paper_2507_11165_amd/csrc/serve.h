// Scheduler core of the hiz serving loop: continuous batching of compression
// and decompression requests over a fixed set of device slots.
//
// A request waits in a FIFO queue until a slot is free. A free slot takes the
// oldest waiting request and, behind it, further requests of the same kind
// (compress or decompress) in arrival order, as long as the batch stays within
// the slot's workspace (device memory admission) and the batch-size limit; a
// same-kind request that does not fit ends the batch, so nothing is starved.
// The slot runs the batch asynchronously; requests that arrive meanwhile are
// batched onto the next free slot, so work from several batches overlaps on
// the device. A completed batch releases its slot and reports one completion
// per request with its submit, start and end times.
//
// The core is independent of HIP: it drives any Device with
//   bool submit(int slot, const std::vector<const Req *> &batch)
//   bool ready(int slot)                           (never blocks)
//   void finish(int slot, std::vector<Done> &out)  (one Done per request)
//   double now()                                   (seconds, monotonic)
// which lets the same loop run against the GPU and against a CPU mock.
#pragma once

#include <atomic>
#include <cstdint>
#include <deque>
#include <mutex>
#include <vector>

namespace hiz {
namespace serve {

struct Req {
    uint64_t id = 0;     // caller tag, returned in the completion
    int op = 0;          // 0 compress, 1 decompress
    uint64_t need = 0;   // device workspace bytes the request needs
    double t_submit = 0; // when the request entered the queue
    uint64_t payload = 0; // device-side argument block index (opaque to the core)
};

struct Done {
    uint64_t id = 0;
    int status = 0;
    uint64_t size = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int batch_size = 0;
    int slot = -1;
};

struct Policy {
    int max_batch = 32;          // requests per batch
    uint64_t slot_capacity = 0;  // workspace bytes per slot
};

// Indices (into q) of the batch a free slot takes now; empty if q is empty.
// A request that can never fit (need above the slot capacity) is returned
// alone, so that the device rejects it and it does not block the queue.
inline std::vector<size_t> form_batch(const std::deque<Req> &q, const Policy &p)
{
    std::vector<size_t> pick;
    if (q.empty())
        return pick;
    const int op = q.front().op;
    uint64_t used = 0;
    for (size_t i = 0; i < q.size() && (int)pick.size() < p.max_batch; i++) {
        const Req &r = q[i];
        if (r.op != op)
            continue; // other kind: waits for a batch of its own, keeps its order
        if (pick.empty() && r.need > p.slot_capacity) {
            pick.push_back(i);
            break;
        }
        if (used + r.need > p.slot_capacity)
            break;
        used += r.need;
        pick.push_back(i);
    }
    return pick;
}

// The scheduling loop state; step() advances it once without blocking.
template <class Device> class Scheduler {
  public:
    Scheduler(Device &dev, int slots, const Policy &p)
        : dev_(dev), policy_(p), busy_(slots, false), batch_(slots), started_(slots)
    {
    }

    // Thread-safe: queue one request (t_submit taken now if it is 0).
    void submit(Req r)
    {
        if (r.t_submit == 0)
            r.t_submit = dev_.now();
        std::lock_guard<std::mutex> g(mu_);
        queue_.push_back(r);
        submitted_++;
    }

    // Collect finished batches, then start batches on free slots. Returns the
    // number of completions produced.
    size_t step()
    {
        size_t made = 0;
        std::vector<Done> fresh;
        for (int s = 0; s < (int)busy_.size(); s++) {
            if (!busy_[s] || !dev_.ready(s))
                continue;
            std::vector<Done> out;
            dev_.finish(s, out);
            const double t = dev_.now();
            for (size_t k = 0; k < out.size() && k < batch_[s].size(); k++) {
                Done d = out[k];
                d.id = batch_[s][k].id;
                d.t_submit = batch_[s][k].t_submit;
                d.t_start = started_[s];
                d.t_done = t;
                d.batch_size = (int)batch_[s].size();
                d.slot = s;
                fresh.push_back(d);
                made++;
            }
            batch_[s].clear();
            busy_[s] = false;
            running_--;
        }
        for (int s = 0; s < (int)busy_.size(); s++) {
            if (busy_[s])
                continue;
            std::vector<Req> take;
            {
                std::lock_guard<std::mutex> g(mu_);
                const std::vector<size_t> pick = form_batch(queue_, policy_);
                if (pick.empty())
                    break;
                for (size_t i : pick)
                    take.push_back(queue_[i]);
                // erase picked entries, keeping the others in order
                std::deque<Req> rest;
                size_t j = 0;
                for (size_t i = 0; i < queue_.size(); i++) {
                    if (j < pick.size() && pick[j] == i) {
                        j++;
                        continue;
                    }
                    rest.push_back(queue_[i]);
                }
                queue_.swap(rest);
            }
            batch_[s] = take;
            std::vector<const Req *> ptrs;
            for (const Req &r : batch_[s])
                ptrs.push_back(&r);
            started_[s] = dev_.now();
            if (dev_.submit(s, ptrs)) {
                busy_[s] = true;
                running_++;
                batches_++;
                if (running_ > max_running_)
                    max_running_ = running_.load();
            } else {
                // the device rejected the batch as a whole: complete it with its error
                std::vector<Done> out;
                dev_.finish(s, out);
                const double t = dev_.now();
                for (size_t k = 0; k < batch_[s].size(); k++) {
                    Done d = k < out.size() ? out[k] : Done();
                    d.id = batch_[s][k].id;
                    d.t_submit = batch_[s][k].t_submit;
                    d.t_start = started_[s];
                    d.t_done = t;
                    d.batch_size = (int)batch_[s].size();
                    d.slot = s;
                    fresh.push_back(d);
                    made++;
                }
                batch_[s].clear();
            }
        }
        if (!fresh.empty()) {
            std::lock_guard<std::mutex> g(done_mu_);
            for (const Done &d : fresh)
                done_.push_back(d);
            produced_ += fresh.size();
        }
        return made;
    }

    // Move out up to max completions (oldest first).
    size_t poll(Done *out, size_t max)
    {
        std::lock_guard<std::mutex> g(done_mu_);
        size_t n = 0;
        while (n < max && !done_.empty()) {
            out[n++] = done_.front();
            done_.pop_front();
        }
        delivered_ += n;
        return n;
    }

    // Every submitted request has produced its completion.
    bool drained() const { return produced_ == submitted_; }
    size_t waiting()
    {
        std::lock_guard<std::mutex> g(mu_);
        return queue_.size();
    }
    int running() const { return running_; }
    int max_running() const { return max_running_; }
    uint64_t batches() const { return batches_; }
    uint64_t submitted() const { return submitted_; }
    uint64_t delivered() const { return delivered_; }
    uint64_t produced() const { return produced_; }
    size_t pending_completions()
    {
        std::lock_guard<std::mutex> g(done_mu_);
        return done_.size();
    }

  private:
    Device &dev_;
    Policy policy_;
    std::mutex mu_, done_mu_;
    std::deque<Req> queue_;
    std::vector<bool> busy_;
    std::vector<std::vector<Req>> batch_;
    std::vector<double> started_;
    std::deque<Done> done_;
    std::atomic<int> running_{0}, max_running_{0};
    std::atomic<uint64_t> batches_{0}, submitted_{0}, delivered_{0}, produced_{0};
};

} // namespace serve
} // namespace hiz
