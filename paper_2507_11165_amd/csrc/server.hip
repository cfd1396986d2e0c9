// Serving loop of the hiz library: continuous batching of compression and
// decompression requests on one device (the C ABI hiz_server_* of hiz.h).
//
// The server owns `slots` contexts, each with its own non-blocking stream and
// a workspace sized up front to an equal share of the memory budget, so no
// allocation happens while requests are served and codebooks, tables and code
// buffers stay resident. A scheduler thread runs the loop of serve.h: a free
// slot takes the next batch of waiting requests that fits its workspace and
// enqueues it with the batched submit entry points, followed on the slot's
// stream by a host callback that wakes the loop when the batch is done; the
// loop also wakes on every submit and never waits for the device itself, so
// batches on different slots overlap on the GPU. Each slot's pinned staging is
// reserved for max_batch requests at creation, and a decompression request's
// header bytes are read on the submitting thread, so a batch submit never
// synchronizes.
#include "hiz.h"
#include "hiz_internal.h"
#include "serve.h"

#include <chrono>
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

double clock_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Wakes the scheduling loop: on a submit, and from a stream host callback when
// a batch completes on the device.
struct Waker {
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    bool kick = false;

    void wake()
    {
        {
            std::lock_guard<std::mutex> g(mu);
            kick = true;
        }
        cv.notify_one();
    }
};

void wake_from_stream(void *w) { static_cast<Waker *>(w)->wake(); }

// A request's arguments, with the header bytes of a stream to decompress.
struct Pending {
    hiz_request r;
    uint8_t hdr[hiz::kOffChunks];
};

// The GPU side of the scheduler: batched submits on per-slot contexts.
struct GpuDevice {
    struct Slot {
        hiz_ctx *ctx = nullptr;
        hipStream_t stream = nullptr;
        int n = 0;
        hiz_status submit_rc = HIZ_OK;
        std::vector<uint64_t> sizes, dims;
        std::vector<hiz_status> status;
    };
    int device = 0;
    uint64_t capacity = 0; // workspace bytes of each slot
    bool have_params = false;
    hiz_params params;
    std::vector<Slot> slots;
    std::mutex args_mu;
    std::unordered_map<uint64_t, Pending> args; // payload key -> request
    Waker *waker = nullptr;

    double now() { return clock_s(); }

    bool submit(int s, const std::vector<const hiz::serve::Req *> &batch)
    {
        Slot &sl = slots[s];
        const int n = (int)batch.size();
        sl.n = n;
        sl.sizes.assign(n, 0);
        sl.dims.assign(3 * (size_t)n, 0);
        sl.status.assign(n, HIZ_OK);
        uint64_t need = 0;
        for (const hiz::serve::Req *q : batch)
            need += q->need;
        if (need > capacity) {
            // larger than a slot's workspace: rejected without touching the device
            std::lock_guard<std::mutex> g(args_mu);
            for (const hiz::serve::Req *q : batch)
                args.erase(q->payload);
            sl.submit_rc = HIZ_ERR_NOMEM;
            return false;
        }
        std::vector<hiz_request> rq(n);
        std::vector<uint8_t> hdrs;
        {
            std::lock_guard<std::mutex> g(args_mu);
            if (batch[0]->op == HIZ_OP_DECOMPRESS)
                hdrs.resize((size_t)hiz::kOffChunks * n);
            for (int i = 0; i < n; i++) {
                const Pending &p = args[batch[i]->payload];
                rq[i] = p.r;
                if (!hdrs.empty())
                    memcpy(&hdrs[(size_t)hiz::kOffChunks * i], p.hdr, hiz::kOffChunks);
                args.erase(batch[i]->payload);
            }
        }
        hiz_status rc;
        hipSetDevice(device);
        if (rq[0].op == HIZ_OP_COMPRESS) {
            std::vector<const float *> f(n);
            std::vector<uint64_t> dims(3 * (size_t)n);
            std::vector<int> modes(n);
            std::vector<double> ebs(n);
            std::vector<void *> outs(n);
            std::vector<uint64_t> caps(n);
            for (int i = 0; i < n; i++) {
                f[i] = static_cast<const float *>(rq[i].d_in);
                memcpy(&dims[3 * (size_t)i], rq[i].dims, sizeof(rq[i].dims));
                modes[i] = rq[i].mode;
                ebs[i] = rq[i].eb;
                outs[i] = rq[i].d_out;
                caps[i] = rq[i].out_cap;
            }
            rc = hiz_compress_batch_submit(sl.ctx, n, f.data(), dims.data(), modes.data(),
                                           ebs.data(), have_params ? &params : nullptr,
                                           outs.data(), caps.data(),
                                           reinterpret_cast<hiz_stream_t>(sl.stream));
        } else {
            std::vector<const void *> ins(n);
            std::vector<uint64_t> in_sizes(n);
            std::vector<float *> outs(n);
            std::vector<uint64_t> caps(n);
            for (int i = 0; i < n; i++) {
                ins[i] = rq[i].d_in;
                in_sizes[i] = rq[i].in_size;
                outs[i] = static_cast<float *>(rq[i].d_out);
                caps[i] = rq[i].out_cap;
            }
            rc = hiz::ctx_decompress_submit_hdrs(sl.ctx, n, ins.data(), in_sizes.data(),
                                                 outs.data(), caps.data(), sl.stream,
                                                 hdrs.data());
        }
        sl.submit_rc = rc;
        if (rc == HIZ_OK && waker)
            hipLaunchHostFunc(sl.stream, wake_from_stream, waker);
        return rc == HIZ_OK;
    }

    bool ready(int s) { return hiz_batch_ready(slots[s].ctx) != 0; }

    void finish(int s, std::vector<hiz::serve::Done> &out)
    {
        Slot &sl = slots[s];
        out.assign(sl.n, hiz::serve::Done());
        if (sl.submit_rc != HIZ_OK) {
            for (int i = 0; i < sl.n; i++)
                out[i].status = sl.submit_rc;
            return;
        }
        hiz_batch_finish(sl.ctx, sl.sizes.data(), sl.dims.data(), sl.status.data());
        for (int i = 0; i < sl.n; i++) {
            out[i].status = sl.status[i];
            out[i].size = sl.sizes[i];
        }
    }
};

} // namespace

struct hiz_server {
    GpuDevice dev;
    hiz::serve::Policy policy;
    hiz::serve::Scheduler<GpuDevice> *sched = nullptr;
    std::thread worker;
    Waker waker;
    uint64_t next_key = 1;
    std::string err;
    // header reads of decompression requests (on the submitting thread)
    std::mutex hdr_mu;
    hipStream_t hdr_stream = nullptr;
    uint8_t *hdr_pinned = nullptr;
};

namespace {

void serve_loop(hiz_server *S)
{
    hipSetDevice(S->dev.device);
    Waker &W = S->waker;
    while (true) {
        {
            std::lock_guard<std::mutex> g(W.mu);
            W.kick = false;
        }
        const size_t made = S->sched->step();
        std::unique_lock<std::mutex> lk(W.mu);
        if (S->sched->drained() && W.stop)
            break;
        if (made)
            continue;
        // nothing changed: sleep until a submit or a batch completion wakes
        // the loop (the timeout only guards against a lost wake-up)
        W.cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return W.kick || W.stop; });
    }
}

} // namespace

extern "C" {

hiz_status hiz_server_create(int device, int slots, uint64_t mem_budget, int max_batch,
                             const hiz_params *params, hiz_server **out)
{
    if (!out || slots < 1 || slots > 16 || max_batch < 1 || max_batch > 4096)
        return HIZ_ERR_ARG;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) {
        hipGetLastError();
        return HIZ_ERR_ARG;
    }
    if (mem_budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
            return HIZ_ERR_HIP;
        mem_budget = free_b / 4; // a quarter of what is free now
    }
    hiz_server *S = new (std::nothrow) hiz_server();
    if (!S)
        return HIZ_ERR_NOMEM;
    S->dev.device = device;
    if (params) {
        S->dev.have_params = true;
        S->dev.params = *params;
    }
    S->policy.max_batch = max_batch;
    // the context grows its workspace by an eighth plus 1 MiB over a request
    S->policy.slot_capacity = (mem_budget / (uint64_t)slots) * 8 / 9;
    S->dev.capacity = S->policy.slot_capacity;
    S->dev.slots.resize(slots);
    for (int s = 0; s < slots; s++) {
        GpuDevice::Slot &sl = S->dev.slots[s];
        hiz_status rc = hiz_create(device, S->policy.slot_capacity, &sl.ctx);
        if (rc == HIZ_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
            rc = HIZ_ERR_HIP;
        if (rc != HIZ_OK) {
            for (GpuDevice::Slot &o : S->dev.slots) {
                if (o.stream)
                    hipStreamDestroy(o.stream);
                if (o.ctx)
                    hiz_destroy(o.ctx);
            }
            delete S;
            return rc;
        }
    }
    hiz_status rc = HIZ_OK;
    for (GpuDevice::Slot &sl : S->dev.slots)
        if (rc == HIZ_OK)
            rc = hiz::ctx_reserve_pinned(sl.ctx, max_batch);
    if (rc == HIZ_OK && hipStreamCreateWithFlags(&S->hdr_stream, hipStreamNonBlocking) != hipSuccess)
        rc = HIZ_ERR_HIP;
    if (rc == HIZ_OK && hipHostMalloc((void **)&S->hdr_pinned, hiz::kOffChunks,
                                      hipHostMallocDefault) != hipSuccess)
        rc = HIZ_ERR_NOMEM;
    if (rc != HIZ_OK) {
        hipGetLastError();
        for (GpuDevice::Slot &o : S->dev.slots) {
            hipStreamDestroy(o.stream);
            hiz_destroy(o.ctx);
        }
        if (S->hdr_stream)
            hipStreamDestroy(S->hdr_stream);
        delete S;
        return rc;
    }
    S->dev.waker = &S->waker;
    S->sched = new hiz::serve::Scheduler<GpuDevice>(S->dev, slots, S->policy);
    S->worker = std::thread(serve_loop, S);
    *out = S;
    return HIZ_OK;
}

hiz_status hiz_server_submit(hiz_server *S, const hiz_request *r)
{
    if (!S || !r || (r->op != HIZ_OP_COMPRESS && r->op != HIZ_OP_DECOMPRESS) || !r->d_in ||
        !r->d_out)
        return HIZ_ERR_ARG;
    uint64_t need;
    if (r->op == HIZ_OP_COMPRESS) {
        uint64_t n_elems = 1;
        for (int k = 0; k < 3; k++) {
            if (r->dims[k] == 0 || n_elems > (1ull << 40) / r->dims[k])
                return HIZ_ERR_ARG;
            n_elems *= r->dims[k];
        }
        need = hiz_workspace_bound(r->dims);
    } else {
        // the field the stream decodes into bounds its size; its shape is in
        // the stream's header on the device, so the bound covers every shape
        if (r->out_cap == 0)
            return HIZ_ERR_ARG;
        need = hiz::workspace_bound_points(r->out_cap);
    }
    if (need == 0)
        return HIZ_ERR_ARG;
    Pending p;
    p.r = *r;
    memset(p.hdr, 0, sizeof(p.hdr));
    if (r->op == HIZ_OP_DECOMPRESS) {
        // the stream's header and code lengths, read here so that the batch
        // submit on the scheduler thread never waits for the device
        const size_t nh = (size_t)std::min<uint64_t>(r->in_size, hiz::kOffChunks);
        std::lock_guard<std::mutex> g(S->hdr_mu);
        hipSetDevice(S->dev.device);
        if (hipMemcpyAsync(S->hdr_pinned, r->d_in, nh, hipMemcpyDeviceToHost, S->hdr_stream) !=
                hipSuccess ||
            hipStreamSynchronize(S->hdr_stream) != hipSuccess) {
            hipGetLastError();
            return HIZ_ERR_HIP;
        }
        memcpy(p.hdr, S->hdr_pinned, nh);
    }
    hiz::serve::Req q;
    q.id = r->id;
    q.op = r->op;
    q.need = need;
    {
        std::lock_guard<std::mutex> g(S->dev.args_mu);
        q.payload = S->next_key++;
        S->dev.args[q.payload] = p;
    }
    S->sched->submit(q);
    S->waker.wake();
    return HIZ_OK;
}

int hiz_server_poll(hiz_server *S, hiz_completion *out, int max)
{
    if (!S || !out || max <= 0)
        return 0;
    std::vector<hiz::serve::Done> d(max);
    const size_t n = S->sched->poll(d.data(), (size_t)max);
    for (size_t i = 0; i < n; i++) {
        out[i].id = d[i].id;
        out[i].status = (hiz_status)d[i].status;
        out[i].size = d[i].size;
        out[i].t_submit = d[i].t_submit;
        out[i].t_start = d[i].t_start;
        out[i].t_done = d[i].t_done;
        out[i].batch_size = d[i].batch_size;
        out[i].slot = d[i].slot;
    }
    return (int)n;
}

hiz_status hiz_server_drain(hiz_server *S, double timeout_s)
{
    if (!S)
        return HIZ_ERR_ARG;
    const double t_end = clock_s() + (timeout_s > 0 ? timeout_s : 1e30);
    while (!S->sched->drained()) {
        if (clock_s() > t_end)
            return HIZ_ERR_HIP;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return HIZ_OK;
}

void hiz_server_get_stats(hiz_server *S, hiz_server_stats *st)
{
    if (!S || !st)
        return;
    memset(st, 0, sizeof(*st));
    st->submitted = S->sched->submitted();
    st->completed = S->sched->produced();
    st->batches = S->sched->batches();
    st->max_running = S->sched->max_running();
    st->slots = (int)S->dev.slots.size();
    st->slot_capacity = S->policy.slot_capacity;
}

double hiz_server_clock(void) { return clock_s(); }

void hiz_server_destroy(hiz_server *S)
{
    if (!S)
        return;
    {
        std::lock_guard<std::mutex> g(S->waker.mu);
        S->waker.stop = true;
    }
    S->waker.cv.notify_one();
    // the loop finishes what was submitted before it stops
    if (S->worker.joinable())
        S->worker.join();
    delete S->sched;
    for (GpuDevice::Slot &sl : S->dev.slots) {
        if (sl.stream) {
            hipStreamSynchronize(sl.stream);
            hipStreamDestroy(sl.stream);
        }
        if (sl.ctx)
            hiz_destroy(sl.ctx);
    }
    if (S->hdr_stream)
        hipStreamDestroy(S->hdr_stream);
    if (S->hdr_pinned)
        hipHostFree(S->hdr_pinned);
    delete S;
}

} // extern "C"
