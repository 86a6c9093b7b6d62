// Served renders: a request queue drained by one worker thread into batches
// (declared in include/vtx.h, vtx_server_*).
//
// The paper's renderer draws one interactive view per frame; a server that
// renders the frames of many clients (each a session of consecutive frames of
// one resident molecule) gathers the requests that are waiting whenever the
// device can take more work and renders them as one batch, so many small
// views share each launch (continuous batching).  At most `max_inflight`
// batches are queued on the device at once: arrivals during a batch form the
// next one.  Completion is stamped by a host callback queued on the stream
// after each batch, so a request's latency runs from its submission to the
// moment its batch has finished on the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "vtx.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    vtx_job job;
    uint64_t ticket;
    double submit_s;
};

struct Batch;

}  // namespace

struct vtx_server {
    vtx_context* ctx = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    int32_t max_batch = 64;
    int32_t max_inflight = 2;
    std::mutex mu;
    std::condition_variable cv_work;     // requests arrived / stop
    std::condition_variable cv_done;     // a batch completed
    std::deque<Request> queue;
    std::vector<vtx_completion> done;    // completed, not yet polled
    uint64_t next_ticket = 1;
    uint64_t submitted = 0, completed = 0;
    int32_t inflight = 0;
    bool stop = false;
    std::thread worker;
    vtx_server_stats stats{};
};

namespace {

struct Batch {
    vtx_server* srv;
    std::vector<Request> reqs;
    double launch_s;
};

// Runs on the runtime's callback thread once the batch's work has finished
// on the device: stamps and files the completions (no HIP calls here).
void batch_done(void* p) {
    Batch* b = static_cast<Batch*>(p);
    const double t = now_s();
    vtx_server* s = b->srv;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (const Request& r : b->reqs) {
            vtx_completion c;
            std::memset(&c, 0, sizeof(c));
            c.ticket = r.ticket;
            c.submit_s = r.submit_s;
            c.launch_s = b->launch_s;
            c.done_s = t;
            c.batch_size = (int32_t)b->reqs.size();
            c.status = VTX_OK;
            s->done.push_back(c);
        }
        s->completed += b->reqs.size();
        s->inflight -= 1;
    }
    s->cv_done.notify_all();
    delete b;
}

void fail_batch(vtx_server* s, Batch* b, int rc) {
    const double t = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (const Request& r : b->reqs) {
            vtx_completion c;
            std::memset(&c, 0, sizeof(c));
            c.ticket = r.ticket;
            c.submit_s = r.submit_s;
            c.launch_s = b->launch_s;
            c.done_s = t;
            c.batch_size = (int32_t)b->reqs.size();
            c.status = rc;
            s->done.push_back(c);
        }
        s->completed += b->reqs.size();
        s->stats.failed += b->reqs.size();
        s->inflight -= 1;
    }
    s->cv_done.notify_all();
    delete b;
}

void worker_loop(vtx_server* s) {
    (void)hipSetDevice(s->device);
    std::vector<vtx_job> jobs;
    for (;;) {
        Batch* b = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
            if (s->queue.empty()) return;   // stop requested and nothing left
            // the device takes at most max_inflight batches: arrivals meanwhile
            // join the next one
            s->cv_done.wait(lk, [&] { return s->inflight < s->max_inflight; });
            b = new Batch();
            b->srv = s;
            const size_t take = std::min(s->queue.size(), (size_t)s->max_batch);
            for (size_t i = 0; i < take; ++i) {
                b->reqs.push_back(s->queue.front());
                s->queue.pop_front();
            }
            s->inflight += 1;
            s->stats.batches += 1;
            s->stats.max_batch_seen = std::max<uint64_t>(s->stats.max_batch_seen, take);
        }
        jobs.clear();
        for (const Request& r : b->reqs) jobs.push_back(r.job);
        b->launch_s = now_s();
        int rc = vtx_render_batch(s->ctx, jobs.data(), (int32_t)jobs.size(), s->stream);
        if (rc == VTX_OK && hipLaunchHostFunc(s->stream, batch_done, b) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(s->stream);
            rc = VTX_EHIP;
        }
        if (rc != VTX_OK) fail_batch(s, b, rc);
    }
}

}  // namespace

extern "C" {

double vtx_clock_s(void) { return now_s(); }

int vtx_server_create(vtx_context* ctx, int32_t max_batch, int32_t max_inflight, void* stream, vtx_server** out) {
    if (!ctx || !out) return VTX_EINVAL;
    if (max_batch < 1 || max_batch > 4096 || max_inflight < 1 || max_inflight > 64) return VTX_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return VTX_EHIP;
    vtx_server* s = new vtx_server();
    s->ctx = ctx;
    s->stream = (hipStream_t)stream;
    s->device = dev;
    s->max_batch = max_batch;
    s->max_inflight = max_inflight;
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return VTX_OK;
}

int vtx_server_submit(vtx_server* s, const vtx_job* job, uint64_t* ticket) {
    if (!s || !job) return VTX_EINVAL;
    // a request that cannot render is refused here rather than failing its batch
    const int rc = vtx_check_job(s->ctx, job);
    if (rc != VTX_OK) return rc;
    Request r;
    r.job = *job;
    r.submit_s = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return VTX_EINVAL;
        r.ticket = s->next_ticket++;
        s->queue.push_back(r);
        s->submitted += 1;
    }
    s->cv_work.notify_one();
    if (ticket) *ticket = r.ticket;
    return VTX_OK;
}

int vtx_server_poll(vtx_server* s, vtx_completion* out, int32_t max, int32_t wait_ms, int32_t* n) {
    if (!s || !n || max < 0 || (max > 0 && !out)) return VTX_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    const size_t k = std::min(s->done.size(), (size_t)max);
    for (size_t i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + (ptrdiff_t)k);
    *n = (int32_t)k;
    return VTX_OK;
}

int vtx_server_drain(vtx_server* s) {
    if (!s) return VTX_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
    return VTX_OK;
}

int vtx_server_stats_read(vtx_server* s, vtx_server_stats* out) {
    if (!s || !out) return VTX_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->queued = s->queue.size();
    return VTX_OK;
}

void vtx_server_destroy(vtx_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->inflight == 0; });
    }
    delete s;
}

}  // extern "C"
