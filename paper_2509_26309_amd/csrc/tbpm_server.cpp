// Request server: continuous batching of TBPM propagations on one GPU.
//
// Submitted requests wait in a FIFO.  A scheduler thread admits the head of
// the queue while its footprint fits the remaining HBM budget and a slot is
// free (head-of-line order, so a large request is not overtaken forever),
// gives each admitted request its own stream and resident buffers, and then
// feeds every running request a chunk of time steps per round.  Chunks of
// different requests run concurrently on the device; a request that finishes
// frees its slot and memory at once, and the next queued request is admitted
// while the others keep running.  Each request's kernels, launch shapes and
// reduction order are those of a lone tbpm_propagate_dos call, so its result
// does not depend on what else is running.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "tbpm_engine.h"
#include "tbpm_trace.h"

using namespace tbpm;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const tbpm_ham *ham = nullptr;
    tbpm_params params{};
    std::vector<int64_t> sites;
    std::unique_ptr<Job> job;
    size_t footprint = 0;
    hipStream_t stream = nullptr;
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};
    int chunks_out = 0;        // chunks recorded and not yet seen complete (0..2)
    int chunk_head = 0;
    int chunk_steps = 1;
    bool admitted = false;
    bool done = false;                 // written under the server's mutex
    std::atomic<bool> cancel{false};   // set by tbpm_cancel, read by the scheduler
    tbpm_status status = TBPM_PENDING;
    std::string error;
    double t_submit = 0, t_admit = -1, t_done = -1;
    std::vector<double> corr;  // [R][N_t+1] complex
};

}  // namespace

struct tbpm_server {
    tbpm_ctx *ctx = nullptr;
    size_t budget = 0;
    int max_slots = 1;
    size_t used = 0;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::map<uint64_t, std::unique_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    bool admit_locked(std::vector<Request *> &admitted);
    void start_request(Request *r);
    void finish_request(Request *r, tbpm_status s, const std::string &err);
    void feed(Request *r);
};

// work per chunk: about 64 MB of algorithmic traffic (or at least one step),
// so that every running request gets device time each round
static int chunk_steps_for(const tbpm_ham *ham, const Job &job)
{
    const double per_step = (double)(job.M - 1) * ((double)ham->bytes + 5.0 * (double)ham->n * job.elem * job.bmax);
    int s = (int)(64e6 / (per_step > 1 ? per_step : 1));
    if (s < 1)
        s = 1;
    if (s > 256)
        s = 256;
    return s;
}

bool tbpm_server::admit_locked(std::vector<Request *> &admitted)
{
    bool any = false;
    while (!queue.empty()) {
        Request *r = queue.front();
        if (r->cancel) {
            queue.pop_front();
            r->status = TBPM_ERR_CANCELLED;
            r->done = true;
            r->t_done = now();
            r->ham->users.fetch_sub(1);
            continue;
        }
        if ((int)active.size() >= max_slots || used + r->footprint > budget)
            break;
        queue.pop_front();
        used += r->footprint;
        r->admitted = true;
        r->t_admit = now();
        active.push_back(r);
        admitted.push_back(r);
        any = true;
    }
    return any;
}

void tbpm_server::finish_request(Request *r, tbpm_status s, const std::string &err)
{
    if (r->job)
        r->job->release();
    r->job.reset();
    for (auto &e : r->chunk_ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    if (r->stream) {
        (void)hipStreamDestroy(r->stream);
        r->stream = nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    used -= r->footprint;
    r->status = s;
    r->error = err;
    r->done = true;
    r->t_done = now();
    r->ham->users.fetch_sub(1);
    for (size_t i = 0; i < active.size(); ++i)
        if (active[i] == r) {
            active.erase(active.begin() + (long)i);
            break;
        }
    cv.notify_all();
}

void tbpm_server::start_request(Request *r)
{
    r->job.reset(new Job());
    Job &job = *r->job;
    tbpm_params prm = r->params;
    prm.ldos_sites = r->sites.empty() ? nullptr : r->sites.data();
    tbpm_status s = hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking) == hipSuccess ? TBPM_OK : TBPM_ERR_HIP;
    if (s == TBPM_OK && (hipEventCreateWithFlags(&r->chunk_ev[0], hipEventDisableTiming) != hipSuccess ||
                         hipEventCreateWithFlags(&r->chunk_ev[1], hipEventDisableTiming) != hipSuccess))
        s = TBPM_ERR_HIP;
    if (s == TBPM_OK)
        s = job.setup(ctx, r->ham, &prm, r->stream);
    if (s == TBPM_OK)
        s = job.allocate();
    if (s != TBPM_OK) {
        finish_request(r, s, job.error.empty() ? "request start failed" : job.error);
        return;
    }
    r->chunk_steps = chunk_steps_for(r->ham, job);
}

// enqueue one chunk when fewer than two are outstanding; complete the request
// once everything is enqueued and the device has drained its stream
void tbpm_server::feed(Request *r)
{
    // retire completed chunks in order
    while (r->chunks_out > 0) {
        const int tail = (r->chunk_head - r->chunks_out + 2) % 2;
        hipError_t q = hipEventQuery(r->chunk_ev[tail]);
        if (q == hipErrorNotReady)
            break;
        if (q != hipSuccess) {
            finish_request(r, TBPM_ERR_HIP, std::string("device error: ") + hipGetErrorString(q));
            return;
        }
        --r->chunks_out;
        if (r->job->flag_set()) {
            // a norm left norm_tol in a completed chunk: stop now and free the slot
            (void)hipStreamSynchronize(r->stream);
            finish_request(r, TBPM_ERR_DIVERGED, "a vector's norm left norm_tol during the run");
            return;
        }
    }
    Job &job = *r->job;
    if (r->cancel) {
        if (r->chunks_out == 0)
            finish_request(r, TBPM_ERR_CANCELLED, "cancelled");
        return;
    }
    if (job.all_enqueued()) {
        if (r->chunks_out > 0)
            return;
        r->corr.assign((size_t)r->params.num_vectors * ((size_t)r->params.num_time_steps + 1) * 2, 0.0);
        tbpm_status s = job.finish(r->corr.data(), nullptr, nullptr);
        finish_request(r, s, s == TBPM_OK ? "" : job.error);
        return;
    }
    if (r->chunks_out >= 2)
        return;
    TraceRange range("tbpm_server_chunk");
    tbpm_status s = job.advance(r->chunk_steps), s2 = TBPM_OK;
    if (s == TBPM_OK || s == TBPM_PENDING)
        s2 = job.queue_flag_read();
    if ((s != TBPM_OK && s != TBPM_PENDING) || s2 != TBPM_OK) {
        (void)hipStreamSynchronize(r->stream);
        finish_request(r, s2 != TBPM_OK ? s2 : s, job.error);
        return;
    }
    if (hipEventRecord(r->chunk_ev[r->chunk_head], r->stream) != hipSuccess) {
        (void)hipStreamSynchronize(r->stream);
        finish_request(r, TBPM_ERR_HIP, "event record failed");
        return;
    }
    r->chunk_head = (r->chunk_head + 1) % 2;
    ++r->chunks_out;
}

void tbpm_server::run()
{
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<Request *> admitted;
        std::vector<Request *> running;
        {
            std::unique_lock<std::mutex> lk(mu);
            admit_locked(admitted);
            if (stop && queue.empty() && active.empty())
                break;
            if (active.empty() && admitted.empty()) {
                cv.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            running = active;
        }
        for (Request *r : admitted)
            start_request(r);
        for (Request *r : running) {
            bool still;
            {
                std::lock_guard<std::mutex> lk(mu);
                still = !r->done;
            }
            if (still && r->job)
                feed(r);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

extern "C" {

tbpm_status tbpm_server_create(tbpm_ctx *ctx, size_t hbm_budget, int32_t max_slots, tbpm_server **out)
{
    if (!ctx || !out || max_slots < 1 || hbm_budget == 0)
        return TBPM_ERR_ARG;
    tbpm_server *s = new (std::nothrow) tbpm_server();
    if (!s)
        return TBPM_ERR_OOM;
    s->ctx = ctx;
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->t0 = Clock::now();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return TBPM_OK;
}

tbpm_status tbpm_submit(tbpm_server *srv, const tbpm_ham *ham, const tbpm_params *params, uint64_t *ticket)
{
    if (!srv || !ham || !params || !ticket)
        return TBPM_ERR_ARG;
    if (ham->ctx != srv->ctx)
        return TBPM_ERR_ARG;
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r)
        return TBPM_ERR_OOM;
    r->ham = ham;
    r->params = *params;
    if (params->num_ldos_sites > 0 && params->ldos_sites)
        r->sites.assign(params->ldos_sites, params->ldos_sites + params->num_ldos_sites);
    r->params.ldos_sites = nullptr;
    // validate and size the request with a job that allocates nothing
    {
        Job probe;
        tbpm_params prm = r->params;
        prm.ldos_sites = r->sites.empty() ? nullptr : r->sites.data();
        tbpm_status s = probe.setup(srv->ctx, ham, &prm, nullptr);
        if (s != TBPM_OK)
            return s;
        r->footprint = probe.footprint();
        probe.ctx = nullptr;
    }
    if (r->footprint > srv->budget)
        return TBPM_ERR_TOO_LARGE;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop)
        return TBPM_ERR_ARG;
    r->ticket = srv->next_ticket++;
    r->t_submit = srv->now();
    ham->users.fetch_add(1);
    *ticket = r->ticket;
    srv->queue.push_back(r.get());
    srv->all[r->ticket] = std::move(r);
    srv->cv.notify_all();
    return TBPM_OK;
}

tbpm_status tbpm_poll(tbpm_server *srv, uint64_t ticket, double *corr, int64_t corr_len, double *corr_mean,
                      int64_t mean_len, double *timings)
{
    if (!srv)
        return TBPM_ERR_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end())
        return TBPM_ERR_UNKNOWN;
    Request *r = it->second.get();
    const int64_t R = r->params.num_vectors, nt1 = (int64_t)r->params.num_time_steps + 1;
    // capacities are checked before anything is written, finished or not
    if ((corr && corr_len < R * nt1) || (corr_mean && mean_len < nt1))
        return TBPM_ERR_ARG;
    if (timings) {
        timings[0] = r->t_submit;
        timings[1] = r->t_admit;
        timings[2] = r->t_done;
    }
    if (!r->done)
        return TBPM_PENDING;
    if (r->status == TBPM_OK) {
        if (corr)
            std::copy(r->corr.begin(), r->corr.end(), corr);
        if (corr_mean)
            sample_mean(r->corr.data(), (size_t)R, (size_t)nt1, true, corr_mean);
    }
    return r->status;
}

tbpm_status tbpm_cancel(tbpm_server *srv, uint64_t ticket)
{
    if (!srv)
        return TBPM_ERR_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end())
        return TBPM_ERR_UNKNOWN;
    it->second->cancel = true;
    srv->cv.notify_all();
    return TBPM_OK;
}

tbpm_status tbpm_server_destroy(tbpm_server *srv)
{
    if (!srv)
        return TBPM_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
    }
    if (srv->worker.joinable())
        srv->worker.join();
    delete srv;
    return TBPM_OK;
}

}  // extern "C"
