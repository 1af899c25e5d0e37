// Serving: many resident matrices, requests submitted from any thread, merged
// per matrix into multi-column passes and issued on a few HIP streams.
//
// Threads: one dispatcher (takes groups from the queue with sched_pick and
// issues them) and one completion thread per stream (waits for the event
// recorded after each group, in issue order, and retires its requests).  The
// multi-column kernels reduce every column exactly as a single request would,
// so a request's output does not depend on which other requests shared its
// pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "spw_internal.h"
#include "spw_sched.h"

namespace spw {
namespace {

constexpr int32_t PASS_COLS = 8;           // columns per column-dot pass (kernel limit)

spw_status sfail(spw_status s, const std::string &msg)
{
    set_error(msg);
    return s;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Pending {
    spw_request r;
    double t_submit;
    double model_bytes;
};

struct Group {
    hipEvent_t done;
    std::vector<uint64_t> tickets;
    int32_t mat;
    spw_status st;
};

struct StreamSlot {
    hipStream_t stream = nullptr;
    std::deque<Group> fifo;                // issued, not yet retired
    std::thread completer;
};

}  // namespace
}  // namespace spw

struct spw_server_s {
    spw_serve_opts opts{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work;       // dispatcher: queue or capacity changed
    std::condition_variable cv_done;       // waiters and completers
    std::deque<spw::SchedReq> queue;
    std::unordered_map<uint64_t, spw::Pending> pending;   // queued or in flight
    std::unordered_map<uint64_t, spw_status> failed;      // retired with an error
    std::set<uint64_t> live;               // tickets queued or in flight
    uint64_t next_ticket = 1;
    std::vector<spw_matrix> mats;
    spw::SchedState sched;
    std::vector<spw::StreamSlot> streams;
    std::vector<hipEvent_t> event_pool;
    std::vector<int32_t> mat_groups;       // per matrix: groups picked and not yet retired
    std::thread dispatcher;
    bool paused = false;
    bool stopping = false;
    bool dispatch_done = false;            // the dispatcher has exited
    int64_t hbm_used = 0;
    // statistics
    int64_t submitted = 0, completed = 0, rejected_busy = 0, groups = 0, merged = 0, passes = 0;
    std::vector<double> latencies_us;
    double model_bytes_done = 0.0;
    double t_first_submit = 0.0, t_last_done = 0.0;
};

namespace spw {
namespace {

int64_t elt_bytes(spw_dtype t) { return t == SPW_F64 ? 8 : t == SPW_F32 ? 4 : 2; }

// Algorithmic bytes of one request: the matrix once (values, 4-byte indices
// and pointers) plus k input and k output vectors.
double request_bytes(const spw_matrix_s &A, const spw_request &r)
{
    const double sx = (double)elt_bytes(r.vdt);
    return (double)A.nnz * (double)(elt_bytes(A.value_storage) + 4) + 4.0 * (double)(A.cols + 1) +
           (double)r.k * sx * (double)(A.m + A.n);
}

// Issues one group; returns the status of the launches and the number of passes.
spw_status issue_group(spw_matrix_s &A, const std::vector<spw_request> &reqs, hipStream_t stream, int64_t *passes)
{
    const spw_request &h = reqs[0];
    const bool scatter = (A.format == SPW_CSC) == (h.op == SPW_OP_MV);
    const size_t es = (size_t)elt_bytes(h.vdt);
    // flatten the columns of every request
    std::vector<const void *> in;
    std::vector<void *> out;
    std::vector<int64_t> li, lo;
    for (const spw_request &r : reqs)
        for (int32_t c = 0; c < r.k; ++c) {
            in.push_back((const char *)r.in + (size_t)c * es);
            out.push_back((char *)r.out + (size_t)c * es);
            li.push_back(r.ldi);
            lo.push_back(r.ldo);
        }
    const int32_t total = (int32_t)in.size();
    for (int32_t c0 = 0; c0 < total; c0 += PASS_COLS) {
        const int32_t kk = std::min(PASS_COLS, total - c0);
        const int e = scatter ? launch_mv_cols(A, h.vdt, kk, &in[(size_t)c0], &li[(size_t)c0], &out[(size_t)c0],
                                               &lo[(size_t)c0], stream)
                              : launch_vtm_cols(A, h.vdt, kk, &in[(size_t)c0], &li[(size_t)c0], &out[(size_t)c0],
                                                &lo[(size_t)c0], stream);
        if (e) {
            set_error(std::string("serve: kernel launch failed: ") + hipGetErrorString((hipError_t)e));
            return SPW_ERR_DEVICE;
        }
        *passes += (scatter && A.scratch.pcols < kk) ? kk : 1;
    }
    return SPW_OK;
}

void dispatcher_main(spw_server_s *S)
{
    (void)hipSetDevice(S->device);
    std::vector<size_t> picked;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        int s = -1;
        S->cv_work.wait(lk, [&] {
            if (S->stopping && S->queue.empty()) return true;
            if (S->paused || S->queue.empty()) return false;
            s = sched_pick(S->queue, S->sched, S->opts.max_batch_cols, picked);
            return s >= 0;
        });
        if (s < 0) {                       // stopping with an empty queue
            S->dispatch_done = true;
            S->cv_done.notify_all();
            break;
        }
        std::vector<spw_request> reqs;
        std::vector<uint64_t> tickets;
        for (size_t i : picked) {
            const uint64_t t = S->queue[i].ticket;
            tickets.push_back(t);
            reqs.push_back(S->pending[t].r);
        }
        for (size_t n = picked.size(); n-- > 0;) S->queue.erase(S->queue.begin() + (long)picked[n]);
        const int32_t mat = reqs[0].matrix;
        S->sched.stream_busy[(size_t)s]++;
        S->sched.mat_stream[(size_t)mat] = s;
        S->mat_groups[(size_t)mat]++;
        ++S->groups;
        if (reqs.size() > 1) S->merged += (int64_t)reqs.size();
        hipEvent_t ev;
        if (S->event_pool.empty()) {
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                ev = nullptr;
            }
        } else {
            ev = S->event_pool.back();
            S->event_pool.pop_back();
        }
        StreamSlot &slot = S->streams[(size_t)s];
        spw_matrix_s *Am = S->mats[(size_t)mat];
        lk.unlock();
        // launches happen outside the lock; this stream's completer only looks
        // at groups already in its fifo
        int64_t npass = 0;
        spw_status st = SPW_ERR_DEVICE;
        if (ev) {
            try {
                st = issue_group(*Am, reqs, slot.stream, &npass);
            } catch (const std::bad_alloc &) {   // the group fails; the server goes on
                st = SPW_ERR_OUT_OF_MEMORY;
            }
        }
        if (ev && hipEventRecord(ev, slot.stream) != hipSuccess) {
            (void)hipGetLastError();
            st = SPW_ERR_DEVICE;
        }
        lk.lock();
        S->passes += npass;
        slot.fifo.push_back(Group{ev, std::move(tickets), mat, st});
        S->cv_done.notify_all();
    }
}

void completer_main(spw_server_s *S, int s)
{
    (void)hipSetDevice(S->device);
    StreamSlot &slot = S->streams[(size_t)s];
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_done.wait(lk, [&] { return !slot.fifo.empty() || S->dispatch_done; });
        if (slot.fifo.empty()) break;      // stopping and drained
        Group g = slot.fifo.front();
        lk.unlock();
        spw_status st = g.st;
        if (g.done && hipEventSynchronize(g.done) != hipSuccess) {
            (void)hipGetLastError();
            st = SPW_ERR_DEVICE;
        }
        const double t = now_s();
        lk.lock();
        slot.fifo.pop_front();
        if (g.done) S->event_pool.push_back(g.done);
        for (uint64_t tk : g.tickets) {
            auto it = S->pending.find(tk);
            if (it != S->pending.end()) {
                S->latencies_us.push_back((t - it->second.t_submit) * 1e6);
                S->model_bytes_done += it->second.model_bytes;
                S->pending.erase(it);
            }
            if (st != SPW_OK) S->failed[tk] = st;
            S->live.erase(tk);
            ++S->completed;
        }
        S->t_last_done = t;
        S->sched.stream_busy[(size_t)s]--;
        // the matrix stays bound to this stream while any of its groups is
        // picked (possibly still being issued) and not retired
        if (--S->mat_groups[(size_t)g.mat] == 0) S->sched.mat_stream[(size_t)g.mat] = -1;
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    const size_t i = std::min(v.size() - 1, (size_t)(q / 100.0 * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (long)i, v.end());
    return v[i];
}

}  // namespace
}  // namespace spw

using namespace spw;

extern "C" {

static spw_status spw_serve_opts_default_impl(spw_serve_opts *o)
{
    if (!o) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_opts_default: NULL opts");
    *o = spw_serve_opts{};
    o->struct_size = sizeof(*o);
    o->hbm_budget_bytes = (int64_t)64 << 30;
    o->max_inflight = 4096;
    o->streams = 4;
    o->max_batch_cols = 64;
    o->depth = 2;
    o->device = -1;
    o->start_paused = 0;
    return SPW_OK;
}

spw_status spw_serve_opts_default(spw_serve_opts *o)
{
    return guarded("spw_serve_opts_default", [&] { return spw_serve_opts_default_impl(o); });
}

static spw_status spw_serve_create_impl(spw_server *out, const spw_serve_opts *o_in)
{
    if (!out) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_create: NULL out");
    *out = nullptr;
    spw_serve_opts o;
    spw_serve_opts_default(&o);
    if (o_in) {
        if (o_in->struct_size != sizeof(spw_serve_opts))
            return sfail(SPW_ERR_INVALID_ARG, "spw_serve_create: opts.struct_size must be sizeof(spw_serve_opts)");
        o = *o_in;
    }
    if (o.hbm_budget_bytes <= 0 || o.max_inflight < 1 || o.streams < 1 || o.streams > 16 || o.max_batch_cols < 1 ||
        o.depth < 1)
        return sfail(SPW_ERR_INVALID_ARG, "spw_serve_create: budget, max_inflight, streams (1..16), "
                                          "max_batch_cols and depth must be positive");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return sfail(SPW_ERR_DEVICE, "spw_serve_create: no usable GPU");
    }
    if (o.device >= 0) dev = o.device;
    if (hipSetDevice(dev) != hipSuccess) {
        (void)hipGetLastError();
        return sfail(SPW_ERR_DEVICE, "spw_serve_create: hipSetDevice failed");
    }
    std::unique_ptr<spw_server_s> S(new spw_server_s());
    S->opts = o;
    S->device = dev;
    S->paused = o.start_paused != 0;
    S->sched.depth = o.depth;
    S->sched.stream_busy.assign((size_t)o.streams, 0);
    S->streams.resize((size_t)o.streams);
    for (auto &sl : S->streams) {
        // default priority: streams of other priorities are not used here
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            for (auto &q : S->streams)
                if (q.stream) (void)hipStreamDestroy(q.stream);
            return sfail(SPW_ERR_DEVICE, "spw_serve_create: hipStreamCreate failed");
        }
    }
    spw_server_s *raw = S.get();
    raw->dispatcher = std::thread(dispatcher_main, raw);
    for (int s = 0; s < o.streams; ++s) raw->streams[(size_t)s].completer = std::thread(completer_main, raw, s);
    *out = S.release();
    return SPW_OK;
}

spw_status spw_serve_create(spw_server *out, const spw_serve_opts *o_in)
{
    return guarded("spw_serve_create", [&] { return spw_serve_create_impl(out, o_in); });
}

static spw_status spw_serve_register_impl(spw_server S, spw_matrix A, int32_t *handle)
{
    if (!S || !A || !handle) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_register: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return sfail(SPW_ERR_SHUTDOWN, "spw_serve_register: server is shutting down");
    if (A->device != S->device) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_register: matrix is on another device");
    for (spw_matrix M : S->mats)
        if (M == A) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_register: matrix already registered");
    // the scratch of a pass (up to PASS_COLS columns) is allocated now, so that
    // serving never allocates; all of it is charged to the budget
    const int64_t before = A->device_bytes;
    {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(S->device);
        spw_status st = grow_scratch(*A, PASS_COLS);
        if (!st) st = grow_partial_cols(*A, PASS_COLS);
        (void)hipSetDevice(prev);
        if (st) return st;
    }
    const int64_t charge = A->device_bytes;
    if (S->hbm_used + charge > S->opts.hbm_budget_bytes)
        return sfail(SPW_ERR_BUDGET, "spw_serve_register: matrix needs " + std::to_string(charge) +
                                         " device bytes; " + std::to_string(S->opts.hbm_budget_bytes - S->hbm_used) +
                                         " of the budget are left (scratch grew by " +
                                         std::to_string(charge - before) + " bytes and stays with the matrix)");
    S->hbm_used += charge;
    S->mats.push_back(A);
    S->sched.mat_stream.push_back(-1);
    S->mat_groups.push_back(0);
    *handle = (int32_t)(S->mats.size() - 1);
    return SPW_OK;
}

spw_status spw_serve_register(spw_server S, spw_matrix A, int32_t *handle)
{
    return guarded("spw_serve_register", [&] { return spw_serve_register_impl(S, A, handle); });
}

static spw_status spw_serve_submit_impl(spw_server S, const spw_request *r, uint64_t *ticket)
{
    if (!S || !r || !ticket) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: NULL argument");
    if (r->struct_size != sizeof(spw_request))
        return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: request.struct_size must be sizeof(spw_request)");
    if (r->op != SPW_OP_MV && r->op != SPW_OP_VTM) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: bad op");
    if (r->vdt != SPW_F64 && r->vdt != SPW_F32) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: bad vector dtype");
    if (r->k < 1 || r->k > 64) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: k must be in [1, 64]");
    if (r->ldi < r->k || r->ldo < r->k) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: leading dimension < k");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return sfail(SPW_ERR_SHUTDOWN, "spw_serve_submit: server is shutting down");
    if (r->matrix < 0 || (size_t)r->matrix >= S->mats.size())
        return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: unknown matrix handle");
    const spw_matrix_s &A = *S->mats[(size_t)r->matrix];
    const int64_t in_len = r->op == SPW_OP_MV ? A.n : A.m;
    const int64_t out_len = r->op == SPW_OP_MV ? A.m : A.n;
    if ((in_len > 0 && !r->in) || (out_len > 0 && !r->out))
        return sfail(SPW_ERR_INVALID_ARG, "spw_serve_submit: NULL vector");
    const bool column_dots = (r->op == SPW_OP_VTM) == (A.format == SPW_CSC);
    if (column_dots && r->ldo >= CHUNK_OUT_LD_LIMIT)
        return sfail(SPW_ERR_UNSUPPORTED, "spw_serve_submit: output leading dimension must be below 2^18 for "
                                          "this matrix and op");
    if ((int64_t)S->live.size() >= S->opts.max_inflight) {
        ++S->rejected_busy;
        return sfail(SPW_ERR_BUSY, "spw_serve_submit: " + std::to_string(S->opts.max_inflight) +
                                       " requests already queued or running");
    }
    const uint64_t t = S->next_ticket++;
    const double now = now_s();
    if (S->submitted == 0) S->t_first_submit = now;
    ++S->submitted;
    S->pending[t] = Pending{*r, now, request_bytes(A, *r)};
    S->live.insert(t);
    S->queue.push_back(SchedReq{t, r->matrix, (int32_t)r->op, (int32_t)r->vdt, r->k});
    *ticket = t;
    S->cv_work.notify_one();
    return SPW_OK;
}

spw_status spw_serve_submit(spw_server S, const spw_request *r, uint64_t *ticket)
{
    return guarded("spw_serve_submit", [&] { return spw_serve_submit_impl(S, r, ticket); });
}

static spw_status spw_serve_resume_impl(spw_server S)
{
    if (!S) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_resume: NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    S->paused = false;
    S->cv_work.notify_all();
    return SPW_OK;
}

spw_status spw_serve_resume(spw_server S)
{
    return guarded("spw_serve_resume", [&] { return spw_serve_resume_impl(S); });
}

static spw_status ticket_state(spw_server S, uint64_t ticket, bool *done)
{
    if (ticket == 0 || ticket >= S->next_ticket) return sfail(SPW_ERR_INVALID_ARG, "unknown ticket");
    *done = S->live.find(ticket) == S->live.end();
    if (*done) {
        auto it = S->failed.find(ticket);
        if (it != S->failed.end()) return sfail(it->second, "request failed on the device");
    }
    return SPW_OK;
}

static spw_status spw_serve_poll_impl(spw_server S, uint64_t ticket, int32_t *done)
{
    if (!S || !done) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_poll: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    bool d = false;
    const spw_status st = ticket_state(S, ticket, &d);
    *done = d ? 1 : 0;
    return st;
}

spw_status spw_serve_poll(spw_server S, uint64_t ticket, int32_t *done)
{
    return guarded("spw_serve_poll", [&] { return spw_serve_poll_impl(S, ticket, done); });
}

static spw_status spw_serve_wait_impl(spw_server S, uint64_t ticket, int64_t timeout_us)
{
    if (!S) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_wait: NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    bool d = false;
    spw_status st = ticket_state(S, ticket, &d);
    if (st || d) return st;
    auto pred = [&] { return S->live.find(ticket) == S->live.end(); };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, pred);
    } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred)) {
        return sfail(SPW_ERR_TIMEOUT, "spw_serve_wait: request " + std::to_string(ticket) + " still pending");
    }
    return ticket_state(S, ticket, &d);
}

spw_status spw_serve_wait(spw_server S, uint64_t ticket, int64_t timeout_us)
{
    return guarded("spw_serve_wait", [&] { return spw_serve_wait_impl(S, ticket, timeout_us); });
}

static spw_status spw_serve_stats_impl(spw_server S, spw_server_stats *o)
{
    if (!S || !o) return sfail(SPW_ERR_INVALID_ARG, "spw_serve_stats: NULL argument");
    if (o->struct_size != sizeof(spw_server_stats))
        return sfail(SPW_ERR_INVALID_ARG, "spw_serve_stats: out->struct_size must be sizeof(spw_server_stats)");
    std::lock_guard<std::mutex> lk(S->mu);
    o->submitted = S->submitted;
    o->completed = S->completed;
    o->rejected_busy = S->rejected_busy;
    o->groups = S->groups;
    o->merged_requests = S->merged;
    o->passes = S->passes;
    o->inflight = (int64_t)S->live.size();
    o->registered = (int64_t)S->mats.size();
    o->hbm_budget_bytes = S->opts.hbm_budget_bytes;
    o->hbm_used_bytes = S->hbm_used;
    o->latency_p50_us = percentile(S->latencies_us, 50.0);
    o->latency_p99_us = percentile(S->latencies_us, 99.0);
    double sum = 0.0;
    for (double x : S->latencies_us) sum += x;
    o->latency_mean_us = S->latencies_us.empty() ? 0.0 : sum / (double)S->latencies_us.size();
    o->model_bytes = S->model_bytes_done;
    o->busy_seconds = S->completed > 0 ? S->t_last_done - S->t_first_submit : 0.0;
    o->gbps = o->busy_seconds > 0 ? o->model_bytes / o->busy_seconds / 1e9 : 0.0;
    return SPW_OK;
}

spw_status spw_serve_stats(spw_server S, spw_server_stats *o)
{
    return guarded("spw_serve_stats", [&] { return spw_serve_stats_impl(S, o); });
}

static spw_status spw_serve_destroy_impl(spw_server S)
{
    if (!S) return SPW_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        S->paused = false;                 // drain what is queued
        S->cv_work.notify_all();
    }
    if (S->dispatcher.joinable()) S->dispatcher.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->cv_done.notify_all();
    }
    for (auto &sl : S->streams)
        if (sl.completer.joinable()) sl.completer.join();
    (void)hipSetDevice(S->device);
    for (auto &sl : S->streams)
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
    delete S;
    return SPW_OK;
}

spw_status spw_serve_destroy(spw_server S)
{
    return guarded("spw_serve_destroy", [&] { return spw_serve_destroy_impl(S); });
}

}  // extern "C"
