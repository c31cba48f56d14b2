// Continuous-batching request server.
//
// Motif significance needs the same count on many graphs (Section 1: the
// original and an ensemble of randomised graphs), and such counts arrive as
// independent (graph, k) requests.  The server keeps graphs and class tables
// resident and runs the requests through the same kernels as mk_count:
//
//   submit   -> FIFO queue
//   admit    -> while the head fits the HBM budget and a slot is free: plan it
//               (typed adjacency + work units) on one of the server's streams
//   slices   -> every admitted request has one slice of at most tick_units
//               of its work units in flight on its stream; a HIP event marks
//               the slice's end, and the server thread (polling the events)
//               launches the request's next slice as soon as it is done
//   complete -> a request whose units are all done has its histogram copied
//               out on a separate copy stream, its memory released, and its
//               waiter woken
//
// A request that arrives while others run is admitted as soon as a slot and
// the memory budget allow, and its slices then share the device with
// everyone else's; a long request holds a stream for at most one slice at a
// time.  There is no global barrier between slices.  Each request has its
// own histogram and its slices cover its units exactly once, so its result
// is the same as when it runs alone.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "internal.h"

using namespace mk;

namespace {

constexpr int kServerStreams = 8;
constexpr uint64_t kDefaultBudget = 8ull << 30;
constexpr int kDefaultSlots = 64;
constexpr int kDefaultTickUnits = 8192;

enum class State { Queued, Active, Done, Failed };

struct Request {
    uint64_t ticket = 0;
    const mk_graph *g = nullptr;
    int k = 0;
    uint64_t est_bytes = 0;
    uint64_t bytes = 0;
    State state = State::Queued;
    int status = MK_OK;
    std::string error;
    mk_batch *batch = nullptr;
    uint64_t units = 0, cursor = 0;
    int stream = 0;
    hipEvent_t ev = nullptr;  // end of the work last launched for the request
    bool inflight = false;
    std::vector<uint64_t> hist;
    mk_request_times times{};
};

}  // namespace

struct mk_server {
    mk_ctx *ctx = nullptr;
    mk_server_opts opts{};
    std::thread thread;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    uint64_t used_bytes = 0;
    bool stopping = false;
    int next_stream = 0;
    hipStream_t streams[kServerStreams] = {};
    hipStream_t copy_stream = nullptr;
    // finished requests' batches, freed only when nothing runs (a free can
    // wait for every kernel in flight); their bytes stay in used_bytes
    std::vector<std::pair<mk_batch *, uint64_t>> graveyard;
    std::chrono::steady_clock::time_point t0;

    double now_us() const
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
            .count();
    }
};

static void finish(mk_server *s, Request *r, State st, int status, const char *why)
{
    std::lock_guard<std::mutex> lock(s->mu);
    if (r->batch) {
        s->graveyard.emplace_back(r->batch, r->bytes);
        r->batch = nullptr;
    } else {
        s->used_bytes -= std::min(s->used_bytes, r->bytes);
    }
    if (r->ev) {
        (void)hipEventDestroy(r->ev);
        r->ev = nullptr;
    }
    r->state = st;
    r->status = status;
    if (why) r->error = why;
    r->times.done_us = s->now_us();
    s->cv_done.notify_all();
}

// free the finished batches (call when no request is in flight, or when
// their memory is needed)
static void bury(mk_server *s)
{
    std::vector<std::pair<mk_batch *, uint64_t>> g;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        g.swap(s->graveyard);
    }
    uint64_t freed = 0;
    for (auto &e : g) {
        mk_batch_free(e.first);
        freed += e.second;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    s->used_bytes -= std::min(s->used_bytes, freed);
}

// plan an admitted request on its stream; false if it failed
static bool start_request(mk_server *s, Request *r)
{
    mk_table *t = nullptr;
    int rc = mk_table_build(s->ctx, r->k, &t);
    if (rc == MK_OK) {
        mk_batch_opts o{};
        o.use_graph = -1;
        rc = mk_batch_create(s->ctx, &r->g, 1, t, &o, &r->batch);
    }
    if (rc == MK_OK) rc = batch_prepare(r->batch, s->streams[r->stream]);
    if (rc == MK_OK) {
        hipError_t e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r->ev, s->streams[r->stream]);
        if (e != hipSuccess) rc = fail(MK_EDEVICE, "server event: %s", hipGetErrorString(e));
        r->inflight = true;
    }
    if (rc != MK_OK) {
        finish(s, r, State::Failed, rc, mk_last_error());
        return false;
    }
    r->units = batch_units(r->batch);
    r->hist.assign(t->num_classes, 0);
    std::lock_guard<std::mutex> lock(s->mu);
    const uint64_t actual = batch_device_bytes(r->batch);
    s->used_bytes = s->used_bytes - std::min(s->used_bytes, r->bytes) + actual;
    r->bytes = actual;
    return true;
}

static void server_loop(mk_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    const uint64_t budget = s->opts.hbm_budget_bytes;
    const size_t slots = (size_t)s->opts.max_slots;
    const uint64_t tick = (uint64_t)s->opts.tick_units;
    for (;;) {
        bool need_bury = false;
        {
            std::lock_guard<std::mutex> lock(s->mu);
            const bool blocked = !s->queue.empty() &&
                                 s->used_bytes + s->queue.front()->est_bytes > budget;
            need_bury = !s->graveyard.empty() && (s->active.empty() || blocked);
        }
        if (need_bury) bury(s);
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            auto can_admit = [&] {
                return !s->queue.empty() && s->active.size() + admitted.size() < slots &&
                       s->used_bytes + s->queue.front()->est_bytes <= budget;
            };
            if (s->active.empty() && s->graveyard.empty())
                s->cv_work.wait(lock, [&] { return s->stopping || can_admit(); });
            if (s->stopping && s->queue.empty() && s->active.empty() && s->graveyard.empty())
                break;
            while (can_admit()) {
                Request *r = s->queue.front();
                s->queue.pop_front();
                r->state = State::Active;
                r->times.admit_us = s->now_us();
                r->bytes = r->est_bytes;
                s->used_bytes += r->est_bytes;
                r->stream = s->next_stream++ % kServerStreams;
                admitted.push_back(r);
            }
        }
        for (Request *r : admitted)
            if (start_request(s, r)) s->active.push_back(r);

        bool progress = !admitted.empty();
        // finished slices
        for (Request *r : s->active) {
            if (!r->inflight) continue;
            const hipError_t q = hipEventQuery(r->ev);
            if (q == hipSuccess) {
                r->inflight = false;
                progress = true;
            } else if (q != hipErrorNotReady) {
                r->status = fail(MK_EDEVICE, "request %llu: %s", (unsigned long long)r->ticket,
                                 hipGetErrorString(q));
                r->error = mk_last_error();
                r->inflight = false;
                r->cursor = r->units;
            }
        }
        // next slices, and completions
        std::vector<Request *> still;
        for (Request *r : s->active) {
            if (r->inflight) {
                still.push_back(r);
                continue;
            }
            if (r->cursor < r->units && r->status == MK_OK) {
                const uint64_t end = std::min(r->units, r->cursor + tick);
                hipStream_t st = s->streams[r->stream];
                int rc = batch_enum_slice(r->batch, (uint32_t)r->cursor, (uint32_t)end, st);
                if (rc == MK_OK && hipEventRecord(r->ev, st) != hipSuccess)
                    rc = fail(MK_EDEVICE, "server event record failed");
                if (rc == MK_OK) {
                    r->cursor = end;
                    r->inflight = true;
                    progress = true;
                    still.push_back(r);
                    continue;
                }
                // a failed launch ends the request now (reported below)
                r->status = rc;
                r->error = mk_last_error();
                r->cursor = r->units;
            }
            int rc = r->status;
            if (rc == MK_OK) rc = batch_collect(r->batch, r->hist.data(), s->copy_stream);
            if (rc == MK_OK) finish(s, r, State::Done, MK_OK, nullptr);
            else finish(s, r, State::Failed, rc, r->error.empty() ? mk_last_error() : r->error.c_str());
            progress = true;
        }
        s->active.swap(still);
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

extern "C" int mk_server_start(mk_ctx *ctx, const mk_server_opts *opts, mk_server **out)
{
    if (!ctx || !out) return fail(MK_EINVAL, "mk_server_start: NULL argument");
    *out = nullptr;
    mk_server *s = new mk_server();
    s->ctx = ctx;
    if (opts) s->opts = *opts;
    if (s->opts.hbm_budget_bytes == 0) s->opts.hbm_budget_bytes = kDefaultBudget;
    if (s->opts.max_slots <= 0) s->opts.max_slots = kDefaultSlots;
    if (s->opts.tick_units <= 0) s->opts.tick_units = kDefaultTickUnits;
    hipError_t e = hipSetDevice(ctx->device);
    for (int i = 0; i < kServerStreams && e == hipSuccess; ++i)
        e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        for (hipStream_t st : s->streams)
            if (st) (void)hipStreamDestroy(st);
        if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
        delete s;
        return fail(MK_EDEVICE, "mk_server_start: %s", hipGetErrorString(e));
    }
    s->t0 = std::chrono::steady_clock::now();
    s->thread = std::thread(server_loop, s);
    *out = s;
    return MK_OK;
}

extern "C" int mk_submit(mk_server *s, const mk_graph *g, int k, uint64_t *ticket)
{
    if (!s || !g || !ticket) return fail(MK_EINVAL, "mk_submit: NULL argument");
    if (k < 3 || k > 6) return fail(MK_ERANGE, "mk_submit: k=%d outside 3..6", k);
    if (g->ctx != s->ctx) return fail(MK_EINVAL, "mk_submit: graph of another context");
    uint64_t est = 0;
    int rc = mk_graph_footprint(g, k, &est);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stopping) return fail(MK_EBUSY, "mk_submit: server is stopping");
    if (est > s->opts.hbm_budget_bytes)
        return fail(MK_EBUSY, "request needs ~%llu bytes, budget is %llu",
                    (unsigned long long)est, (unsigned long long)s->opts.hbm_budget_bytes);
    Request *r = new Request();
    r->ticket = s->next_ticket++;
    r->g = g;
    r->k = k;
    r->est_bytes = est;
    r->times.submit_us = s->now_us();
    r->times.admit_us = -1;
    r->times.done_us = -1;
    s->queue.push_back(r);
    s->all[r->ticket] = r;
    *ticket = r->ticket;
    s->cv_work.notify_all();
    return MK_OK;
}

extern "C" int mk_wait(mk_server *s, uint64_t ticket, uint64_t *hist, uint32_t capacity,
                       int32_t timeout_ms, mk_request_times *times)
{
    if (!s) return fail(MK_EINVAL, "mk_wait: NULL server");
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(MK_ENOTFOUND, "mk_wait: unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    auto ready = [&] { return r->state == State::Done || r->state == State::Failed; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lock, ready);
    } else if (!s->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), ready)) {
        return fail(MK_ETIMEDOUT, "mk_wait: request %llu not done after %d ms",
                    (unsigned long long)ticket, timeout_ms);
    }
    int rc = r->status;
    if (rc == MK_OK) {
        if (hist && capacity < r->hist.size()) {
            return fail(MK_ERANGE, "mk_wait: capacity %u < %zu classes", capacity, r->hist.size());
        }
        if (hist) std::copy(r->hist.begin(), r->hist.end(), hist);
    } else {
        fail(rc, "request %llu failed: %s", (unsigned long long)ticket, r->error.c_str());
    }
    if (times) *times = r->times;
    s->all.erase(it);
    delete r;
    return rc;
}

extern "C" int mk_server_stop(mk_server *s)
{
    if (!s) return fail(MK_EINVAL, "mk_server_stop: NULL server");
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stopping = true;
        s->cv_work.notify_all();
    }
    if (s->thread.joinable()) s->thread.join();
    bury(s);
    for (auto &kv : s->all) {
        if (kv.second->batch) mk_batch_free(kv.second->batch);
        if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    (void)hipSetDevice(s->ctx->device);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
    return MK_OK;
}
