// Continuous-batching request server.
//
// Motif significance needs the same count on many graphs (Section 1: the
// original and an ensemble of randomised graphs), and such counts arrive as
// independent (graph, k) requests.  The server keeps graphs and class tables
// resident and runs the requests through the same kernels as mk_count:
//
//   submit   -> FIFO queue
//   admit    -> while the head fits the HBM budget and a slot is free; the
//               requests admitted together are grouped by k and by size
//               class of n (ceil log2), and each group becomes one batch (one typed-adjacency and plan pass, one
//               persistent launch per slice for all its graphs), its graphs
//               ordered by size so that the small ones come first in the
//               unit queue
//   slices   -> every group keeps two slices of its work units queued on
//               its stream (the first of tick_units, each next one twice
//               the last); a HIP event marks each slice's end, and the
//               server thread (polling the events) queues the group's next
//               slice as soon as one ends
//   complete -> after each slice, every request whose units all lie in the
//               finished slices has its histogram finished and copied out
//               on a separate copy stream, and its waiter is woken; the
//               group's memory is released when its last request is done
//
// Requests that arrive while others run form new groups as soon as a slot
// and the memory budget allow; their slices share the device with the
// running groups' (the streams run concurrently), so small late requests do
// not wait for a long one to end.  Each request has its own histogram rows
// and the slices cover every unit exactly once, so its result is the same
// as when it runs alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "internal.h"
#include "server_hooks.h"

using namespace mk;

namespace {

constexpr int kServerStreams = 4;  // the hardware queues a process gets
constexpr uint64_t kDefaultBudget = 8ull << 30;
constexpr int kDefaultSlots = 64;
constexpr int kDefaultTickUnits = 8192;
// slices of a group queued on its stream at once: the next one is already
// there when one ends, so the host's polling leaves no gap
constexpr int kInFlight = 2;

enum class State { Queued, Active, Done, Failed };

struct Group;

struct Request {
    uint64_t ticket = 0;
    const mk_graph *g = nullptr;
    int k = 0;
    uint64_t est_bytes = 0;
    State state = State::Queued;
    int status = MK_OK;
    std::string error;
    Group *group = nullptr;
    int gi = 0;  // graph index in its group's batch
    std::vector<uint64_t> hist;
    mk_request_times times{};
};

// requests of one k admitted together, counted as one batch
struct Group {
    int k = 0;
    mk_batch *batch = nullptr;
    std::vector<Request *> reqs;       // in graph order
    std::vector<uint32_t> unit_begin;  // per graph, plus the total
    uint64_t units = 0;
    uint64_t launched = 0;             // units of the slices launched so far
    uint64_t done = 0;                 // units of the slices known to be done
    uint64_t slice = 0;                // size of the next slice
    size_t next = 0;                   // first request not yet collected
    int stream = 0;
    // slices in flight, oldest first: their end events and end units
    hipEvent_t ev[kInFlight] = {};
    uint64_t ev_end[kInFlight] = {};
    int head = 0, inflight = 0;
    bool prepared = false;             // the planning pass is known to be done
    uint64_t bytes = 0;                // device bytes charged to the budget
    int status = MK_OK;
    std::string error;
};

}  // namespace

struct mk_server {
    mk_ctx *ctx = nullptr;
    mk_server_opts opts{};
    std::thread thread;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Group *> groups;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    uint64_t used_bytes = 0;
    size_t active_requests = 0;
    bool stopping = false;
    int next_stream = 0;
    hipStream_t streams[kServerStreams] = {};
    hipStream_t copy_stream = nullptr;
    // finished groups' batches, freed only when nothing runs (a free can
    // wait for every kernel in flight); their bytes stay in used_bytes
    std::vector<std::pair<mk_batch *, uint64_t>> graveyard;
    std::chrono::steady_clock::time_point t0;

    double now_us() const
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
            .count();
    }
};

// vertex-count class of a graph: ceil(log2(n)), at least 10 (n <= 1024)
static int size_class(int n)
{
    int c = 10;
    while (c < 31 && (1 << c) < n) ++c;
    return c;
}

// a request leaves the server (its waiter is woken)
static void finish_request(mk_server *s, Request *r, State st, int status, const char *why)
{
    std::lock_guard<std::mutex> lock(s->mu);
    r->state = st;
    r->status = status;
    if (why) r->error = why;
    r->times.done_us = s->now_us();
    s->active_requests -= std::min<size_t>(s->active_requests, 1);
    s->cv_done.notify_all();
}

// the group's batch goes to the graveyard (freed when nothing runs)
static void retire_group(mk_server *s, Group *gp)
{
    for (hipEvent_t e : gp->ev)
        if (e) (void)hipEventDestroy(e);
    std::lock_guard<std::mutex> lock(s->mu);
    if (gp->batch) s->graveyard.emplace_back(gp->batch, gp->bytes);
    else s->used_bytes -= std::min(s->used_bytes, gp->bytes);
    delete gp;
}

// free the finished batches (call when no group is in flight, or when their
// memory is needed)
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

// fail every request of a group that is not collected yet
static void fail_group(mk_server *s, Group *gp, int status, const char *why)
{
    for (size_t i = gp->next; i < gp->reqs.size(); ++i)
        finish_request(s, gp->reqs[i], State::Failed, status, why);
    gp->next = gp->reqs.size();
}

// one batch for the admitted requests of one k, planned on the group's stream
static Group *start_group(mk_server *s, int k, std::vector<Request *> reqs, uint64_t est_bytes)
{
    // small graphs first: their units come first in the queue, so they are
    // done after the first slices
    std::stable_sort(reqs.begin(), reqs.end(), [](const Request *a, const Request *b) {
        return a->g->nnz_u < b->g->nnz_u;
    });
    Group *gp = new Group();
    gp->k = k;
    gp->reqs = reqs;
    gp->bytes = est_bytes;
    gp->stream = s->next_stream++ % kServerStreams;
    for (size_t i = 0; i < reqs.size(); ++i) {
        reqs[i]->group = gp;
        reqs[i]->gi = (int)i;
    }
    mk_table *t = nullptr;
    int rc = mk_table_build(s->ctx, k, &t);
    std::vector<const mk_graph *> gs;
    for (Request *r : reqs) gs.push_back(r->g);
    if (rc == MK_OK) {
        mk_batch_opts o{};
        o.use_graph = -1;
        rc = mk_batch_create(s->ctx, gs.data(), (int32_t)gs.size(), t, &o, &gp->batch);
    }
    if (rc == MK_OK) rc = batch_unit_begins(gp->batch, &gp->unit_begin);
    if (rc == MK_OK) rc = batch_prepare(gp->batch, s->streams[gp->stream]);
    for (int i = 0; i < kInFlight && rc == MK_OK; ++i) {
        hipError_t e = hipEventCreateWithFlags(&gp->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) rc = fail(MK_EDEVICE, "server event: %s", hipGetErrorString(e));
    }
    if (rc == MK_OK) {
        // the planning pass counts as a slice of no units: requests are
        // collected only after it (the histograms are cleared there)
        if (hipEventRecord(gp->ev[0], s->streams[gp->stream]) != hipSuccess)
            rc = fail(MK_EDEVICE, "server event record failed");
        gp->ev_end[0] = 0;
        gp->inflight = 1;
    }
    if (rc == MK_OK) {
        gp->units = gp->unit_begin.back();
        for (Request *r : reqs) r->hist.assign(t->num_classes, 0);
        std::lock_guard<std::mutex> lock(s->mu);
        const uint64_t actual = batch_device_bytes(gp->batch);
        s->used_bytes = s->used_bytes - std::min(s->used_bytes, gp->bytes) + actual;
        gp->bytes = actual;
    } else {
        gp->status = rc;
        gp->error = mk_last_error();
    }
    return gp;
}

// collect the requests whose units all lie in finished slices
static void collect_done(mk_server *s, Group *gp)
{
    while (gp->prepared && gp->next < gp->reqs.size() &&
           gp->unit_begin[gp->next + 1] <= gp->done) {
        Request *r = gp->reqs[gp->next];
        int rc = batch_collect_graph(gp->batch, r->gi, r->hist.data(), s->copy_stream);
        if (rc == MK_OK) finish_request(s, r, State::Done, MK_OK, nullptr);
        else finish_request(s, r, State::Failed, rc, mk_last_error());
        ++gp->next;
    }
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
            need_bury = !s->graveyard.empty() && (s->groups.empty() || blocked);
        }
        if (need_bury) bury(s);
        // admit: FIFO while a slot is free and the head fits the budget
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            auto can_admit = [&] {
                return !s->queue.empty() && s->active_requests < slots &&
                       s->used_bytes + s->queue.front()->est_bytes <= budget;
            };
            if (s->groups.empty() && s->graveyard.empty())
                s->cv_work.wait(lock, [&] { return s->stopping || can_admit(); });
            if (s->stopping && s->queue.empty() && s->groups.empty() && s->graveyard.empty())
                break;
            while (can_admit()) {
                Request *r = s->queue.front();
                s->queue.pop_front();
                r->state = State::Active;
                r->times.admit_us = s->now_us();
                s->used_bytes += r->est_bytes;
                ++s->active_requests;
                admitted.push_back(r);
            }
        }
        bool progress = !admitted.empty();
        // groups: one per k and vertex-count class (a batch sizes every
        // wave's LDS marks for its largest graph, so graphs of very
        // different n are not mixed: the small ones would run at the large
        // one's occupancy)
        std::vector<std::pair<int, std::vector<Request *>>> parts;
        for (Request *r : admitted) {
            const int key = r->k * 64 + size_class(r->g->n);
            auto it = std::find_if(parts.begin(), parts.end(),
                                   [key](const auto &p) { return p.first == key; });
            if (it == parts.end()) {
                parts.emplace_back(key, std::vector<Request *>{});
                it = parts.end() - 1;
            }
            it->second.push_back(r);
        }
        for (auto &part : parts) {
            uint64_t bytes = 0;
            for (Request *r : part.second) bytes += r->est_bytes;
            Group *gp = start_group(s, part.first / 64, part.second, bytes);
            if (gp->status != MK_OK) {
                fail_group(s, gp, gp->status, gp->error.c_str());
                retire_group(s, gp);
            } else {
                s->groups.push_back(gp);
            }
        }
        // finished slices (oldest first) and the requests they complete
        for (Group *gp : s->groups) {
            while (gp->inflight > 0 && gp->status == MK_OK) {
                const hipError_t q = hipEventQuery(gp->ev[gp->head]);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    gp->status = fail(MK_EDEVICE, "server group: %s", hipGetErrorString(q));
                    gp->error = mk_last_error();
                    break;
                }
                gp->done = gp->ev_end[gp->head];
                gp->prepared = true;
                gp->head = (gp->head + 1) % kInFlight;
                --gp->inflight;
                progress = true;
            }
            if (gp->status == MK_OK) collect_done(s, gp);
        }
        // next slices: each group keeps kInFlight queued on its stream; the
        // first covers tick units and every next one twice the last (the
        // small graphs first in the queue finish early, the rest in few
        // launches)
        std::vector<Group *> still;
        for (Group *gp : s->groups) {
            while (gp->status == MK_OK && gp->inflight < kInFlight && gp->launched < gp->units) {
                if (gp->slice == 0) gp->slice = tick;
                const uint64_t end = std::min(gp->units, gp->launched + gp->slice);
                gp->slice *= 2;
                hipStream_t st = s->streams[gp->stream];
                const int slot = (gp->head + gp->inflight) % kInFlight;
                int rc = batch_enum_slice(gp->batch, (uint32_t)gp->launched, (uint32_t)end, st);
                if (rc == MK_OK && hipEventRecord(gp->ev[slot], st) != hipSuccess)
                    rc = fail(MK_EDEVICE, "server event record failed");
                if (rc != MK_OK) {
                    gp->status = rc;
                    gp->error = mk_last_error();
                    break;
                }
                gp->ev_end[slot] = end;
                gp->launched = end;
                ++gp->inflight;
                progress = true;
            }
            if (gp->status == MK_OK && (gp->inflight > 0 || gp->next < gp->reqs.size())) {
                still.push_back(gp);
                continue;
            }
            if (gp->status != MK_OK) {
                // wait for its slices before the batch can go
                for (int i = 0; i < gp->inflight; ++i)
                    (void)hipEventSynchronize(gp->ev[(gp->head + i) % kInFlight]);
                fail_group(s, gp, gp->status, gp->error.c_str());
            }
            retire_group(s, gp);
            progress = true;
        }
        s->groups.swap(still);
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
    for (auto &kv : s->all) delete kv.second;
    (void)hipSetDevice(s->ctx->device);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
    return MK_OK;
}
