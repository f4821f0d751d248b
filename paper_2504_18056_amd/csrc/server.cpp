// Serving: a request loop that runs the frames of many concurrent sessions.
//
// BATCHED mode serves two lanes side by side.  Frames of sessions large
// enough to fill the device on their own (a round of evaluation tiles) are
// launched as they arrive with the per-session launches on the session's own
// stream, so they overlap each other and the ticks.  Frames of smaller sessions form ticks: the oldest pending
// frame, then the smallest frames of other sessions (at most one per session)
// while the tick's work stays under a cap; a tick writes one compact table of
// step descriptors and per-stage work items into pinned host memory, copies
// it to the device in one transfer and replays a HIP graph of persistent
// kernels captured once per table buffer.  Two table buffers alternate so a
// tick can be prepared and queued while the previous one runs.  CONCURRENT mode launches every request as soon as it arrives on
// its session's own stream, so frames of different sessions overlap on the
// device without a tick boundary.  SERIAL mode runs one request at a time
// with the per-session launches and waits for it.
//
// A worker thread launches work; a completion thread watches the events of
// the work in flight and retires requests as soon as their work is done.
#include "state.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <unordered_set>

using namespace mcs;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    int64_t id;
    int32_t session_id;
    const float *scan;
    int32_t M;
    const float *noise;
    mcs_step_params p;
    mcs_request_times t;
    int64_t evals;
    bool big;                         // BATCHED mode: runs in the large-session lane
};

// One table buffer of BATCHED mode.  Device and pinned host images share one
// layout: a header (per-stage item counts and offsets), max_batch step
// descriptors, then the work items of all stages packed back to back.  A tick
// copies the header, the descriptors and the used items in one transfer.
struct TableBuf {
    void *dev = nullptr;
    void *host = nullptr;
    size_t items_off = 0, bytes = 0;
    int32_t *counts_h = nullptr, *offs_h = nullptr;
    StepDesc *descs_h = nullptr;
    int2 *items_h = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t stream = nullptr;     // ticks of this buffer run here
    std::vector<int64_t> reqs;        // requests of the tick in flight
    std::unordered_set<int32_t> sessions;   // their sessions
    bool busy = false;
};

// A CONCURRENT-mode request in flight and the event recorded after its work.
struct InFlight {
    int64_t id;
    hipEvent_t ev;
};

constexpr int kMaxInFlight = 256;

}  // namespace

struct mcs_server {
    mcs_ctx *ctx = nullptr;
    int mode = MCS_SERVE_BATCHED;
    int dtype = 0, oob = 0, max_batch = 1, max_items = 0;
    hipStream_t stream = nullptr;     // SERIAL mode
    TableBuf buf[2];
    int next_buf = 0;
    // BATCHED mode, large-session lane: sessions of at least big_tiles
    // evaluation tiles; each frame launched on its session's stream as soon
    // as it arrives (tracked with the in-flight events).
    int big_tiles = 0;
    int64_t tick_cap = 0;             // evaluations per tick (its first frame always fits)
    std::deque<int64_t> pending_big;
    std::deque<InFlight> inflight;    // CONCURRENT mode, launch order
    std::vector<hipEvent_t> ev_free;
    std::vector<hipEvent_t> ev_all;
    std::thread worker, completer;
    std::mutex mu;
    std::condition_variable cv_work, cv_flight, cv_done;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Request> reqs;
    int64_t next_id = 1;
    int64_t completed = 0, submitted = 0;
    int64_t ticks = 0, evals = 0;
    int32_t max_batch_seen = 0;
    bool stop = false, stop_completer = false;
    mcs_status error = MCS_OK;
    std::string error_msg;
};

namespace {

mcs_status alloc_tables(mcs_server *s, TableBuf &b)
{
    const size_t n_hdr = align_up(2 * kNumKinds * sizeof(int32_t));
    const size_t n_desc = align_up((size_t)s->max_batch * sizeof(StepDesc));
    const size_t n_items = align_up((size_t)kNumKinds * s->max_items * sizeof(int2));
    b.items_off = n_hdr + n_desc;
    b.bytes = b.items_off + n_items;
    HIP_TRY(hipMalloc(&b.dev, b.bytes), "hipMalloc(server tables)");
    HIP_TRY(hipHostMalloc(&b.host, b.bytes, hipHostMallocDefault), "hipHostMalloc(server tables)");
    HIP_TRY(hipMemset(b.dev, 0, b.bytes), "hipMemset(server tables)");
    std::memset(b.host, 0, b.bytes);
    char *h = (char *)b.host;
    b.counts_h = (int32_t *)h;
    b.offs_h = b.counts_h + kNumKinds;
    b.descs_h = (StepDesc *)(h + n_hdr);
    b.items_h = (int2 *)(h + b.items_off);
    HIP_TRY(hipEventCreateWithFlags(&b.done, hipEventDisableTiming), "hipEventCreate");
    HIP_TRY(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking), "hipStreamCreate");
    char *d = (char *)b.dev;
    BatchTables t{};
    t.counts = (const int32_t *)d;
    t.offs = t.counts + kNumKinds;
    t.descs = (const StepDesc *)(d + n_hdr);
    t.items = (const int2 *)(d + b.items_off);
    HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal), "capture begin");
    hipError_t e = launch_batch(t, s->dtype, s->oob == MCS_OOB_SKIP, b.stream);
    hipError_t e2 = hipStreamEndCapture(b.stream, &b.graph);
    if (e != hipSuccess) return hip_fail(e, "capture launch");
    if (e2 != hipSuccess) return hip_fail(e2, "capture end");
    HIP_TRY(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return MCS_OK;
}

void free_tables(TableBuf &b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.stream) (void)hipStreamDestroy(b.stream);
    if (b.dev) (void)hipFree(b.dev);
    if (b.host) (void)hipHostFree(b.host);
    b = TableBuf{};
}

// Record the first error (s->mu held).
void set_error_locked(mcs_server *s, mcs_status st, const char *msg)
{
    if (s->error == MCS_OK) {
        s->error = st;
        s->error_msg = msg;
    }
}

// Retire one request at time t (s->mu held).
void retire(mcs_server *s, int64_t id, int64_t t, bool ok)
{
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return;
    it->second.t.done_ns = ok ? t : -1;
    if (ok) s->evals += it->second.evals;
    s->completed++;
}

// Build and launch one tick from the pending queue (mutex held by caller on
// entry; released while touching the device).  Returns false if nothing ran.
bool launch_tick(mcs_server *s, std::unique_lock<std::mutex> &lk, TableBuf &b, TableBuf &other)
{
    // The oldest pending frame, then the smallest frames of other sessions
    // (each session's oldest) while the tick's evaluations stay under the cap.
    std::vector<int64_t> heads;
    {
        std::unordered_set<int32_t> seen;
        for (int64_t id : s->pending) {
            const Request &r = s->reqs[id];
            if (seen.insert(r.session_id).second) heads.push_back(id);
        }
    }
    if (heads.empty()) return false;
    std::vector<int64_t> take = {heads[0]};
    int64_t work = s->reqs[heads[0]].evals;
    std::vector<int64_t> rest(heads.begin() + 1, heads.end());
    std::stable_sort(rest.begin(), rest.end(),
                     [&](int64_t a, int64_t b) { return s->reqs[a].evals < s->reqs[b].evals; });
    for (int64_t id : rest) {
        if ((int)take.size() >= s->max_batch) break;
        const int64_t w = s->reqs[id].evals;
        if (work + w > s->tick_cap) break;
        take.push_back(id);
        work += w;
    }
    {
        std::unordered_set<int64_t> taken(take.begin(), take.end());
        std::deque<int64_t> keep;
        for (int64_t id : s->pending)
            if (!taken.count(id)) keep.push_back(id);
        s->pending.swap(keep);
    }
    std::vector<Request> rq;
    for (int64_t id : take) rq.push_back(s->reqs[id]);
    // A session still running in the other buffer's tick orders this tick
    // after it; otherwise the two ticks may overlap on the device.
    bool depends = false;
    if (other.busy)
        for (auto &r : rq) depends = depends || other.sessions.count(r.session_id) > 0;
    lk.unlock();
    const int64_t t_launch = now_ns();
    std::vector<std::array<int, kNumKinds>> needs;
    std::vector<int64_t> run, deferred;
    std::unordered_set<int32_t> tick_sessions;
    int32_t counts[kNumKinds] = {0};
    int used = 0;
    for (auto &r : rq) {
        Session *ss = find_session(s->ctx, r.session_id);
        if (!ss) {
            run.push_back(r.id);   // validated at submission; a destroyed session is skipped
            continue;
        }
        StepDesc d = make_desc(ss, r.scan, r.M, r.noise, &r.p);
        d.order = nullptr;   // the batched stages evaluate in slot order
        const int nb = weight_blocks(d.N), nt = particle_tiles(d.N), ns = scan_blocks(d.M);
        // A session whose tail buffer holds all its tiles (one small enough not
        // to fill the device) is split whole, as on its own stream.
        const bool split = d.tail_tiles >= nt && d.iters + d.post_eval <= kBatchSplitPasses;
        const std::array<int, kNumKinds> need = {ns, d.predict ? nb : 0, split ? 0 : nt, nb, 1, nb, 1, nb, nb,
                                                 d.policy == MCS_RESAMPLE_PRUNE ? nb : 0,
                                                 split ? nt * (kSubChunks / 8) : 0, split ? nt : 0};
        bool fits = true;
        for (int k = 0; k < kNumKinds; ++k) fits = fits && counts[k] + need[k] <= s->max_items;
        if (!fits) {
            deferred.push_back(r.id);   // too much work for one tick's lists: a later tick
            continue;
        }
        for (int k = 0; k < kNumKinds; ++k) counts[k] += need[k];
        b.descs_h[used++] = d;
        needs.push_back(need);
        run.push_back(r.id);
        tick_sessions.insert(r.session_id);
    }
    hipError_t e = hipSuccess;
    if (used > 0) {
        // Stage k's items start at offs[k]; an item is (descriptor, block).
        int total = 0;
        for (int k = 0; k < kNumKinds; ++k) {
            b.counts_h[k] = counts[k];
            b.offs_h[k] = total;
            total += counts[k];
        }
        int fill[kNumKinds];
        for (int k = 0; k < kNumKinds; ++k) fill[k] = b.offs_h[k];
        for (int q = 0; q < used; ++q)
            for (int k = 0; k < kNumKinds; ++k)
                for (int blk = 0; blk < needs[q][k]; ++blk) b.items_h[fill[k]++] = make_int2(q, blk);
        if (depends) e = hipStreamWaitEvent(b.stream, other.done, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.dev, b.host, b.items_off + (size_t)total * sizeof(int2),
                               hipMemcpyHostToDevice, b.stream);
        if (e == hipSuccess) e = hipGraphLaunch(b.exec, b.stream);
        if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
    }
    lk.lock();
    for (auto it = deferred.rbegin(); it != deferred.rend(); ++it) s->pending.push_front(*it);
    if (e != hipSuccess) {
        const mcs_status fs = hip_fail(e, "server tick");
        set_error_locked(s, fs, mcs_last_error());
        // Fail the tick's requests so waiters do not hang.
        for (int64_t id : run) retire(s, id, 0, false);
        s->cv_done.notify_all();
        return false;
    }
    const int64_t t_now = now_ns();
    for (int64_t id : run) {
        Request &r = s->reqs[id];
        r.t.launch_ns = t_launch;
        r.t.tick = (int32_t)s->ticks;
        if (used == 0) retire(s, id, t_now, true);   // only skipped sessions
    }
    if (used == 0) {
        s->cv_done.notify_all();
        return false;
    }
    b.reqs = run;
    b.sessions = tick_sessions;
    b.busy = true;
    s->ticks++;
    if (used > s->max_batch_seen) s->max_batch_seen = used;
    s->cv_flight.notify_all();
    return true;
}

// CONCURRENT mode (and BATCHED mode's large-session lane): launch the oldest
// request of `queue` on its session's stream.
void launch_concurrent(mcs_server *s, std::unique_lock<std::mutex> &lk, std::deque<int64_t> &queue)
{
    const int64_t id = queue.front();
    queue.pop_front();
    const Request r = s->reqs[id];
    hipEvent_t ev = s->ev_free.back();
    s->ev_free.pop_back();
    lk.unlock();
    const int64_t t0 = now_ns();
    mcs_status st = MCS_OK;
    Session *ss = find_session(s->ctx, r.session_id);
    if (ss) {
        st = enqueue_step(ss, r.scan, r.M, r.noise, &r.p, ss->stream);
        if (st == MCS_OK) {
            const hipError_t e = hipEventRecord(ev, ss->stream);
            if (e != hipSuccess) st = hip_fail(e, "event record");
        }
    }
    lk.lock();
    Request &rr = s->reqs[id];
    rr.t.launch_ns = t0;
    rr.t.tick = (int32_t)s->ticks++;
    if (!ss || st != MCS_OK) {
        if (st != MCS_OK) set_error_locked(s, st, mcs_last_error());
        s->ev_free.push_back(ev);
        retire(s, id, now_ns(), false);
        s->cv_done.notify_all();
        return;
    }
    s->inflight.push_back(InFlight{id, ev});
    if ((int32_t)s->inflight.size() > s->max_batch_seen) s->max_batch_seen = (int32_t)s->inflight.size();
    s->cv_flight.notify_all();
}

void run_serial(mcs_server *s, std::unique_lock<std::mutex> &lk)
{
    const int64_t id = s->pending.front();
    s->pending.pop_front();
    Request r = s->reqs[id];
    lk.unlock();
    const int64_t t0 = now_ns();
    mcs_status st = MCS_OK;
    Session *ss = find_session(s->ctx, r.session_id);
    if (ss) {
        st = enqueue_step(ss, r.scan, r.M, r.noise, &r.p, s->stream);
        if (st == MCS_OK) {
            hipError_t e = hipStreamSynchronize(s->stream);
            if (e != hipSuccess) st = hip_fail(e, "serial step");
        }
    }
    const int64_t t1 = now_ns();
    lk.lock();
    if (st != MCS_OK) set_error_locked(s, st, mcs_last_error());
    Request &rr = s->reqs[id];
    rr.t.launch_ns = t0;
    rr.t.tick = (int32_t)s->ticks++;
    retire(s, id, t1, st == MCS_OK);
    if (s->max_batch_seen < 1) s->max_batch_seen = 1;
    s->cv_done.notify_all();
}

bool can_launch(const mcs_server *s)
{
    if (s->mode == MCS_SERVE_BATCHED)
        return (!s->pending.empty() && !s->buf[s->next_buf].busy) ||
               (!s->pending_big.empty() && !s->ev_free.empty());
    if (s->pending.empty()) return false;
    if (s->mode == MCS_SERVE_CONCURRENT) return !s->ev_free.empty();
    return true;
}

void worker_main(mcs_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (!can_launch(s)) {
            if (s->stop && s->pending.empty() && s->pending_big.empty()) break;
            s->cv_work.wait(lk);
            continue;
        }
        if (s->mode == MCS_SERVE_SERIAL) {
            run_serial(s, lk);
        } else if (s->mode == MCS_SERVE_CONCURRENT) {
            launch_concurrent(s, lk, s->pending);
        } else if (!s->pending_big.empty() && !s->ev_free.empty()) {
            launch_concurrent(s, lk, s->pending_big);
        } else {
            TableBuf &nb = s->buf[s->next_buf];
            if (launch_tick(s, lk, nb, s->buf[s->next_buf ^ 1])) s->next_buf ^= 1;
        }
    }
}

// Watches the work in flight without sleeping and retires each request as
// soon as its event has completed.
void completer_main(mcs_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        const bool any = s->buf[0].busy || s->buf[1].busy || !s->inflight.empty();
        if (!any) {
            if (s->stop_completer) break;
            s->cv_flight.wait(lk);
            continue;
        }
        // Snapshot the events to query: buffers k >= 0, in-flight entries -1 - k.
        std::vector<std::pair<int, hipEvent_t>> q;
        for (int k = 0; k < 2; ++k)
            if (s->buf[k].busy) q.emplace_back(k, s->buf[k].done);

        for (size_t k = 0; k < s->inflight.size(); ++k) q.emplace_back(-1 - (int)k, s->inflight[k].ev);
        lk.unlock();
        std::vector<std::pair<int, hipError_t>> ready;
        for (auto &x : q) {
            const hipError_t e = hipEventQuery(x.second);
            if (e != hipErrorNotReady) ready.emplace_back(x.first, e);
        }
        const int64_t t = now_ns();
        if (ready.empty()) {
            std::this_thread::yield();
            lk.lock();
            continue;
        }
        lk.lock();
        std::vector<bool> gone(s->inflight.size(), false);
        bool any_gone = false;
        for (auto &x : ready) {
            const bool ok = x.second == hipSuccess;
            if (!ok) {
                const mcs_status fs = hip_fail(x.second, "server work");
                set_error_locked(s, fs, mcs_last_error());
            }
            if (x.first >= 0) {
                TableBuf &b = s->buf[x.first];
                for (int64_t id : b.reqs) retire(s, id, t, ok);
                b.reqs.clear();
                b.sessions.clear();
                b.busy = false;
            } else {
                // Only this thread removes entries, so the snapshot's indices still hold.
                const size_t k = (size_t)(-1 - x.first);
                retire(s, s->inflight[k].id, t, ok);
                s->ev_free.push_back(s->inflight[k].ev);
                gone[k] = true;
                any_gone = true;
            }
        }
        if (any_gone) {
            std::deque<InFlight> keep;
            for (size_t k = 0; k < s->inflight.size(); ++k)
                if (k >= gone.size() || !gone[k]) keep.push_back(s->inflight[k]);
            s->inflight.swap(keep);
        }
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
}

void destroy_server(mcs_server *s)
{
    for (auto &b : s->buf) free_tables(b);
    for (hipEvent_t e : s->ev_all) (void)hipEventDestroy(e);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // namespace

extern "C" {

mcs_status mcs_server_create(mcs_ctx *ctx, int32_t mode, int32_t dtype, int32_t oob,
                             int32_t max_batch, int32_t max_items, mcs_server **out)
{
    if (!ctx || !out) return fail(MCS_EINVAL, "NULL argument");
    *out = nullptr;
    if (mode != MCS_SERVE_BATCHED && mode != MCS_SERVE_SERIAL && mode != MCS_SERVE_CONCURRENT)
        return fail(MCS_EINVAL, "bad mode");
    if (dtype < MCS_GRID_FP32 || dtype > MCS_GRID_BF16) return fail(MCS_EINVAL, "bad dtype");
    if (oob != MCS_OOB_FLOOR && oob != MCS_OOB_SKIP) return fail(MCS_EINVAL, "bad oob");
    if (max_batch < 1 || max_batch > 4096) return fail(MCS_EINVAL, "max_batch outside [1, 4096]");
    if (max_items < 0 || max_items > (1 << 24)) return fail(MCS_EINVAL, "max_items outside [0, 2^24]");
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    mcs_server *s = new mcs_server;
    s->ctx = ctx;
    s->mode = mode;
    s->dtype = dtype;
    s->oob = oob;
    s->max_batch = max_batch;
    s->max_items = max_items > 0 ? max_items : 262144;
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        s->stream = nullptr;
        destroy_server(s);
        return hip_fail(e, "hipStreamCreate");
    }
    if (mode == MCS_SERVE_BATCHED) {
        // One round of evaluation tiles (0 if the device cannot be queried:
        // then every session goes through the ticks).  A tick holds at most a
        // round's worth of work at 2,048 points and 3 passes.
        s->big_tiles = eval_round_tiles(dtype);
        s->tick_cap = s->big_tiles > 0 ? (int64_t)s->big_tiles * kParticleTile * 2048 * 3 : INT64_MAX;
        for (auto &b : s->buf) {
            if ((st = alloc_tables(s, b)) != MCS_OK) {
                destroy_server(s);
                return st;
            }
        }
    }
    if (mode == MCS_SERVE_CONCURRENT || mode == MCS_SERVE_BATCHED) {
        for (int k = 0; k < kMaxInFlight; ++k) {
            hipEvent_t ev;
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
                destroy_server(s);
                return hip_fail(e, "hipEventCreate");
            }
            s->ev_all.push_back(ev);
            s->ev_free.push_back(ev);
        }
    }
    s->worker = std::thread(worker_main, s);
    s->completer = std::thread(completer_main, s);
    *out = s;
    return MCS_OK;
}

mcs_status mcs_server_drain(mcs_server *s)
{
    if (!s) return fail(MCS_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_work.notify_all();
    s->cv_done.wait(lk, [&] { return s->completed >= s->submitted; });
    if (s->error != MCS_OK) return fail(s->error, "%s", s->error_msg.c_str());
    return MCS_OK;
}

mcs_status mcs_server_destroy(mcs_server *s)
{
    if (!s) return MCS_OK;
    mcs_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_completer = true;
        s->cv_flight.notify_all();
    }
    s->completer.join();
    (void)hipSetDevice(s->ctx->device);
    (void)hipDeviceSynchronize();
    destroy_server(s);
    return MCS_OK;
}

mcs_status mcs_server_submit(mcs_server *s, int32_t sid, const float *scan_dev, int32_t M,
                             const float *noise_dev, const mcs_step_params *p, int64_t *request_id)
{
    if (!s || !scan_dev || !p || !request_id) return fail(MCS_EINVAL, "NULL argument");
    Session *ss = find_session(s->ctx, sid);
    if (!ss) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = validate_params(ss, p, M);
    if (st != MCS_OK) return st;
    if (ss->K_cap > 0) return fail(MCS_EINVAL, "the server runs single-grid sessions only");
    if (ss->map->desc.dtype != s->dtype) return fail(MCS_EINVAL, "session grid dtype differs from the server's");
    if ((p->oob == MCS_OOB_SKIP) != (s->oob == MCS_OOB_SKIP))
        return fail(MCS_EINVAL, "out-of-grid rule differs from the server's");
    StepDesc probe = make_desc(ss, scan_dev, M, noise_dev, p);
    if (!eval_supported(probe)) return fail(MCS_EINVAL, "map not supported");
    // A wide grid (64-bit record addresses) always takes the large-session
    // lane, whose kernels are the plain session's.
    const bool big = s->mode == MCS_SERVE_BATCHED &&
                     ((s->big_tiles > 0 && particle_tiles(ss->N) >= s->big_tiles) || grid_is_wide(probe));
    if (!big && (particle_tiles(ss->N) > s->max_items || weight_blocks(ss->N) > s->max_items ||
                 scan_blocks(M) > s->max_items))
        return fail(MCS_EINVAL, "session work exceeds the server's per-tick work lists");
    Request r{};
    r.session_id = sid;
    r.scan = scan_dev;
    r.M = M;
    r.noise = p->predict ? noise_dev : nullptr;
    r.p = *p;
    r.t.session_id = sid;
    r.t.submit_ns = now_ns();
    r.t.tick = -1;
    r.evals = (int64_t)ss->N * M * (p->iters + (p->post_eval ? 1 : 0));
    r.big = big;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(MCS_EBUSY, "server is stopping");
    r.id = s->next_id++;
    s->reqs[r.id] = r;
    (big ? s->pending_big : s->pending).push_back(r.id);
    s->submitted++;
    *request_id = r.id;
    s->cv_work.notify_one();
    return MCS_OK;
}

mcs_status mcs_server_times(mcs_server *s, int64_t id, mcs_request_times *out)
{
    if (!s || !out) return fail(MCS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MCS_ENOTFOUND, "no request %lld", (long long)id);
    if (it->second.t.done_ns == 0) return fail(MCS_EBUSY, "request %lld pending", (long long)id);
    if (it->second.t.done_ns < 0) return fail(MCS_EDEVICE, "request %lld failed", (long long)id);
    *out = it->second.t;
    return MCS_OK;
}

mcs_status mcs_server_stats_get(mcs_server *s, mcs_server_stats *out)
{
    if (!s || !out) return fail(MCS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->requests = s->completed;
    out->ticks = s->ticks;
    out->evals = s->evals;
    out->max_batch_seen = s->max_batch_seen;
    out->pad = 0;
    return MCS_OK;
}

}  // extern "C"
