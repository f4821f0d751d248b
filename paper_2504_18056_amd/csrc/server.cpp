// Serving: a request loop that runs the frames of many concurrent sessions.
//
// BATCHED mode forms ticks of at most one pending frame per session, writes
// one table of step descriptors and per-stage work items into pinned host
// memory, copies it to the device and replays a HIP graph of persistent
// kernels captured once per table buffer.  Two table buffers alternate so a
// tick can be prepared and queued while the previous one runs.  SERIAL mode
// runs one request at a time with the per-session launches and waits for it.
#include "state.h"

#include <chrono>
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
};

// One table buffer: device tables, their pinned host mirror and the graph
// that reads them.
struct TableBuf {
    void *dev = nullptr;
    void *host = nullptr;
    size_t bytes = 0;
    StepDesc *descs_d = nullptr, *descs_h = nullptr;
    int2 *items_d[kNumKinds] = {}, *items_h[kNumKinds] = {};
    int32_t *counts_d = nullptr, *counts_h = nullptr;
    unsigned int *heads_d = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t stream = nullptr;     // ticks of this buffer run here
    std::vector<int64_t> reqs;        // requests of the tick in flight
    std::unordered_set<int32_t> sessions;   // their sessions
    bool busy = false;
};

}  // namespace

struct mcs_server {
    mcs_ctx *ctx = nullptr;
    int mode = MCS_SERVE_BATCHED;
    int dtype = 0, oob = 0, max_batch = 1, max_items = 0;
    hipStream_t stream = nullptr;
    TableBuf buf[2];
    int next_buf = 0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Request> reqs;
    int64_t next_id = 1;
    int64_t completed = 0, submitted = 0;
    int64_t ticks = 0, evals = 0;
    int32_t max_batch_seen = 0;
    bool stop = false;
    mcs_status error = MCS_OK;
    std::string error_msg;
};

namespace {

mcs_status alloc_tables(mcs_server *s, TableBuf &b)
{
    const size_t n_desc = align_up((size_t)s->max_batch * sizeof(StepDesc));
    const size_t n_items = align_up((size_t)s->max_items * sizeof(int2));
    const size_t n_counts = align_up(kNumKinds * sizeof(int32_t));
    const size_t n_heads = align_up(kNumKinds * sizeof(unsigned int));
    b.bytes = n_desc + kNumKinds * n_items + n_counts + n_heads;
    HIP_TRY(hipMalloc(&b.dev, b.bytes), "hipMalloc(server tables)");
    HIP_TRY(hipHostMalloc(&b.host, b.bytes, hipHostMallocDefault), "hipHostMalloc(server tables)");
    HIP_TRY(hipMemset(b.dev, 0, b.bytes), "hipMemset(server tables)");
    std::memset(b.host, 0, b.bytes);
    char *d = (char *)b.dev, *h = (char *)b.host;
    size_t o = 0;
    b.descs_d = (StepDesc *)(d + o); b.descs_h = (StepDesc *)(h + o); o += n_desc;
    for (int k = 0; k < kNumKinds; ++k) {
        b.items_d[k] = (int2 *)(d + o);
        b.items_h[k] = (int2 *)(h + o);
        o += n_items;
    }
    b.counts_d = (int32_t *)(d + o); b.counts_h = (int32_t *)(h + o); o += n_counts;
    b.heads_d = (unsigned int *)(d + o);
    HIP_TRY(hipEventCreateWithFlags(&b.done, hipEventDisableTiming), "hipEventCreate");
    HIP_TRY(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking), "hipStreamCreate");
    if (s->mode == MCS_SERVE_BATCHED) {
        BatchTables t{};
        t.descs = b.descs_d;
        for (int k = 0; k < kNumKinds; ++k) t.items[k] = b.items_d[k];
        t.counts = b.counts_d;
        t.heads = b.heads_d;
        HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal), "capture begin");
        hipError_t e = launch_batch(t, s->dtype, s->oob == MCS_OOB_SKIP, b.stream);
        hipError_t e2 = hipStreamEndCapture(b.stream, &b.graph);
        if (e != hipSuccess) return hip_fail(e, "capture launch");
        if (e2 != hipSuccess) return hip_fail(e2, "capture end");
        HIP_TRY(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
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

void set_error(mcs_server *s, mcs_status st)
{
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error == MCS_OK) {
        s->error = st;
        s->error_msg = mcs_last_error();
    }
}

// Mark the requests of a finished tick complete.
void finish_tick(mcs_server *s, TableBuf &b)
{
    const int64_t t = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    for (int64_t id : b.reqs) {
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) continue;
        it->second.t.done_ns = t;
        s->evals += it->second.evals;
        s->completed++;
    }
    b.reqs.clear();
    b.sessions.clear();
    b.busy = false;
    s->cv_done.notify_all();
}

// Build and launch one tick from the pending queue (mutex held by caller on
// entry; released while touching the device).  Returns false if nothing ran.
bool launch_tick(mcs_server *s, std::unique_lock<std::mutex> &lk, TableBuf &b, TableBuf &other)
{
    // Pick at most one pending frame per session, oldest first.
    std::vector<int64_t> take;
    std::unordered_set<int32_t> seen;
    for (auto it = s->pending.begin(); it != s->pending.end() && (int)take.size() < s->max_batch;) {
        const Request &r = s->reqs[*it];
        if (seen.count(r.session_id)) { ++it; continue; }
        seen.insert(r.session_id);
        take.push_back(*it);
        it = s->pending.erase(it);
    }
    if (take.empty()) return false;
    std::vector<Request> rq;
    for (int64_t id : take) rq.push_back(s->reqs[id]);
    lk.unlock();
    int32_t counts[kNumKinds] = {0};
    int used = 0;
    const int64_t t_launch = now_ns();
    std::vector<int64_t> run;
    // A session still running in the other buffer's tick orders this tick
    // after it; otherwise the two ticks may overlap on the device.
    bool depends = false;
    if (other.busy)
        for (auto &r : rq) depends = depends || other.sessions.count(r.session_id) > 0;
    std::unordered_set<int32_t> tick_sessions;
    for (auto &r : rq) {
        Session *ss = find_session(s->ctx, r.session_id);
        if (!ss) continue;   // validated at submission; a destroyed session is skipped
        const StepDesc d = make_desc(ss, r.scan, r.M, r.noise, &r.p);
        const int nb = weight_blocks(d.N), nt = particle_tiles(d.N), ns = scan_blocks(d.M);
        const int need[kNumKinds] = {ns, d.predict ? nb : 0, nt, nb, nb, nb, nb};
        bool fits = true;
        for (int k = 0; k < kNumKinds; ++k) fits = fits && counts[k] + need[k] <= s->max_items;
        if (!fits) {
            // Too much work for one tick's lists: run it in a later tick.
            std::lock_guard<std::mutex> g(s->mu);
            s->pending.push_front(r.id);
            continue;
        }
        b.descs_h[used] = d;
        for (int k = 0; k < kNumKinds; ++k)
            for (int q = 0; q < need[k]; ++q) b.items_h[k][counts[k]++] = make_int2(used, q);
        ++used;
        run.push_back(r.id);
        tick_sessions.insert(r.session_id);
    }
    for (int k = 0; k < kNumKinds; ++k) b.counts_h[k] = counts[k];
    hipError_t e = hipSuccess;
    if (used > 0) {
        if (depends) e = hipStreamWaitEvent(b.stream, other.done, 0);
        // Copy only the used parts of the tables.
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.descs_d, b.descs_h, used * sizeof(StepDesc), hipMemcpyHostToDevice,
                               b.stream);
        for (int k = 0; k < kNumKinds && e == hipSuccess; ++k)
            if (counts[k] > 0)
                e = hipMemcpyAsync(b.items_d[k], b.items_h[k], counts[k] * sizeof(int2),
                                   hipMemcpyHostToDevice, b.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.counts_d, b.counts_h, kNumKinds * sizeof(int32_t),
                               hipMemcpyHostToDevice, b.stream);
        if (e == hipSuccess) e = hipGraphLaunch(b.exec, b.stream);
        if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
    }
    lk.lock();
    if (e != hipSuccess) {
        lk.unlock();
        set_error(s, hip_fail(e, "server tick"));
        lk.lock();
        // Fail the tick's requests so waiters do not hang.
        for (int64_t id : run) s->reqs[id].t.done_ns = -1, s->completed++;
        s->cv_done.notify_all();
        return false;
    }
    if (used == 0) return false;
    for (int64_t id : run) {
        Request &r = s->reqs[id];
        r.t.launch_ns = t_launch;
        r.t.tick = (int32_t)s->ticks;
    }
    b.reqs = run;
    b.sessions = tick_sessions;
    b.busy = true;
    s->ticks++;
    if (used > s->max_batch_seen) s->max_batch_seen = used;
    return true;
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
    if (st != MCS_OK) set_error(s, st);
    lk.lock();
    Request &rr = s->reqs[id];
    rr.t.launch_ns = t0;
    rr.t.done_ns = st == MCS_OK ? t1 : -1;
    rr.t.tick = (int32_t)s->ticks++;
    s->evals += st == MCS_OK ? rr.evals : 0;
    s->completed++;
    if (s->max_batch_seen < 1) s->max_batch_seen = 1;
    s->cv_done.notify_all();
}

void worker_main(mcs_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->mode == MCS_SERVE_SERIAL) {
            if (s->pending.empty()) {
                if (s->stop) break;
                s->cv_work.wait(lk);
                continue;
            }
            run_serial(s, lk);
            continue;
        }
        // Retire finished ticks without blocking.
        for (auto &b : s->buf) {
            if (!b.busy) continue;
            const hipError_t q = hipEventQuery(b.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) set_error(s, hip_fail(q, "server tick"));
            lk.unlock();
            finish_tick(s, b);
            lk.lock();
        }
        // Queue a tick into a free buffer (ticks alternate between the two).
        bool launched = false;
        TableBuf &nb = s->buf[s->next_buf];
        if (!nb.busy && !s->pending.empty()) {
            launched = launch_tick(s, lk, nb, s->buf[s->next_buf ^ 1]);
            if (launched) s->next_buf ^= 1;
        }
        if (launched) continue;
        const bool any_busy = s->buf[0].busy || s->buf[1].busy;
        if (!any_busy && s->pending.empty()) {
            if (s->stop) break;
            s->cv_work.wait(lk);
        } else {
            // Work in flight: wake on a new submission or after a short poll interval.
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

extern "C" {

mcs_status mcs_server_create(mcs_ctx *ctx, int32_t mode, int32_t dtype, int32_t oob,
                             int32_t max_batch, int32_t max_items, mcs_server **out)
{
    if (!ctx || !out) return fail(MCS_EINVAL, "NULL argument");
    *out = nullptr;
    if (mode != MCS_SERVE_BATCHED && mode != MCS_SERVE_SERIAL) return fail(MCS_EINVAL, "bad mode");
    if (dtype < MCS_GRID_FP32 || dtype > MCS_GRID_BF16) return fail(MCS_EINVAL, "bad dtype");
    if (oob != MCS_OOB_FLOOR && oob != MCS_OOB_SKIP) return fail(MCS_EINVAL, "bad oob");
    if (max_batch < 1 || max_batch > 4096) return fail(MCS_EINVAL, "max_batch outside [1, 4096]");
    if (max_items < 0) return fail(MCS_EINVAL, "max_items < 0");
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
        delete s;
        return hip_fail(e, "hipStreamCreate");
    }
    for (auto &b : s->buf) {
        if ((st = alloc_tables(s, b)) != MCS_OK) {
            for (auto &bb : s->buf) free_tables(bb);
            (void)hipStreamDestroy(s->stream);
            delete s;
            return st;
        }
    }
    s->worker = std::thread(worker_main, s);
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
    (void)hipSetDevice(s->ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &b : s->buf) free_tables(b);
    (void)hipStreamDestroy(s->stream);
    delete s;
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
    if (ss->K > 0) return fail(MCS_EINVAL, "the server runs single-grid sessions only");
    if (ss->map->desc.dtype != s->dtype) return fail(MCS_EINVAL, "session grid dtype differs from the server's");
    if ((p->oob == MCS_OOB_SKIP) != (s->oob == MCS_OOB_SKIP))
        return fail(MCS_EINVAL, "out-of-grid rule differs from the server's");
    StepDesc probe = make_desc(ss, scan_dev, M, noise_dev, p);
    if (!eval_supported(probe)) return fail(MCS_EINVAL, "map not supported");
    if (weight_blocks(ss->N) > s->max_items || scan_blocks(M) > s->max_items)
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
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(MCS_EBUSY, "server is stopping");
    r.id = s->next_id++;
    s->reqs[r.id] = r;
    s->pending.push_back(r.id);
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
