// C ABI of the MI355X gradient-guided Monte Carlo SLAM particle update: the
// context, the map store, sessions, admission by HBM budget and the step
// sequence enqueued on a session's stream.  Kernels live in kernels.hip.
#include "state.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace mcs;

namespace {
thread_local std::string g_err;
}  // namespace

namespace mcs {

mcs_status fail(mcs_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

mcs_status hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(MCS_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(MCS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

struct Layout {
    size_t off[24];
    size_t total;
};

// Tail tiles of a session on grid map m (single grid or keyframes), and their buffer.
int session_tail_tiles(const Map *m, int N)
{
    return m->kind == kGridMap ? eval_tail_tiles(N, m->desc.dtype, m->K_cap > 0) : 0;
}

size_t tail_bytes(const Map *m, int tail)
{
    return (size_t)tail * (m->K_cap > 0 ? kKfTailBytesPerTile : kTailBytesPerTile);
}

Layout session_layout(int N, int M_max, int K, bool gicp, size_t tail_size)
{
    const size_t n = (size_t)N, nb = (size_t)weight_blocks(N);
    const size_t sizes[] = {
        7 * n * 4,                  // 0 pose
        7 * n * 4,                  // 1 pose_tmp
        n * 4,                      // 2 loglik
        6 * n * 4,                  // 3 grad
        (size_t)K * 7 * n * 4,      // 4 kf_pose
        (size_t)K * 7 * n * 4,      // 5 kf_pose_tmp
        6 * n * 4,                  // 6 noise
        (size_t)M_max * 3 * 4,      // 7 scan3
        (size_t)M_max * 16,         // 8 scan4
        n * 8,                      // 9 logw
        n * 8,                      // 10 cdf_local
        nb * kPartPerBlock * 8,     // 11 part
        n * 4,                      // 12 parents
        (K > 0 ? (size_t)kMaxNeighbors * n * 4 : 0),  // 13 neighbors
        sizeof(StepStatsDev),       // 14 stats
        (size_t)M_max * 32,         // 15 scan8
        n * 4,                      // 16 copies
        (gicp ? (size_t)M_max * kVoxelRecordBytes : 0),   // 17 scan_g
        (gicp ? (size_t)M_max * 6 * 4 : 0),                // 18 cov6
        (gicp ? 21 * n * 4 : 0),                           // 19 hess
        tail_size,                                         // 20 tail sub-chunk sums
        (K == 0 || gicp ? 3 * n * 4 : 0),                  // 21 evaluation order: order, ocell, orank
        (K == 0 || gicp ? (size_t)kOrderCells * 4 : 0),    // 22 ocount
        (K == 0 || gicp ? nb * 2 * kOrderDims * 4 : 0),    // 23 obounds
    };
    Layout L{};
    size_t o = 0;
    for (size_t k = 0; k < sizeof sizes / sizeof sizes[0]; ++k) {
        L.off[k] = o;
        o += align_up(sizes[k]);
    }
    L.total = o;
    return L;
}

}  // namespace


namespace mcs {

mcs_status set_device(mcs_ctx *ctx)
{
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    return MCS_OK;
}

bool budget_allows(const mcs_ctx *ctx, uint64_t extra)
{
    return ctx->budget == 0 || ctx->in_use + extra <= ctx->budget;
}

mcs_status validate_desc(const mcs_grid_desc *d)
{
    if (!d) return fail(MCS_EINVAL, "grid desc is NULL");
    if (d->nx < 2 || d->ny < 2 || d->nz < 2)
        return fail(MCS_EINVAL, "grid dims must be >= 2 (got %d x %d x %d)", d->nx, d->ny, d->nz);
    if (!(d->res > 0.0f) || !std::isfinite(d->res)) return fail(MCS_EINVAL, "grid res must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->origin[a])) return fail(MCS_EINVAL, "grid origin not finite");
    if (d->dtype < MCS_GRID_FP32 || d->dtype > MCS_GRID_BF16)
        return fail(MCS_EINVAL, "unknown grid dtype %d", d->dtype);
    const double cells = (double)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
    if (cells >= 2147483647.0) return fail(MCS_EINVAL, "grid has too many cells (%.0f)", cells);
    if (d->nx > (1 << 24) || d->ny > (1 << 24) || d->nz > (1 << 24))
        return fail(MCS_EINVAL, "grid axis too long");
    return MCS_OK;
}

// Likelihood samples must be finite and in [0, 1].
mcs_status check_samples(const float *v, size_t n, int k)
{
    for (size_t i = 0; i < n; ++i)
        if (!(v[i] >= 0.0f && v[i] <= 1.0f))
            return fail(MCS_EINVAL, "grid %d: sample %zu = %g is not in [0, 1]", k, i, (double)v[i]);
    return MCS_OK;
}

// Upload K host FP32 grids of one shape and convert them into cell records.
mcs_status build_map(mcs_ctx *ctx, int K, const mcs_grid_desc *descs, const float *const *values,
                     int32_t *map_id)
{
    const mcs_grid_desc &d0 = descs[0];
    const size_t samples = (size_t)d0.nx * d0.ny * d0.nz;
    for (int k = 0; k < (K > 0 ? K : 1); ++k) {
        const mcs_status s = check_samples(values[k], samples, k);
        if (s != MCS_OK) return s;
    }
    const int64_t recs = (int64_t)grid_records(d0.nx, d0.ny, d0.nz);
    const size_t grid_bytes = (size_t)recs * record_bytes(d0.dtype);
    const int G = K > 0 ? K : 1;
    const size_t total = align_up(grid_bytes) * G + align_up((size_t)G * 3 * sizeof(float));
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!budget_allows(ctx, total))
            return fail(MCS_EBUDGET, "map needs %zu bytes; budget %llu, in use %llu", total,
                        (unsigned long long)ctx->budget, (unsigned long long)ctx->in_use);
        ctx->in_use += total;
    }
    Map *m = new Map;
    m->K = K;
    m->K_cap = K;
    m->desc = d0;
    m->records = recs;
    m->bytes = total;
    for (int k = 0; k < G; ++k)
        for (int a = 0; a < 3; ++a) m->origins.push_back(descs[k].origin[a]);
    auto undo = [&](mcs_status s) {
        if (m->cells) (void)hipFree(m->cells);
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use -= total;
        delete m;
        return s;
    };
    hipError_t e = hipMalloc(&m->cells, total);
    if (e != hipSuccess) { m->cells = nullptr; return undo(hip_fail(e, "hipMalloc(map)")); }
    m->origins_dev = reinterpret_cast<float *>((char *)m->cells + align_up(grid_bytes) * G);
    float *tmp = nullptr;
    e = hipMalloc(&tmp, samples * sizeof(float));
    if (e != hipSuccess) return undo(hip_fail(e, "hipMalloc(grid staging)"));
    for (int k = 0; k < G && e == hipSuccess; ++k) {
        e = hipMemcpy(tmp, values[k], samples * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_build_cells(tmp, (char *)m->cells + align_up(grid_bytes) * k, d0.nx, d0.ny,
                                   d0.nz, d0.dtype, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e == hipSuccess)
        e = hipMemcpy(m->origins_dev, m->origins.data(), (size_t)G * 3 * sizeof(float),
                      hipMemcpyHostToDevice);
    (void)hipFree(tmp);
    if (e != hipSuccess) return undo(hip_fail(e, "map upload"));
    std::lock_guard<std::mutex> lk(ctx->mu);
    m->id = ctx->next_id++;
    ctx->maps[m->id] = m;
    *map_id = m->id;
    return MCS_OK;
}

Session *find_session(mcs_ctx *ctx, int32_t sid)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->sessions.find(sid);
    return it == ctx->sessions.end() ? nullptr : it->second;
}

void aos_to_soa(const float *aos, float *soa, size_t n, int C)
{
    for (size_t i = 0; i < n; ++i)
        for (int c = 0; c < C; ++c) soa[(size_t)c * n + i] = aos[i * C + c];
}

// Poses: normalise quaternions on the host side of the upload and reject
// non-finite values.
mcs_status check_poses(const float *p, size_t n)
{
    for (size_t i = 0; i < n; ++i) {
        double qq = 0.0;
        for (int c = 0; c < 7; ++c) {
            if (!std::isfinite(p[7 * i + c]) || std::fabs(p[7 * i + c]) > 1e15f)
                return fail(MCS_EINVAL, "pose %zu not finite or beyond 1e15", i);
            if (c >= 3) qq += (double)p[7 * i + c] * p[7 * i + c];
        }
        if (!(qq > 1e-20)) return fail(MCS_EINVAL, "pose %zu has a zero quaternion", i);
    }
    return MCS_OK;
}

mcs_status upload_kf(Session *s, const float *kf_poses)
{
    // Host layout (i, k, c) -> device rows (k*7 + c) of length N.
    const size_t N = s->N, K = s->K;
    std::vector<float> soa(K * 7 * N);
    for (size_t i = 0; i < N; ++i)
        for (size_t k = 0; k < K; ++k)
            for (int c = 0; c < 7; ++c) soa[(k * 7 + c) * N + i] = kf_poses[(i * K + k) * 7 + c];
    HIP_TRY(hipMemcpyAsync(s->kf_pose, soa.data(), soa.size() * 4, hipMemcpyHostToDevice,
                           s->stream), "upload kf poses");
    HIP_TRY(hipStreamSynchronize(s->stream), "sync");
    return MCS_OK;
}

mcs_status validate_params(const Session *s, const mcs_step_params *p, int M)
{
    if (!p) return fail(MCS_EINVAL, "params is NULL");
    if (M < 1 || M > s->M_max) return fail(MCS_EINVAL, "M=%d outside [1, %d]", M, s->M_max);
    if (p->iters < 1 || p->iters > 64) return fail(MCS_EINVAL, "iters=%d outside [1, 64]", p->iters);
    const float fs[] = {p->alpha_t, p->alpha_r, p->rho_max, p->phi_max, p->eps, p->beta};
    for (float f : fs)
        if (!std::isfinite(f)) return fail(MCS_EINVAL, "non-finite step parameter");
    if (!(p->eps > 0.0f)) return fail(MCS_EINVAL, "eps must be > 0");
    // The point loop multiplies up to four factors G + eps (one log2 and one
    // reciprocal per product).  The interpolant of samples in [0, 1] is
    // evaluated with an error below 3e-6 (coefficient rounding and the FMA
    // chain, worst case), so eps >= 1e-5 keeps every factor positive, and
    // eps <= 1 keeps the product of four a normal FP32 number.
    if (s->map->kind == kGridMap && !(p->eps >= 1e-5f && p->eps <= 1.0f))
        return fail(MCS_EINVAL, "eps=%g outside [1e-5, 1]", (double)p->eps);
    if (p->rho_max < 0.0f || p->phi_max < 0.0f) return fail(MCS_EINVAL, "clamps must be >= 0");
    if (p->oob != MCS_OOB_FLOOR && p->oob != MCS_OOB_SKIP) return fail(MCS_EINVAL, "bad oob mode");
    if (p->resample < MCS_RESAMPLE_NEVER || p->resample > MCS_RESAMPLE_PRUNE)
        return fail(MCS_EINVAL, "bad resample policy");
    if (p->resample == MCS_RESAMPLE_PRUNE &&
        !(p->prune_post > 0.0f && p->prune_lik > 0.0f && std::isfinite(p->prune_post) &&
          std::isfinite(p->prune_lik)))
        return fail(MCS_EINVAL, "pruning thresholds must be finite and > 0");
    if (p->noise_mode != MCS_NOISE_INPUT && p->noise_mode != MCS_NOISE_DEVICE)
        return fail(MCS_EINVAL, "bad noise mode");
    if (p->predict && p->noise_mode == MCS_NOISE_DEVICE)
        for (int c = 0; c < 6; ++c)
            if (!(p->noise_sigma[c] >= 0.0f && std::isfinite(p->noise_sigma[c])))
                return fail(MCS_EINVAL, "noise_sigma must be finite and >= 0");
    if (!(p->u >= 0.0 && p->u < 1.0)) return fail(MCS_EINVAL, "u must be in [0, 1)");
    if (p->resample == MCS_RESAMPLE_ESS && !std::isfinite(p->ess_frac))
        return fail(MCS_EINVAL, "ess_frac not finite");
    if (p->predict) {
        double qq = 0.0;
        for (int c = 0; c < 7; ++c) {
            if (!std::isfinite(p->delta_T[c])) return fail(MCS_EINVAL, "delta_T not finite");
            if (c >= 3) qq += (double)p->delta_T[c] * p->delta_T[c];
        }
        if (!(qq > 1e-20)) return fail(MCS_EINVAL, "delta_T has a zero quaternion");
    }
    if (s->K_cap > 0 && s->K == 0)
        return fail(MCS_EINVAL, "the session has no keyframe yet (mcs_session_add_keyframe)");
    if (s->K > 0 && (p->n_neighbors < 1 || p->n_neighbors > std::min(s->K, kMaxNeighbors)))
        return fail(MCS_EINVAL, "n_neighbors=%d outside [1, %d]", p->n_neighbors,
                    std::min(s->K, kMaxNeighbors));
    if (p->kf_update != MCS_KF_FIXED && p->kf_update != MCS_KF_LOOP)
        return fail(MCS_EINVAL, "bad kf_update mode");
    if (p->kf_update == MCS_KF_LOOP && s->K == 0)
        return fail(MCS_EINVAL, "MCS_KF_LOOP needs a keyframe map");
    if (p->kf_update == MCS_KF_LOOP && p->n_recent < 0)
        return fail(MCS_EINVAL, "n_recent=%d must be >= 0", p->n_recent);
    if (s->trace && p->iters + (p->post_eval ? 1 : 0) > s->trace_passes)
        return fail(MCS_EINVAL, "%d passes exceed the trace's %d", p->iters + (p->post_eval ? 1 : 0),
                    s->trace_passes);
    return MCS_OK;
}

// The device-side description of one step of session s.
StepDesc make_desc(const Session *s, const float *scan3_dev, int M, const float *noise_dev,
                   const mcs_step_params *p, const float *cov_dev)
{
    const Map *m = s->map;
    StepDesc d{};
    d.cells = m->cells;
    d.grid_stride = (int64_t)align_up((size_t)m->records * (m->kind == kVoxelMap
                                                                ? kVoxelDeviceBytes
                                                                : record_bytes(m->desc.dtype)));
    d.gicp = m->kind == kVoxelMap;
    d.cov6 = cov_dev;
    d.scan_g = s->scan_g;
    d.hess = s->hess;
    d.origins = m->origins_dev;
    d.vox_occ = m->occ_dev;
    d.occ_stride = (int64_t)align_up((size_t)m->records);
    d.tail_l = s->tail_l;
    d.tail_g = s->tail_g;
    d.tail_tiles = s->tail_tiles;
    d.nx = m->desc.nx; d.ny = m->desc.ny; d.nz = m->desc.nz;
    d.dtype = m->desc.dtype;
    d.ox = m->desc.origin[0]; d.oy = m->desc.origin[1]; d.oz = m->desc.origin[2];
    d.h = m->desc.res;
    d.inv_h = 1.0f / m->desc.res;
    d.K = s->K;
    d.n_nb = s->K > 0 ? p->n_neighbors : 0;
    d.kf_loop = s->K > 0 && p->kf_update == MCS_KF_LOOP;
    d.n_recent = p->n_recent;
    d.noise_rng = p->predict && p->noise_mode == MCS_NOISE_DEVICE;
    d.rng_seed = p->rng_seed;
    d.rng_frame = p->rng_frame;
    for (int c = 0; c < 6; ++c) d.noise_sigma[c] = p->noise_sigma[c];
    d.ln_prune_post = std::log((double)p->prune_post);
    d.ln_prune_lik = std::log((double)p->prune_lik);
    d.pose = s->pose; d.pose_tmp = s->pose_tmp;
    d.kf_pose = s->kf_pose; d.kf_pose_tmp = s->kf_pose_tmp;
    d.loglik = s->loglik; d.grad = s->grad;
    d.logw = s->logw; d.cdf_local = s->cdf_local; d.part = s->part;
    d.parents = s->parents; d.copies = s->copies; d.neighbors = s->neighbors;
    d.stats = s->stats;
    d.N = s->N; d.M = M;
    d.scan3 = scan3_dev; d.scan4 = s->scan4; d.scan8 = s->scan8;
    d.noise = p->predict ? noise_dev : nullptr;
    d.iters = p->iters;
    d.post_eval = p->post_eval ? 1 : 0;
    d.oob_skip = p->oob == MCS_OOB_SKIP;
    d.predict = p->predict ? 1 : 0;
    d.policy = p->resample;
    d.alpha_t = p->alpha_t; d.alpha_r = p->alpha_r;
    d.rho_max = p->rho_max; d.phi_max = p->phi_max;
    d.eps = p->eps;
    d.beta = (double)p->beta;
    d.ess_frac = p->ess_frac;
    d.u = p->u;
    for (int c = 0; c < 7; ++c) d.dT[c] = p->delta_T[c];
    d.trace = s->trace;
    if (s->order && s->N >= kOrderMinParticles) {
        d.order = s->order;
        d.ocell = s->ocell;
        d.orank = s->orank;
        d.ocount = s->ocount;
        d.obounds = s->obounds;
    }
    return d;
}

// Events of the next profiled step (nullptr entries when not profiling).
mcs_status prof_begin(Session *s, std::array<hipEvent_t, 5> *&ev)
{
    ev = nullptr;
    if (!s->profiling) return MCS_OK;
    if (s->prof_used == s->prof_events.size()) {
        std::array<hipEvent_t, 5> a{};
        for (auto &e : a) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
        s->prof_events.push_back(a);
    }
    ev = &s->prof_events[s->prof_used++];
    return MCS_OK;
}

#define PROF_MARK(k)                                                     \
    do {                                                                 \
        if (ev) HIP_TRY(hipEventRecord((*ev)[k], st), "hipEventRecord"); \
    } while (0)

// The step sequence of one session on stream st.
mcs_status enqueue_step(Session *s, const float *scan3_dev, int M, const float *noise_dev,
                        const mcs_step_params *p, hipStream_t st, const float *cov_dev)
{
    if ((s->map->kind == kVoxelMap) != (cov_dev != nullptr))
        return fail(MCS_EINVAL, s->map->kind == kVoxelMap
                                    ? "a GICP map needs scan covariances (mcs_filter_step_gicp*)"
                                    : "scan covariances are for GICP maps only");
    const StepDesc d = make_desc(s, scan3_dev, M, noise_dev, p, cov_dev);
    if (!eval_supported(d)) return fail(MCS_EINVAL, "map or neighbour count not supported");
    std::array<hipEvent_t, 5> *ev = nullptr;
    mcs_status ps = prof_begin(s, ev);
    if (ps != MCS_OK) return ps;
    if (ev) s->prof_evals += (int64_t)s->N * M * (p->iters + (p->post_eval ? 1 : 0)) *
                             (s->K > 0 ? p->n_neighbors : 1);
    PROF_MARK(0);
    HIP_TRY(launch_pack_predict(d, st), "pack/predict");
    HIP_TRY(launch_order(d, st), "order");
    PROF_MARK(1);
    const TailAux aux{s->tail_stream, s->tail_fork, s->tail_join};
    HIP_TRY(launch_eval(d, st, s->tail_stream ? &aux : nullptr), "eval");
    if (s->K > 0) s->last_nb = p->n_neighbors;
    PROF_MARK(2);
    HIP_TRY(launch_weights(d, st), "weights");
    PROF_MARK(3);
    HIP_TRY(launch_resample(d, st), "resample");
    PROF_MARK(4);
    return MCS_OK;
}

// Fold the recorded events into the accumulated stage times.
mcs_status prof_collect(Session *s)
{
    for (size_t k = 0; k < s->prof_used; ++k) {
        auto &e = s->prof_events[k];
        HIP_TRY(hipEventSynchronize(e[4]), "hipEventSynchronize");
        for (int j = 0; j < 4; ++j) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e[j], e[j + 1]), "hipEventElapsedTime");
            s->prof_ms[j] += ms;
        }
        s->prof_steps++;
    }
    s->prof_used = 0;
    return MCS_OK;
}

void prof_release(Session *s)
{
    for (auto &a : s->prof_events)
        for (auto e : a) (void)hipEventDestroy(e);
    s->prof_events.clear();
    s->prof_used = 0;
}

}  // namespace

extern "C" {

const char *mcs_version(void) { return "mcslam-gfx950 0.1"; }

const char *mcs_last_error(void) { return g_err.c_str(); }

mcs_status mcs_create(int32_t device, uint64_t hbm_budget_bytes, mcs_ctx **out)
{
    if (!out) return fail(MCS_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(MCS_EINVAL, "device %d not in [0, %d)", device, n);
    HIP_TRY(hipSetDevice(device), "hipSetDevice");
    void *scr = nullptr;
    HIP_TRY(scratch_init(device, &scr), "hipGetSymbolAddress(scratch)");
    mcs_ctx *c = new mcs_ctx;
    c->device = device;
    c->budget = hbm_budget_bytes;
    c->scratch = scr;
    *out = c;
    return MCS_OK;
}

mcs_status mcs_session_destroy(mcs_ctx *ctx, int32_t sid);

mcs_status mcs_destroy(mcs_ctx *ctx)
{
    if (!ctx) return MCS_OK;
    std::vector<int> ids;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &kv : ctx->sessions) ids.push_back(kv.first);
    }
    for (int id : ids) mcs_session_destroy(ctx, id);
    for (auto &kv : ctx->maps) {
        (void)hipFree(kv.second->cells);
        delete kv.second;
    }
    delete ctx;
    return MCS_OK;
}

mcs_status mcs_memory_in_use(mcs_ctx *ctx, uint64_t *bytes)
{
    if (!ctx || !bytes) return fail(MCS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    *bytes = ctx->in_use;
    return MCS_OK;
}

mcs_status mcs_init_map(mcs_ctx *ctx, const mcs_grid_desc *desc, const float *values,
                        int32_t *map_id)
{
    if (!ctx || !values || !map_id) return fail(MCS_EINVAL, "NULL argument");
    mcs_status s = validate_desc(desc);
    if (s != MCS_OK) return s;
    if (!grid_supported(desc->nx, desc->ny, desc->nz, desc->dtype, false))
        return fail(MCS_EINVAL, "grid has 2^32 or more records");
    if ((s = set_device(ctx)) != MCS_OK) return s;
    const float *v[1] = {values};
    return build_map(ctx, 0, desc, v, map_id);
}

mcs_status mcs_load_keyframes(mcs_ctx *ctx, int32_t K, const mcs_grid_desc *descs,
                              const float *const *values, int32_t *map_id)
{
    if (!ctx || !descs || !values || !map_id) return fail(MCS_EINVAL, "NULL argument");
    if (K < 1) return fail(MCS_EINVAL, "K must be >= 1");
    for (int k = 0; k < K; ++k) {
        mcs_status s = validate_desc(&descs[k]);
        if (s != MCS_OK) return s;
        if (!values[k]) return fail(MCS_EINVAL, "keyframe grid %d is NULL", k);
        if (descs[k].nx != descs[0].nx || descs[k].ny != descs[0].ny || descs[k].nz != descs[0].nz ||
            descs[k].res != descs[0].res || descs[k].dtype != descs[0].dtype)
            return fail(MCS_EINVAL, "keyframe grid %d differs in shape, res or dtype", k);
    }
    if (!grid_supported(descs[0].nx, descs[0].ny, descs[0].nz, descs[0].dtype, true))
        return fail(MCS_EINVAL, "keyframe grid too large (32-bit record offsets, 24-bit row and slab products)");
    mcs_status s = set_device(ctx);
    if (s != MCS_OK) return s;
    return build_map(ctx, K, descs, values, map_id);
}

mcs_status mcs_load_gicp_keyframes(mcs_ctx *ctx, int32_t K, const mcs_voxel_desc *descs,
                                   const float *const *voxels, int32_t *map_id)
{
    if (!ctx || !descs || !voxels || !map_id) return fail(MCS_EINVAL, "NULL argument");
    if (K < 1) return fail(MCS_EINVAL, "K must be >= 1");
    const mcs_voxel_desc &d0 = descs[0];
    for (int k = 0; k < K; ++k) {
        const mcs_voxel_desc &d = descs[k];
        if (d.nx < 1 || d.ny < 1 || d.nz < 1 || d.nx > (1 << 16) || d.ny > (1 << 16) || d.nz > (1 << 16))
            return fail(MCS_EINVAL, "voxel map %d: dims outside [1, 65536]", k);
        if (!(d.edge > 0.0f) || !std::isfinite(d.edge)) return fail(MCS_EINVAL, "voxel map %d: bad edge", k);
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(d.origin[a])) return fail(MCS_EINVAL, "voxel map %d: bad origin", k);
        if (d.nx != d0.nx || d.ny != d0.ny || d.nz != d0.nz || d.edge != d0.edge)
            return fail(MCS_EINVAL, "voxel map %d differs in shape or edge", k);
        if (!voxels[k]) return fail(MCS_EINVAL, "voxel map %d is NULL", k);
    }
    const int64_t recs = (int64_t)d0.nx * d0.ny * d0.nz;
    if (recs >= (int64_t)1 << 31) return fail(MCS_EINVAL, "voxel map has 2^31 or more voxels");
    if ((int64_t)d0.nx * d0.ny >= (int64_t)1 << 24)
        return fail(MCS_EINVAL, "voxel map rows times columns must stay below 2^24");
    mcs_status s = set_device(ctx);
    if (s != MCS_OK) return s;
    const size_t map_bytes = (size_t)recs * kVoxelDeviceBytes;
    const size_t occ_stride = align_up((size_t)recs);
    if (occ_stride * (size_t)K >= ((size_t)1 << 32) - 1)
        return fail(MCS_EINVAL, "voxel maps hold 2^32 or more voxels in total");
    const size_t total = align_up(map_bytes) * K + align_up((size_t)K * 3 * sizeof(float)) + occ_stride * K;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!budget_allows(ctx, total))
            return fail(MCS_EBUDGET, "map needs %zu bytes; budget %llu, in use %llu", total,
                        (unsigned long long)ctx->budget, (unsigned long long)ctx->in_use);
        ctx->in_use += total;
    }
    Map *m = new Map;
    m->kind = kVoxelMap;
    m->K = K;
    m->K_cap = K;
    m->desc.nx = d0.nx; m->desc.ny = d0.ny; m->desc.nz = d0.nz;
    for (int a = 0; a < 3; ++a) m->desc.origin[a] = d0.origin[a];
    m->desc.res = d0.edge;
    m->desc.dtype = MCS_GRID_FP32;
    m->records = recs;
    m->bytes = total;
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < 3; ++a) m->origins.push_back(descs[k].origin[a]);
    hipError_t e = hipMalloc(&m->cells, total);
    if (e == hipSuccess) {
        m->origins_dev = reinterpret_cast<float *>((char *)m->cells + align_up(map_bytes) * K);
        m->occ_dev = reinterpret_cast<uint8_t *>((char *)m->origins_dev + align_up((size_t)K * 3 * sizeof(float)));
        std::vector<uint8_t> occ(occ_stride, 0);
        std::vector<unsigned char> padded(map_bytes, 0);
        for (int k = 0; k < K && e == hipSuccess; ++k) {
            // Records padded to their device stride on the host, then one copy.
            for (int64_t v = 0; v < recs; ++v)
                std::memcpy(&padded[(size_t)v * kVoxelDeviceBytes], &voxels[k][(size_t)v * 12], kVoxelRecordBytes);
            e = hipMemcpy((char *)m->cells + align_up(map_bytes) * k, padded.data(), map_bytes,
                          hipMemcpyHostToDevice);
            // Occupied: a positive point count (the test the kernel makes on the record).
            for (int64_t v = 0; v < recs; ++v) occ[v] = voxels[k][(size_t)v * 12 + 3] > 0.0f ? 1 : 0;
            if (e == hipSuccess)
                e = hipMemcpy(m->occ_dev + occ_stride * k, occ.data(), occ_stride, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess)
            e = hipMemcpy(m->origins_dev, m->origins.data(), (size_t)K * 3 * sizeof(float),
                          hipMemcpyHostToDevice);
    } else {
        m->cells = nullptr;
    }
    if (e != hipSuccess) {
        if (m->cells) (void)hipFree(m->cells);
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->in_use -= total;
        }
        delete m;
        return hip_fail(e, "voxel map upload");
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    m->id = ctx->next_id++;
    ctx->maps[m->id] = m;
    *map_id = m->id;
    return MCS_OK;
}

mcs_status mcs_create_keyframe_map(mcs_ctx *ctx, int32_t K_cap, const mcs_grid_desc *desc,
                                   int32_t *map_id)
{
    if (!ctx || !desc || !map_id) return fail(MCS_EINVAL, "NULL argument");
    if (K_cap < 1 || K_cap > (1 << 16)) return fail(MCS_EINVAL, "K_cap=%d outside [1, 65536]", K_cap);
    mcs_status s = validate_desc(desc);
    if (s != MCS_OK) return s;
    if (!grid_supported(desc->nx, desc->ny, desc->nz, desc->dtype, true))
        return fail(MCS_EINVAL, "keyframe grid too large (32-bit record offsets, 24-bit row and slab products)");
    if ((s = set_device(ctx)) != MCS_OK) return s;
    const int64_t recs = (int64_t)grid_records(desc->nx, desc->ny, desc->nz);
    const size_t grid_bytes = (size_t)recs * record_bytes(desc->dtype);
    const size_t total =
        align_up(grid_bytes) * K_cap + align_up((size_t)K_cap * 3 * sizeof(float));
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!budget_allows(ctx, total))
            return fail(MCS_EBUDGET, "map needs %zu bytes; budget %llu, in use %llu", total,
                        (unsigned long long)ctx->budget, (unsigned long long)ctx->in_use);
        ctx->in_use += total;
    }
    Map *m = new Map;
    m->K = 0;
    m->K_cap = K_cap;
    m->desc = *desc;
    m->records = recs;
    m->bytes = total;
    m->origins.assign((size_t)K_cap * 3, 0.0f);
    hipError_t e = hipMalloc(&m->cells, total);
    if (e != hipSuccess) {
        m->cells = nullptr;
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use -= total;
        delete m;
        return hip_fail(e, "hipMalloc(map)");
    }
    m->origins_dev = reinterpret_cast<float *>((char *)m->cells + align_up(grid_bytes) * K_cap);
    std::lock_guard<std::mutex> lk(ctx->mu);
    m->id = ctx->next_id++;
    ctx->maps[m->id] = m;
    *map_id = m->id;
    return MCS_OK;
}

mcs_status mcs_append_keyframe(mcs_ctx *ctx, int32_t map_id, const mcs_grid_desc *desc,
                               const float *values, int32_t *index)
{
    if (!ctx || !desc || !values || !index) return fail(MCS_EINVAL, "NULL argument");
    mcs_status s = validate_desc(desc);
    if (s != MCS_OK) return s;
    if ((s = set_device(ctx)) != MCS_OK) return s;
    Map *m = nullptr;
    int k = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->maps.find(map_id);
        if (it == ctx->maps.end()) return fail(MCS_ENOTFOUND, "no map %d", map_id);
        m = it->second;
        if (m->kind != kGridMap || m->K_cap == 0) return fail(MCS_EINVAL, "map %d is not a keyframe grid map", map_id);
        if (m->K >= m->K_cap) return fail(MCS_EBUSY, "map %d is full (%d keyframes)", map_id, m->K_cap);
        if (desc->nx != m->desc.nx || desc->ny != m->desc.ny || desc->nz != m->desc.nz ||
            desc->res != m->desc.res || desc->dtype != m->desc.dtype)
            return fail(MCS_EINVAL, "keyframe grid differs in shape, res or dtype");
        k = m->K;
    }
    const size_t samples = (size_t)desc->nx * desc->ny * desc->nz;
    if ((s = check_samples(values, samples, k)) != MCS_OK) return s;
    const size_t grid_bytes = (size_t)m->records * record_bytes(desc->dtype);
    float *tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, samples * sizeof(float)), "hipMalloc(grid staging)");
    hipError_t e = hipMemcpy(tmp, values, samples * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_build_cells(tmp, (char *)m->cells + align_up(grid_bytes) * k, desc->nx, desc->ny,
                               desc->nz, desc->dtype, nullptr);
    if (e == hipSuccess) e = hipMemcpy(m->origins_dev + 3 * k, desc->origin, 3 * sizeof(float),
                                       hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "keyframe upload");
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (int a = 0; a < 3; ++a) m->origins[3 * (size_t)k + a] = desc->origin[a];
    m->K = k + 1;
    *index = k;
    return MCS_OK;
}

mcs_status mcs_session_add_keyframe(mcs_ctx *ctx, int32_t sid, int32_t *index)
{
    if (!ctx || !index) return fail(MCS_EINVAL, "NULL argument");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    int map_k = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        map_k = s->map->K;
    }
    if (s->K_cap == 0) return fail(MCS_EINVAL, "session %d has no keyframe map", sid);
    if (s->K >= map_k) return fail(MCS_EINVAL, "the map has no keyframe %d yet", s->K);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    // Every particle's pose of the new keyframe is its current pose.
    const size_t N = s->N;
    HIP_TRY(hipMemcpyAsync(s->kf_pose + (size_t)s->K * 7 * N, s->pose, 7 * N * sizeof(float),
                           hipMemcpyDeviceToDevice, s->stream), "copy keyframe poses");
    *index = s->K;
    s->K++;
    return MCS_OK;
}

mcs_status mcs_release_map(mcs_ctx *ctx, int32_t map_id)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Map *m = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->maps.find(map_id);
        if (it == ctx->maps.end()) return fail(MCS_ENOTFOUND, "no map %d", map_id);
        if (it->second->users > 0) return fail(MCS_EBUSY, "map %d is used by a session", map_id);
        m = it->second;
        ctx->maps.erase(it);
        ctx->in_use -= m->bytes;
    }
    mcs_status s = set_device(ctx);
    if (s != MCS_OK) return s;
    (void)hipFree(m->cells);
    delete m;
    return MCS_OK;
}

mcs_status mcs_session_bytes(mcs_ctx *ctx, int32_t map_id, int32_t N, int32_t M_max,
                             uint64_t *bytes)
{
    if (!ctx || !bytes) return fail(MCS_EINVAL, "NULL argument");
    if (N < 1 || M_max < 1) return fail(MCS_EINVAL, "N and M_max must be >= 1");
    int K = 0, tail = 0;
    bool gicp = false;
    if (mcs_status s = set_device(ctx)) return s;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->maps.find(map_id);
        if (it == ctx->maps.end()) return fail(MCS_ENOTFOUND, "no map %d", map_id);
        K = it->second->K_cap;
        gicp = it->second->kind == kVoxelMap;
        tail = session_tail_tiles(it->second, N);
        *bytes = session_layout(N, M_max, K, gicp, tail_bytes(it->second, tail)).total;
    }
    return MCS_OK;
}

mcs_status mcs_session_create(mcs_ctx *ctx, int32_t map_id, int32_t N, int32_t M_max,
                              const float *poses, const float *kf_poses, int32_t *session_id)
{
    if (!ctx || !poses || !session_id) return fail(MCS_EINVAL, "NULL argument");
    if (N < 1 || N > (1 << 28)) return fail(MCS_EINVAL, "N=%d outside [1, 2^28]", N);
    if (M_max < 1 || M_max > (1 << 24)) return fail(MCS_EINVAL, "M_max=%d outside [1, 2^24]", M_max);
    mcs_status s = set_device(ctx);
    if (s != MCS_OK) return s;
    if ((s = check_poses(poses, (size_t)N)) != MCS_OK) return s;
    Map *m = nullptr;
    const Layout *Lp = nullptr;
    Layout L{};
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->maps.find(map_id);
        if (it == ctx->maps.end()) return fail(MCS_ENOTFOUND, "no map %d", map_id);
        m = it->second;
        if (m->K > 0 && !kf_poses) return fail(MCS_EINVAL, "keyframe map needs kf_poses");
        L = session_layout(N, M_max, m->K_cap, m->kind == kVoxelMap, tail_bytes(m, session_tail_tiles(m, N)));
        Lp = &L;
        if (!budget_allows(ctx, L.total))
            return fail(MCS_EBUDGET, "session needs %zu bytes; budget %llu, in use %llu", L.total,
                        (unsigned long long)ctx->budget, (unsigned long long)ctx->in_use);
        ctx->in_use += L.total;
        m->users++;
    }
    if (m->K > 0 && (s = check_poses(kf_poses, (size_t)N * m->K)) != MCS_OK) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use -= L.total;
        m->users--;
        return s;
    }
    Session *ss = new Session;
    ss->map = m;
    ss->N = N;
    ss->M_max = M_max;
    ss->K = m->K;
    ss->K_cap = m->K_cap;
    ss->bytes = Lp->total;
    auto undo = [&](mcs_status st) {
        if (ss->block) (void)hipFree(ss->block);
        if (ss->stream) (void)hipStreamDestroy(ss->stream);
        if (ss->staged) (void)hipEventDestroy(ss->staged);
        if (ss->tail_stream) (void)hipStreamDestroy(ss->tail_stream);
        if (ss->tail_fork) (void)hipEventDestroy(ss->tail_fork);
        if (ss->tail_join) (void)hipEventDestroy(ss->tail_join);
        if (ss->pinned) (void)hipHostFree(ss->pinned);
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use -= L.total;
        m->users--;
        delete ss;
        return st;
    };
    hipError_t e = hipMalloc(&ss->block, L.total);
    if (e != hipSuccess) { ss->block = nullptr; return undo(hip_fail(e, "hipMalloc(session)")); }
    e = hipStreamCreateWithFlags(&ss->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { ss->stream = nullptr; return undo(hip_fail(e, "hipStreamCreate")); }
    e = hipEventCreateWithFlags(&ss->staged, hipEventDisableTiming);
    if (e != hipSuccess) { ss->staged = nullptr; return undo(hip_fail(e, "hipEventCreate")); }
    char *b = (char *)ss->block;
    ss->pose = (float *)(b + L.off[0]);
    ss->pose_tmp = (float *)(b + L.off[1]);
    ss->loglik = (float *)(b + L.off[2]);
    ss->grad = (float *)(b + L.off[3]);
    ss->kf_pose = (float *)(b + L.off[4]);
    ss->kf_pose_tmp = (float *)(b + L.off[5]);
    ss->noise = (float *)(b + L.off[6]);
    ss->scan3 = (float *)(b + L.off[7]);
    ss->scan4 = (float4 *)(b + L.off[8]);
    ss->logw = (double *)(b + L.off[9]);
    ss->cdf_local = (double *)(b + L.off[10]);
    ss->part = (double *)(b + L.off[11]);
    ss->parents = (int32_t *)(b + L.off[12]);
    ss->neighbors = (int32_t *)(b + L.off[13]);
    ss->stats = (StepStatsDev *)(b + L.off[14]);
    ss->scan8 = (double4 *)(b + L.off[15]);
    ss->copies = (int32_t *)(b + L.off[16]);
    if ((m->K_cap == 0 && m->kind == kGridMap) || m->kind == kVoxelMap) {
        ss->order = (int32_t *)(b + L.off[21]);
        ss->ocell = ss->order + N;
        ss->orank = ss->ocell + N;
        ss->ocount = (int32_t *)(b + L.off[22]);
        ss->obounds = (float *)(b + L.off[23]);
    }
    if (m->kind == kVoxelMap) {
        ss->scan_g = (float4 *)(b + L.off[17]);
        ss->cov6 = (float *)(b + L.off[18]);
        ss->hess = (float *)(b + L.off[19]);
    }
    if (L.off[20] < L.total) {
        const int tail = session_tail_tiles(m, N);
        ss->tail_tiles = tail;
        ss->tail_l = (double *)(b + L.off[20]);
        e = hipStreamCreateWithFlags(&ss->tail_stream, hipStreamNonBlocking);
        if (e != hipSuccess) { ss->tail_stream = nullptr; return undo(hip_fail(e, "hipStreamCreate")); }
        e = hipEventCreateWithFlags(&ss->tail_fork, hipEventDisableTiming);
        if (e != hipSuccess) { ss->tail_fork = nullptr; return undo(hip_fail(e, "hipEventCreate")); }
        e = hipEventCreateWithFlags(&ss->tail_join, hipEventDisableTiming);
        if (e != hipSuccess) { ss->tail_join = nullptr; return undo(hip_fail(e, "hipEventCreate")); }
        if (m->K_cap == 0) ss->tail_g = (float *)(b + L.off[20] + (size_t)tail * kSubChunks * 64 * 8);
    }
    e = hipMemsetAsync(ss->block, 0, L.total, ss->stream);
    if (e != hipSuccess) return undo(hip_fail(e, "hipMemset(session)"));
    // Initial state: poses, uniform log-weights, identity parents.
    std::vector<float> soa((size_t)7 * N);
    aos_to_soa(poses, soa.data(), (size_t)N, 7);
    std::vector<double> lw((size_t)N, -std::log((double)N));
    std::vector<int32_t> par((size_t)N);
    for (int i = 0; i < N; ++i) par[i] = i;
    e = hipMemcpyAsync(ss->pose, soa.data(), soa.size() * 4, hipMemcpyHostToDevice, ss->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ss->logw, lw.data(), lw.size() * 8, hipMemcpyHostToDevice, ss->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ss->parents, par.data(), par.size() * 4, hipMemcpyHostToDevice,
                           ss->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ss->stream);
    if (e != hipSuccess) return undo(hip_fail(e, "session init upload"));
    if (ss->K > 0 && (s = upload_kf(ss, kf_poses)) != MCS_OK) return undo(s);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ss->id = ctx->next_id++;
    ctx->sessions[ss->id] = ss;
    *session_id = ss->id;
    return MCS_OK;
}

mcs_status mcs_session_destroy(mcs_ctx *ctx, int32_t sid)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->sessions.find(sid);
        if (it == ctx->sessions.end()) return fail(MCS_ENOTFOUND, "no session %d", sid);
        s = it->second;
        ctx->sessions.erase(it);
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->tail_stream) (void)hipStreamSynchronize(s->tail_stream);
    (void)hipFree(s->block);
    (void)hipStreamDestroy(s->stream);
    (void)hipEventDestroy(s->staged);
    if (s->tail_stream) {
        (void)hipStreamDestroy(s->tail_stream);
        (void)hipEventDestroy(s->tail_fork);
        (void)hipEventDestroy(s->tail_join);
    }
    if (s->pinned) (void)hipHostFree(s->pinned);
    if (s->trace) (void)hipFree(s->trace);
    prof_release(s);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->in_use -= s->bytes + s->trace_bytes;
    s->map->users--;
    delete s;
    return MCS_OK;
}

mcs_status mcs_set_particles(mcs_ctx *ctx, int32_t sid, const float *poses, const double *logw,
                             const float *kf_poses)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(hipStreamSynchronize(s->stream), "sync");
    if (poses) {
        if ((st = check_poses(poses, (size_t)s->N)) != MCS_OK) return st;
        std::vector<float> soa((size_t)7 * s->N);
        aos_to_soa(poses, soa.data(), (size_t)s->N, 7);
        HIP_TRY(hipMemcpyAsync(s->pose, soa.data(), soa.size() * 4, hipMemcpyHostToDevice,
                               s->stream), "upload poses");
        HIP_TRY(hipStreamSynchronize(s->stream), "sync");
    }
    if (logw) {
        for (int i = 0; i < s->N; ++i)
            if (std::isnan(logw[i]) || logw[i] == INFINITY)
                return fail(MCS_EINVAL, "logw[%d] is NaN or +inf", i);
        HIP_TRY(hipMemcpyAsync(s->logw, logw, (size_t)s->N * 8, hipMemcpyHostToDevice, s->stream),
                "upload logw");
        HIP_TRY(hipStreamSynchronize(s->stream), "sync");
    }
    if (kf_poses) {
        if (s->K == 0) return fail(MCS_EINVAL, "session has no keyframes");
        if ((st = check_poses(kf_poses, (size_t)s->N * s->K)) != MCS_OK) return st;
        if ((st = upload_kf(s, kf_poses)) != MCS_OK) return st;
    }
    return MCS_OK;
}

}  // extern "C"

namespace {

// A step on host inputs: stage scan (and covariances, noise) through pinned
// memory on the session's stream, then enqueue the step.
mcs_status filter_step_host(mcs_ctx *ctx, int32_t sid, const float *scan, const float *cov, int32_t M,
                            const float *noise, const mcs_step_params *p)
{
    if (!ctx || !scan) return fail(MCS_EINVAL, "NULL argument");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = validate_params(s, p, M);
    if (st != MCS_OK) return st;
    if ((s->map->kind == kVoxelMap) != (cov != nullptr))
        return fail(MCS_EINVAL, s->map->kind == kVoxelMap
                                    ? "a GICP map needs scan covariances (mcs_filter_step_gicp)"
                                    : "scan covariances are for GICP maps only");
    for (int64_t k = 0; k < (int64_t)M * 3; ++k)
        if (!std::isfinite(scan[k])) return fail(MCS_EINVAL, "scan value %lld not finite", (long long)k);
    if (cov)
        for (int64_t k = 0; k < (int64_t)M * 6; ++k)
            if (!std::isfinite(cov[k])) return fail(MCS_EINVAL, "covariance value %lld not finite", (long long)k);
    const bool use_noise = p->predict && noise && p->noise_mode == MCS_NOISE_INPUT;
    if (use_noise)
        for (int64_t k = 0; k < (int64_t)s->N * 6; ++k)
            if (!std::isfinite(noise[k])) return fail(MCS_EINVAL, "noise value not finite");
    if ((st = set_device(ctx)) != MCS_OK) return st;
    // Stage through pinned host memory; wait for the previous upload from it.
    const size_t n_scan = (size_t)M * 3, n_cov = cov ? (size_t)M * 6 : 0;
    const size_t need = n_scan + n_cov + (use_noise ? (size_t)s->N * 6 : 0);
    if (s->staged_pending) HIP_TRY(hipEventSynchronize(s->staged), "wait staging");
    s->staged_pending = false;
    if (s->pinned_floats < need) {
        if (s->pinned) (void)hipHostFree(s->pinned);
        s->pinned = nullptr;
        s->pinned_floats = 0;
        HIP_TRY(hipHostMalloc((void **)&s->pinned, need * sizeof(float), hipHostMallocDefault),
                "hipHostMalloc");
        s->pinned_floats = need;
    }
    std::memcpy(s->pinned, scan, n_scan * sizeof(float));
    HIP_TRY(hipMemcpyAsync(s->scan3, s->pinned, n_scan * sizeof(float), hipMemcpyHostToDevice,
                           s->stream), "upload scan");
    if (cov) {
        std::memcpy(s->pinned + n_scan, cov, n_cov * sizeof(float));
        HIP_TRY(hipMemcpyAsync(s->cov6, s->pinned + n_scan, n_cov * sizeof(float),
                               hipMemcpyHostToDevice, s->stream), "upload covariances");
    }
    if (use_noise) {
        std::memcpy(s->pinned + n_scan + n_cov, noise, (size_t)s->N * 6 * sizeof(float));
        HIP_TRY(hipMemcpyAsync(s->noise, s->pinned + n_scan + n_cov, (size_t)s->N * 6 * sizeof(float),
                               hipMemcpyHostToDevice, s->stream), "upload noise");
    }
    HIP_TRY(hipEventRecord(s->staged, s->stream), "event");
    s->staged_pending = true;
    return enqueue_step(s, s->scan3, M, use_noise ? s->noise : nullptr, p, s->stream,
                        cov ? s->cov6 : nullptr);
}

mcs_status filter_step_dev(mcs_ctx *ctx, int32_t sid, const float *scan_dev, const float *cov_dev,
                           int32_t M, const float *noise_dev, const mcs_step_params *p, void *stream)
{
    if (!ctx || !scan_dev) return fail(MCS_EINVAL, "NULL argument");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = validate_params(s, p, M);
    if (st != MCS_OK) return st;
    if ((st = set_device(ctx)) != MCS_OK) return st;
    hipStream_t hs = stream ? (hipStream_t)stream : s->stream;
    return enqueue_step(s, scan_dev, M, p->predict ? noise_dev : nullptr, p, hs, cov_dev);
}

}  // namespace

extern "C" {

mcs_status mcs_filter_step(mcs_ctx *ctx, int32_t sid, const float *scan, int32_t M,
                           const float *noise, const mcs_step_params *p)
{
    return filter_step_host(ctx, sid, scan, nullptr, M, noise, p);
}

mcs_status mcs_filter_step_dev(mcs_ctx *ctx, int32_t sid, const float *scan_dev, int32_t M,
                               const float *noise_dev, const mcs_step_params *p, void *stream)
{
    return filter_step_dev(ctx, sid, scan_dev, nullptr, M, noise_dev, p, stream);
}

// The public statistics are the leading fields of the device-side record.
static_assert(offsetof(StepStatsDev, lse) == offsetof(mcs_step_stats, lse) &&
                  offsetof(StepStatsDev, ess) == offsetof(mcs_step_stats, ess) &&
                  offsetof(StepStatsDev, resampled) == offsetof(mcs_step_stats, resampled) &&
                  offsetof(StepStatsDev, best) == offsetof(mcs_step_stats, best) &&
                  offsetof(StepStatsDev, best_pose) == offsetof(mcs_step_stats, best_pose) &&
                  offsetof(StepStatsDev, degenerate) == offsetof(mcs_step_stats, degenerate) &&
                  offsetof(StepStatsDev, pruned) == offsetof(mcs_step_stats, pruned),
              "mcs_step_stats must be a prefix of StepStatsDev");

mcs_status mcs_filter_step_noalloc(mcs_ctx *ctx, int32_t map_id, int32_t N, float *pose_dev,
                                   double *logw_dev, float *loglik_dev, float *grad_dev,
                                   int32_t *parents_dev, const float *scan_dev, int32_t M,
                                   const float *noise_dev, const mcs_step_params *p,
                                   mcs_step_stats *stats_dev, void *stream)
{
    if (!ctx || !pose_dev || !logw_dev || !loglik_dev || !grad_dev || !parents_dev || !scan_dev)
        return fail(MCS_EINVAL, "NULL argument");
    if (N < 1 || N > MCS_NOALLOC_MAX_PARTICLES)
        return fail(MCS_EINVAL, "N=%d outside [1, %d] (the static area's limit)", N,
                    MCS_NOALLOC_MAX_PARTICLES);
    if (M < 1 || M > MCS_NOALLOC_MAX_POINTS)
        return fail(MCS_EINVAL, "M=%d outside [1, %d] (the static area's limit)", M,
                    MCS_NOALLOC_MAX_POINTS);
    if (!ctx->scratch) return fail(MCS_EDEVICE, "no static area on device %d", ctx->device);
    Map *m = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->maps.find(map_id);
        if (it == ctx->maps.end()) return fail(MCS_ENOTFOUND, "no map %d", map_id);
        m = it->second;
    }
    if (m->kind != kGridMap || m->K_cap > 0)
        return fail(MCS_EINVAL, "the allocation-free step takes single-grid maps only");
    // The step's temporaries, carved out of the static area.
    const size_t n = (size_t)N, nb = (size_t)weight_blocks(N);
    const size_t sizes[] = {7 * n * 4, n * 8, nb * kPartPerBlock * 8, n * 4, (size_t)M * 16,
                            (size_t)M * 32, sizeof(StepStatsDev), 3 * n * 4, (size_t)kOrderCells * 4,
                            nb * 2 * kOrderDims * 4};
    constexpr int kParts = sizeof sizes / sizeof sizes[0];
    size_t off[kParts + 1], o = 0;
    for (int k = 0; k < kParts; ++k) {
        off[k] = o;
        o += align_up(sizes[k]);
    }
    off[kParts] = o;
    if (o > kNoAllocScratchBytes) return fail(MCS_EINVAL, "step temporaries exceed the static area");
    // A small last round of tiles is spread over one wave per sub-chunk when
    // its partial sums fit the rest of the area (same results either way).
    int tail = eval_tail_tiles(N, m->desc.dtype, false);
    if (o + (size_t)tail * kTailBytesPerTile > kNoAllocScratchBytes) tail = 0;
    char *b = (char *)ctx->scratch;
    Session tmp;
    tmp.map = m;
    tmp.N = N;
    tmp.M_max = M;
    tmp.pose = pose_dev;
    tmp.pose_tmp = (float *)(b + off[0]);
    tmp.cdf_local = (double *)(b + off[1]);
    tmp.part = (double *)(b + off[2]);
    tmp.copies = (int32_t *)(b + off[3]);
    tmp.scan4 = (float4 *)(b + off[4]);
    tmp.scan8 = (double4 *)(b + off[5]);
    tmp.stats = (StepStatsDev *)(b + off[6]);
    tmp.order = (int32_t *)(b + off[7]);
    tmp.ocell = tmp.order + N;
    tmp.orank = tmp.ocell + N;
    tmp.ocount = (int32_t *)(b + off[8]);
    tmp.obounds = (float *)(b + off[9]);
    tmp.loglik = loglik_dev;
    tmp.grad = grad_dev;
    tmp.logw = logw_dev;
    tmp.parents = parents_dev;
    if (tail > 0) {
        tmp.tail_tiles = tail;
        tmp.tail_l = (double *)(b + off[kParts]);
        tmp.tail_g = (float *)(b + off[kParts] + (size_t)tail * kSubChunks * 64 * 8);
    }
    mcs_status st = validate_params(&tmp, p, M);
    if (st != MCS_OK) return st;
    if ((st = set_device(ctx)) != MCS_OK) return st;
    const hipStream_t hs = (hipStream_t)stream;
    const StepDesc d = make_desc(&tmp, scan_dev, M, p->predict ? noise_dev : nullptr, p);
    if (!eval_supported(d)) return fail(MCS_EINVAL, "map not supported");
    HIP_TRY(launch_pack_predict(d, hs), "pack/predict");
    HIP_TRY(launch_order(d, hs), "order");
    HIP_TRY(launch_eval(d, hs, nullptr), "eval");
    HIP_TRY(launch_weights(d, hs), "weights");
    HIP_TRY(launch_resample(d, hs), "resample");
    if (stats_dev)
        HIP_TRY(hipMemcpyAsync(stats_dev, d.stats, sizeof(mcs_step_stats), hipMemcpyDeviceToDevice, hs),
                "stats");
    return MCS_OK;
}

mcs_status mcs_gather_floor_dev(mcs_ctx *ctx, int32_t sid, const float *scan_dev, int32_t M,
                                const mcs_step_params *p, void *stream)
{
    if (!ctx || !scan_dev) return fail(MCS_EINVAL, "NULL argument");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    if (s->map->kind != kGridMap || s->K_cap > 0)
        return fail(MCS_EINVAL, "the gather floor runs on single-grid sessions only");
    mcs_status st = validate_params(s, p, M);
    if (st != MCS_OK) return st;
    if ((st = set_device(ctx)) != MCS_OK) return st;
    hipStream_t hs = stream ? (hipStream_t)stream : s->stream;
    StepDesc d = make_desc(s, scan_dev, M, nullptr, p);
    d.predict = 0;
    d.noise = nullptr;
    d.post_eval = 0;
    d.oob_skip = 0;
    d.trace = nullptr;
    d.floor_only = 1;
    if (!eval_supported(d)) return fail(MCS_EINVAL, "map not supported");
    std::array<hipEvent_t, 5> *ev = nullptr;
    if ((st = prof_begin(s, ev)) != MCS_OK) return st;
    if (ev) s->prof_evals += (int64_t)s->N * M * p->iters;
#define FLOOR_MARK(k)                                                        \
    do {                                                                     \
        if (ev) HIP_TRY(hipEventRecord((*ev)[k], hs), "hipEventRecord");     \
    } while (0)
    FLOOR_MARK(0);
    HIP_TRY(launch_pack_predict(d, hs), "pack");
    HIP_TRY(launch_order(d, hs), "order");
    FLOOR_MARK(1);
    const TailAux aux{s->tail_stream, s->tail_fork, s->tail_join};
    HIP_TRY(launch_eval(d, hs, s->tail_stream ? &aux : nullptr), "gather floor");
    FLOOR_MARK(2);
    FLOOR_MARK(3);
    FLOOR_MARK(4);
#undef FLOOR_MARK
    return MCS_OK;
}

mcs_status mcs_measure_issue_rates(mcs_ctx *ctx, double *rates, int32_t n)
{
    if (!ctx || !rates) return fail(MCS_EINVAL, "NULL argument");
    if (n < MCS_RATE_COUNT) return fail(MCS_EINVAL, "rates holds %d entries, %d needed", n, (int)MCS_RATE_COUNT);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(measure_issue_rates(rates), "issue-rate kernels");
    return MCS_OK;
}

mcs_status mcs_filter_step_gicp(mcs_ctx *ctx, int32_t sid, const float *mu, const float *cov,
                                int32_t M, const float *noise, const mcs_step_params *p)
{
    if (!cov) return fail(MCS_EINVAL, "NULL covariances");
    return filter_step_host(ctx, sid, mu, cov, M, noise, p);
}

mcs_status mcs_filter_step_gicp_dev(mcs_ctx *ctx, int32_t sid, const float *mu_dev,
                                    const float *cov_dev, int32_t M, const float *noise_dev,
                                    const mcs_step_params *p, void *stream)
{
    if (!cov_dev) return fail(MCS_EINVAL, "NULL covariances");
    return filter_step_dev(ctx, sid, mu_dev, cov_dev, M, noise_dev, p, stream);
}

mcs_status mcs_get_gicp_system(mcs_ctx *ctx, int32_t sid, float *H, float *b)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    if (s->map->kind != kVoxelMap) return fail(MCS_EINVAL, "session %d has no GICP map", sid);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    const size_t N = s->N;
    if (H) {
        std::vector<float> soa(21 * N);
        HIP_TRY(hipMemcpy(soa.data(), s->hess, soa.size() * 4, hipMemcpyDeviceToHost), "hess");
        for (size_t i = 0; i < N; ++i)
            for (int c = 0; c < 21; ++c) H[21 * i + c] = soa[c * N + i];
    }
    if (b) {
        std::vector<float> soa(6 * N);
        HIP_TRY(hipMemcpy(soa.data(), s->grad, soa.size() * 4, hipMemcpyDeviceToHost), "b");
        for (size_t i = 0; i < N; ++i)
            for (int c = 0; c < 6; ++c) b[6 * i + c] = soa[c * N + i];
    }
    return MCS_OK;
}

mcs_status mcs_get_neighbors(mcs_ctx *ctx, int32_t sid, int32_t *out, int32_t *n_neighbors)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    if (s->K == 0) return fail(MCS_EINVAL, "session %d has no keyframe map", sid);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (n_neighbors) *n_neighbors = s->last_nb;
    if (out && s->last_nb > 0) {
        const size_t N = s->N, nb = s->last_nb;
        std::vector<int32_t> soa(nb * N);
        HIP_TRY(hipMemcpy(soa.data(), s->neighbors, soa.size() * 4, hipMemcpyDeviceToHost),
                "neighbors");
        for (size_t i = 0; i < N; ++i)
            for (size_t k = 0; k < nb; ++k) out[i * nb + k] = soa[k * N + i];
    }
    return MCS_OK;
}

mcs_status mcs_session_sync(mcs_ctx *ctx, int32_t sid)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    return MCS_OK;
}

mcs_status mcs_session_stream(mcs_ctx *ctx, int32_t sid, void **stream)
{
    if (!ctx || !stream) return fail(MCS_EINVAL, "NULL argument");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    *stream = (void *)s->stream;
    return MCS_OK;
}

mcs_status mcs_get_particles(mcs_ctx *ctx, int32_t sid, float *poses, double *logw,
                             int32_t *parents, float *loglik, float *grad, float *kf_poses,
                             mcs_step_stats *stats)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    // Waits for everything queued on the device, whichever stream it used.
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    const size_t N = s->N;
    if (poses) {
        std::vector<float> soa(7 * N);
        HIP_TRY(hipMemcpy(soa.data(), s->pose, soa.size() * 4, hipMemcpyDeviceToHost), "poses");
        for (size_t i = 0; i < N; ++i) {
            for (int c = 0; c < 7; ++c) poses[7 * i + c] = soa[c * N + i];
            if (poses[7 * i + 3] < 0.0f)
                for (int c = 3; c < 7; ++c) poses[7 * i + c] = -poses[7 * i + c];
        }
    }
    if (logw) HIP_TRY(hipMemcpy(logw, s->logw, N * 8, hipMemcpyDeviceToHost), "logw");
    if (parents) HIP_TRY(hipMemcpy(parents, s->parents, N * 4, hipMemcpyDeviceToHost), "parents");
    if (loglik) HIP_TRY(hipMemcpy(loglik, s->loglik, N * 4, hipMemcpyDeviceToHost), "loglik");
    if (grad) {
        std::vector<float> soa(6 * N);
        HIP_TRY(hipMemcpy(soa.data(), s->grad, soa.size() * 4, hipMemcpyDeviceToHost), "grad");
        for (size_t i = 0; i < N; ++i)
            for (int c = 0; c < 6; ++c) grad[6 * i + c] = soa[c * N + i];
    }
    if (kf_poses && s->K > 0) {
        const size_t K = s->K;
        std::vector<float> soa(K * 7 * N);
        HIP_TRY(hipMemcpy(soa.data(), s->kf_pose, soa.size() * 4, hipMemcpyDeviceToHost), "kf");
        for (size_t i = 0; i < N; ++i)
            for (size_t k = 0; k < K; ++k) {
                float *o = kf_poses + (i * K + k) * 7;
                for (int c = 0; c < 7; ++c) o[c] = soa[(k * 7 + c) * N + i];
                if (o[3] < 0.0f)
                    for (int c = 3; c < 7; ++c) o[c] = -o[c];
            }
    }
    if (stats) {
        StepStatsDev d{};
        HIP_TRY(hipMemcpy(&d, s->stats, sizeof d, hipMemcpyDeviceToHost), "stats");
        stats->lse = d.lse;
        stats->ess = d.ess;
        stats->resampled = d.resampled;
        stats->best = d.best;
        for (int c = 0; c < 7; ++c) stats->best_pose[c] = d.best_pose[c];
        if (stats->best_pose[3] < 0.0f)
            for (int c = 3; c < 7; ++c) stats->best_pose[c] = -stats->best_pose[c];
        stats->degenerate = d.degenerate;
        stats->pruned = d.pruned;
    }
    return MCS_OK;
}

mcs_status mcs_session_info(mcs_ctx *ctx, int32_t sid, int32_t *N, int32_t *K, int32_t *M_max,
                            int32_t *last_nb)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    if (N) *N = s->N;
    if (K) *K = s->K;
    if (M_max) *M_max = s->M_max;
    if (last_nb) *last_nb = s->last_nb;
    return MCS_OK;
}

mcs_status mcs_session_trace(mcs_ctx *ctx, int32_t sid, int32_t max_passes)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    if (max_passes < 0 || max_passes > 65) return fail(MCS_EINVAL, "max_passes=%d outside [0, 65]", max_passes);
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    if (max_passes > 0 && s->map->kind != kGridMap)
        return fail(MCS_EINVAL, "pass traces are for likelihood-grid maps only");
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(hipStreamSynchronize(s->stream), "sync");
    if (s->tail_stream) HIP_TRY(hipStreamSynchronize(s->tail_stream), "sync");
    if (s->trace) {
        (void)hipFree(s->trace);
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use -= s->trace_bytes;
        s->trace = nullptr;
        s->trace_bytes = 0;
        s->trace_passes = 0;
    }
    if (max_passes == 0) return MCS_OK;
    const size_t bytes = (size_t)max_passes * kTraceRows * s->N * sizeof(float);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!budget_allows(ctx, bytes)) return fail(MCS_EBUDGET, "trace needs %zu bytes", bytes);
        ctx->in_use += bytes;
    }
    hipError_t e = hipMalloc((void **)&s->trace, bytes);
    if (e == hipSuccess) e = hipMemset(s->trace, 0, bytes);
    if (e != hipSuccess) {
        if (s->trace) (void)hipFree(s->trace);
        s->trace = nullptr;
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use -= bytes;
        return hip_fail(e, "hipMalloc(trace)");
    }
    s->trace_bytes = bytes;
    s->trace_passes = max_passes;
    return MCS_OK;
}

mcs_status mcs_get_pass_trace(mcs_ctx *ctx, int32_t sid, int32_t pass, float *poses,
                              float *loglik, float *grad)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    if (!s->trace) return fail(MCS_EINVAL, "session %d has no pass trace", sid);
    if (pass < 0 || pass >= s->trace_passes)
        return fail(MCS_EINVAL, "pass=%d outside [0, %d)", pass, s->trace_passes);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    const size_t N = s->N;
    std::vector<float> soa(kTraceRows * N);
    HIP_TRY(hipMemcpy(soa.data(), s->trace + (size_t)pass * kTraceRows * N, soa.size() * 4,
                      hipMemcpyDeviceToHost), "trace");
    for (size_t i = 0; i < N; ++i) {
        if (poses)
            for (int c = 0; c < 7; ++c) poses[7 * i + c] = soa[c * N + i];
        if (loglik) loglik[i] = soa[7 * N + i];
        if (grad)
            for (int c = 0; c < 6; ++c) grad[6 * i + c] = soa[(8 + c) * N + i];
    }
    return MCS_OK;
}

mcs_status mcs_session_profile(mcs_ctx *ctx, int32_t sid, int32_t enable)
{
    if (!ctx) return fail(MCS_EINVAL, "NULL context");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    s->prof_used = 0;
    s->prof_evals = 0;
    s->prof_steps = 0;
    for (double &v : s->prof_ms) v = 0.0;
    s->profiling = enable != 0;
    return MCS_OK;
}

mcs_status mcs_session_profile_read(mcs_ctx *ctx, int32_t sid, mcs_profile *out)
{
    if (!ctx || !out) return fail(MCS_EINVAL, "NULL argument");
    Session *s = find_session(ctx, sid);
    if (!s) return fail(MCS_ENOTFOUND, "no session %d", sid);
    mcs_status st = set_device(ctx);
    if (st != MCS_OK) return st;
    if ((st = prof_collect(s)) != MCS_OK) return st;
    out->predict_ms = s->prof_ms[0];
    out->eval_ms = s->prof_ms[1];
    out->weights_ms = s->prof_ms[2];
    out->resample_ms = s->prof_ms[3];
    out->steps = s->prof_steps;
    out->evals = s->prof_evals;
    return MCS_OK;
}

}  // extern "C"
