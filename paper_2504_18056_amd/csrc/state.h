// Host-side state of the C ABI shared by mcslam.cpp and server.cpp: maps,
// sessions, the context, error reporting and the per-session step.
#pragma once

#include "../../include/mcslam.h"
#include "internal.h"

#include <array>
#include <map>
#include <mutex>
#include <vector>

namespace mcs {

mcs_status fail(mcs_status code, const char *fmt, ...);
mcs_status hip_fail(hipError_t e, const char *what);

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxNeighbors = 8;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline size_t record_bytes(int dtype) { return dtype == MCS_GRID_FP32 ? 32 : 16; }

enum MapKind { kGridMap = 0, kVoxelMap = 1 };
constexpr size_t kVoxelRecordBytes = 48;   // mean (3), count, covariance (6), 2 unused
// On the device each voxel record takes 64 B (the 48 B above, then padding), so
// that a record never straddles a 128 B cache line: a wave's record reads
// touch one line per distinct voxel.
constexpr size_t kVoxelDeviceBytes = 64;

struct Map {
    int id = 0;
    int kind = kGridMap;             // likelihood grids, or GICP voxel Gaussians
    int K = 0;                       // grids loaded (keyframe maps); 0 for a single grid
    int K_cap = 0;                   // keyframe capacity; 0: single-grid map
    mcs_grid_desc desc{};            // dims, res, dtype (origin of grid 0)
    std::vector<float> origins;      // K x 3 (or 1 x 3)
    void *cells = nullptr;
    size_t bytes = 0;
    int64_t records = 0;             // per grid (cells or voxels)
    float *origins_dev = nullptr;
    uint8_t *occ_dev = nullptr;      // voxel maps: occupancy bytes, align_up(records) per map
    int users = 0;
};

struct Session {
    int id = 0;
    Map *map = nullptr;
    int N = 0, M_max = 0, K = 0;     // K: keyframes this session has (<= the map's)
    int K_cap = 0;                   // keyframe rows allocated (the map's capacity)
    hipStream_t stream = nullptr;
    void *block = nullptr;           // one device allocation holding every buffer
    size_t bytes = 0;
    float *pose = nullptr, *pose_tmp = nullptr, *loglik = nullptr, *grad = nullptr;
    float *kf_pose = nullptr, *kf_pose_tmp = nullptr, *noise = nullptr, *scan3 = nullptr;
    float4 *scan4 = nullptr;
    double4 *scan8 = nullptr;
    double *logw = nullptr, *cdf_local = nullptr, *part = nullptr;
    int32_t *parents = nullptr, *neighbors = nullptr, *copies = nullptr;
    StepStatsDev *stats = nullptr;
    float4 *scan_g = nullptr;        // GICP: packed points and covariances
    float *cov6 = nullptr;           // GICP: uploaded covariances (host-pointer steps)
    float *hess = nullptr;           // GICP: [21][N] Gauss-Newton H
    double *tail_l = nullptr;        // single grid: tail tiles' sub-chunk log sums
    float *tail_g = nullptr;         // and gradient sums (null: no tail split)
    int tail_tiles = 0;
    hipStream_t tail_stream = nullptr;   // with tail tiles: the tail's passes run on it
    hipEvent_t tail_fork = nullptr, tail_join = nullptr;
    float *pinned = nullptr;         // host staging for host-pointer steps
    size_t pinned_floats = 0;
    int last_nb = 0;                 // neighbours per particle in the last keyframe step
    int32_t *order = nullptr, *ocell = nullptr, *orank = nullptr, *ocount = nullptr;
    float *obounds = nullptr;        // single-grid sessions: evaluation order buffers
    float *trace = nullptr;          // pass trace [trace_passes][kTraceRows][N] (null: off)
    int trace_passes = 0;
    size_t trace_bytes = 0;
    hipEvent_t staged = nullptr;     // last upload from `pinned` done
    bool staged_pending = false;
    // Stage timing: 5 events per profiled step (start, after predict, after
    // eval, after weights, after resample).
    bool profiling = false;
    std::vector<std::array<hipEvent_t, 5>> prof_events;
    size_t prof_used = 0;
    int64_t prof_evals = 0;
    double prof_ms[4] = {0, 0, 0, 0};
    int64_t prof_steps = 0;
};

}  // namespace mcs

struct mcs_ctx {
    int device = 0;
    uint64_t budget = 0;
    uint64_t in_use = 0;
    std::mutex mu;
    std::map<int, mcs::Map *> maps;
    std::map<int, mcs::Session *> sessions;
    int next_id = 1;
    void *scratch = nullptr;         // this device's static area (mcs_filter_step_noalloc)
};

namespace mcs {

mcs_status set_device(mcs_ctx *ctx);
Session *find_session(mcs_ctx *ctx, int32_t sid);
mcs_status validate_params(const Session *s, const mcs_step_params *p, int M);
StepDesc make_desc(const Session *s, const float *scan3_dev, int M, const float *noise_dev,
                   const mcs_step_params *p, const float *cov_dev = nullptr);
mcs_status enqueue_step(Session *s, const float *scan3_dev, int M, const float *noise_dev,
                        const mcs_step_params *p, hipStream_t st, const float *cov_dev = nullptr);

}  // namespace mcs
