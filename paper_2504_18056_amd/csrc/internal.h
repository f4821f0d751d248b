// Internal interface between the C ABI host code (mcslam.cpp, server.cpp) and
// the HIP kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mcs {

// Device-side statistics of the last step (mirrors mcs_step_stats).
struct StepStatsDev {
    double lse;
    double ess;
    int32_t resampled;
    int32_t best;
    float best_pose[7];
    int32_t degenerate;
    int32_t pruned;          // dead particles respawned (pruning policy)
    // Device-only: shared between the stages of one step.
    int32_t prune;           // the pruning stages run in this step
    double lmax;             // max_i l_i
    double live_mass;        // W, sum of the live weights
    int32_t last_live;       // largest live index
    int32_t pad2;
};

// One session's filter step as every kernel sees it.  The grid is stored
// cell-major with a zero layer around the cells: cell (i, j, k), i < nx-1,
// j < ny-1, k < nz-1, is record (i+1) + (nx+1)*((j+1) + (ny+1)*(k+1)) and holds
// either the 8 coefficients of its trilinear polynomial (FP32, 32 B) or its
// corner samples (i+a, j+b, k+c) at slot a + 2b + 4c (FP16/BF16, 16 B);
// records with an index 0 or n on some axis are zero.
struct StepDesc {
    // Map.  Keyframe maps (K > 0) hold K grids of equal dims, grid_stride
    // bytes apart, each with its own origin (origins[3k..3k+2]).
    const void *cells;
    int64_t grid_stride;
    const float *origins;
    // GICP voxel maps: one byte per voxel, nonzero where the voxel holds
    // points (its count is positive), occ_stride bytes per map.
    const uint8_t *vox_occ;
    int64_t occ_stride;
    int32_t nx, ny, nz, dtype;
    float ox, oy, oz;
    float h, inv_h;
    int32_t K, n_nb;
    // Particle state (SoA rows of length N).
    float *pose;             // [7][N]: tx ty tz qw qx qy qz
    float *pose_tmp;         // [7][N]
    float *kf_pose;          // [K*7][N]
    float *kf_pose_tmp;      // [K*7][N]
    float *loglik;           // [N]
    float *grad;             // [6][N]
    double *logw;            // [N]
    double *cdf_local;       // [N]
    double *part;            // [kPartPerBlock * weight_blocks(N)]
    int32_t *copies;         // [N], pruning: copies drawn of each particle
    int32_t *parents;        // [N]
    int32_t *neighbors;      // [n_nb][N]
    StepStatsDev *stats;
    int32_t N, M;
    // Inputs of this step.
    const float *scan3;      // [M][3]
    float4 *scan4;           // [M] packed copy
    double4 *scan8;          // [M] packed FP64 copy
    const float *noise;      // [N][6] or null
    // Step parameters.
    int32_t iters, post_eval, oob_skip, predict, policy;
    float alpha_t, alpha_r, rho_max, phi_max, eps;
    double beta, ess_frac, u;
    float dT[7];
    int32_t kf_loop;         // keyframe maps: loop-gated correction with propagation
    int32_t n_recent;        // with kf_loop: neighbours with index >= K - n_recent are recent
    int32_t noise_rng;       // prediction noise drawn on the device
    uint64_t rng_seed, rng_frame;
    float noise_sigma[6];
    double ln_prune_post, ln_prune_lik;   // pruning thresholds, natural log
    // GICP likelihood with Gauss-Newton passes on voxel keyframe maps: cells
    // then holds K maps of nx*ny*nz voxel records (48 B), h the voxel edge.
    int32_t gicp;
    const float *cov6;       // [M][6] scan point covariances (xx xy xz yy yz zz)
    float4 *scan_g;          // [3M] packed points: (mu, 0), (xx xy xz yy), (yz zz 0 0)
    float *hess;             // [21][N] H of the last pass (upper triangle, row-major)
    // Tail tiles (eval_tail_tiles).  Single grid: per (tile, sub-chunk,
    // particle) partial sums, [tail][kSubChunks][64] log sums and
    // [tail][kSubChunks][6][64].  Keyframe maps: tail_l is the base of the
    // buffer kf_tail() lays out (kKfTailBytesPerTile per tile).
    double *tail_l;
    float *tail_g;
    int32_t tail_tiles;      // tiles the session's tail buffers hold (0: no split)
    // Pass trace (null: off): per pass, [pass][kTraceRows][N] with the pose the
    // pass evaluates (7 rows), its l (1) and its body-frame gradient (6).
    float *trace;
    // Gather-floor measurement (1): the evaluation passes keep the transform
    // and the record loads and replace the arithmetic by a checksum of the
    // gathered words (l = checksum, g = 0, so the poses stay put).
    int32_t floor_only;
    // Evaluation order (null: slot s takes particle s): the particles grouped
    // by a coarse cell of their pose, recomputed each step after the
    // prediction.  order [N] (slot -> particle), ocell and orank [N], ocount
    // [kOrderCells] (counts, then offsets), obounds [weight_blocks(N)][2 * 6]
    // (per-block ranges of the six coordinates).
    int32_t *order, *ocell, *orank, *ocount;
    float *obounds;
};

constexpr int kTraceRows = 14;
constexpr int kOrderDims = 6;
constexpr int kOrderBits = 3;                                  // per coordinate
constexpr int kOrderDrop = 3;                                  // low Morton bits dropped
constexpr int kOrderCells = 1 << (kOrderDims * kOrderBits - kOrderDrop);   // 32768
// Sessions of at least this many particles evaluate in the grouped order.
constexpr int kOrderMinParticles = 4096;

constexpr int kWeightBlock = 256;
constexpr int kPartPerBlock = 6;   // doubles of per-block partials
constexpr int kParticleTile = 64;
constexpr int kKfMaxNb = 8;
// Sub-chunks of the scan in the single-grid evaluation's fixed summation order.
constexpr int kSubChunks = 32;
constexpr size_t kTailBytesPerTile = (size_t)kSubChunks * 64 * (8 + 6 * 4);
constexpr size_t kKfTailBytesPerTile =
    (size_t)(kKfMaxNb + 1) * 64 * 4 + (size_t)kSubChunks * kKfMaxNb * 64 * (8 + 6 * 4);

// Cell records of a grid of nx x ny x nz samples: the (nx - 1)(ny - 1)(nz - 1)
// cells and a zero layer around them, (nx + 1)(ny + 1)(nz + 1) in all.
__host__ __device__ inline uint64_t grid_records(int nx, int ny, int nz)
{
    return (uint64_t)(nx + 1) * (uint64_t)(ny + 1) * (uint64_t)(nz + 1);
}
// Largest byte range of one buffer of records (32-bit offsets).
constexpr uint32_t kMaxRecordBytes = 0xFFFFFFE0u;

__host__ __device__ inline int weight_blocks(int N) { return (N + kWeightBlock - 1) / kWeightBlock; }
__host__ __device__ inline int particle_tiles(int N) { return (N + kParticleTile - 1) / kParticleTile; }
__host__ __device__ inline int scan_blocks(int M) { return (M + kWeightBlock - 1) / kWeightBlock; }

// Launchers (kernels.hip); all enqueue on `st` and return hipError_t.
hipError_t launch_build_cells(const float *grid, void *cells, int nx, int ny, int nz, int dtype,
                              hipStream_t st);
// The stages of one step of one session.
hipError_t launch_pack_predict(const StepDesc &d, hipStream_t st);
// aux: a second stream and two events of the session; with them the tail
// tiles' kernels run beside the main launch (fork after the stages before,
// join before the stages after).
struct TailAux {
    hipStream_t stream;
    hipEvent_t fork, join;
};
hipError_t launch_eval(const StepDesc &d, hipStream_t st, const TailAux *aux = nullptr);
// Evaluation order of the step (nothing when d.order is null).
hipError_t launch_order(const StepDesc &d, hipStream_t st);
hipError_t launch_weights(const StepDesc &d, hipStream_t st);
hipError_t launch_resample(const StepDesc &d, hipStream_t st);
// Whether the eval kernels accept this map (record buffer under 4 GiB).
bool eval_supported(const StepDesc &d);
// Tiles of a single-grid session of N particles that the evaluation spreads
// over one wave per sub-chunk (the last, partly filled round of tiles), or 0.
int eval_tail_tiles(int N, int dtype, bool keyframes);
// Single-grid evaluation tiles resident on the device at once (0 if unknown).
int eval_round_tiles(int dtype);
bool grid_supported(int nx, int ny, int nz, int dtype, bool keyframe);
// A single grid read through 64-bit record addresses (beyond one buffer's
// range, or with rows or slabs of 2^24 records and more).
bool grid_is_wide(const StepDesc &d);

// Batched steps of many sessions (the serving path).  Work lists in device
// memory name (descriptor, block) pairs per stage; every stage kernel is
// persistent (fixed grid) and strides over its list, so one captured graph
// serves any batch composition.
enum BatchKind {
    kPack = 0, kPredict, kEval, kWeights, kWCombine, kNormScan, kPrefix, kSearch, kCommit, kFill,
    kChunk,    // sessions split whole: (descriptor, tile * 4 + group of 8 sub-chunks)
    kTStep,    // their per-pass reduce and epilogue: (descriptor, tile)
    kNumKinds
};
// Passes that a tick runs on split sessions (requests with more take kEval).
constexpr int kBatchSplitPasses = 4;

struct BatchTables {
    const StepDesc *descs;
    const int2 *items;              // (descriptor index, block index); stage k at offs[k]
    const int32_t *counts;          // [kNumKinds]
    const int32_t *offs;            // [kNumKinds]
};

// Enqueue one tick of every stage for single-grid sessions of one grid dtype
// and out-of-grid rule.
hipError_t launch_batch(const BatchTables &t, int dtype, int skip, hipStream_t st);

// The allocation-free step's static device area: its size, and its address on
// `device` (which must be current), looked up once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
hipError_t scratch_init(int device, void **ptr);

// VALU lane-operations per second by instruction class (mcs_rate_class
// order, MCS_RATE_COUNT entries), on the current device.
hipError_t measure_issue_rates(double *rates);

}  // namespace mcs
