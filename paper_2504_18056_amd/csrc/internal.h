// Internal interface between the C ABI host code (mcslam.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
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
    int32_t pad;
};

// One likelihood grid in the cell-major layout: cell (i, j, k), for
// i < nx-1, j < ny-1, k < nz-1, is record i + (nx-1)*(j + (ny-1)*k) and holds
// the corner samples (i+a, j+b, k+c) at slot a + 2b + 4c.  A record is 8 FP32
// (32 B) or 8 FP16/BF16 (16 B).
struct GridDev {
    const void *cells;
    int32_t nx, ny, nz;
    int32_t dtype;
    float ox, oy, oz;
    float inv_h;
};

// Parameters of one single-grid likelihood/gradient/step launch.
struct EvalArgs {
    const float4 *scan;      // M points (x, y, z, unused)
    int32_t M;
    GridDev grid;
    float *pose;             // SoA [7][N]: tx ty tz qw qx qy qz
    float *loglik;           // [N]
    float *grad;             // SoA [6][N]
    int32_t N;
    int32_t iters;           // gradient passes
    int32_t post_eval;       // one extra likelihood-only pass
    int32_t oob_skip;
    float alpha_t, alpha_r, rho_max, phi_max;
    float eps;
};

// Keyframe map: K grids of equal dims; per-particle keyframe poses.
struct KfEvalArgs {
    const float4 *scan;
    int32_t M;
    const void *cells;       // K grids back to back
    int64_t grid_records;    // records per grid
    const float *origins;    // [K][3]
    int32_t nx, ny, nz, dtype;
    float inv_h;
    int32_t K, n_nb;
    float *pose;             // SoA [7][N]
    const float *kf_pose;    // SoA [K][7][N]
    float *loglik;
    float *grad;
    int32_t *neighbors;      // [n_nb][N] (last pass)
    int32_t N;
    int32_t iters, post_eval, oob_skip;
    float alpha_t, alpha_r, rho_max, phi_max, eps;
};

struct WeightArgs {
    double *logw;            // [N]
    const float *loglik;     // [N]
    int32_t N;
    double beta;
    double *part;            // [nblocks][4]
    unsigned int *counter;   // self-resetting arrival counter
    StepStatsDev *stats;
    int32_t policy;
    double ess_frac;
    const float *pose;       // SoA [7][N], for the representative
};

struct ResampleArgs {
    double *logw;            // [N]
    double *cdf_local;       // [N]
    double *part;            // [nblocks] block totals, then exclusive offsets
    unsigned int *counter;
    const StepStatsDev *stats;
    int32_t N;
    double u;
    int32_t *parents;        // [N]
    float *pose;             // SoA [7][N]
    float *pose_tmp;         // SoA [7][N]
    float *kf_pose;          // SoA [K][7][N] or null
    float *kf_pose_tmp;
    int32_t K;
};

constexpr int kWeightBlock = 256;

// Launchers (kernels.hip).  All enqueue on `st` and return hipError_t.
hipError_t launch_pack_scan(const float *scan3, float4 *scan4, int M, hipStream_t st);
hipError_t launch_build_cells(const float *grid, void *cells, int nx, int ny, int nz, int dtype,
                              hipStream_t st);
hipError_t launch_predict(float *pose, int N, const float dT[7], const float *noise,
                          hipStream_t st);
hipError_t launch_eval_step(const EvalArgs &a, hipStream_t st);
hipError_t launch_kf_eval_step(const KfEvalArgs &a, hipStream_t st);
hipError_t launch_weights(const WeightArgs &a, hipStream_t st);
hipError_t launch_resample(const ResampleArgs &a, hipStream_t st);
hipError_t launch_soa_from_aos(const float *aos, float *soa, int N, int C, hipStream_t st);
hipError_t launch_fill_f64(double *p, double v, int n, hipStream_t st);
hipError_t launch_fill_u32(unsigned int *p, unsigned int v, int n, hipStream_t st);

inline int weight_blocks(int N) { return (N + kWeightBlock - 1) / kWeightBlock; }

}  // namespace mcs
