// HIP kernels (gfx950) of the gradient-guided Monte Carlo SLAM particle update.
//
// Paper: T. Nakao et al., "Range-based 6-DoF Monte Carlo SLAM with
// Gradient-guided Particle Filter on GPU" (arXiv 2504.18056).  Each particle
// is updated independently (Sec. III-A, algorithm overview), which is what the
// launch shapes below exploit.
//
// Hot kernel k_eval_step: one lane per particle, 64 particles per workgroup,
// the scan split over the W waves of the workgroup.  The scan point of an
// inner-loop iteration is the same for every lane of a wave, so it is read
// with scalar loads and enters the VALU as an SGPR operand.  Each particle's
// pose lives in VGPRs as the grid-index affine map u = A p + b with
// A = R / h and b = (t - o) / h - 1/2.  Each evaluation is one record load of
// the cell-major grid (8 corner samples in 32 B or 16 B), a trilinear value
// and gradient, ln via the hardware log2, and 7 running sums (the log term in
// FP64, the six gradient sums in FP32).  The W partial sums are combined in
// LDS in a fixed order, then wave 0 takes the pose step (Eq. 7) per lane.
// No MFMA: the work is a gather plus a few dozen scalar FLOPs per point, not
// a dense contraction.
#include "internal.h"

#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

namespace mcs {
namespace {

constexpr double kLn2 = 0.693147180559945309417232121458176568;

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Rotation matrix (row-major) of a unit quaternion (w, x, y, z).
__device__ __forceinline__ void rot_of_quat(float w, float x, float y, float z, float R[9])
{
#pragma clang fp contract(off)
    const float x2 = x + x, y2 = y + y, z2 = z + z;
    const float wx = w * x2, wy = w * y2, wz = w * z2;
    const float xx = x * x2, xy = x * y2, xz = x * z2;
    const float yy = y * y2, yz = y * z2, zz = z * z2;
    R[0] = 1.0f - (yy + zz); R[1] = xy - wz;          R[2] = xz + wy;
    R[3] = xy + wz;          R[4] = 1.0f - (xx + zz); R[5] = yz - wx;
    R[6] = xz - wy;          R[7] = yz + wx;          R[8] = 1.0f - (xx + yy);
}

__device__ __forceinline__ void normalize_quat(float &w, float &x, float &y, float &z)
{
#pragma clang fp contract(off)
    const float s = __builtin_amdgcn_rsqf(w * w + x * x + y * y + z * z);
    w *= s; x *= s; y *= s; z *= s;
    if (w < 0.0f) { w = -w; x = -x; y = -y; z = -z; }
}

// Coefficients of Exp on SE(3) for rotation vector phi with |phi|^2 = th2:
//   a = (1 - cos th) / th^2, b = (th - sin th) / th^3 (the V matrix
//   V = I + a [phi]x + b [phi]x^2), and the quaternion of exp([phi]x),
//   (cos(th/2), c phi) with c = sin(th/2) / th.
// Below 0.1 rad, series truncated after the th^4 term (error < 3e-11).
__device__ __forceinline__ void exp_coeffs(float th2, float &a, float &b, float &c, float &cw)
{
    if (th2 < 0.01f) {
        a = 0.5f - th2 * (1.0f / 24.0f) + th2 * th2 * (1.0f / 720.0f);
        b = (1.0f / 6.0f) - th2 * (1.0f / 120.0f) + th2 * th2 * (1.0f / 5040.0f);
        c = 0.5f - th2 * (1.0f / 48.0f) + th2 * th2 * (1.0f / 3840.0f);
        cw = 1.0f - th2 * 0.125f + th2 * th2 * (1.0f / 384.0f);
    } else {
        const float th = sqrtf(th2);
        float s, co, sh, ch;
        sincosf(th, &s, &co);
        sincosf(0.5f * th, &sh, &ch);
        a = 2.0f * sh * sh / th2;
        b = (th - s) / (th2 * th);
        c = sh / th;
        cw = ch;
    }
}

// (t, q) <- (t, q) * Exp([rho; phi]): t += R V(phi) rho, q <- q (x) q(phi).
__device__ __forceinline__ void right_exp(float t[3], float q[4], const float rho[3],
                                          const float phi[3])
{
#pragma clang fp contract(off)
    const float th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    float a, b, c, cw;
    exp_coeffs(th2, a, b, c, cw);
    // V rho = rho + a (phi x rho) + b (phi x (phi x rho)).
    const float c1x = phi[1] * rho[2] - phi[2] * rho[1];
    const float c1y = phi[2] * rho[0] - phi[0] * rho[2];
    const float c1z = phi[0] * rho[1] - phi[1] * rho[0];
    const float c2x = phi[1] * c1z - phi[2] * c1y;
    const float c2y = phi[2] * c1x - phi[0] * c1z;
    const float c2z = phi[0] * c1y - phi[1] * c1x;
    const float vx = rho[0] + a * c1x + b * c2x;
    const float vy = rho[1] + a * c1y + b * c2y;
    const float vz = rho[2] + a * c1z + b * c2z;
    float R[9];
    rot_of_quat(q[0], q[1], q[2], q[3], R);
    t[0] += R[0] * vx + R[1] * vy + R[2] * vz;
    t[1] += R[3] * vx + R[4] * vy + R[5] * vz;
    t[2] += R[6] * vx + R[7] * vy + R[8] * vz;
    const float dw = cw, dx = c * phi[0], dy = c * phi[1], dz = c * phi[2];
    float nw = q[0] * dw - q[1] * dx - q[2] * dy - q[3] * dz;
    float nx = q[0] * dx + q[1] * dw + q[2] * dz - q[3] * dy;
    float ny = q[0] * dy - q[1] * dz + q[2] * dw + q[3] * dx;
    float nz = q[0] * dz + q[1] * dy - q[2] * dx + q[3] * dw;
    normalize_quat(nw, nx, ny, nz);
    q[0] = nw; q[1] = nx; q[2] = ny; q[3] = nz;
}

// Rotation matrix of a unit quaternion, FP64.
__device__ __forceinline__ void rot_of_quat_d(double w, double x, double y, double z, double R[9])
{
#pragma clang fp contract(off)
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// (t, q) <- (t, q) Exp([rho; phi]) in FP64: t += R V(phi) rho,
// q <- q (x) q(phi), renormalised with w >= 0.  q must be a unit quaternion.
__device__ __forceinline__ void right_exp_d(double t[3], double q[4], const double rho[3],
                                            const double phi[3])
{
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double a, b, c, cw;
    if (th2 < 1e-4) {
        // Series in th^2 (th < 0.01): truncation below 1e-17.
        a = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        b = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
        c = 0.5 - th2 / 48.0 + th2 * th2 / 3840.0;
        cw = 1.0 - th2 / 8.0 + th2 * th2 / 384.0;
    } else {
        const double th = sqrt(th2);
        double s, co, sh, ch;
        sincos(th, &s, &co);
        sincos(0.5 * th, &sh, &ch);
        a = 2.0 * sh * sh / th2;
        b = (th - s) / (th2 * th);
        c = sh / th;
        cw = ch;
    }
    const double c1x = phi[1] * rho[2] - phi[2] * rho[1];
    const double c1y = phi[2] * rho[0] - phi[0] * rho[2];
    const double c1z = phi[0] * rho[1] - phi[1] * rho[0];
    const double c2x = phi[1] * c1z - phi[2] * c1y;
    const double c2y = phi[2] * c1x - phi[0] * c1z;
    const double c2z = phi[0] * c1y - phi[1] * c1x;
    const double vx = rho[0] + a * c1x + b * c2x;
    const double vy = rho[1] + a * c1y + b * c2y;
    const double vz = rho[2] + a * c1z + b * c2z;
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    double R[9];
    rot_of_quat_d(w, x, y, z, R);
    t[0] += R[0] * vx + R[1] * vy + R[2] * vz;
    t[1] += R[3] * vx + R[4] * vy + R[5] * vz;
    t[2] += R[6] * vx + R[7] * vy + R[8] * vz;
    const double dx = c * phi[0], dy = c * phi[1], dz = c * phi[2];
    const double nw = w * cw - x * dx - y * dy - z * dz;
    const double nx = w * dx + x * cw + y * dz - z * dy;
    const double ny = w * dy - x * dz + y * cw + z * dx;
    const double nz = w * dz + x * dy - y * dx + z * cw;
    const double m = (nw < 0.0 ? -1.0 : 1.0) / sqrt(nw * nw + nx * nx + ny * ny + nz * nz);
    q[0] = nw * m; q[1] = nx * m; q[2] = ny * m; q[3] = nz * m;
}

__device__ __forceinline__ void load_pose_d(const float t[3], const float q[4], double td[3],
                                            double qd[4])
{
#pragma clang fp contract(off)
    for (int a = 0; a < 3; ++a) td[a] = t[a];
    const double n = 1.0 / sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] +
                                (double)q[3] * q[3]);
    for (int a = 0; a < 4; ++a) qd[a] = q[a] * n;
}

__device__ __forceinline__ void store_pose_d(const double td[3], const double qd[4], float t[3],
                                             float q[4])
{
    for (int a = 0; a < 3; ++a) t[a] = (float)td[a];
    for (int a = 0; a < 4; ++a) q[a] = (float)qd[a];
}

// Gradient-guided step of Eq. 7 from the body-frame gradient g: each block
// of psi = [a_t g_rho; a_r g_phi] is scaled down to its bound, then
// T <- T Exp(psi).  FP32: the increment is at most a decimetre, so t + dt is
// rounded once at t's own precision.
// psi = [a_t g_rho; a_r g_phi], each block scaled down to its norm bound.
__device__ __forceinline__ void step_vector(const float g[6], float alpha_t, float alpha_r,
                                            float rho_max, float phi_max, float rho[3], float phi[3])
{
#pragma clang fp contract(off)
    rho[0] = alpha_t * g[0]; rho[1] = alpha_t * g[1]; rho[2] = alpha_t * g[2];
    phi[0] = alpha_r * g[3]; phi[1] = alpha_r * g[4]; phi[2] = alpha_r * g[5];
    const float nr = sqrtf(rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2]);
    const float np = sqrtf(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (nr > rho_max) {
        const float k = rho_max / nr;
        rho[0] *= k; rho[1] *= k; rho[2] *= k;
    }
    if (np > phi_max) {
        const float k = phi_max / np;
        phi[0] *= k; phi[1] *= k; phi[2] *= k;
    }
}

__device__ __forceinline__ void take_step(float t[3], float q[4], const float g[6], float alpha_t,
                                          float alpha_r, float rho_max, float phi_max)
{
#pragma clang fp contract(off)
    float rho[3], phi[3];
    step_vector(g, alpha_t, alpha_r, rho_max, phi_max, rho, phi);
    right_exp(t, q, rho, phi);
}

// ---------------------------------------------------------------------------
// Grid records
// ---------------------------------------------------------------------------

typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
// Scan points are wave-uniform: reading them through the constant address
// space lets the compiler use scalar loads.
typedef const __attribute__((address_space(4))) f4v *scan_ptr;

constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, gfx9 family

// One cell record as loaded: 8 FP32 (two 16 B loads) or 8 16-bit samples.
template <int DT> struct Cell;
template <> struct Cell<0> { f4v a, b; };
template <> struct Cell<1> { u4v a; };
template <> struct Cell<2> { u4v a; };

template <int DT> __device__ __forceinline__ constexpr uint32_t record_shift() { return DT == 0 ? 5 : 4; }

template <int DT>
__device__ __forceinline__ void load_cell(__amdgpu_buffer_rsrc_t rs, uint32_t off, Cell<DT> &c);

template <>
__device__ __forceinline__ void load_cell<0>(__amdgpu_buffer_rsrc_t rs, uint32_t off, Cell<0> &c)
{
    c.a = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    c.b = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0));
}
template <>
__device__ __forceinline__ void load_cell<1>(__amdgpu_buffer_rsrc_t rs, uint32_t off, Cell<1> &c)
{
    c.a = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
}
template <>
__device__ __forceinline__ void load_cell<2>(__amdgpu_buffer_rsrc_t rs, uint32_t off, Cell<2> &c)
{
    c.a = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
}

// The same record through a 64-bit address (maps beyond one buffer's range).
template <int DT>
__device__ __forceinline__ void load_cell_g(uint64_t addr, Cell<DT> &c);
template <>
__device__ __forceinline__ void load_cell_g<0>(uint64_t addr, Cell<0> &c)
{
    const f4v *p = reinterpret_cast<const f4v *>(addr);
    c.a = p[0];
    c.b = p[1];
}
template <>
__device__ __forceinline__ void load_cell_g<1>(uint64_t addr, Cell<1> &c)
{
    c.a = *reinterpret_cast<const u4v *>(addr);
}
template <>
__device__ __forceinline__ void load_cell_g<2>(uint64_t addr, Cell<2> &c)
{
    c.a = *reinterpret_cast<const u4v *>(addr);
}

__device__ __forceinline__ float half_lo(uint32_t v)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu));
}

// Corner samples of a BF16 record (FP32 records hold polynomial coefficients
// and FP16 records feed mixed-precision FMAs, so neither is decoded).
template <int DT> __device__ __forceinline__ void decode(const Cell<DT> &c, float v[8]);
template <> __device__ __forceinline__ void decode<2>(const Cell<2> &c, float v[8])
{
    v[0] = __uint_as_float(c.a.x << 16); v[1] = __uint_as_float(c.a.x & 0xffff0000u);
    v[2] = __uint_as_float(c.a.y << 16); v[3] = __uint_as_float(c.a.y & 0xffff0000u);
    v[4] = __uint_as_float(c.a.z << 16); v[5] = __uint_as_float(c.a.z & 0xffff0000u);
    v[6] = __uint_as_float(c.a.w << 16); v[7] = __uint_as_float(c.a.w & 0xffff0000u);
}

// Running sums of one particle over its share of the scan.
struct Acc {
    double l;              // sum of log2(G + eps)
    float ax, ay, az;      // sum of dG/du / (G + eps)
    float bx, by, bz;      // sum of v' x (dG/du / (G + eps)), v' = A p
};

// Point-loop form of the sums: with d = dG/du / (G + eps) per point, the
// loop keeps sum d and the outer products S = sum d p^T (p the scan point,
// sensor frame) instead of sum v' x d.  Since v' = A p, the cross-product sum
// is recovered per range of points as B_a = e_abc A_be S_ce (e_abc the
// permutation symbol), so the loop needs neither v' nor a separate
// translation add.
struct PtAcc {
    double l;
    float ax, ay, az;
    float s[9];            // s[3c + e] = sum d_c p_e
};

__device__ __forceinline__ void add_acc(Acc &a, const Acc &b)
{
#pragma clang fp contract(off)
    a.l += b.l;
    a.ax += b.ax; a.ay += b.ay; a.az += b.az;
    a.bx += b.bx; a.by += b.by; a.bz += b.bz;
}

// The single-grid scan is cut into kSubChunks sub-chunks of Q points (Q a
// multiple of 4), each summed from zero on its own; a wave adds its
// consecutive sub-chunks in order, and the W wave sums are added in wave
// order.  This fixed order lets a tile's sub-chunks also be spread over
// separate waves (the tail tiles of a launch) with bit-identical results.
__host__ __device__ __forceinline__ int sub_chunk_len(int M)
{
    return 4 * ((M + 4 * kSubChunks - 1) / (4 * kSubChunks));
}

// Grid constants of one evaluation loop.  Records are laid out with a zero
// layer around the cells (grid_records): record (I, J, K), 0 <= I <= nx and so
// on, x fastest; the cell (i, j, k) of the samples is record (i + 1, j + 1,
// k + 1), and records with an index 0 or n on some axis are zero.
struct GridK {
    __amdgpu_buffer_rsrc_t rs;
    const char *gbase;       // 64-bit addressing: the grid's records
    int32_t ixm, iym, izm;   // largest record index per axis (n)
    uint32_t nxm, nym, nzm;  // cells per axis (n - 1): inside records have indices 1 .. n - 1
    uint32_t cx, cxy;        // record strides: records per row and per slab
    float eps;
};

__device__ __forceinline__ void grid_layout(const StepDesc &d, GridK &g)
{
    g.ixm = d.nx; g.iym = d.ny; g.izm = d.nz;
    g.nxm = (uint32_t)(d.nx - 1); g.nym = (uint32_t)(d.ny - 1); g.nzm = (uint32_t)(d.nz - 1);
    g.cx = (uint32_t)(d.nx + 1);
    g.cxy = (uint32_t)(d.nx + 1) * (uint32_t)(d.ny + 1);
    g.eps = d.eps;
}

// The records of a single grid: a buffer over them (its range capped at 32
// bits; grids beyond it are read through 64-bit addresses) and their base.
template <int DT>
__device__ __forceinline__ void single_grid_records(const StepDesc &d, GridK &g)
{
    const uint64_t bytes = grid_records(d.nx, d.ny, d.nz) << record_shift<DT>();
    g.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(d.cells), (short)0,
                                             (int)(uint32_t)(bytes < kMaxRecordBytes ? bytes : kMaxRecordBytes),
                                             kRsrcWord3);
    g.gbase = static_cast<const char *>(d.cells);
}

// Cell fractions and record offset of a transformed point.
struct Pt {
    float fx, fy, fz;      // position inside the cell
    uint32_t off;          // byte offset of the cell's record (a zero record when outside)
    bool inside;
};

// Trilinear value and gradient (index units) of one cell record.
template <int DT>
__device__ __forceinline__ void trilinear(const Cell<DT> &cell, float fx, float fy, float fz,
                                          float &G, float &gx, float &gy, float &gz)
{
#pragma clang fp contract(off)
    float c[8];
    decode<DT>(cell, c);
    // Corner records: lerps along x on the four y/z edges, then y, then z.
    const float d00 = c[1] - c[0], d10 = c[3] - c[2], d01 = c[5] - c[4], d11 = c[7] - c[6];
    const float e00 = fmaf(fx, d00, c[0]), e10 = fmaf(fx, d10, c[2]);
    const float e01 = fmaf(fx, d01, c[4]), e11 = fmaf(fx, d11, c[6]);
    const float gy0 = e10 - e00, gy1 = e11 - e01;
    const float f0 = fmaf(fy, gy0, e00), f1 = fmaf(fy, gy1, e01);
    gz = f1 - f0;
    G = fmaf(fz, gz, f0);
    gy = fmaf(fz, gy1 - gy0, gy0);
    const float dx0 = fmaf(fy, d10 - d00, d00), dx1 = fmaf(fy, d11 - d01, d01);
    gx = fmaf(fz, dx1 - dx0, dx0);
}

// hi(c) - lo(c) of two packed FP16 samples in one mixed-precision FMA
// (hi * 1 - lo, rounded once: the FP32 difference of the decoded samples).
__device__ __forceinline__ float half_hi_minus_lo(uint32_t c)
{
#pragma clang fp contract(off)
    float r;
    asm("v_fma_mix_f32 %0, %1, %2, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]"
        : "=v"(r) : "v"(c), "s"(1.0f));
    return r;
}

// FP16 corners: the first x lerps read the packed samples directly through
// mixed-precision FMAs, so no sample is decoded separately.  Same arithmetic,
// and results, as the generic form applied to the decoded FP16 samples.
template <>
__device__ __forceinline__ void trilinear<1>(const Cell<1> &cell, float fx, float fy, float fz,
                                             float &G, float &gx, float &gy, float &gz)
{
#pragma clang fp contract(off)
    const float d00 = half_hi_minus_lo(cell.a.x), d10 = half_hi_minus_lo(cell.a.y);
    const float d01 = half_hi_minus_lo(cell.a.z), d11 = half_hi_minus_lo(cell.a.w);
    const float e00 = fmaf(fx, d00, half_lo(cell.a.x)), e10 = fmaf(fx, d10, half_lo(cell.a.y));
    const float e01 = fmaf(fx, d01, half_lo(cell.a.z)), e11 = fmaf(fx, d11, half_lo(cell.a.w));
    const float gy0 = e10 - e00, gy1 = e11 - e01;
    const float f0 = fmaf(fy, gy0, e00), f1 = fmaf(fy, gy1, e01);
    gz = f1 - f0;
    G = fmaf(fz, gz, f0);
    gy = fmaf(fz, gy1 - gy0, gy0);
    const float dx0 = fmaf(fy, d10 - d00, d00), dx1 = fmaf(fy, d11 - d01, d01);
    gx = fmaf(fz, dx1 - dx0, dx0);
}

// FP32 grids store each cell as the coefficients of its trilinear polynomial
//   G(x, y, z) = a0 + a1 x + a2 y + a3 z + a4 xy + a5 xz + a6 yz + a7 xyz
// (x, y, z the fractions in the cell), so value and gradient take 11 FMAs.
template <>
__device__ __forceinline__ void trilinear<0>(const Cell<0> &cell, float fx, float fy, float fz,
                                             float &G, float &gx, float &gy, float &gz)
{
#pragma clang fp contract(off)
    const float a0 = cell.a.x, a1 = cell.a.y, a2 = cell.a.z, a3 = cell.a.w;
    const float a4 = cell.b.x, a5 = cell.b.y, a6 = cell.b.z, a7 = cell.b.w;
    const float p = fmaf(a6, fy, a3);      // dG/dz at x = 0
    const float q = fmaf(a7, fy, a5);      // d2G/dxdz
    const float r = fmaf(a4, fy, a1);      // dG/dx at z = 0
    const float s = fmaf(a2, fy, a0);      // G at x = z = 0
    gz = fmaf(q, fx, p);
    gx = fmaf(q, fz, r);
    G = fmaf(gz, fz, fmaf(r, fx, s));
    gy = fmaf(fmaf(a7, fx, a6), fz, fmaf(a4, fx, a2));
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) f4v *scan32_ptr;

// Gradient sums of one point (scan point pf, uniform over the wave) given
// 1/(G + eps).
__device__ __forceinline__ void add_grad(const f4v &pf, float gx, float gy, float gz, float inv,
                                         PtAcc &acc)
{
#pragma clang fp contract(off)
    const float dx = gx * inv, dy = gy * inv, dz = gz * inv;
    acc.ax += dx; acc.ay += dy; acc.az += dz;
    acc.s[0] = fmaf(dx, pf.x, acc.s[0]); acc.s[1] = fmaf(dx, pf.y, acc.s[1]); acc.s[2] = fmaf(dx, pf.z, acc.s[2]);
    acc.s[3] = fmaf(dy, pf.x, acc.s[3]); acc.s[4] = fmaf(dy, pf.y, acc.s[4]); acc.s[5] = fmaf(dy, pf.z, acc.s[5]);
    acc.s[6] = fmaf(dz, pf.x, acc.s[6]); acc.s[7] = fmaf(dz, pf.y, acc.s[7]); acc.s[8] = fmaf(dz, pf.z, acc.s[8]);
}

template <int DT, bool SKIP>
__device__ __forceinline__ void accumulate1(const GridK &g, const Pt &p, const f4v &pf,
                                            const Cell<DT> &c, PtAcc &acc)
{
#pragma clang fp contract(off)
    float G, x, y, z;
    trilinear<DT>(c, p.fx, p.fy, p.fz, G, x, y, z);
    float d = G + g.eps;
    if (SKIP) d = p.inside ? d : 1.0f;
    acc.l += (double)fast_log2(d);
    add_grad(pf, x, y, z, fast_rcp(d), acc);
}

// The per-point transform runs in FP64: the grid map A = R/h, b stays in
// FP64, points arrive as FP64 (scalar loads of the FP64 copy of the scan), and
// u = A p + b, floor(u) and the fraction are computed in FP64; only the
// fraction is rounded to FP32.  An FP32 A would carry one rounding
// shared by every point of the particle, a systematic error that the peaked
// likelihood turns into gradient errors of order 1e-4 of the summation scale.
typedef double d4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) d4v *scan64_ptr;
typedef double d16v __attribute__((ext_vector_type(16)));

struct GridMap64 {
    double A[9];
    double b[3];
    uint32_t base;         // byte offset of the grid in the record buffer (keyframe maps)
};

__device__ __forceinline__ void grid_map64(const float *t, const float *q, double ox, double oy,
                                           double oz, double h, GridMap64 &m)
{
#pragma clang fp contract(off)
    double w = q[0], x = q[1], y = q[2], z = q[3];
    const double n = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= n; x *= n; y *= n; z *= n;
    double R[9];
    rot_of_quat_d(w, x, y, z, R);
    const double ih = 1.0 / h;
    for (int e = 0; e < 9; ++e) m.A[e] = R[e] * ih;
    // u + 1 = (x - o)/h - 1/2 + 1: the record index of the zero-layer layout.
    m.b[0] = ((double)t[0] - ox) * ih + 0.5;
    m.b[1] = ((double)t[1] - oy) * ih + 0.5;
    m.b[2] = ((double)t[2] - oz) * ih + 0.5;
    m.base = 0;
}

// floor(x) as int32 in one instruction (saturating for out-of-range x).
// Conversion toward zero, saturating (NaN gives 0).
__device__ __forceinline__ int cvt_trunc_d(double x)
{
    int r;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// v clamped to [0, hi] in one instruction (hi is wave-uniform).
__device__ __forceinline__ int clamp_index(int v, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(v), "s"(hi));
    return r;
}

template <int DT, bool BIG, bool KF = false>
__device__ __forceinline__ Pt prep_point64(const GridK &g, const GridMap64 &gm, double px,
                                           double py, double pz)
{
#pragma clang fp contract(off)
    Pt p;
    const double *A = gm.A;
    // u + 1 per axis (the map's b carries the +1): for u + 1 >= 0 the
    // truncation is the floor, so a point inside the grid (0 <= u < n - 1)
    // takes record index floor(u) + 1 in [1, n - 1]; every other point, NaN
    // included, lands in the zero layer (index 0 or n) after the clamp.
    const double ux = fma(A[0], px, fma(A[1], py, fma(A[2], pz, gm.b[0])));
    const double uy = fma(A[3], px, fma(A[4], py, fma(A[5], pz, gm.b[1])));
    const double uz = fma(A[6], px, fma(A[7], py, fma(A[8], pz, gm.b[2])));
    const int ix = clamp_index(cvt_trunc_d(ux), g.ixm);
    const int iy = clamp_index(cvt_trunc_d(uy), g.iym);
    const int iz = clamp_index(cvt_trunc_d(uz), g.izm);
    p.fx = (float)__builtin_amdgcn_fract(ux);
    p.fy = (float)__builtin_amdgcn_fract(uy);
    p.fz = (float)__builtin_amdgcn_fract(uz);
    p.inside = ((uint32_t)(ix - 1) < g.nxm) & ((uint32_t)(iy - 1) < g.nym) & ((uint32_t)(iz - 1) < g.nzm);
    const uint32_t rec = BIG ? (uint32_t)ix + g.cx * (uint32_t)iy + g.cxy * (uint32_t)iz
                             : (uint32_t)ix + __umul24(g.cx, (uint32_t)iy) +
                                   __umul24(g.cxy, (uint32_t)iz);
    if constexpr (BIG && !KF)
        p.off = rec;   // a record index: the record is read through a 64-bit address
    else
        p.off = KF ? gm.base + (rec << record_shift<DT>()) : (rec << record_shift<DT>());
    return p;
}

// Four points share one log2 and one reciprocal:
//   log2(d0 d1 d2 d3),  r = 1 / (d0 d1 d2 d3),  1/(d0 d1) = d2 d3 r,  1/(d2 d3) = d0 d1 r,
// then 1/d0 = d1 / (d0 d1) and so on.  With grid values in [0, 1] and
// eps >= 1e-5 every d lies in [eps - 3e-6, 1 + eps] (the interpolant's rounding
// error stays below 3e-6), so the product of four stays a normal FP32 number.
template <int DT, bool SKIP>
__device__ __forceinline__ void accumulate4(const GridK &g, const Pt *p, const f4v *pf,
                                            const Cell<DT> *c, PtAcc &acc)
{
#pragma clang fp contract(off)
    float G[4], x[4], y[4], z[4], d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        trilinear<DT>(c[k], p[k].fx, p[k].fy, p[k].fz, G[k], x[k], y[k], z[k]);
        d[k] = G[k] + g.eps;
        if (SKIP) d[k] = p[k].inside ? d[k] : 1.0f;
    }
    const float p01 = d[0] * d[1], p23 = d[2] * d[3];
    const float prod = p01 * p23;
    acc.l += (double)fast_log2(prod);
    const float r = fast_rcp(prod);
    const float r01 = p23 * r, r23 = p01 * r;
    add_grad(pf[0], x[0], y[0], z[0], d[1] * r01, acc);
    add_grad(pf[1], x[1], y[1], z[1], d[0] * r01, acc);
    add_grad(pf[2], x[2], y[2], z[2], d[3] * r23, acc);
    add_grad(pf[3], x[3], y[3], z[3], d[2] * r23, acc);
}

// Gather floor: the words of a record folded into one (keeps the loads live
// with the least arithmetic).
template <int DT> __device__ __forceinline__ uint32_t cell_xor(const Cell<DT> &c);
template <> __device__ __forceinline__ uint32_t cell_xor<0>(const Cell<0> &c)
{
    return (__float_as_uint(c.a.x) ^ __float_as_uint(c.a.y) ^ __float_as_uint(c.a.z) ^
            __float_as_uint(c.a.w)) ^
           (__float_as_uint(c.b.x) ^ __float_as_uint(c.b.y) ^ __float_as_uint(c.b.z) ^
            __float_as_uint(c.b.w));
}
template <> __device__ __forceinline__ uint32_t cell_xor<1>(const Cell<1> &c)
{
    return c.a.x ^ c.a.y ^ c.a.z ^ c.a.w;
}
template <> __device__ __forceinline__ uint32_t cell_xor<2>(const Cell<2> &c)
{
    return c.a.x ^ c.a.y ^ c.a.z ^ c.a.w;
}

// Record of a prepared point: from the buffer or, with GLB, through a 64-bit
// address; with WIDE (a single grid beyond one buffer's range or with slabs of
// 2^24 records and more) p.off is the record index and the address is formed
// in 64 bits.  An outside point reads a record of the zero layer either way.
template <int DT, bool GLB, bool WIDE = false>
__device__ __forceinline__ void fetch(const GridK &g, const Pt &p, Cell<DT> &c)
{
    if (WIDE)
        load_cell_g<DT>((uint64_t)g.gbase + ((uint64_t)p.off << record_shift<DT>()), c);
    else if (GLB)
        load_cell_g<DT>((uint64_t)(g.gbase + p.off), c);
    else
        load_cell<DT>(g.rs, p.off, c);
}

// Points [j0, j1) of the scan against one pose, four at a time: the four
// points' FP64 coordinates arrive in one 128 B scalar load, and each point's
// record loads are issued as soon as its offset is known (a scheduling
// barrier keeps them ahead of the next point's transform), before any of the
// four points' arithmetic.  The range's sums are stored in acc (l, sum d and
// B = sum v' x d, v' = A p).
template <int DT, bool BIG, bool SKIP, bool KF = false, bool GLB = false, bool FLOOR = false>
__device__ __forceinline__ void eval_range64(const GridK &g, scan64_ptr scan, scan32_ptr scanf,
                                             int j0, int j1, const GridMap64 &gm, Acc &acc)
{
#pragma clang fp contract(off)
    PtAcc pa = {0.0, 0.0f, 0.0f, 0.0f, {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f}};
    uint32_t fl = 0;                      // FLOOR: checksum of the gathered words
    int j = j0;
    constexpr int U = 4;
    for (; j + U <= j1; j += U) {
        Pt p[U];
        f4v pf[U];
        Cell<DT> c[U];
        // Raised wave priority while the four points' loads are being
        // issued: a wave that reaches its loads gets them out ahead of other
        // waves' arithmetic, so more of their latency overlaps.
        __builtin_amdgcn_s_setprio(2);
        const d16v sq = *(const __attribute__((address_space(4))) d16v *)(scan + j);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            p[k] = prep_point64<DT, BIG, KF>(g, gm, sq[4 * k], sq[4 * k + 1], sq[4 * k + 2]);
            fetch<DT, GLB, BIG && !KF>(g, p[k], c[k]);
            __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_s_setprio(0);
        if constexpr (FLOOR) {
#pragma unroll
            for (int k = 0; k < U; ++k) fl ^= cell_xor<DT>(c[k]);
        } else {
#pragma unroll
            for (int k = 0; k < U; ++k) pf[k] = scanf[j + k];
            accumulate4<DT, SKIP>(g, p, pf, c, pa);
        }
    }
    for (; j < j1; ++j) {
        const d4v s = scan[j];
        const Pt p = prep_point64<DT, BIG, KF>(g, gm, s.x, s.y, s.z);
        Cell<DT> c;
        fetch<DT, GLB, BIG && !KF>(g, p, c);
        if constexpr (FLOOR) {
            fl ^= cell_xor<DT>(c);
        } else {
            const f4v pf = scanf[j];
            accumulate1<DT, SKIP>(g, p, pf, c, pa);
        }
    }
    if constexpr (FLOOR) {
        acc = {(double)fl, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        return;
    }
    // B_a = e_abc A_be S_ce, in FP64 from the FP32 sums.
    const double *A = gm.A;
    double S[9];
    for (int e = 0; e < 9; ++e) S[e] = (double)pa.s[e];
    double B[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < 3; ++e) {
        B[0] = fma(A[3 + e], S[6 + e], fma(-A[6 + e], S[3 + e], B[0]));
        B[1] = fma(A[6 + e], S[e], fma(-A[e], S[6 + e], B[1]));
        B[2] = fma(A[e], S[3 + e], fma(-A[3 + e], S[e], B[2]));
    }
    acc.l = pa.l;
    acc.ax = pa.ax; acc.ay = pa.ay; acc.az = pa.az;
    acc.bx = (float)B[0]; acc.by = (float)B[1]; acc.bz = (float)B[2];
}

// ---------------------------------------------------------------------------
// Likelihood + gradient + pose step, single grid: one 64-particle tile
// ---------------------------------------------------------------------------

// Body-frame gradient of the 7 sums: g_rho = R^T (sum d') / h,
// g_phi = R^T sum (v' x d'), R from the tile's pose q.
__device__ __forceinline__ void body_gradient(const float q[4], const float s[6], float inv_h,
                                              float gr[6])
{
#pragma clang fp contract(off)
    float qn[4] = {q[0], q[1], q[2], q[3]};
    normalize_quat(qn[0], qn[1], qn[2], qn[3]);
    float R[9];
    rot_of_quat(qn[0], qn[1], qn[2], qn[3], R);
    const float ax = s[0] * inv_h, ay = s[1] * inv_h, az = s[2] * inv_h;
    gr[0] = R[0] * ax + R[3] * ay + R[6] * az;
    gr[1] = R[1] * ax + R[4] * ay + R[7] * az;
    gr[2] = R[2] * ax + R[5] * ay + R[8] * az;
    gr[3] = R[0] * s[3] + R[3] * s[4] + R[6] * s[5];
    gr[4] = R[1] * s[3] + R[4] * s[4] + R[7] * s[5];
    gr[5] = R[2] * s[3] + R[5] * s[4] + R[8] * s[5];
}

// The particle a slot of the evaluation takes (N for the slots past the last).
__device__ __forceinline__ int slot_particle(const StepDesc &d, int slot)
{
    return d.order ? (slot < d.N ? d.order[slot] : d.N) : slot;
}

// Load the tile's poses into LDS as stored: the first pass evaluates the
// pose itself (its quaternion normalised in FP64 by the grid map); the FP32
// normalisation happens before the first step.
__device__ __forceinline__ void load_tile_pose(const StepDesc &d, int i, int lane, float (*s_pose)[64])
{
    const int N = d.N;
    const int ic = i < N ? i : N - 1;
    for (int c = 0; c < 7; ++c) s_pose[c][lane] = d.pose[c * N + ic];
}

// Reduce the W partial sums (fixed order), store l and g, take the step.
// With s_upd (keyframe maps, loop-gated correction) only lanes with s_loop >= 0
// step, and each of them leaves psi (rows 0-5) and its translation before the
// step (rows 6-8) in s_upd for the keyframe propagation.
// Sub-chunk sc (in summation order) of wave w of a tile: the waves take the
// sub-chunks in turn, so that at any time the 8 waves of a tile, and the tiles
// running beside it, evaluate neighbouring parts of the scan (whose points
// land in overlapping cells).
template <int W>
__device__ __forceinline__ constexpr int wave_sub_chunk(int w, int sc) { return sc * W + w; }

template <int W>
__device__ __forceinline__ void tile_epilogue(const StepDesc &d, int i, int lane, int pass,
                                              const double (*s_l)[64], const float (*s_g)[W][64],
                                              float (*s_pose)[64], const int *s_loop = nullptr,
                                              float (*s_upd)[64] = nullptr)
{
#pragma clang fp contract(off)
    double l = 0.0;
    float s[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int w = 0; w < W; ++w) {
        l += s_l[w][lane];
        for (int c = 0; c < 6; ++c) s[c] += s_g[c][w][lane];
    }
    float t[3] = {s_pose[0][lane], s_pose[1][lane], s_pose[2][lane]};
    float q[4] = {s_pose[3][lane], s_pose[4][lane], s_pose[5][lane], s_pose[6][lane]};
    float gr[6];
    if (d.K > 0) {
        for (int c = 0; c < 6; ++c) gr[c] = s[c];   // already body-frame, summed over neighbours
    } else {
        body_gradient(q, s, d.inv_h, gr);
    }
    const int N = d.N;
    const bool stepping = pass < d.iters;
    if (i < N) {
        // Only the last pass's log-likelihood and the last step's gradient are
        // outputs; earlier passes' would be overwritten (and, with the
        // evaluation order, scattered writes cost a partial line each).
        if (pass == d.iters + d.post_eval - 1) d.loglik[i] = (float)(l * kLn2);
        if (pass == d.iters - 1)
            for (int c = 0; c < 6; ++c) d.grad[c * N + i] = gr[c];
        if (d.trace) {
            float *tr = d.trace + (size_t)pass * kTraceRows * N + i;
            for (int c = 0; c < 3; ++c) tr[(size_t)c * N] = t[c];
            for (int c = 0; c < 4; ++c) tr[(size_t)(3 + c) * N] = q[c];
            tr[(size_t)7 * N] = (float)(l * kLn2);
            for (int c = 0; c < 6; ++c) tr[(size_t)(8 + c) * N] = gr[c];
        }
    }
    // The stored pose may carry any nonzero quaternion; the step composes
    // with its normalisation (later passes hold the step's own unit result).
    if (stepping && pass == 0) normalize_quat(q[0], q[1], q[2], q[3]);
    if (stepping && s_upd) {
        if (s_loop[lane] >= 0) {
            float rho[3], phi[3];
            step_vector(gr, d.alpha_t, d.alpha_r, d.rho_max, d.phi_max, rho, phi);
            for (int c = 0; c < 3; ++c) {
                s_upd[c][lane] = rho[c];
                s_upd[3 + c][lane] = phi[c];
                s_upd[6 + c][lane] = t[c];
            }
            right_exp(t, q, rho, phi);
        }
    } else if (stepping) {
        take_step(t, q, gr, d.alpha_t, d.alpha_r, d.rho_max, d.phi_max);
    }
    if (stepping) {
        s_pose[0][lane] = t[0]; s_pose[1][lane] = t[1]; s_pose[2][lane] = t[2];
        s_pose[3][lane] = q[0]; s_pose[4][lane] = q[1]; s_pose[5][lane] = q[2]; s_pose[6][lane] = q[3];
    }
}

__device__ __forceinline__ void store_tile_pose(const StepDesc &d, int i, int lane,
                                                const float (*s_pose)[64])
{
#pragma clang fp contract(off)
    const int N = d.N;
    if (i < N) {
        d.pose[i] = s_pose[0][lane]; d.pose[N + i] = s_pose[1][lane]; d.pose[2 * N + i] = s_pose[2][lane];
        d.pose[3 * N + i] = s_pose[3][lane]; d.pose[4 * N + i] = s_pose[4][lane];
        d.pose[5 * N + i] = s_pose[5][lane]; d.pose[6 * N + i] = s_pose[6][lane];
    }
}

template <int DT, bool BIG, bool SKIP, int W, bool FLOOR = false>
__device__ __forceinline__ void eval_tile(const StepDesc &d, int tile)
{
#pragma clang fp contract(off)
    __shared__ double s_l[W][64];
    __shared__ float s_g[6][W][64];
    __shared__ float s_pose[7][64];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = slot_particle(d, tile * 64 + lane);
    if (wave == 0) load_tile_pose(d, i, lane, s_pose);

    GridK g;
    grid_layout(d, g);
    single_grid_records<DT>(d, g);
    const int M = d.M;
    const int Q = sub_chunk_len(M);
    constexpr int S = kSubChunks / W;      // sub-chunks per wave
    const int passes = d.iters + d.post_eval;
    __syncthreads();

    for (int pass = 0; pass < passes; ++pass) {
        Acc acc = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        {
            const float t[3] = {s_pose[0][lane], s_pose[1][lane], s_pose[2][lane]};
            const float q[4] = {s_pose[3][lane], s_pose[4][lane], s_pose[5][lane], s_pose[6][lane]};
            GridMap64 gm;
            grid_map64(t, q, d.ox, d.oy, d.oz, d.h, gm);
            for (int sc = 0; sc < S; ++sc) {
                const int c = wave_sub_chunk<W>(wave, sc);
                Acc part = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                eval_range64<DT, BIG, SKIP, false, false, FLOOR>(g, (scan64_ptr)d.scan8, (scan32_ptr)d.scan4,
                                                                 min(M, c * Q), min(M, (c + 1) * Q), gm, part);
                add_acc(acc, part);
            }
        }
        s_l[wave][lane] = acc.l;
        s_g[0][wave][lane] = acc.ax; s_g[1][wave][lane] = acc.ay; s_g[2][wave][lane] = acc.az;
        s_g[3][wave][lane] = acc.bx; s_g[4][wave][lane] = acc.by; s_g[5][wave][lane] = acc.bz;
        __syncthreads();
        if (wave == 0) tile_epilogue<W>(d, i, lane, pass, s_l, s_g, s_pose);
        __syncthreads();
    }
    if (wave == 0) store_tile_pose(d, i, lane, s_pose);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Tail tiles: one wave per sub-chunk, then a per-tile reduce and step
// ---------------------------------------------------------------------------

// Pose of particle i as the tile holds it before pass `pass`: the input pose
// as stored (pass 0, as load_tile_pose) or the pose the previous pass's step
// stored.
__device__ __forceinline__ void tail_pose(const StepDesc &d, int i, int pass, float t[3], float q[4])
{
    (void)pass;
    const int N = d.N;
    const int ic = i < N ? i : N - 1;
    t[0] = d.pose[ic]; t[1] = d.pose[N + ic]; t[2] = d.pose[2 * N + ic];
    q[0] = d.pose[3 * N + ic]; q[1] = d.pose[4 * N + ic]; q[2] = d.pose[5 * N + ic]; q[3] = d.pose[6 * N + ic];
}

// One sub-chunk of one tail tile per wave: the same sub-chunk sums eval_tile forms.
template <int DT, bool BIG, bool SKIP, bool FLOOR = false>
__device__ __forceinline__ void tail_chunk(const StepDesc &d, int tile0, int pass, int rel, int c)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int i = slot_particle(d, (tile0 + rel) * 64 + lane);
    GridK g;
    grid_layout(d, g);
    single_grid_records<DT>(d, g);
    const int M = d.M, Q = sub_chunk_len(M);
    float t[3], q[4];
    tail_pose(d, i, pass, t, q);
    GridMap64 gm;
    grid_map64(t, q, d.ox, d.oy, d.oz, d.h, gm);
    Acc part = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    eval_range64<DT, BIG, SKIP, false, false, FLOOR>(g, (scan64_ptr)d.scan8, (scan32_ptr)d.scan4,
                                                     min(M, c * Q), min(M, (c + 1) * Q), gm, part);
    const size_t r = (size_t)rel * kSubChunks + c;
    d.tail_l[r * 64 + lane] = part.l;
    float *tg = d.tail_g + r * 6 * 64 + lane;
    tg[0] = part.ax; tg[64] = part.ay; tg[128] = part.az;
    tg[192] = part.bx; tg[256] = part.by; tg[320] = part.bz;
}

// Reduce a tail tile's sub-chunk sums in eval_tile's order (W waves of
// kSubChunks / W consecutive sub-chunks each), then the same epilogue; the
// pose goes back to memory after every pass.  One wave per tile.
template <int W>
__device__ __forceinline__ void tail_step(const StepDesc &d, int tile0, int pass, int rel)
{
#pragma clang fp contract(off)
    __shared__ double s_l[W][64];
    __shared__ float s_g[6][W][64];
    __shared__ float s_pose[7][64];
    const int lane = threadIdx.x & 63;
    const int i = slot_particle(d, (tile0 + rel) * 64 + lane);
    float t[3], q[4];
    tail_pose(d, i, pass, t, q);
    s_pose[0][lane] = t[0]; s_pose[1][lane] = t[1]; s_pose[2][lane] = t[2];
    s_pose[3][lane] = q[0]; s_pose[4][lane] = q[1]; s_pose[5][lane] = q[2]; s_pose[6][lane] = q[3];
    constexpr int S = kSubChunks / W;
    for (int w = 0; w < W; ++w) {
        Acc acc = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int sc = 0; sc < S; ++sc) {
            const size_t r = (size_t)rel * kSubChunks + wave_sub_chunk<W>(w, sc);
            const float *tg = d.tail_g + r * 6 * 64 + lane;
            const Acc part = {d.tail_l[r * 64 + lane], tg[0], tg[64], tg[128], tg[192], tg[256], tg[320]};
            add_acc(acc, part);
        }
        s_l[w][lane] = acc.l;
        s_g[0][w][lane] = acc.ax; s_g[1][w][lane] = acc.ay; s_g[2][w][lane] = acc.az;
        s_g[3][w][lane] = acc.bx; s_g[4][w][lane] = acc.by; s_g[5][w][lane] = acc.bz;
    }
    tile_epilogue<W>(d, i, lane, pass, s_l, s_g, s_pose);
    store_tile_pose(d, i, lane, s_pose);
}

// ---------------------------------------------------------------------------
// Keyframe map: sum over neighbour keyframes (Eq. 2) under T_k^-1 T (Eq. 4)
// ---------------------------------------------------------------------------

// Squared translation distance in FP32 with a fixed operation order (no
// contraction): the neighbour choice is an integer decision that the checks
// reproduce bit for bit.
__device__ __forceinline__ float dist2_rn(float ax, float ay, float az, float bx, float by, float bz)
{
    const float dx = __fsub_rn(ax, bx), dy = __fsub_rn(ay, by), dz = __fsub_rn(az, bz);
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// |a - b| with every operation rounded on its own (no contraction), so that
// the path lengths below do not depend on how a loop body is compiled.
__device__ __forceinline__ float seg_len(float ax, float ay, float az, float bx, float by, float bz)
{
    return __fsqrt_rn(dist2_rn(ax, ay, az, bx, by, bz));
}

// Keyframe propagation of the loop-gated correction (Eq. 8-10) for the tile's
// particles: keyframe k in (o, K) moves by psi_k = (d_k / d_t) psi, where d_k
// is the path length along the particle's keyframe translations from its
// oldest neighbour o to k and d_t = d_{K-1} + |t_pre - t_{K-1}|.  The keyframes
// (o, K) are split into W contiguous chunks, one per wave.  Phase 1 (reads
// only) sums each chunk's segments, in keyframe order, into LDS; after the
// barrier every wave adds the sums of the chunks before its own (in chunk
// order) and phase 2 rewrites its chunk.  Loads are issued B keyframes at a
// time so that their latencies overlap.
template <int W>
__device__ __forceinline__ void kf_propagate(const StepDesc &d, int i, int lane, int wave,
                                             const int *s_loop, const float (*s_upd)[64],
                                             float (*s_seg)[64])
{
#pragma clang fp contract(off)
    constexpr int B = 4;
    const int N = d.N, K = d.K;
    const int o = s_loop[lane];
    const bool act = o >= 0 && i < N;
    float *kp = d.kf_pose;
    const size_t col = act ? (size_t)i : 0;
    const int len = act ? K - 1 - o : 0;
    const int chunk = (len + W - 1) / W;
    const int ka = act ? o + 1 + wave * chunk : 0;
    const int kb = act ? min(K, ka + chunk) : 0;
    // Phase 1: segments (k-1, k) for k in [ka, kb), and the translations
    // before the chunk and of the newest keyframe, all read before any write.
    float seg = 0.0f, ax = 0.0f, ay = 0.0f, az = 0.0f, lx = 0.0f, ly = 0.0f, lz = 0.0f;
    if (act) {
        const size_t rl = (size_t)(K - 1) * 7 * N + col;
        lx = kp[rl]; ly = kp[rl + N]; lz = kp[rl + 2 * N];
    }
    if (ka < kb) {
        const size_t r0 = (size_t)(ka - 1) * 7 * N + col;
        float px = kp[r0], py = kp[r0 + N], pz = kp[r0 + 2 * N];
        ax = px; ay = py; az = pz;
        for (int k = ka; k < kb; k += B) {
            float x[B], y[B], z[B];
            for (int b = 0; b < B; ++b) {
                const size_t r = (size_t)min(k + b, kb - 1) * 7 * N + col;
                x[b] = kp[r]; y[b] = kp[r + N]; z[b] = kp[r + 2 * N];
            }
            for (int b = 0; b < B; ++b) {
                if (k + b < kb) {
                    seg = __fadd_rn(seg, seg_len(x[b], y[b], z[b], px, py, pz));
                    px = x[b]; py = y[b]; pz = z[b];
                }
            }
        }
    }
    s_seg[wave][lane] = seg;
    __syncthreads();
    float da = 0.0f, dsum = 0.0f;
    for (int w = 0; w < W; ++w) {
        if (w == wave) da = dsum;
        dsum = __fadd_rn(dsum, s_seg[w][lane]);
    }
    const float dt = __fadd_rn(dsum, seg_len(s_upd[6][lane], s_upd[7][lane], s_upd[8][lane], lx, ly, lz));
    if (!(ka < kb && dt > 0.0f)) return;
    const float psi_rho[3] = {s_upd[0][lane], s_upd[1][lane], s_upd[2][lane]};
    const float psi_phi[3] = {s_upd[3][lane], s_upd[4][lane], s_upd[5][lane]};
    constexpr int B2 = 2;
    for (int k = ka; k < kb; k += B2) {
        float v[B2][7];
        for (int b = 0; b < B2; ++b) {
            const size_t r = (size_t)min(k + b, kb - 1) * 7 * N + col;
            for (int c = 0; c < 7; ++c) v[b][c] = kp[r + (size_t)c * N];
        }
        for (int b = 0; b < B2; ++b) {
            if (k + b >= kb) break;
            float t[3] = {v[b][0], v[b][1], v[b][2]};
            float q[4] = {v[b][3], v[b][4], v[b][5], v[b][6]};
            da = __fadd_rn(da, seg_len(t[0], t[1], t[2], ax, ay, az));
            ax = t[0]; ay = t[1]; az = t[2];
            const float ratio = __fdiv_rn(da, dt);
            const float rho[3] = {ratio * psi_rho[0], ratio * psi_rho[1], ratio * psi_rho[2]};
            const float phi[3] = {ratio * psi_phi[0], ratio * psi_phi[1], ratio * psi_phi[2]};
            right_exp(t, q, rho, phi);
            const size_t r = (size_t)(k + b) * 7 * N + col;
            kp[r] = t[0]; kp[r + N] = t[1]; kp[r + 2 * N] = t[2];
            kp[r + 3 * N] = q[0]; kp[r + 4 * N] = q[1]; kp[r + 5 * N] = q[2]; kp[r + 6 * N] = q[3];
        }
    }
}

// Wave 0 of a keyframe tile: the tile's poses into LDS, each particle's
// neighbour keyframes (the n_nb smallest FP32 squared translation distances,
// ties to the smaller k) and its loop flag (Sec. III-C.2: an old keyframe
// among the neighbours; the oldest neighbour, else -1).
__device__ __forceinline__ void kf_select(const StepDesc &d, int i, int lane, float (*s_pose)[64],
                                          int (*s_nb)[64], int *s_loop)
{
#pragma clang fp contract(off)
    const int N = d.N, K = d.K, n_nb = d.n_nb;
    const int ic = i < N ? i : N - 1;
    load_tile_pose(d, i, lane, s_pose);
    const float tx = s_pose[0][lane], ty = s_pose[1][lane], tz = s_pose[2][lane];
    float bd[kKfMaxNb];
    int bk[kKfMaxNb];
    for (int s = 0; s < kKfMaxNb; ++s) { bd[s] = INFINITY; bk[s] = K; }
    for (int k = 0; k < K; ++k) {
        const size_t r = (size_t)k * 7 * N + ic;
        const float dd = dist2_rn(tx, ty, tz, d.kf_pose[r], d.kf_pose[r + N], d.kf_pose[r + 2 * N]);
        // Insert (dd, k) into the sorted list; k ascending keeps ties on the smaller k.
        float cd = dd;
        int ck = k;
        for (int s = 0; s < kKfMaxNb; ++s) {
            if (s < n_nb && cd < bd[s]) {
                const float td = bd[s];
                const int tk = bk[s];
                bd[s] = cd; bk[s] = ck;
                cd = td; ck = tk;
            }
        }
    }
    // Every slot below n_nb <= K is filled (distances are finite); guard anyway.
    for (int s = 0; s < kKfMaxNb; ++s) bk[s] = bk[s] < K ? bk[s] : 0;
    if (i < N)
        for (int s = 0; s < n_nb; ++s) d.neighbors[(size_t)s * N + i] = bk[s];
    // The point loops visit a particle's neighbours in keyframe order, so that
    // the lanes of a wave (particles with mostly the same neighbours) read the
    // same keyframe's grid at the same time.
    for (int s = 1; s < kKfMaxNb; ++s) {
        if (s >= n_nb) break;
        const int v = bk[s];
        int t = s;
        while (t > 0 && bk[t - 1] > v) {
            bk[t] = bk[t - 1];
            --t;
        }
        bk[t] = v;
    }
    for (int s = 0; s < kKfMaxNb; ++s) s_nb[s][lane] = bk[s];
    const int o = bk[0];
    s_loop[lane] = (d.kf_loop && o < K - d.n_recent) ? o : -1;
}

// ---------------------------------------------------------------------------
// GICP likelihood with voxel correspondences and Gauss-Newton passes (Eq. 2-7)
// ---------------------------------------------------------------------------

// Upper-triangle index of H[r][c], r <= c, row-major over the 6x6 system.
__host__ __device__ constexpr int htri(int r, int c) { return r * 6 - r * (r - 1) / 2 + (c - r); }

// psi = -H^-1 b by Cholesky in FP64; false when H is not positive definite
// (a pivot at most 1e-12 of the largest diagonal entry).
__device__ __forceinline__ bool gn_solve(const float h[21], const float b[6], float psi[6])
{
    double L[21];
    double dmax = 0.0;
    for (int r = 0; r < 6; ++r) dmax = fmax(dmax, (double)h[htri(r, r)]);
    if (!(dmax > 0.0)) return false;
    // L stored as the transpose of the upper triangle: L[htri(c, r)] = L_rc for r >= c.
    for (int c = 0; c < 6; ++c) {
        double sd = h[htri(c, c)];
        for (int k = 0; k < c; ++k) sd -= L[htri(k, c)] * L[htri(k, c)];
        if (!(sd > 1e-12 * dmax)) return false;
        const double lc = sqrt(sd);
        L[htri(c, c)] = lc;
        const double il = 1.0 / lc;
        for (int r = c + 1; r < 6; ++r) {
            double sv = h[htri(c, r)];
            for (int k = 0; k < c; ++k) sv -= L[htri(k, r)] * L[htri(k, c)];
            L[htri(c, r)] = sv * il;
        }
    }
    double y[6], x[6];
    for (int r = 0; r < 6; ++r) {
        double sv = -(double)b[r];
        for (int k = 0; k < r; ++k) sv -= L[htri(k, r)] * y[k];
        y[r] = sv / L[htri(r, r)];
    }
    for (int r = 5; r >= 0; --r) {
        double sv = y[r];
        for (int k = r + 1; k < 6; ++k) sv -= L[htri(r, k)] * x[k];
        x[r] = sv / L[htri(r, r)];
    }
    for (int r = 0; r < 6; ++r) psi[r] = (float)x[r];
    return true;
}

typedef const __attribute__((address_space(4))) f4v *gscan_ptr;

// One (particle, point, keyframe) term of Eq. 3-6 in the scan's frame:
// x = R' mu + t' (FP64) selects the voxel, taken in voxel units as
// y = (R'/vs) mu + ((t' - o)/vs + 1) and x = y vs + (o - vs); e = mu_v - x; with R'^T the
// rotation back, e_s = R'^T e, Omega_s = (R'^T S_v R' + Sigma)^-1 (FP64
// inverse), w = Omega_s e_s; l -= e_s^T w; b += J_s^T w and
// H += J_s^T Omega_s J_s with J_s = [-I, [mu]x].
typedef const __attribute__((address_space(1))) f4v *gf4_ptr;

// 1/x for a positive normal x: the hardware's reciprocal estimate refined by
// two Newton steps, each of which roughly doubles its correct bits (to about
// one ulp; IEEE division's scaling and fix-up steps are not needed here).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Voxel coordinates of point p in a neighbour's map: y = (x - o)/vs + 1 (FP64),
// truncated to floor + 1 for y >= 0 and to 0 or less (outside, as are NaN and
// the saturated out-of-range results) below; returns the record index, or
// 0xFFFFFFFF outside the map.  The index products take 24-bit multiplies
// (nx and nx * ny below 2^24, voxels below 2^31: checked at load), formed for
// every lane and then selected, so that no branch is taken.
__device__ __forceinline__ uint32_t gicp_voxel(const double Rs[9], const double ts[3], uint32_t nx,
                                               uint32_t ny, uint32_t nz, uint32_t nxy, double px,
                                               double py, double pz, double y[3])
{
    y[0] = fma(Rs[0], px, fma(Rs[1], py, fma(Rs[2], pz, ts[0])));
    y[1] = fma(Rs[3], px, fma(Rs[4], py, fma(Rs[5], pz, ts[1])));
    y[2] = fma(Rs[6], px, fma(Rs[7], py, fma(Rs[8], pz, ts[2])));
    const uint32_t i0 = (uint32_t)cvt_trunc_d(y[0]) - 1u, i1 = (uint32_t)cvt_trunc_d(y[1]) - 1u,
                   i2 = (uint32_t)cvt_trunc_d(y[2]) - 1u;
    const bool in = (i0 < nx) & (i1 < ny) & (i2 < nz);
    const uint32_t rec = i0 + __umul24(nx, i1) + __umul24(nxy, i2);
    return in ? rec : 0xFFFFFFFFu;
}

// Points whose occupancy is probed together.
constexpr int kGicpProbe = 4;

struct GicpFetch {
    f4v va, vb, vc;
    double x0, x1, x2;
};

__device__ __forceinline__ void gicp_point(const GicpFetch &f, const float Rf[9], const f4v p4,
                                           const f4v c4a, const f4v c4b, double &l, float acc[27])
{
    // Called only for a lane whose voxel is occupied (its occupancy byte is
    // set exactly when the record's count is positive).
    const f4v va = f.va, vb = f.vb, vc = f.vc;
    const double x0 = f.x0, x1 = f.x1, x2 = f.x2;
    // Residual in the keyframe frame (FP64 difference, then FP32) and in the scan frame.
    const float e0 = (float)((double)va.x - x0), e1 = (float)((double)va.y - x1),
                e2 = (float)((double)va.z - x2);
    const float es0 = Rf[0] * e0 + Rf[3] * e1 + Rf[6] * e2;
    const float es1 = Rf[1] * e0 + Rf[4] * e1 + Rf[7] * e2;
    const float es2 = Rf[2] * e0 + Rf[5] * e1 + Rf[8] * e2;
    // S_v (xx xy xz yy yz zz) = (vb.x vb.y vb.z vb.w vc.x vc.y); T = S_v R', Ss = R'^T T;
    // C = Ss + Sigma in FP32, then inverted in FP64.
    const float S00 = vb.x, S01 = vb.y, S02 = vb.z, S11 = vb.w, S12 = vc.x, S22 = vc.y;
    float T[9];
    for (int c = 0; c < 3; ++c) {
        T[c] = S00 * Rf[c] + S01 * Rf[3 + c] + S02 * Rf[6 + c];
        T[3 + c] = S01 * Rf[c] + S11 * Rf[3 + c] + S12 * Rf[6 + c];
        T[6 + c] = S02 * Rf[c] + S12 * Rf[3 + c] + S22 * Rf[6 + c];
    }
    const double C00 = (double)(Rf[0] * T[0] + Rf[3] * T[3] + Rf[6] * T[6] + c4a.x);
    const double C01 = (double)(Rf[0] * T[1] + Rf[3] * T[4] + Rf[6] * T[7] + c4a.y);
    const double C02 = (double)(Rf[0] * T[2] + Rf[3] * T[5] + Rf[6] * T[8] + c4a.z);
    const double C11 = (double)(Rf[1] * T[1] + Rf[4] * T[4] + Rf[7] * T[7] + c4a.w);
    const double C12 = (double)(Rf[1] * T[2] + Rf[4] * T[5] + Rf[7] * T[8] + c4b.x);
    const double C22 = (double)(Rf[2] * T[2] + Rf[5] * T[5] + Rf[8] * T[8] + c4b.y);
    // Inverse of the symmetric C by its adjugate.
    const double a00 = C11 * C22 - C12 * C12, a01 = C02 * C12 - C01 * C22, a02 = C01 * C12 - C02 * C11;
    const double det = C00 * a00 + C01 * a01 + C02 * a02;
    if (!(det > 0.0)) return;
    const double id = rcp_nr(det);
    const double O00 = a00 * id, O01 = a01 * id, O02 = a02 * id;
    const double O11 = (C00 * C22 - C02 * C02) * id, O12 = (C01 * C02 - C00 * C12) * id,
                 O22 = (C00 * C11 - C01 * C01) * id;
    const double w0 = O00 * es0 + O01 * es1 + O02 * es2;
    const double w1 = O01 * es0 + O11 * es1 + O12 * es2;
    const double w2 = O02 * es0 + O12 * es1 + O22 * es2;
    l -= (double)es0 * w0 + (double)es1 * w1 + (double)es2 * w2;
    const float px = p4.x, py = p4.y, pz = p4.z;
    const float fw0 = (float)w0, fw1 = (float)w1, fw2 = (float)w2;
    // b = J_s^T w = [-w; -(mu x w)]
    acc[21] -= fw0; acc[22] -= fw1; acc[23] -= fw2;
    acc[24] -= py * fw2 - pz * fw1;
    acc[25] -= pz * fw0 - px * fw2;
    acc[26] -= px * fw1 - py * fw0;
    const float o00 = (float)O00, o01 = (float)O01, o02 = (float)O02, o11 = (float)O11,
                o12 = (float)O12, o22 = (float)O22;
    // H_rho,rho = Omega
    acc[htri(0, 0)] += o00; acc[htri(0, 1)] += o01; acc[htri(0, 2)] += o02;
    acc[htri(1, 1)] += o11; acc[htri(1, 2)] += o12; acc[htri(2, 2)] += o22;
    // OK = Omega [mu]x, rows r: (Om[r][1] pz - Om[r][2] py, Om[r][2] px - Om[r][0] pz, Om[r][0] py - Om[r][1] px)
    const float k00 = o01 * pz - o02 * py, k01 = o02 * px - o00 * pz, k02 = o00 * py - o01 * px;
    const float k10 = o11 * pz - o12 * py, k11 = o12 * px - o01 * pz, k12 = o01 * py - o11 * px;
    const float k20 = o12 * pz - o22 * py, k21 = o22 * px - o02 * pz, k22 = o02 * py - o12 * px;
    // H_rho,phi = -OK
    acc[htri(0, 3)] -= k00; acc[htri(0, 4)] -= k01; acc[htri(0, 5)] -= k02;
    acc[htri(1, 3)] -= k10; acc[htri(1, 4)] -= k11; acc[htri(1, 5)] -= k12;
    acc[htri(2, 3)] -= k20; acc[htri(2, 4)] -= k21; acc[htri(2, 5)] -= k22;
    // H_phi,phi = [mu]x^T OK: row 0 = pz OK[1] - py OK[2], row 1 = px OK[2] - pz OK[0],
    // row 2 = py OK[0] - px OK[1] (upper triangle).
    acc[htri(3, 3)] += pz * k10 - py * k20;
    acc[htri(3, 4)] += pz * k11 - py * k21;
    acc[htri(3, 5)] += pz * k12 - py * k22;
    acc[htri(4, 4)] += px * k21 - pz * k01;
    acc[htri(4, 5)] += px * k22 - pz * k02;
    acc[htri(5, 5)] += py * k02 - px * k12;
}

template <int W>
__device__ __forceinline__ void gicp_tile(const StepDesc &d, int tile)
{
    // The relative poses of a pass (s_rel, written before the point loops) and
    // the per-wave partial sums (s_h, written after them) share one area.
    constexpr size_t kRelBytes = (size_t)kKfMaxNb * 12 * 64 * sizeof(double);
    constexpr size_t kSumBytes = (size_t)27 * W * 64 * sizeof(float);
    __shared__ __attribute__((aligned(16))) unsigned char s_area[kRelBytes > kSumBytes ? kRelBytes : kSumBytes];
    double(*s_rel)[12][64] = reinterpret_cast<double(*)[12][64]>(s_area);   // [neighbour][Rs 9, ts 3][lane]
    float(*s_h)[W][64] = reinterpret_cast<float(*)[W][64]>(s_area);         // H (21) and b (6) per wave
    __shared__ double s_l[W][64];
    __shared__ float s_pose[7][64];
    __shared__ int s_nb[kKfMaxNb][64];
    __shared__ int s_loop[64];
    __shared__ float s_upd[9][64];
    __shared__ float s_seg[W][64];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int N = d.N, n_nb = d.n_nb;
    const int i = slot_particle(d, tile * 64 + lane);
    const int ic = i < N ? i : N - 1;
    const gscan_ptr scan = (gscan_ptr)d.scan_g;           // [3M]: (mu, 0), covariance
    const scan64_ptr scan8 = (scan64_ptr)d.scan8;         // [M] FP64 means
    const double vs = (double)d.h, inv_vs = 1.0 / vs;
    const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz, nxy = nx * ny;
    // Occupancy bytes of all K maps (below 4 GiB, checked at load).
    const __amdgpu_buffer_rsrc_t occ_rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(d.vox_occ), (short)0, (int)(uint32_t)(d.K * d.occ_stride), kRsrcWord3);

    if (wave == 0) kf_select(d, i, lane, s_pose, s_nb, s_loop);
    const int passes = d.iters + d.post_eval;
    __syncthreads();

    for (int pass = 0; pass < passes; ++pass) {
        // Relative pose T_k^-1 T (Eq. 4) of each neighbour in FP64, one
        // neighbour per wave: R' = R_k^T R, t' = R_k^T (t - t_k), kept as
        // R'/vs and (t' - o)/vs + 1 for the voxel index.
        for (int s = wave; s < n_nb; s += W) {
            const float tf[3] = {s_pose[0][lane], s_pose[1][lane], s_pose[2][lane]};
            const float qf[4] = {s_pose[3][lane], s_pose[4][lane], s_pose[5][lane], s_pose[6][lane]};
            double tp[3], qp[4], Rp[9];
            load_pose_d(tf, qf, tp, qp);
            rot_of_quat_d(qp[0], qp[1], qp[2], qp[3], Rp);
            const int k = s_nb[s][lane];
            const size_t r = (size_t)k * 7 * N + ic;
            const float ktf[3] = {d.kf_pose[r], d.kf_pose[r + N], d.kf_pose[r + 2 * N]};
            const float kqf[4] = {d.kf_pose[r + 3 * N], d.kf_pose[r + 4 * N], d.kf_pose[r + 5 * N],
                                  d.kf_pose[r + 6 * N]};
            double kt[3], kq[4], Rk[9];
            load_pose_d(ktf, kqf, kt, kq);
            rot_of_quat_d(kq[0], kq[1], kq[2], kq[3], Rk);
            const double dt[3] = {tp[0] - kt[0], tp[1] - kt[1], tp[2] - kt[2]};
            for (int row = 0; row < 3; ++row) {
                for (int col = 0; col < 3; ++col)
                    s_rel[s][3 * row + col][lane] =
                        (Rk[row] * Rp[col] + Rk[3 + row] * Rp[3 + col] + Rk[6 + row] * Rp[6 + col]) * inv_vs;
                const double o = (double)d.origins[3 * k + row];
                s_rel[s][9 + row][lane] =
                    ((Rk[row] * dt[0] + Rk[3 + row] * dt[1] + Rk[6 + row] * dt[2]) - o) * inv_vs + 1.0;
            }
        }
        __syncthreads();
        double l = 0.0;
        float acc[27];
        for (int c = 0; c < 27; ++c) acc[c] = 0.0f;
        for (int s = 0; s < n_nb; ++s) {
            const int k = s_nb[s][lane];
            double Rs[9], ts[3], ob[3];
            float Rf[9];
            for (int c = 0; c < 9; ++c) {
                Rs[c] = s_rel[s][c][lane];
                Rf[c] = (float)(Rs[c] * vs);
            }
            for (int c = 0; c < 3; ++c) {
                ts[c] = s_rel[s][9 + c][lane];
                ob[c] = (double)d.origins[3 * k + c] - vs;
            }
            const uint64_t vbase = (uint64_t)d.cells + (uint64_t)k * (uint64_t)d.grid_stride;
            // Most (point, neighbour) pairs fall outside the map or in an empty
            // voxel, for every lane at once.  So kGicpProbe points (their FP64
            // means in one 128 B scalar load) have their occupancy bytes
            // requested together, and only a point that some lane finds
            // occupied has its whole record read and its terms formed.
            const gf4_ptr vrec = reinterpret_cast<gf4_ptr>(vbase);
            const uint32_t occ_base = (uint32_t)k * (uint32_t)d.occ_stride;
            const auto point = [&](int j, double px, double py, double pz) {
                double y[3];
                const uint32_t rec = gicp_voxel(Rs, ts, nx, ny, nz, nxy, px, py, pz, y);
                GicpFetch f;
                const gf4_ptr vr = vrec + 4 * (size_t)rec;   // 64 B per record
                f.va = vr[0];
                f.vb = vr[1];
                f.vc = vr[2];
                // The record's three parts are requested together (one round trip).
                asm volatile("" ::"v"(f.va), "v"(f.vb), "v"(f.vc));
                f.x0 = fma(y[0], vs, ob[0]);
                f.x1 = fma(y[1], vs, ob[1]);
                f.x2 = fma(y[2], vs, ob[2]);
                const f4v p4 = {(float)px, (float)py, (float)pz, 0.0f};
                gicp_point(f, Rf, p4, scan[3 * j + 1], scan[3 * j + 2], l, acc);
            };
            // Batches of kGicpProbe points are dealt to the waves in turn (at any
            // time the waves of a tile probe neighbouring points); the last
            // M mod kGicpProbe points go to the last wave.
            const int n_batch = d.M / kGicpProbe;
            for (int bt = wave; bt < n_batch; bt += W) {
                const int jb = bt * kGicpProbe;
                const d16v sq = *(const __attribute__((address_space(4))) d16v *)(scan8 + jb);
                uint32_t occ[kGicpProbe];
#pragma unroll
                for (int b = 0; b < kGicpProbe; ++b) {
                    double y[3];
                    const uint32_t rec =
                        gicp_voxel(Rs, ts, nx, ny, nz, nxy, sq[4 * b], sq[4 * b + 1], sq[4 * b + 2], y);
                    // A lane outside the map reads past the buffer's end,
                    // which returns 0 (empty): no branch, all issued before the first wait.
                    occ[b] = __builtin_amdgcn_raw_buffer_load_b8(
                        occ_rs, rec != 0xFFFFFFFFu ? occ_base + rec : 0xFFFFFFFFu, 0, 0);
                }
#pragma unroll
                for (int b = 0; b < kGicpProbe; ++b) {
                    if (__builtin_amdgcn_ballot_w64(occ[b] != 0u) == 0) continue;
                    if (occ[b] != 0u) point(jb + b, sq[4 * b], sq[4 * b + 1], sq[4 * b + 2]);
                }
            }
            for (int jb = wave == W - 1 ? n_batch * kGicpProbe : d.M; jb < d.M; ++jb) {
                const d4v p = scan8[jb];
                double y[3];
                const uint32_t rec = gicp_voxel(Rs, ts, nx, ny, nz, nxy, p.x, p.y, p.z, y);
                const uint32_t o = __builtin_amdgcn_raw_buffer_load_b8(
                    occ_rs, rec != 0xFFFFFFFFu ? occ_base + rec : 0xFFFFFFFFu, 0, 0);
                if (__builtin_amdgcn_ballot_w64(o != 0u) == 0) continue;
                if (o != 0u) point(jb, p.x, p.y, p.z);
            }
        }
        __syncthreads();   // every wave is done with s_rel before s_h reuses it
        s_l[wave][lane] = l;
        for (int c = 0; c < 27; ++c) s_h[c][wave][lane] = acc[c];
        __syncthreads();
        if (wave == 0) {
            double lt = 0.0;
            float h[27];
            for (int c = 0; c < 27; ++c) h[c] = 0.0f;
            for (int w = 0; w < W; ++w) {
                lt += s_l[w][lane];
                for (int c = 0; c < 27; ++c) h[c] += s_h[c][w][lane];
            }
            const bool stepping = pass < d.iters;
            if (i < N) {
                d.loglik[i] = (float)lt;
                if (stepping) {
                    for (int c = 0; c < 6; ++c) d.grad[(size_t)c * N + i] = h[21 + c];
                    for (int c = 0; c < 21; ++c) d.hess[(size_t)c * N + i] = h[c];
                }
            }
            const bool gate = !d.kf_loop || s_loop[lane] >= 0;
            float psi[6];
            if (stepping && gate && gn_solve(h, h + 21, psi)) {
                float rho[3] = {psi[0], psi[1], psi[2]}, phi[3] = {psi[3], psi[4], psi[5]};
                const float nr = sqrtf(rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2]);
                const float np = sqrtf(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
                if (nr > d.rho_max) {
                    const float f = d.rho_max / nr;
                    rho[0] *= f; rho[1] *= f; rho[2] *= f;
                }
                if (np > d.phi_max) {
                    const float f = d.phi_max / np;
                    phi[0] *= f; phi[1] *= f; phi[2] *= f;
                }
                float t3[3] = {s_pose[0][lane], s_pose[1][lane], s_pose[2][lane]};
                float q4[4] = {s_pose[3][lane], s_pose[4][lane], s_pose[5][lane], s_pose[6][lane]};
                if (pass == 0) normalize_quat(q4[0], q4[1], q4[2], q4[3]);   // the stored quaternion
                for (int c = 0; c < 3; ++c) {
                    s_upd[c][lane] = rho[c];
                    s_upd[3 + c][lane] = phi[c];
                    s_upd[6 + c][lane] = t3[c];
                }
                right_exp(t3, q4, rho, phi);
                s_pose[0][lane] = t3[0]; s_pose[1][lane] = t3[1]; s_pose[2][lane] = t3[2];
                s_pose[3][lane] = q4[0]; s_pose[4][lane] = q4[1]; s_pose[5][lane] = q4[2];
                s_pose[6][lane] = q4[3];
            } else if (d.kf_loop) {
                // No step: nothing to propagate for this particle.
                for (int c = 0; c < 6; ++c) s_upd[c][lane] = 0.0f;
                s_upd[6][lane] = s_pose[0][lane]; s_upd[7][lane] = s_pose[1][lane];
                s_upd[8][lane] = s_pose[2][lane];
            }
        }
        __syncthreads();
        if (d.kf_loop && pass < d.iters) {
            kf_propagate<W>(d, i, lane, wave, s_loop, s_upd, s_seg);
            __syncthreads();
        }
    }
    if (wave == 0) store_tile_pose(d, i, lane, s_pose);
    __syncthreads();
}

// Relative grid map of keyframe k for a particle at (tf, qf): T_k^-1 T (Eq. 4)
// in FP64, R' = R_k^T R, t' = R_k^T (t - t_k), as A' = R'/h and
// b' = (t' - o_k)/h - 1/2 of keyframe k's grid.
__device__ __forceinline__ void kf_grid_map(const StepDesc &d, int k, int ic, const float tf[3],
                                            const float qf[4], double ih, GridMap64 &gm)
{
#pragma clang fp contract(off)
    const int N = d.N;
    double tp[3], qp[4], Rp[9];
    load_pose_d(tf, qf, tp, qp);
    rot_of_quat_d(qp[0], qp[1], qp[2], qp[3], Rp);
    const size_t r = (size_t)k * 7 * N + ic;
    const float ktf[3] = {d.kf_pose[r], d.kf_pose[r + N], d.kf_pose[r + 2 * N]};
    const float kqf[4] = {d.kf_pose[r + 3 * N], d.kf_pose[r + 4 * N], d.kf_pose[r + 5 * N],
                          d.kf_pose[r + 6 * N]};
    double kt[3], kq[4], Rk[9];
    load_pose_d(ktf, kqf, kt, kq);
    rot_of_quat_d(kq[0], kq[1], kq[2], kq[3], Rk);
    const double dt[3] = {tp[0] - kt[0], tp[1] - kt[1], tp[2] - kt[2]};
    for (int row = 0; row < 3; ++row) {
        for (int col = 0; col < 3; ++col)
            gm.A[3 * row + col] =
                (Rk[row] * Rp[col] + Rk[3 + row] * Rp[3 + col] + Rk[6 + row] * Rp[6 + col]) * ih;
        const double tr = Rk[row] * dt[0] + Rk[3 + row] * dt[1] + Rk[6 + row] * dt[2];
        gm.b[row] = (tr - (double)d.origins[3 * k + row]) * ih + 0.5;   // u + 1
    }
}

// Add one neighbour's sums, rotated into the body frame: R'^T A_n / h = A'^T A_n,
// R'^T B_n = h A'^T B_n.
__device__ __forceinline__ void kf_add_neighbour(const GridMap64 &gm, float h, const Acc &acc, double &l,
                                                 float gsum[6])
{
#pragma clang fp contract(off)
    l += acc.l;
    float A[9];
    for (int e = 0; e < 9; ++e) A[e] = (float)gm.A[e];
    gsum[0] += A[0] * acc.ax + A[3] * acc.ay + A[6] * acc.az;
    gsum[1] += A[1] * acc.ax + A[4] * acc.ay + A[7] * acc.az;
    gsum[2] += A[2] * acc.ax + A[5] * acc.ay + A[8] * acc.az;
    gsum[3] += h * (A[0] * acc.bx + A[3] * acc.by + A[6] * acc.bz);
    gsum[4] += h * (A[1] * acc.bx + A[4] * acc.by + A[7] * acc.bz);
    gsum[5] += h * (A[2] * acc.bx + A[5] * acc.by + A[8] * acc.bz);
}

// Keyframe tile with the single-grid point loop.  When all K keyframe grids
// fit one buffer's 32-bit range, each lane adds the byte offset of its
// neighbour's grid to the record offsets, and an outside point still reads
// zeros past the buffer's end; otherwise (GLB) each lane reads its
// neighbour's grid through 64-bit addresses and an outside point reads the
// map's zero record.  Every wave builds the relative grid maps itself (FP64,
// per neighbour), so no map is held in LDS.
template <int DT, bool SKIP, int W, bool GLB>
__device__ __forceinline__ void kf_tile_buf(const StepDesc &d, int tile)
{
#pragma clang fp contract(off)
    __shared__ double s_l[W][64];
    __shared__ float s_g[6][W][64];
    __shared__ float s_pose[7][64];
    __shared__ int s_nb[kKfMaxNb][64];
    __shared__ int s_loop[64];
    __shared__ float s_upd[9][64];
    __shared__ float s_seg[W][64];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int N = d.N, n_nb = d.n_nb;
    const int i = tile * 64 + lane;
    const int ic = i < N ? i : N - 1;
    GridK g;
    grid_layout(d, g);
    g.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(d.cells), (short)0,
                                             GLB ? 0 : (int)((uint32_t)d.grid_stride * (uint32_t)d.K),
                                             kRsrcWord3);
    g.gbase = static_cast<const char *>(d.cells);
    const double ih = 1.0 / (double)d.h;

    if (wave == 0) kf_select(d, i, lane, s_pose, s_nb, s_loop);
    const int M = d.M, Q = sub_chunk_len(M);
    constexpr int S = kSubChunks / W;      // sub-chunks per wave
    const int passes = d.iters + d.post_eval;
    __syncthreads();

    for (int pass = 0; pass < passes; ++pass) {
        double l = 0.0;
        float gsum[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int s = 0; s < n_nb; ++s) {
            // The particle's pose is re-read from LDS per neighbour so that it
            // holds no registers during the point loop.
            const float tf[3] = {s_pose[0][lane], s_pose[1][lane], s_pose[2][lane]};
            const float qf[4] = {s_pose[3][lane], s_pose[4][lane], s_pose[5][lane], s_pose[6][lane]};
            const int k = s_nb[s][lane];
            GridMap64 gm;
            kf_grid_map(d, k, ic, tf, qf, ih, gm);
            gm.base = GLB ? 0u : (uint32_t)k * (uint32_t)d.grid_stride;
            if (GLB) g.gbase = static_cast<const char *>(d.cells) + (uint64_t)k * (uint64_t)d.grid_stride;
            Acc acc = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            for (int sc = 0; sc < S; ++sc) {
                const int c = wave_sub_chunk<W>(wave, sc);
                Acc part = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                eval_range64<DT, false, SKIP, !GLB, GLB>(g, (scan64_ptr)d.scan8, (scan32_ptr)d.scan4, min(M, c * Q),
                                                         min(M, (c + 1) * Q), gm, part);
                add_acc(acc, part);
            }
            kf_add_neighbour(gm, d.h, acc, l, gsum);
        }
        s_l[wave][lane] = l;
        for (int c = 0; c < 6; ++c) s_g[c][wave][lane] = gsum[c];
        __syncthreads();
        if (wave == 0) {
            if (d.kf_loop)
                tile_epilogue<W>(d, i, lane, pass, s_l, s_g, s_pose, s_loop, s_upd);
            else
                tile_epilogue<W>(d, i, lane, pass, s_l, s_g, s_pose);
        }
        __syncthreads();
        if (d.kf_loop && pass < d.iters) {
            kf_propagate<W>(d, i, lane, wave, s_loop, s_upd, s_seg);
            __syncthreads();
        }
    }
    if (wave == 0) store_tile_pose(d, i, lane, s_pose);
    __syncthreads();
}

// Keyframe-map tail tiles (the last, small round of a launch): per tile the
// neighbours in keyframe order and the loop flag, then per (sub-chunk,
// neighbour) the seven sums; the step adds them in kf_tile_buf's order.
struct KfTail {
    int32_t *nb;        // [tile][kKfMaxNb][64]
    int32_t *loop;      // [tile][64]
    double *l;          // [tile][kSubChunks][kKfMaxNb][64]
    float *g;           // [tile][kSubChunks][kKfMaxNb][6][64]
};
__device__ __forceinline__ KfTail kf_tail(const StepDesc &d)
{
    const size_t T = (size_t)d.tail_tiles;
    char *b = reinterpret_cast<char *>(d.tail_l);
    KfTail t;
    t.nb = reinterpret_cast<int32_t *>(b);
    t.loop = t.nb + T * kKfMaxNb * 64;
    t.l = reinterpret_cast<double *>(b + T * (kKfMaxNb + 1) * 64 * 4);
    t.g = reinterpret_cast<float *>(t.l + T * kSubChunks * kKfMaxNb * 64);
    return t;
}

// Neighbours (in keyframe order) and loop flags of the tail tiles, once per step.
__device__ __forceinline__ void kf_tail_select(const StepDesc &d, int tile0, int rel)
{
    __shared__ float s_pose[7][64];
    __shared__ int s_nb[kKfMaxNb][64];
    __shared__ int s_loop[64];
    const int lane = threadIdx.x & 63;
    const int i = (tile0 + rel) * 64 + lane;
    kf_select(d, i, lane, s_pose, s_nb, s_loop);
    const KfTail t = kf_tail(d);
    for (int s = 0; s < kKfMaxNb; ++s) t.nb[((size_t)rel * kKfMaxNb + s) * 64 + lane] = s_nb[s][lane];
    t.loop[(size_t)rel * 64 + lane] = s_loop[lane];
}

// One sub-chunk c of one tail tile for every neighbour (the sums kf_tile_buf forms).
template <int DT, bool SKIP, bool GLB>
__device__ __forceinline__ void kf_tail_chunk(const StepDesc &d, int tile0, int pass, int rel, int c)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int N = d.N, n_nb = d.n_nb;
    const int i = (tile0 + rel) * 64 + lane;
    const int ic = i < N ? i : N - 1;
    GridK g;
    grid_layout(d, g);
    g.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(d.cells), (short)0,
                                             GLB ? 0 : (int)((uint32_t)d.grid_stride * (uint32_t)d.K),
                                             kRsrcWord3);
    g.gbase = static_cast<const char *>(d.cells);
    const double ih = 1.0 / (double)d.h;
    const int M = d.M, Q = sub_chunk_len(M);
    float tf[3], qf[4];
    tail_pose(d, i, pass, tf, qf);
    const KfTail t = kf_tail(d);
    for (int s = 0; s < n_nb; ++s) {
        const int k = t.nb[((size_t)rel * kKfMaxNb + s) * 64 + lane];
        GridMap64 gm;
        kf_grid_map(d, k, ic, tf, qf, ih, gm);
        gm.base = GLB ? 0u : (uint32_t)k * (uint32_t)d.grid_stride;
        if (GLB) g.gbase = static_cast<const char *>(d.cells) + (uint64_t)k * (uint64_t)d.grid_stride;
        Acc part = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        eval_range64<DT, false, SKIP, !GLB, GLB>(g, (scan64_ptr)d.scan8, (scan32_ptr)d.scan4, min(M, c * Q), min(M, (c + 1) * Q),
                                                 gm, part);
        const size_t r = ((size_t)rel * kSubChunks + c) * kKfMaxNb + s;
        t.l[r * 64 + lane] = part.l;
        float *tg = t.g + r * 6 * 64 + lane;
        tg[0] = part.ax; tg[64] = part.ay; tg[128] = part.az;
        tg[192] = part.bx; tg[256] = part.by; tg[320] = part.bz;
    }
}

// Reduce one tail tile's sums in kf_tile_buf's order (wave w: neighbour by
// neighbour, its kSubChunks / W sub-chunks each), the same epilogue and
// keyframe propagation, and the pose back to memory.  W waves per tile.
template <int W>
__device__ __forceinline__ void kf_tail_step(const StepDesc &d, int tile0, int pass, int rel)
{
#pragma clang fp contract(off)
    __shared__ double s_l[W][64];
    __shared__ float s_g[6][W][64];
    __shared__ float s_pose[7][64];
    __shared__ int s_loop[64];
    __shared__ float s_upd[9][64];
    __shared__ float s_seg[W][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int N = d.N, n_nb = d.n_nb;
    const int i = (tile0 + rel) * 64 + lane;
    const int ic = i < N ? i : N - 1;
    const KfTail t = kf_tail(d);
    if (wave == 0) {
        float tf[3], qf[4];
        tail_pose(d, i, pass, tf, qf);
        s_pose[0][lane] = tf[0]; s_pose[1][lane] = tf[1]; s_pose[2][lane] = tf[2];
        s_pose[3][lane] = qf[0]; s_pose[4][lane] = qf[1]; s_pose[5][lane] = qf[2]; s_pose[6][lane] = qf[3];
        s_loop[lane] = t.loop[(size_t)rel * 64 + lane];
    }
    __syncthreads();
    const double ih = 1.0 / (double)d.h;
    constexpr int S = kSubChunks / W;
    double l = 0.0;
    float gsum[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int s = 0; s < n_nb; ++s) {
        const float tf[3] = {s_pose[0][lane], s_pose[1][lane], s_pose[2][lane]};
        const float qf[4] = {s_pose[3][lane], s_pose[4][lane], s_pose[5][lane], s_pose[6][lane]};
        const int k = t.nb[((size_t)rel * kKfMaxNb + s) * 64 + lane];
        GridMap64 gm;
        kf_grid_map(d, k, ic, tf, qf, ih, gm);
        Acc acc = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int sc = 0; sc < S; ++sc) {
            const size_t r = ((size_t)rel * kSubChunks + wave_sub_chunk<W>(wave, sc)) * kKfMaxNb + s;
            const float *tg = t.g + r * 6 * 64 + lane;
            const Acc part = {t.l[r * 64 + lane], tg[0], tg[64], tg[128], tg[192], tg[256], tg[320]};
            add_acc(acc, part);
        }
        kf_add_neighbour(gm, d.h, acc, l, gsum);
    }
    s_l[wave][lane] = l;
    for (int c = 0; c < 6; ++c) s_g[c][wave][lane] = gsum[c];
    __syncthreads();
    if (wave == 0) {
        if (d.kf_loop)
            tile_epilogue<W>(d, i, lane, pass, s_l, s_g, s_pose, s_loop, s_upd);
        else
            tile_epilogue<W>(d, i, lane, pass, s_l, s_g, s_pose);
    }
    __syncthreads();
    if (d.kf_loop && pass < d.iters) {
        kf_propagate<W>(d, i, lane, wave, s_loop, s_upd, s_seg);
        __syncthreads();
    }
    if (wave == 0) store_tile_pose(d, i, lane, s_pose);
}

// ---------------------------------------------------------------------------
// Scan packing, grid records, prediction
// ---------------------------------------------------------------------------

// Packs points [256 b, 256 b + 256) into float4.  A point with a non-finite
// or huge coordinate becomes (1e30, 1e30, 1e30): outside every grid, with
// finite products in the kernels, so it contributes as an outside point.
__device__ __forceinline__ void pack_blk(const StepDesc &d, int b)
{
    const int j = b * kWeightBlock + threadIdx.x;
    if (j >= d.M) return;
    if (d.gicp) {
        // A point with a non-finite mean or covariance is moved far outside
        // every voxel map, so it finds no correspondence.
        const float *c = d.cov6 + 6 * (size_t)j;
        const float x = d.scan3[3 * j], y = d.scan3[3 * j + 1], z = d.scan3[3 * j + 2];
        bool ok = fabsf(x) <= 1e30f && fabsf(y) <= 1e30f && fabsf(z) <= 1e30f;
        for (int e = 0; e < 6; ++e) ok = ok && fabsf(c[e]) <= 1e30f;
        float4 *o = d.scan_g + 3 * (size_t)j;
        o[0] = ok ? make_float4(x, y, z, 0.0f) : make_float4(1e30f, 1e30f, 1e30f, 0.0f);
        o[1] = ok ? make_float4(c[0], c[1], c[2], c[3]) : make_float4(1.0f, 0.0f, 0.0f, 1.0f);
        o[2] = ok ? make_float4(c[4], c[5], 0.0f, 0.0f) : make_float4(0.0f, 1.0f, 0.0f, 0.0f);
        d.scan8[j] = ok ? make_double4(x, y, z, 0.0) : make_double4(1e30, 1e30, 1e30, 0.0);
        return;
    }
    const float x = d.scan3[3 * j], y = d.scan3[3 * j + 1], z = d.scan3[3 * j + 2];
    const bool ok = fabsf(x) <= 1e30f && fabsf(y) <= 1e30f && fabsf(z) <= 1e30f;
    const float4 v = ok ? make_float4(x, y, z, 0.0f) : make_float4(1e30f, 1e30f, 1e30f, 0.0f);
    d.scan4[j] = v;
    d.scan8[j] = make_double4(v.x, v.y, v.z, 0.0);
}

// Counter-based prediction noise: SplitMix64 (Steele, Lea and Flood, 2014)
// outputs by index, turned into normals by Box-Muller.  The stream of frame f
// is keyed by the f-th output of the seed's stream; particle i takes the
// uniforms 6i .. 6i+5 of it.
constexpr uint64_t kSm64Gamma = 0x9e3779b97f4a7c15ull;

__device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double sm64_uniform(uint64_t key, uint64_t j)
{
    return (double)(sm64_mix(key + (j + 1) * kSm64Gamma) >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void noise_normals(uint64_t seed, uint64_t frame, uint64_t i, double z[6])
{
    const uint64_t key = sm64_mix(seed + (frame + 1) * kSm64Gamma);
    for (int m = 0; m < 3; ++m) {
        const double ua = sm64_uniform(key, 6 * i + 2 * m);
        const double ub = sm64_uniform(key, 6 * i + 2 * m + 1);
        const double r = sqrt(-2.0 * log(1.0 - ua));
        double sn, cs;
        sincos(2.0 * M_PI * ub, &sn, &cs);
        z[2 * m] = r * cs;
        z[2 * m + 1] = r * sn;
    }
}

// T_i <- T_i * dT * Exp(delta_i)  (Eq. 1), in FP64, rounded to FP32 once.
__device__ __forceinline__ void predict_blk(const StepDesc &d, int b)
{
    const int i = b * kWeightBlock + threadIdx.x;
    const int N = d.N;
    if (i >= N) return;
    float *pose = d.pose;
    const float tf[3] = {pose[i], pose[N + i], pose[2 * N + i]};
    const float qf[4] = {pose[3 * N + i], pose[4 * N + i], pose[5 * N + i], pose[6 * N + i]};
    double t[3], q[4], R[9];
    load_pose_d(tf, qf, t, q);
    rot_of_quat_d(q[0], q[1], q[2], q[3], R);
    const float *dv = d.dT;
    t[0] += R[0] * dv[0] + R[1] * dv[1] + R[2] * dv[2];
    t[1] += R[3] * dv[0] + R[4] * dv[1] + R[5] * dv[2];
    t[2] += R[6] * dv[0] + R[7] * dv[1] + R[8] * dv[2];
    double bw = dv[3], bx = dv[4], by = dv[5], bz = dv[6];
    const double bn = 1.0 / sqrt(bw * bw + bx * bx + by * by + bz * bz);
    bw *= bn; bx *= bn; by *= bn; bz *= bn;
    double nq[4] = {q[0] * bw - q[1] * bx - q[2] * by - q[3] * bz,
                    q[0] * bx + q[1] * bw + q[2] * bz - q[3] * by,
                    q[0] * by - q[1] * bz + q[2] * bw + q[3] * bx,
                    q[0] * bz + q[1] * by - q[2] * bx + q[3] * bw};
    const double m = (nq[0] < 0.0 ? -1.0 : 1.0) /
                     sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
    for (int a = 0; a < 4; ++a) nq[a] *= m;
    if (d.noise_rng) {
        double z[6];
        noise_normals(d.rng_seed, d.rng_frame, (uint64_t)i, z);
        const double rho[3] = {d.noise_sigma[0] * z[0], d.noise_sigma[1] * z[1], d.noise_sigma[2] * z[2]};
        const double phi[3] = {d.noise_sigma[3] * z[3], d.noise_sigma[4] * z[4], d.noise_sigma[5] * z[5]};
        right_exp_d(t, nq, rho, phi);
    } else if (d.noise) {
        const float *nz = d.noise + 6 * (size_t)i;
        const double rho[3] = {nz[0], nz[1], nz[2]};
        const double phi[3] = {nz[3], nz[4], nz[5]};
        right_exp_d(t, nq, rho, phi);
    }
    float to[3], qo[4];
    store_pose_d(t, nq, to, qo);
    pose[i] = to[0]; pose[N + i] = to[1]; pose[2 * N + i] = to[2];
    pose[3 * N + i] = qo[0]; pose[4 * N + i] = qo[1]; pose[5 * N + i] = qo[2]; pose[6 * N + i] = qo[3];
}

__device__ __forceinline__ uint32_t pack_f16(float lo, float hi)
{
    const unsigned short a = __builtin_bit_cast(unsigned short, (_Float16)lo);
    const unsigned short b = __builtin_bit_cast(unsigned short, (_Float16)hi);
    return (uint32_t)a | ((uint32_t)b << 16);
}

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const unsigned short a = __builtin_bit_cast(unsigned short, (__bf16)lo);
    const unsigned short b = __builtin_bit_cast(unsigned short, (__bf16)hi);
    return (uint32_t)a | ((uint32_t)b << 16);
}

__global__ void k_build_cells(const float *__restrict__ grid, void *__restrict__ cells, int nx,
                              int ny, int nz, int dtype)
{
    const size_t px = (size_t)nx + 1, py = (size_t)ny + 1;
    const size_t n_rec = grid_records(nx, ny, nz);
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rec) return;
    const int I = (int)(r % px);
    const int J = (int)((r / px) % py);
    const int Kz = (int)(r / (px * py));
    if (I == 0 || I == nx || J == 0 || J == ny || Kz == 0 || Kz == nz) {
        // The zero layer: what a point outside the grid reads.
        if (dtype == 0) {
            float4 *o = reinterpret_cast<float4 *>(cells) + 2 * r;
            o[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            o[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        } else {
            reinterpret_cast<uint4 *>(cells)[r] = make_uint4(0u, 0u, 0u, 0u);
        }
        return;
    }
    const int i = I - 1, j = J - 1, k = Kz - 1;
    float c[8];
    for (int s = 0; s < 8; ++s) {
        const int a = s & 1, b = (s >> 1) & 1, cc = s >> 2;
        c[s] = grid[(size_t)(i + a) + (size_t)nx * ((size_t)(j + b) + (size_t)ny * (k + cc))];
    }
    if (dtype == 0) {
        // Coefficients of the cell's trilinear polynomial (slot s = a + 2b + 4c
        // holds corner (a, b, c)), in FP64 and rounded once.
        const double v000 = c[0], v100 = c[1], v010 = c[2], v110 = c[3];
        const double v001 = c[4], v101 = c[5], v011 = c[6], v111 = c[7];
        const double a0 = v000, a1 = v100 - v000, a2 = v010 - v000, a3 = v001 - v000;
        const double a4 = v110 - v100 - v010 + v000;
        const double a5 = v101 - v100 - v001 + v000;
        const double a6 = v011 - v010 - v001 + v000;
        const double a7 = v111 - v110 - v101 - v011 + v100 + v010 + v001 - v000;
        float4 *o = reinterpret_cast<float4 *>(cells) + 2 * r;
        o[0] = make_float4((float)a0, (float)a1, (float)a2, (float)a3);
        o[1] = make_float4((float)a4, (float)a5, (float)a6, (float)a7);
    } else if (dtype == 1) {
        reinterpret_cast<uint4 *>(cells)[r] =
            make_uint4(pack_f16(c[0], c[1]), pack_f16(c[2], c[3]), pack_f16(c[4], c[5]),
                       pack_f16(c[6], c[7]));
    } else {
        reinterpret_cast<uint4 *>(cells)[r] =
            make_uint4(pack_bf16(c[0], c[1]), pack_bf16(c[2], c[3]), pack_bf16(c[4], c[5]),
                       pack_bf16(c[6], c[7]));
    }
}

// ---------------------------------------------------------------------------
// Weights: logw += beta l, log-sum-exp, ESS, representative, resample flag
// ---------------------------------------------------------------------------

// Block sum in a fixed tree order (deterministic for a given block size).
template <int B>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = B / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Block max with the lowest index on ties.
template <int B>
__device__ __forceinline__ void block_argmax(double &v, int &idx, double *shv, int *shi)
{
    const int tid = threadIdx.x;
    shv[tid] = v;
    shi[tid] = idx;
    __syncthreads();
    for (int s = B / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const double o = shv[tid + s];
            const int oi = shi[tid + s];
            if (o > shv[tid] || (o == shv[tid] && oi < shi[tid])) {
                shv[tid] = o;
                shi[tid] = oi;
            }
        }
        __syncthreads();
    }
    v = shv[0];
    idx = shi[0];
    __syncthreads();
}

constexpr int kPolicyAlways = 1, kPolicyEss = 2, kPolicyPrune = 3;

// Per-block partials of the weight update: logw += beta l, then the block's
// max (lowest index on ties), sum of exp(logw - max) and of its square, and
// its largest log-likelihood.
__device__ __forceinline__ void weights_blk(const StepDesc &d, int b)
{
    constexpr int B = kWeightBlock;
    __shared__ double sh[B];
    __shared__ int shi[B];
    const int tid = threadIdx.x;
    const int i = b * B + tid;
    const int N = d.N;
    double lw = -INFINITY, ll = -INFINITY;
    if (i < N) {
        ll = (double)d.loglik[i];
        lw = d.logw[i] + d.beta * ll;
        d.logw[i] = lw;
    }
    double m = lw;
    int am = i < N ? i : INT_MAX;
    block_argmax<B>(m, am, sh, shi);
    const double e = (i < N && m > -INFINITY) ? exp(lw - m) : 0.0;
    const double S = block_sum<B>(e, sh);
    const double Q = block_sum<B>(e * e, sh);
    int li = i;
    block_argmax<B>(ll, li, sh, shi);
    if (tid == 0) {
        double *p = d.part + kPartPerBlock * (size_t)b;
        p[0] = m; p[1] = S; p[2] = Q; p[3] = (double)am; p[4] = ll;
    }
}

// One block per session: combine the per-block partials (fixed order) into
// L = logsumexp(logw), ESS, the representative, max l and the resampling
// decision.
__device__ __forceinline__ void wcombine_blk(const StepDesc &d)
{
    constexpr int B = kWeightBlock;
    __shared__ double sh[B];
    __shared__ int shi[B];
    const int tid = threadIdx.x;
    const int N = d.N;
    const int nb = weight_blocks(N);
    double gm = -INFINITY, lm = -INFINITY;
    int gam = INT_MAX, lmi = 0;
    for (int bk = tid; bk < nb; bk += B) {
        const double *p = d.part + kPartPerBlock * (size_t)bk;
        const double bm = p[0];
        const int bi = (int)p[3];
        if (bm > gm || (bm == gm && bi < gam)) { gm = bm; gam = bi; }
        if (p[4] > lm) lm = p[4];
    }
    block_argmax<B>(gm, gam, sh, shi);
    block_argmax<B>(lm, lmi, sh, shi);
    double s = 0.0, q = 0.0;
    if (gm > -INFINITY) {
        for (int bk = tid; bk < nb; bk += B) {
            const double *p = d.part + kPartPerBlock * (size_t)bk;
            if (p[0] > -INFINITY) {
                const double f = exp(p[0] - gm);
                s += p[1] * f;
                q += p[2] * f * f;
            }
        }
    }
    const double St = block_sum<B>(s, sh);
    const double Qt = block_sum<B>(q, sh);
    if (tid == 0) {
        StepStatsDev *st = d.stats;
        const bool degenerate = !(gm > -INFINITY) || !(St > 0.0) || isnan(St);
        if (degenerate) {
            st->lse = NAN;
            st->ess = (double)N;
            st->resampled = 0;
            st->best = 0;
            st->degenerate = 1;
        } else {
            const double L = gm + log(St);
            const double ess = St * St / Qt;
            st->lse = L;
            st->ess = ess;
            st->resampled = (d.policy == kPolicyAlways) ||
                            (d.policy == kPolicyEss && ess < d.ess_frac * (double)N);
            st->best = gam;
            st->degenerate = 0;
        }
        st->lmax = lm;
        st->prune = 0;
        st->pruned = 0;
        const int bb = degenerate ? 0 : gam;
        for (int c = 0; c < 7; ++c) st->best_pose[c] = d.pose[(size_t)c * N + bb];
    }
}

// ---------------------------------------------------------------------------
// Normalisation, systematic resampling and dead-particle pruning
// ---------------------------------------------------------------------------

// Inclusive scan of one value per thread over the block (Hillis-Steele,
// double-buffered; fixed order).
template <int B>
__device__ __forceinline__ double block_scan(double v, double (*sh)[B])
{
    const int tid = threadIdx.x;
    int cur = 0;
    sh[cur][tid] = v;
    __syncthreads();
    for (int off = 1; off < B; off <<= 1) {
        const double x = sh[cur][tid] + (tid >= off ? sh[cur][tid - off] : 0.0);
        sh[cur ^ 1][tid] = (tid >= off) ? x : sh[cur][tid];
        cur ^= 1;
        __syncthreads();
    }
    v = sh[cur][tid];
    __syncthreads();
    return v;
}

// Dead-particle test of the pruning policy (Sec. III-F) on the normalised
// log-weight: weight below the posterior threshold, or likelihood relative to
// the frame's best below the likelihood threshold.
__device__ __forceinline__ bool is_dead(const StepDesc &d, double lw, float l, double lmax)
{
    return lw < d.ln_prune_post || ((double)l - lmax) < d.ln_prune_lik;
}

// logw -= L (uniform reset when degenerate); when resampling, the block-local
// inclusive scan of w = exp(logw) and the block total.  When pruning, the
// scan runs over the live weights only, and the block's dead count and
// largest live index are kept too.
__device__ __forceinline__ void normscan_blk(const StepDesc &d, int b)
{
    constexpr int B = kWeightBlock;
    __shared__ double sh[2][B];
    __shared__ int shi[B];
    const int tid = threadIdx.x;
    const int i = b * B + tid;
    const int N = d.N;
    const int nb = weight_blocks(N);
    const StepStatsDev *st = d.stats;
    const int degenerate = st->degenerate;
    const int resampled = st->resampled;
    const double L = st->lse;
    double lw = -INFINITY;
    if (i < N) {
        lw = degenerate ? -log((double)N) : d.logw[i] - L;
        d.logw[i] = lw;
    }
    if (d.policy == kPolicyPrune) {
        if (degenerate) return;
        const bool dead = i < N && is_dead(d, lw, d.loglik[i], st->lmax);
        const bool live = i < N && !dead;
        const double v = block_scan<B>(live ? exp(lw) : 0.0, sh);
        if (i < N) {
            d.cdf_local[i] = v;
            d.copies[i] = 0;
        }
        if (tid == B - 1) d.part[b] = v;
        const double nd = block_sum<B>(dead ? 1.0 : 0.0, sh[0]);
        double lv = live ? (double)i : -1.0;
        int dummy = 0;
        block_argmax<B>(lv, dummy, sh[1], shi);
        if (tid == 0) {
            d.part[nb + b] = nd;
            d.part[2 * (size_t)nb + b] = lv;
        }
        return;
    }
    if (!resampled) return;
    const double v = block_scan<B>((i < N) ? exp(lw) : 0.0, sh);
    if (i < N) d.cdf_local[i] = v;
    if (tid == B - 1) d.part[b] = v;
}

// Exclusive prefix of a[0..n) in place by one block; returns the total.
// Thread t owns a contiguous chunk; chunk sums are scanned, then each chunk
// is rewritten sequentially from the previous chunk's inclusive prefix.
template <int B>
__device__ __forceinline__ double block_exclusive_prefix(double *a, int n, double (*sh)[B], double *incl)
{
    const int tid = threadIdx.x;
    const int per = (n + B - 1) / B;
    const int c0 = min(n, tid * per), c1 = min(n, c0 + per);
    double csum = 0.0;
    for (int k = c0; k < c1; ++k) csum += a[k];
    incl[tid] = block_scan<B>(csum, sh);
    __syncthreads();
    double off = tid > 0 ? incl[tid - 1] : 0.0;
    for (int k = c0; k < c1; ++k) {
        const double tot = a[k];
        a[k] = off;
        off += tot;
    }
    const double total = incl[B - 1];
    __syncthreads();
    return total;
}

// One block per session: exclusive prefix of the block totals, in place.
// When pruning, also of the block dead counts, and the decision to prune.
__device__ __forceinline__ void prefix_blk(const StepDesc &d)
{
    constexpr int B = kWeightBlock;
    __shared__ double sh[2][B];
    __shared__ double incl[B];
    __shared__ int shi[B];
    StepStatsDev *st = d.stats;
    const int nb = weight_blocks(d.N);
    if (d.policy == kPolicyPrune) {
        if (st->degenerate) return;
        const double W = block_exclusive_prefix<B>(d.part, nb, sh, incl);
        const double D = block_exclusive_prefix<B>(d.part + nb, nb, sh, incl);
        double lv = -1.0;
        for (int bk = threadIdx.x; bk < nb; bk += B) lv = fmax(lv, d.part[2 * (size_t)nb + bk]);
        int dummy = 0;
        block_argmax<B>(lv, dummy, sh[0], shi);
        if (threadIdx.x == 0) {
            const bool go = D > 0.0 && lv >= 0.0 && W > 0.0;
            st->live_mass = W;
            st->last_live = (int)lv;
            st->prune = go ? 1 : 0;
            st->pruned = go ? (int)D : 0;
        }
        return;
    }
    if (!st->resampled) return;
    block_exclusive_prefix<B>(d.part, nb, sh, incl);
}

// Resampling: a_k = min{i : CDF_i > (u + k)/N} (N - 1 if none) by binary
// search on CDF_i = offset[i / B] + local_i, then gather of the state rows.
// Pruning: dead slot number r (in index order) takes
// a_r = min{i : C_i > (u + r)/D W} over the live CDF, copies the parent's
// pose and keyframe poses, and counts the copy.
__device__ __forceinline__ void search_blk(const StepDesc &d, int b)
{
    constexpr int B = kWeightBlock;
    const int k = b * B + threadIdx.x;
    const int N = d.N;
    const StepStatsDev *st = d.stats;
    if (d.policy == kPolicyPrune) {
        __shared__ double sh[2][B];
        if (!st->prune) {
            if (k < N) d.parents[k] = k;
            return;
        }
        const double lmax = st->lmax;
        const bool dead = k < N && is_dead(d, d.logw[k], d.loglik[k], lmax);
        const double incl = block_scan<B>(dead ? 1.0 : 0.0, sh);
        if (k >= N) return;
        if (!dead) {
            d.parents[k] = k;
            return;
        }
        const int nb = weight_blocks(N);
        const double rank = d.part[nb + b] + incl - 1.0;
        const double target = (d.u + rank) / (double)st->pruned * st->live_mass;
        int lo = 0, hi = N;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const double c = d.part[mid / B] + d.cdf_local[mid];
            if (c > target) hi = mid; else lo = mid + 1;
        }
        // The live CDF is flat over dead entries; a rounding step at a block
        // boundary must not make a dead entry the parent.
        while (lo < N && is_dead(d, d.logw[lo], d.loglik[lo], lmax)) ++lo;
        const int a = lo < N ? lo : st->last_live;
        d.parents[k] = a;
        for (int c = 0; c < 7; ++c) d.pose[(size_t)c * N + k] = d.pose[(size_t)c * N + a];
        for (int r = 0; r < 7 * d.K; ++r) d.kf_pose[(size_t)r * N + k] = d.kf_pose[(size_t)r * N + a];
        __hip_atomic_fetch_add(d.copies + a, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    if (k >= N) return;
    if (!st->resampled) {
        d.parents[k] = k;
        return;
    }
    const double uk = (d.u + (double)k) / (double)N;
    int lo = 0, hi = N;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double c = d.part[mid / B] + d.cdf_local[mid];
        if (c > uk) hi = mid; else lo = mid + 1;
    }
    const int anc = lo < N ? lo : N - 1;
    d.parents[k] = anc;
    for (int c = 0; c < 7; ++c) d.pose_tmp[(size_t)c * N + k] = d.pose[(size_t)c * N + anc];
    for (int r = 0; r < 7 * d.K; ++r) d.kf_pose_tmp[(size_t)r * N + k] = d.kf_pose[(size_t)r * N + anc];
}

// Resampling: copy the gathered rows back, logw = -ln N.  Pruning: a live
// particle shares its weight with its copies and the live mass is
// renormalised, logw_p -= ln(1 + c_p) + ln W.
__device__ __forceinline__ void commit_blk(const StepDesc &d, int b)
{
    const int k = b * kWeightBlock + threadIdx.x;
    const int N = d.N;
    if (k >= N) return;
    if (d.policy == kPolicyPrune) {
        if (d.stats->prune && d.parents[k] == k)
            d.logw[k] = d.logw[k] - log1p((double)d.copies[k]) - log(d.stats->live_mass);
        return;
    }
    if (!d.stats->resampled) return;
    for (int r = 0; r < 7; ++r) d.pose[(size_t)r * N + k] = d.pose_tmp[(size_t)r * N + k];
    for (int r = 0; r < 7 * d.K; ++r) d.kf_pose[(size_t)r * N + k] = d.kf_pose_tmp[(size_t)r * N + k];
    d.logw[k] = -log((double)N);
}

// Pruning: a respawned slot takes its parent's updated log-weight.
__device__ __forceinline__ void fill_blk(const StepDesc &d, int b)
{
    const int k = b * kWeightBlock + threadIdx.x;
    if (k >= d.N || d.policy != kPolicyPrune || !d.stats->prune) return;
    const int a = d.parents[k];
    if (a != k) d.logw[k] = d.logw[a];
}

// ---------------------------------------------------------------------------
// Evaluation order: particles grouped by a coarse cell of their pose
// ---------------------------------------------------------------------------

// Where a particle's transformed points land is set by its translation and
// rotation, so the evaluation takes the particles grouped by a coarse cell of
// six pose coordinates (translation, and the vector part of the quaternion
// taken with w >= 0): each coordinate is cut into 2^kOrderBits equal parts of
// the cloud's range, the parts are ranked along a Morton curve, and cells are
// runs of 2^kOrderDrop consecutive Morton codes.  A wave's
// 64 lanes then hold particles of nearby poses, whose record loads touch
// fewer cache lines.  The order inside a cell is whatever the atomic ranks
// give: every particle's arithmetic, and so its result, is the same in any
// slot.
__device__ __forceinline__ void order_coords(const StepDesc &d, int i, float c[kOrderDims])
{
    const int N = d.N;
    const float w = d.pose[3 * N + i];
    const float sg = w < 0.0f ? -1.0f : 1.0f;
    c[0] = d.pose[i];
    c[1] = d.pose[N + i];
    c[2] = d.pose[2 * N + i];
    c[3] = sg * d.pose[4 * N + i];
    c[4] = sg * d.pose[5 * N + i];
    c[5] = sg * d.pose[6 * N + i];
}

// Blocks of k_order_bounds: at most kOrderBoundBlocks, each taking every
// (blocks x kWeightBlock)-th particle, so that every block of k_order_cell
// reduces a bounded number of partial ranges whatever N is.
constexpr int kOrderBoundBlocks = 256;
__host__ __device__ inline int order_bound_blocks(int N)
{
    const int nb = weight_blocks(N);
    return nb < kOrderBoundBlocks ? nb : kOrderBoundBlocks;
}

// Per block: the low and high ends of each coordinate over its particles
// (non-finite values are left out), written as the block's partial range;
// the blocks also clear the cell counts.
__device__ __forceinline__ void order_bounds_blk(const StepDesc &d, int b)
{
    constexpr int B = kWeightBlock;
    __shared__ float lo[B], hi[B];
    const int tid = threadIdx.x;
    const int stride = order_bound_blocks(d.N) * B;
    float tlo[kOrderDims], thi[kOrderDims];
    for (int k = 0; k < kOrderDims; ++k) { tlo[k] = INFINITY; thi[k] = -INFINITY; }
    for (int i = b * B + tid; i < d.N; i += stride) {
        float c[kOrderDims];
        order_coords(d, i, c);
        for (int k = 0; k < kOrderDims; ++k)
            if (fabsf(c[k]) <= 1e30f) { tlo[k] = fminf(tlo[k], c[k]); thi[k] = fmaxf(thi[k], c[k]); }
    }
    for (int k = 0; k < kOrderDims; ++k) {
        lo[tid] = tlo[k];
        hi[tid] = thi[k];
        __syncthreads();
        for (int st = B / 2; st > 0; st >>= 1) {
            if (tid < st) {
                lo[tid] = fminf(lo[tid], lo[tid + st]);
                hi[tid] = fmaxf(hi[tid], hi[tid + st]);
            }
            __syncthreads();
        }
        if (tid == 0) {
            d.obounds[(size_t)b * 2 * kOrderDims + 2 * k] = lo[0];
            d.obounds[(size_t)b * 2 * kOrderDims + 2 * k + 1] = hi[0];
        }
        __syncthreads();
    }
    for (int k = b * B + tid; k < kOrderCells; k += stride) d.ocount[k] = 0;
}

// Per particle: its cell (over the cloud's range, from all blocks' partial
// ranges) and its rank among the particles of that cell.  The lanes of a
// wave that share a cell take their ranks from one atomic add.
__device__ __forceinline__ void order_cell_blk(const StepDesc &d, int b)
{
    constexpr int B = kWeightBlock;
    __shared__ float lo[kOrderDims][B], hi[kOrderDims][B];
    __shared__ float base[kOrderDims], scale[kOrderDims];
    const int tid = threadIdx.x;
    const int nb = order_bound_blocks(d.N);
    for (int k = 0; k < kOrderDims; ++k) {
        float l = INFINITY, h = -INFINITY;
        for (int q = tid; q < nb; q += B) {
            l = fminf(l, d.obounds[(size_t)q * 2 * kOrderDims + 2 * k]);
            h = fmaxf(h, d.obounds[(size_t)q * 2 * kOrderDims + 2 * k + 1]);
        }
        lo[k][tid] = l;
        hi[k][tid] = h;
    }
    __syncthreads();
    for (int st = B / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int k = 0; k < kOrderDims; ++k) {
                lo[k][tid] = fminf(lo[k][tid], lo[k][tid + st]);
                hi[k][tid] = fmaxf(hi[k][tid], hi[k][tid + st]);
            }
        __syncthreads();
    }
    if (tid < kOrderDims) {
        const float l = lo[tid][0], h = hi[tid][0];
        const float span = h - l;
        base[tid] = l;
        scale[tid] = (span > 0.0f && span <= 1e30f) ? (float)(1 << kOrderBits) / span : 0.0f;
    }
    __syncthreads();
    const int i = b * B + tid;
    const bool valid = i < d.N;
    int cell = -1;
    if (valid) {
        float c[kOrderDims];
        order_coords(d, i, c);
        int q[kOrderDims];
        for (int k = 0; k < kOrderDims; ++k) {
            const float v = (c[k] - base[k]) * scale[k];
            q[k] = (v >= 0.0f) ? min((int)v, (1 << kOrderBits) - 1) : 0;   // NaN and below: part 0
        }
        int code = 0;
        for (int bit = kOrderBits - 1; bit >= 0; --bit)
            for (int k = 0; k < kOrderDims; ++k) code = (code << 1) | ((q[k] >> bit) & 1);
        cell = code >> kOrderDrop;
    }
    // Ranks within the cells: the wave's (cell, lane) keys are sorted across
    // the lanes (bitonic; unused lanes last), each run of equal cells takes its
    // base from one atomic add by its first lane (all runs in one instruction),
    // and every lane of a run adds its place in the run.  The sorted lane
    // writes the cell and rank of the particle its key came from.
    const int lane = __lane_id();
    uint32_t key = valid ? ((uint32_t)cell << 6) | (uint32_t)lane : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t other = (uint32_t)__shfl_xor((int)key, j);
            const bool ascending = (lane & k) == 0, lower = (lane & j) == 0;
            key = (lower == ascending) ? min(key, other) : max(key, other);
        }
    }
    const bool used = key != 0xFFFFFFFFu;
    const uint32_t c = key >> 6;
    const uint32_t c_prev = (uint32_t)__shfl_up((int)c, 1);
    const bool head = used && (lane == 0 || c != c_prev);
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int start = 63 - __clzll((long long)(heads & upto));   // this lane's run starts here
    const uint64_t later = heads & ~upto;                           // heads after this lane
    const int n_used = (int)__popcll(__ballot(used));
    const int next = later ? __ffsll((long long)later) - 1 : n_used;
    int first = 0;
    if (head)
        first = __hip_atomic_fetch_add(d.ocount + c, next - lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    first = __shfl(first, start);
    if (used) {
        const int i_src = b * B + (tid & ~63) + (int)(key & 63u);
        d.ocell[i_src] = (int)c;
        d.orank[i_src] = first + (lane - start);
    }
}

// One block of kOrderPrefixBlock threads: exclusive prefix of the cell
// counts, in place, through LDS (coalesced loads and stores; each thread
// scans a contiguous run of cells, the run totals are scanned across the
// block).
constexpr int kOrderPrefixBlock = 1024;
__device__ __forceinline__ void order_prefix_blk(const StepDesc &d)
{
    constexpr int B = kOrderPrefixBlock;
    constexpr int per = kOrderCells / B;
    constexpr int pad = per + 1;                 // LDS row stride (bank spread)
    __shared__ int cnt[B * pad];
    __shared__ int sh[2][B];
    const int tid = threadIdx.x;
    for (int k = 0; k < per; ++k) {
        const int e = k * B + tid;               // coalesced in global memory
        cnt[(e / per) * pad + e % per] = d.ocount[e];
    }
    __syncthreads();
    int sum = 0;
    for (int k = 0; k < per; ++k) sum += cnt[tid * pad + k];
    int cur = 0;
    sh[cur][tid] = sum;
    __syncthreads();
    for (int off = 1; off < B; off <<= 1) {
        const int x = sh[cur][tid] + (tid >= off ? sh[cur][tid - off] : 0);
        sh[cur ^ 1][tid] = x;
        cur ^= 1;
        __syncthreads();
    }
    int run = sh[cur][tid] - sum;                // exclusive prefix of this thread's cells
    for (int k = 0; k < per; ++k) {
        const int v = cnt[tid * pad + k];
        cnt[tid * pad + k] = run;
        run += v;
    }
    __syncthreads();
    for (int k = 0; k < per; ++k) {
        const int e = k * B + tid;
        d.ocount[e] = cnt[(e / per) * pad + e % per];
    }
}

// Per particle: its slot in the evaluation order.
__device__ __forceinline__ void order_scatter_blk(const StepDesc &d, int b)
{
    const int i = b * kWeightBlock + threadIdx.x;
    if (i >= d.N) return;
    d.order[d.ocount[d.ocell[i]] + d.orank[i]] = i;
}

// ---------------------------------------------------------------------------
// Kernels: one session per launch (grid = that session's blocks)
// ---------------------------------------------------------------------------

// Blocks [0, scan_blocks(M)) pack the scan; the rest (if any) predict.
__global__ __launch_bounds__(kWeightBlock) void k_pack_predict(StepDesc d)
{
    const int ns = scan_blocks(d.M);
    if ((int)blockIdx.x < ns)
        pack_blk(d, blockIdx.x);
    else
        predict_blk(d, blockIdx.x - ns);
}

// The dispatcher hands workgroups to the eight XCDs in turn (workgroup b to
// XCD b % 8), and each XCD has its own L2.  This maps workgroup b of a grid of
// n to a tile so that each XCD works through one contiguous run of tiles:
// particles that are neighbours in the evaluation order (similar poses, so
// overlapping cells) then share an L2 instead of being spread over all eight.
// A bijection on [0, n) for any n; only the cache behaviour depends on the
// dispatch order.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

template <int DT, bool BIG, bool SKIP, int W, bool FLOOR = false>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4))) void k_eval(StepDesc d)
{
    eval_tile<DT, BIG, SKIP, W, FLOOR>(d, xcd_tile(blockIdx.x, gridDim.x));
}

// Eight waves per block, one sub-chunk each: block b covers tail tile
// b / (kSubChunks / 8) and its sub-chunks (b % (kSubChunks / 8)) * 8 + wave.
template <int DT, bool BIG, bool SKIP, bool FLOOR = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_tail(StepDesc d, int tile0,
                                                                                          int pass)
{
    constexpr int G = kSubChunks / 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    tail_chunk<DT, BIG, SKIP, FLOOR>(d, tile0, pass, blockIdx.x / G, (blockIdx.x % G) * 8 + wave);
}

template <int W>
__global__ __launch_bounds__(64) void k_eval_tail_step(StepDesc d, int tile0, int pass)
{
    tail_step<W>(d, tile0, pass, blockIdx.x);
}

// Four waves per SIMD (at most 128 VGPRs; the few spills fall outside the
// point loop) so that all 64-particle tiles of a 50,000-particle session fit
// on the device at once.
template <int DT, bool SKIP, int W, bool GLB>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4))) void k_kf_eval(StepDesc d)
{
    kf_tile_buf<DT, SKIP, W, GLB>(d, xcd_tile(blockIdx.x, gridDim.x));
}

__global__ __launch_bounds__(64) void k_kf_tail_select(StepDesc d, int tile0)
{
    kf_tail_select(d, tile0, blockIdx.x);
}

// Eight waves per block, one sub-chunk each (as k_eval_tail).
template <int DT, bool SKIP, bool GLB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_kf_tail_chunk(StepDesc d, int tile0,
                                                                                              int pass)
{
    constexpr int G = kSubChunks / 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    kf_tail_chunk<DT, SKIP, GLB>(d, tile0, pass, blockIdx.x / G, (blockIdx.x % G) * 8 + wave);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_kf_tail_step(StepDesc d, int tile0, int pass)
{
    kf_tail_step<W>(d, tile0, pass, blockIdx.x);
}

// Four waves per SIMD (128 VGPRs): the spills this costs are cheaper than the
// latency hiding that fewer waves give up.
template <int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4))) void k_gicp_eval(StepDesc d)
{
    gicp_tile<W>(d, xcd_tile(blockIdx.x, gridDim.x));
}

__global__ __launch_bounds__(kWeightBlock) void k_weights(StepDesc d) { weights_blk(d, blockIdx.x); }
__global__ __launch_bounds__(kWeightBlock) void k_wcombine(StepDesc d) { wcombine_blk(d); }
__global__ __launch_bounds__(kWeightBlock) void k_normscan(StepDesc d) { normscan_blk(d, blockIdx.x); }
__global__ __launch_bounds__(kWeightBlock) void k_prefix(StepDesc d) { prefix_blk(d); }
__global__ __launch_bounds__(kWeightBlock) void k_search(StepDesc d) { search_blk(d, blockIdx.x); }
__global__ __launch_bounds__(kWeightBlock) void k_commit(StepDesc d) { commit_blk(d, blockIdx.x); }
__global__ __launch_bounds__(kWeightBlock) void k_fill(StepDesc d) { fill_blk(d, blockIdx.x); }
__global__ __launch_bounds__(kWeightBlock) void k_order_bounds(StepDesc d) { order_bounds_blk(d, blockIdx.x); }
__global__ __launch_bounds__(kWeightBlock) void k_order_cell(StepDesc d) { order_cell_blk(d, blockIdx.x); }
__global__ __launch_bounds__(kOrderPrefixBlock) void k_order_prefix(StepDesc d) { order_prefix_blk(d); }
__global__ __launch_bounds__(kWeightBlock) void k_order_scatter(StepDesc d) { order_scatter_blk(d, blockIdx.x); }

// ---------------------------------------------------------------------------
// Kernels: persistent, batched over many sessions
// ---------------------------------------------------------------------------

// Workgroup g of a persistent grid of G takes the items g, g + G, g + 2G, ...
// of a stage's list: a static assignment, with no shared counter to contend
// on.  The item is uniform across the workgroup.
#define MCS_BATCH_LOOP(KIND, BODY)                                          \
    const int n_items = t.counts[KIND];                                     \
    const int2 *items = t.items + t.offs[KIND];                             \
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {              \
        const int2 v = items[it];                                           \
        int2 w;                                                             \
        w.x = __builtin_amdgcn_readfirstlane(v.x);                          \
        w.y = __builtin_amdgcn_readfirstlane(v.y);                          \
        const StepDesc &d = t.descs[w.x];                                   \
        BODY;                                                               \
        __syncthreads();                                                    \
    }

__global__ __launch_bounds__(kWeightBlock) void kb_pack(BatchTables t) { MCS_BATCH_LOOP(kPack, pack_blk(d, w.y)) }
__global__ __launch_bounds__(kWeightBlock) void kb_predict(BatchTables t) { MCS_BATCH_LOOP(kPredict, predict_blk(d, w.y)) }
__global__ __launch_bounds__(kWeightBlock) void kb_weights(BatchTables t) { MCS_BATCH_LOOP(kWeights, weights_blk(d, w.y)) }
__global__ __launch_bounds__(kWeightBlock) void kb_wcombine(BatchTables t) { MCS_BATCH_LOOP(kWCombine, wcombine_blk(d)) }
__global__ __launch_bounds__(kWeightBlock) void kb_normscan(BatchTables t) { MCS_BATCH_LOOP(kNormScan, normscan_blk(d, w.y)) }
__global__ __launch_bounds__(kWeightBlock) void kb_prefix(BatchTables t) { MCS_BATCH_LOOP(kPrefix, prefix_blk(d)) }
__global__ __launch_bounds__(kWeightBlock) void kb_search(BatchTables t) { MCS_BATCH_LOOP(kSearch, search_blk(d, w.y)) }
__global__ __launch_bounds__(kWeightBlock) void kb_commit(BatchTables t) { MCS_BATCH_LOOP(kCommit, commit_blk(d, w.y)) }
__global__ __launch_bounds__(kWeightBlock) void kb_fill(BatchTables t) { MCS_BATCH_LOOP(kFill, fill_blk(d, w.y)) }

template <int DT, bool SKIP, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4))) void kb_eval(BatchTables t)
{
    MCS_BATCH_LOOP(kEval, (eval_tile<DT, false, SKIP, W>(d, w.y)))
}

// Sessions split whole in a tick (fewer tiles than fill the device): pass
// PASS of every tile as one wave per sub-chunk, then the tile's reduce and
// epilogue, as the per-session tail path does (same sums, same order).
template <int DT, bool SKIP, int PASS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void kb_tail_chunk(BatchTables t)
{
    constexpr int G = kSubChunks / 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    MCS_BATCH_LOOP(kChunk, if (PASS < d.iters + d.post_eval)
                               (tail_chunk<DT, false, SKIP>(d, 0, PASS, w.y / G, (w.y % G) * 8 + wave)))
}

template <int W, int PASS>
__global__ __launch_bounds__(64) void kb_tail_step(BatchTables t)
{
    MCS_BATCH_LOOP(kTStep, if (PASS < d.iters + d.post_eval) (tail_step<W>(d, 0, PASS, w.y)))
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

constexpr int kEvalW = 8;   // waves per workgroup
constexpr int kKfW = 8;
constexpr int kGicpW = 8;

hipError_t launch_build_cells(const float *grid, void *cells, int nx, int ny, int nz, int dtype,
                              hipStream_t st)
{
    const size_t n = grid_records(nx, ny, nz);
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_build_cells, dim3((unsigned)blocks), dim3(256), 0, st, grid, cells, nx,
                       ny, nz, dtype);
    return hipGetLastError();
}

hipError_t launch_pack_predict(const StepDesc &d, hipStream_t st)
{
    const int blocks = scan_blocks(d.M) + (d.predict ? weight_blocks(d.N) : 0);
    hipLaunchKernelGGL(k_pack_predict, dim3(blocks), dim3(kWeightBlock), 0, st, d);
    return hipGetLastError();
}

// A single grid whose record indices need full 32-bit products (rows or slabs
// of 2^24 records and more) or whose records pass one buffer's 32-bit byte
// range: its kernels take BIG (32-bit products, 64-bit record addresses).
static bool wide_grid(int nx, int ny, int nz, int dtype)
{
    const bool slab = (uint64_t)(nx + 1) >= (1u << 24) || (uint64_t)(nx + 1) * (ny + 1) >= (1u << 24);
    return slab || (grid_records(nx, ny, nz) << (dtype == 0 ? 5 : 4)) > (uint64_t)kMaxRecordBytes;
}

bool grid_is_wide(const StepDesc &d) { return d.K == 0 && !d.gicp && wide_grid(d.nx, d.ny, d.nz, d.dtype); }

static bool big_slab(const StepDesc &d) { return wide_grid(d.nx, d.ny, d.nz, d.dtype); }

// A keyframe grid's records must fit a 32-bit byte range (kMaxRecordBytes) and
// take the 24-bit index products; a single grid's record indices must fit 32
// bits.
bool grid_supported(int nx, int ny, int nz, int dtype, bool keyframe)
{
    const uint64_t n_rec = grid_records(nx, ny, nz);
    if (!keyframe) return n_rec <= (uint64_t)0xFFFFFFFFu;
    const bool slab = (uint64_t)(nx + 1) >= (1u << 24) || (uint64_t)(nx + 1) * (ny + 1) >= (1u << 24);
    return (n_rec << (dtype == 0 ? 5 : 4)) <= (uint64_t)kMaxRecordBytes && !slab;
}

// Tiles of the evaluation kernel (single grid, or keyframe map) resident on
// the device at once, and the compute units (cached per device).
static void eval_round(int dtype, bool kf, int &round, int &cus)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::pair<int, int>> cache;
    round = cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    const int key = dtype + (kf ? 3 : 0);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({dev, key});
    if (it != cache.end()) {
        round = it->second.first;
        cus = it->second.second;
        return;
    }
    const void *fn;
    int threads;
    if (kf) {
        fn = dtype == 0   ? reinterpret_cast<const void *>(&k_kf_eval<0, false, kKfW, false>)
             : dtype == 1 ? reinterpret_cast<const void *>(&k_kf_eval<1, false, kKfW, false>)
                          : reinterpret_cast<const void *>(&k_kf_eval<2, false, kKfW, false>);
        threads = 64 * kKfW;
    } else {
        fn = dtype == 0   ? reinterpret_cast<const void *>(&k_eval<0, false, false, kEvalW>)
             : dtype == 1 ? reinterpret_cast<const void *>(&k_eval<1, false, false, kEvalW>)
                          : reinterpret_cast<const void *>(&k_eval<2, false, false, kEvalW>);
        threads = 64 * kEvalW;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        cus = 0;
        return;
    }
    round = per_cu * cus;
    cache[{dev, key}] = {round, cus};
}

int eval_round_tiles(int dtype)
{
    int round = 0, cus = 0;
    eval_round(dtype, false, round, cus);
    return round;
}

// A launch of at least one full round leaves its tiles unevenly spread over
// the compute units when the count is not a multiple of their number: the
// remainder is split when it is at most a quarter of the units.  A single-grid
// session of at most three quarters of one round is split whole (its waves
// then fill the device instead of leaving a quarter of it idle for a whole
// tile's time).
int eval_tail_tiles(int N, int dtype, bool keyframes)
{
    int round = 0, cus = 0;
    eval_round(dtype, keyframes, round, cus);
    if (round <= 0 || cus <= 0) return 0;
    const int tiles = particle_tiles(N);
    if (keyframes && tiles < cus) return 0;
    if (!keyframes && tiles < round) return 4 * tiles <= 3 * round ? tiles : 0;
    const int rem = tiles % cus;
    return rem > 0 && rem <= cus / 4 ? rem : 0;
}

bool eval_supported(const StepDesc &d)
{
    const bool nb_ok = d.n_nb >= 1 && d.n_nb <= kKfMaxNb && d.n_nb <= d.K;
    if (d.gicp) return nb_ok;
    if (d.K > 0) return nb_ok && grid_supported(d.nx, d.ny, d.nz, d.dtype, true);
    return grid_supported(d.nx, d.ny, d.nz, d.dtype, false);
}

template <int DT, bool SKIP, bool FLOOR = false>
static hipError_t launch_eval_dt(const StepDesc &d, hipStream_t st, const TailAux *aux)
{
    const unsigned blocks = (unsigned)particle_tiles(d.N);
    if (d.K > 0) {
        // One buffer can address all keyframe grids when they fit its 32-bit
        // range; larger maps are read through 64-bit addresses.  As for single
        // grids, a small last round of tiles runs as one wave per sub-chunk.
        const bool one_buffer = (uint64_t)d.grid_stride * (uint64_t)d.K <= (uint64_t)kMaxRecordBytes;
        const int tail = d.tail_l ? min(d.tail_tiles, particle_tiles(d.N)) : 0;
        const unsigned main_tiles = blocks - (unsigned)tail;
        const bool fork = tail > 0 && main_tiles > 0 && aux != nullptr;
        const hipStream_t ts = fork ? aux->stream : st;
        if (fork) {
            hipError_t e = hipEventRecord(aux->fork, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(ts, aux->fork, 0);
            if (e != hipSuccess) return e;
        }
        if (tail > 0) {
            const dim3 gb((unsigned)tail * (kSubChunks / 8));
            hipLaunchKernelGGL(k_kf_tail_select, dim3((unsigned)tail), dim3(64), 0, ts, d, (int)main_tiles);
            for (int pass = 0; pass < d.iters + d.post_eval; ++pass) {
                if (one_buffer)
                    hipLaunchKernelGGL((k_kf_tail_chunk<DT, SKIP, false>), gb, dim3(512), 0, ts, d,
                                       (int)main_tiles, pass);
                else
                    hipLaunchKernelGGL((k_kf_tail_chunk<DT, SKIP, true>), gb, dim3(512), 0, ts, d,
                                       (int)main_tiles, pass);
                hipLaunchKernelGGL((k_kf_tail_step<kKfW>), dim3((unsigned)tail), dim3(64 * kKfW), 0, ts, d,
                                   (int)main_tiles, pass);
            }
        }
        if (main_tiles > 0) {
            if (one_buffer)
                hipLaunchKernelGGL((k_kf_eval<DT, SKIP, kKfW, false>), dim3(main_tiles), dim3(64 * kKfW), 0,
                                   st, d);
            else
                hipLaunchKernelGGL((k_kf_eval<DT, SKIP, kKfW, true>), dim3(main_tiles), dim3(64 * kKfW), 0,
                                   st, d);
        }
        if (fork) {
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(aux->join, ts);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, aux->join, 0);
            if (e != hipSuccess) return e;
        }
    } else {
        // Whole rounds of tiles in one launch; a small last round (tail) with
        // one wave per sub-chunk, pass by pass (the same sums and order).
        const int tail = d.tail_l ? min(d.tail_tiles, particle_tiles(d.N)) : 0;
        const unsigned main_tiles = blocks - (unsigned)tail;
        // With a second stream the tail's passes run beside the main launch,
        // whose whole rounds then absorb them.
        const bool fork = tail > 0 && main_tiles > 0 && aux != nullptr;
        const hipStream_t ts = fork ? aux->stream : st;
        if (fork) {
            hipError_t e = hipEventRecord(aux->fork, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(ts, aux->fork, 0);
            if (e != hipSuccess) return e;
        }
        for (int pass = 0; tail > 0 && pass < d.iters + d.post_eval; ++pass) {
            const dim3 gb((unsigned)tail * (kSubChunks / 8));
            if (big_slab(d))
                hipLaunchKernelGGL((k_eval_tail<DT, true, SKIP, FLOOR>), gb, dim3(512), 0, ts, d, (int)main_tiles,
                                   pass);
            else
                hipLaunchKernelGGL((k_eval_tail<DT, false, SKIP, FLOOR>), gb, dim3(512), 0, ts, d, (int)main_tiles,
                                   pass);
            hipLaunchKernelGGL((k_eval_tail_step<kEvalW>), dim3((unsigned)tail), dim3(64), 0, ts, d,
                               (int)main_tiles, pass);
        }
        if (main_tiles > 0) {
            if (big_slab(d))
                hipLaunchKernelGGL((k_eval<DT, true, SKIP, kEvalW, FLOOR>), dim3(main_tiles), dim3(64 * kEvalW),
                                   0, st, d);
            else
                hipLaunchKernelGGL((k_eval<DT, false, SKIP, kEvalW, FLOOR>), dim3(main_tiles), dim3(64 * kEvalW),
                                   0, st, d);
        }
        if (fork) {
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(aux->join, ts);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, aux->join, 0);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

hipError_t launch_eval(const StepDesc &d, hipStream_t st, const TailAux *aux)
{
    if (!eval_supported(d)) return hipErrorInvalidValue;
    if (d.gicp) {
        hipLaunchKernelGGL((k_gicp_eval<kGicpW>), dim3((unsigned)particle_tiles(d.N)),
                           dim3(64 * kGicpW), 0, st, d);
        return hipGetLastError();
    }
    const bool skip = d.oob_skip != 0;
    if (d.floor_only) {
        if (d.K > 0) return hipErrorInvalidValue;
        switch (d.dtype) {
        case 0: return launch_eval_dt<0, false, true>(d, st, aux);
        case 1: return launch_eval_dt<1, false, true>(d, st, aux);
        case 2: return launch_eval_dt<2, false, true>(d, st, aux);
        default: return hipErrorInvalidValue;
        }
    }
    switch (d.dtype) {
    case 0: return skip ? launch_eval_dt<0, true>(d, st, aux) : launch_eval_dt<0, false>(d, st, aux);
    case 1: return skip ? launch_eval_dt<1, true>(d, st, aux) : launch_eval_dt<1, false>(d, st, aux);
    case 2: return skip ? launch_eval_dt<2, true>(d, st, aux) : launch_eval_dt<2, false>(d, st, aux);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_order(const StepDesc &d, hipStream_t st)
{
    if (!d.order) return hipSuccess;
    const dim3 nb((unsigned)weight_blocks(d.N));
    hipLaunchKernelGGL(k_order_bounds, dim3((unsigned)order_bound_blocks(d.N)), dim3(kWeightBlock), 0, st, d);
    hipLaunchKernelGGL(k_order_cell, nb, dim3(kWeightBlock), 0, st, d);
    hipLaunchKernelGGL(k_order_prefix, dim3(1), dim3(kOrderPrefixBlock), 0, st, d);
    hipLaunchKernelGGL(k_order_scatter, nb, dim3(kWeightBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_weights(const StepDesc &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_weights, dim3(weight_blocks(d.N)), dim3(kWeightBlock), 0, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wcombine, dim3(1), dim3(kWeightBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_resample(const StepDesc &d, hipStream_t st)
{
    const unsigned nb = (unsigned)weight_blocks(d.N);
    hipLaunchKernelGGL(k_normscan, dim3(nb), dim3(kWeightBlock), 0, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prefix, dim3(1), dim3(kWeightBlock), 0, st, d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_search, dim3(nb), dim3(kWeightBlock), 0, st, d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_commit, dim3(nb), dim3(kWeightBlock), 0, st, d);
    if ((e = hipGetLastError()) != hipSuccess || d.policy != kPolicyPrune) return e;
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(kWeightBlock), 0, st, d);
    return hipGetLastError();
}

// Persistent grid sizes: enough workgroups to fill 256 CUs several times.
constexpr unsigned kBatchGridSmall = 2048;
constexpr unsigned kBatchGridEval = 1280;
constexpr unsigned kBatchGridOne = 256;     // one-block-per-session stages

template <int DT, bool SKIP>
static hipError_t launch_batch_dt(const BatchTables &t, hipStream_t st)
{
    hipLaunchKernelGGL(kb_pack, dim3(kBatchGridSmall), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL(kb_predict, dim3(kBatchGridSmall), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL((kb_eval<DT, SKIP, kEvalW>), dim3(kBatchGridEval), dim3(64 * kEvalW), 0, st, t);
    static_assert(kBatchSplitPasses == 4, "one chunk and one step launch per split pass");
    hipLaunchKernelGGL((kb_tail_chunk<DT, SKIP, 0>), dim3(kBatchGridEval), dim3(512), 0, st, t);
    hipLaunchKernelGGL((kb_tail_step<kEvalW, 0>), dim3(kBatchGridSmall), dim3(64), 0, st, t);
    hipLaunchKernelGGL((kb_tail_chunk<DT, SKIP, 1>), dim3(kBatchGridEval), dim3(512), 0, st, t);
    hipLaunchKernelGGL((kb_tail_step<kEvalW, 1>), dim3(kBatchGridSmall), dim3(64), 0, st, t);
    hipLaunchKernelGGL((kb_tail_chunk<DT, SKIP, 2>), dim3(kBatchGridEval), dim3(512), 0, st, t);
    hipLaunchKernelGGL((kb_tail_step<kEvalW, 2>), dim3(kBatchGridSmall), dim3(64), 0, st, t);
    hipLaunchKernelGGL((kb_tail_chunk<DT, SKIP, 3>), dim3(kBatchGridEval), dim3(512), 0, st, t);
    hipLaunchKernelGGL((kb_tail_step<kEvalW, 3>), dim3(kBatchGridSmall), dim3(64), 0, st, t);
    hipLaunchKernelGGL(kb_weights, dim3(kBatchGridSmall), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL(kb_wcombine, dim3(kBatchGridOne), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL(kb_normscan, dim3(kBatchGridSmall), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL(kb_prefix, dim3(kBatchGridOne), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL(kb_search, dim3(kBatchGridSmall), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL(kb_commit, dim3(kBatchGridSmall), dim3(kWeightBlock), 0, st, t);
    hipLaunchKernelGGL(kb_fill, dim3(kBatchGridSmall), dim3(kWeightBlock), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchTables &t, int dtype, int skip, hipStream_t st)
{
    switch (dtype * 2 + (skip ? 1 : 0)) {
    case 0: return launch_batch_dt<0, false>(t, st);
    case 1: return launch_batch_dt<0, true>(t, st);
    case 2: return launch_batch_dt<1, false>(t, st);
    case 3: return launch_batch_dt<1, true>(t, st);
    case 4: return launch_batch_dt<2, false>(t, st);
    case 5: return launch_batch_dt<2, true>(t, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Static device area of the allocation-free step (mcs_filter_step_noalloc)
// ---------------------------------------------------------------------------

// One per GPU the library runs on, held until the process ends.  In host code
// the array's name is not a device address: its address on a device comes
// from hipGetSymbolAddress with that device current (scratch_init).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t scratch_init(int device, void **ptr)
{
    static std::mutex mu;
    static std::map<int, void *> by_device;
    std::lock_guard<std::mutex> lk(mu);
    auto it = by_device.find(device);
    if (it != by_device.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    by_device[device] = p;
    *ptr = p;
    return hipSuccess;
}

}  // namespace mcs
