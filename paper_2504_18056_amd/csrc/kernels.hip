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

namespace mcs {
namespace {

constexpr double kLn2 = 0.693147180559945309417232121458176568;

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Rotation matrix (row-major) of a unit quaternion (w, x, y, z).
__device__ __forceinline__ void rot_of_quat(float w, float x, float y, float z, float R[9])
{
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

__device__ __forceinline__ float half_lo(uint32_t v)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu));
}
__device__ __forceinline__ float half_hi(uint32_t v)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
}

template <int DT> __device__ __forceinline__ void decode(const Cell<DT> &c, float v[8]);
template <> __device__ __forceinline__ void decode<0>(const Cell<0> &c, float v[8])
{
    v[0] = c.a.x; v[1] = c.a.y; v[2] = c.a.z; v[3] = c.a.w;
    v[4] = c.b.x; v[5] = c.b.y; v[6] = c.b.z; v[7] = c.b.w;
}
template <> __device__ __forceinline__ void decode<1>(const Cell<1> &c, float v[8])
{
    v[0] = half_lo(c.a.x); v[1] = half_hi(c.a.x); v[2] = half_lo(c.a.y); v[3] = half_hi(c.a.y);
    v[4] = half_lo(c.a.z); v[5] = half_hi(c.a.z); v[6] = half_lo(c.a.w); v[7] = half_hi(c.a.w);
}
template <> __device__ __forceinline__ void decode<2>(const Cell<2> &c, float v[8])
{
    v[0] = __uint_as_float(c.a.x << 16); v[1] = __uint_as_float(c.a.x & 0xffff0000u);
    v[2] = __uint_as_float(c.a.y << 16); v[3] = __uint_as_float(c.a.y & 0xffff0000u);
    v[4] = __uint_as_float(c.a.z << 16); v[5] = __uint_as_float(c.a.z & 0xffff0000u);
    v[6] = __uint_as_float(c.a.w << 16); v[7] = __uint_as_float(c.a.w & 0xffff0000u);
}

// Running sums of one particle over its share of the scan.
struct Acc {
    double l;              // sum of log2(G + eps) (times the skip mask)
    float ax, ay, az;      // sum of dG/du / (G + eps)
    float bx, by, bz;      // sum of v' x (dG/du / (G + eps)), v' = A p
};

// Grid constants of one evaluation loop.
struct GridK {
    __amdgpu_buffer_rsrc_t rs;
    float nxm, nym, nzm;   // n - 1 per axis: the valid index range is [0, n - 1)
    uint32_t cx, cxy;      // record strides: cells per row and per slab
    float eps;
    float skip;            // 1: outside points contribute nothing; 0: ln(eps)
};

// Transformed point, cell fractions, inside mask and record offset.
struct Pt {
    float vx, vy, vz;      // v' = A p (grid units)
    float fx, fy, fz;
    float m;               // 1 inside, 0 outside
    uint32_t off;          // byte offset of the cell record
};

template <int DT, bool BIG>
__device__ __forceinline__ Pt prep_point(const GridK &g, const float A[9], const float b[3],
                                         float px, float py, float pz)
{
    Pt p;
    p.vx = fmaf(A[0], px, fmaf(A[1], py, A[2] * pz));
    p.vy = fmaf(A[3], px, fmaf(A[4], py, A[5] * pz));
    p.vz = fmaf(A[6], px, fmaf(A[7], py, A[8] * pz));
    const float ux = p.vx + b[0], uy = p.vy + b[1], uz = p.vz + b[2];
    const bool inside = (ux >= 0.0f) & (ux < g.nxm) & (uy >= 0.0f) & (uy < g.nym) &
                        (uz >= 0.0f) & (uz < g.nzm);
    p.m = inside ? 1.0f : 0.0f;
    // Outside points read cell 0 and are masked.
    const float sx = inside ? ux : 0.0f, sy = inside ? uy : 0.0f, sz = inside ? uz : 0.0f;
    const float flx = floorf(sx), fly = floorf(sy), flz = floorf(sz);
    p.fx = sx - flx; p.fy = sy - fly; p.fz = sz - flz;
    const uint32_t ix = (uint32_t)flx, iy = (uint32_t)fly, iz = (uint32_t)flz;
    const uint32_t rec = BIG ? ix + g.cx * iy + g.cxy * iz
                             : ix + __umul24(g.cx, iy) + __umul24(g.cxy, iz);
    p.off = rec << record_shift<DT>();
    return p;
}

template <int DT>
__device__ __forceinline__ void accumulate(const GridK &g, const Pt &p, const Cell<DT> &cell,
                                           Acc &acc)
{
    float c[8];
    decode<DT>(cell, c);
    const float fx = p.fx, fy = p.fy, fz = p.fz;
    // Along x on the four y/z edges.
    const float d00 = c[1] - c[0], d10 = c[3] - c[2], d01 = c[5] - c[4], d11 = c[7] - c[6];
    const float e00 = fmaf(fx, d00, c[0]), e10 = fmaf(fx, d10, c[2]);
    const float e01 = fmaf(fx, d01, c[4]), e11 = fmaf(fx, d11, c[6]);
    // Along y.
    const float gy0 = e10 - e00, gy1 = e11 - e01;
    const float f0 = fmaf(fy, gy0, e00), f1 = fmaf(fy, gy1, e01);
    // Along z.
    const float gz = f1 - f0;
    const float G = fmaf(fz, gz, f0) * p.m;
    const float dGy = fmaf(fz, gy1 - gy0, gy0);
    const float dx0 = fmaf(fy, d10 - d00, d00), dx1 = fmaf(fy, d11 - d01, d01);
    const float dGx = fmaf(fz, dx1 - dx0, dx0);
    const float den = G + g.eps;
    // Outside: G = 0 gives log2(eps); with skipping the term is scaled to 0.
    const float keep = fmaf(g.skip, p.m - 1.0f, 1.0f);
    acc.l += (double)(fast_log2(den) * keep);
    const float r = fast_rcp(den) * p.m;
    const float dx = dGx * r, dy = dGy * r, dz = gz * r;
    acc.ax += dx; acc.ay += dy; acc.az += dz;
    acc.bx = fmaf(p.vy, dz, fmaf(-p.vz, dy, acc.bx));
    acc.by = fmaf(p.vz, dx, fmaf(-p.vx, dz, acc.by));
    acc.bz = fmaf(p.vx, dy, fmaf(-p.vy, dx, acc.bz));
}

// Points [j0, j1) of the scan against one pose, U points per batch: the U
// record loads are issued before any of their arithmetic.
template <int DT, bool BIG, int U>
__device__ __forceinline__ void eval_range(const GridK &g, scan_ptr scan, int j0, int j1,
                                           const float A[9], const float b[3], Acc &acc)
{
    int j = j0;
    for (; j + U <= j1; j += U) {
        Pt p[U];
        Cell<DT> c[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const f4v s = scan[j + k];
            p[k] = prep_point<DT, BIG>(g, A, b, s.x, s.y, s.z);
            load_cell<DT>(g.rs, p[k].off, c[k]);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) accumulate<DT>(g, p[k], c[k], acc);
    }
    for (; j < j1; ++j) {
        const f4v s = scan[j];
        const Pt p = prep_point<DT, BIG>(g, A, b, s.x, s.y, s.z);
        Cell<DT> c;
        load_cell<DT>(g.rs, p.off, c);
        accumulate<DT>(g, p, c, acc);
    }
}

// ---------------------------------------------------------------------------
// Likelihood + gradient + pose step, single grid
// ---------------------------------------------------------------------------

template <int DT, bool BIG, int W, int U>
__global__ __launch_bounds__(64 * W) void k_eval_step(EvalArgs a)
{
    __shared__ double s_l[W][64];
    __shared__ float s_g[6][W][64];
    __shared__ float s_pose[7][64];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int N = a.N;
    const int i = blockIdx.x * 64 + lane;
    const int ic = i < N ? i : N - 1;

    float t[3] = {a.pose[ic], a.pose[N + ic], a.pose[2 * N + ic]};
    float q[4] = {a.pose[3 * N + ic], a.pose[4 * N + ic], a.pose[5 * N + ic], a.pose[6 * N + ic]};

    GridK g;
    const uint32_t n_rec = (uint32_t)(a.grid.nx - 1) * (uint32_t)(a.grid.ny - 1) *
                           (uint32_t)(a.grid.nz - 1);
    g.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(a.grid.cells), (short)0,
                                             (int)(n_rec << record_shift<DT>()), kRsrcWord3);
    g.nxm = (float)(a.grid.nx - 1);
    g.nym = (float)(a.grid.ny - 1);
    g.nzm = (float)(a.grid.nz - 1);
    g.cx = (uint32_t)(a.grid.nx - 1);
    g.cxy = (uint32_t)(a.grid.nx - 1) * (uint32_t)(a.grid.ny - 1);
    g.eps = a.eps;
    g.skip = a.oob_skip ? 1.0f : 0.0f;
    const float inv_h = a.grid.inv_h;
    const scan_ptr scan = (scan_ptr)a.scan;

    const int M = a.M;
    const int chunk = (M + W - 1) / W;
    const int j0 = min(M, wave * chunk);
    const int j1 = min(M, j0 + chunk);
    const int passes = a.iters + a.post_eval;

    for (int pass = 0; pass < passes; ++pass) {
        normalize_quat(q[0], q[1], q[2], q[3]);
        float A[9], b[3];
        {
            float R[9];
            rot_of_quat(q[0], q[1], q[2], q[3], R);
            for (int e = 0; e < 9; ++e) A[e] = R[e] * inv_h;
        }
        b[0] = fmaf(t[0] - a.grid.ox, inv_h, -0.5f);
        b[1] = fmaf(t[1] - a.grid.oy, inv_h, -0.5f);
        b[2] = fmaf(t[2] - a.grid.oz, inv_h, -0.5f);

        Acc acc = {0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        eval_range<DT, BIG, U>(g, scan, j0, j1, A, b, acc);

        s_l[wave][lane] = acc.l;
        s_g[0][wave][lane] = acc.ax; s_g[1][wave][lane] = acc.ay; s_g[2][wave][lane] = acc.az;
        s_g[3][wave][lane] = acc.bx; s_g[4][wave][lane] = acc.by; s_g[5][wave][lane] = acc.bz;
        __syncthreads();
        if (wave == 0) {
            double l = 0.0;
            float s[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            for (int w = 0; w < W; ++w) {
                l += s_l[w][lane];
                for (int c = 0; c < 6; ++c) s[c] += s_g[c][w][lane];
            }
            // World gradient of l wrt the point is (sum d') / h; the body-frame
            // gradient is g_rho = R^T (sum d') / h, g_phi = R^T sum (v' x d').
            float R[9];
            rot_of_quat(q[0], q[1], q[2], q[3], R);
            const float ax = s[0] * inv_h, ay = s[1] * inv_h, az = s[2] * inv_h;
            float gr[6];
            gr[0] = R[0] * ax + R[3] * ay + R[6] * az;
            gr[1] = R[1] * ax + R[4] * ay + R[7] * az;
            gr[2] = R[2] * ax + R[5] * ay + R[8] * az;
            gr[3] = R[0] * s[3] + R[3] * s[4] + R[6] * s[5];
            gr[4] = R[1] * s[3] + R[4] * s[4] + R[7] * s[5];
            gr[5] = R[2] * s[3] + R[5] * s[4] + R[8] * s[5];
            const bool stepping = pass < a.iters;
            if (i < N) {
                a.loglik[i] = (float)(l * kLn2);
                if (stepping)
                    for (int c = 0; c < 6; ++c) a.grad[c * N + i] = gr[c];
            }
            if (stepping) {
                float rho[3] = {a.alpha_t * gr[0], a.alpha_t * gr[1], a.alpha_t * gr[2]};
                float phi[3] = {a.alpha_r * gr[3], a.alpha_r * gr[4], a.alpha_r * gr[5]};
                const float nr = sqrtf(rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2]);
                const float np = sqrtf(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
                if (nr > a.rho_max) {
                    const float k = a.rho_max / nr;
                    rho[0] *= k; rho[1] *= k; rho[2] *= k;
                }
                if (np > a.phi_max) {
                    const float k = a.phi_max / np;
                    phi[0] *= k; phi[1] *= k; phi[2] *= k;
                }
                right_exp(t, q, rho, phi);
            }
            s_pose[0][lane] = t[0]; s_pose[1][lane] = t[1]; s_pose[2][lane] = t[2];
            s_pose[3][lane] = q[0]; s_pose[4][lane] = q[1]; s_pose[5][lane] = q[2];
            s_pose[6][lane] = q[3];
        }
        __syncthreads();
        t[0] = s_pose[0][lane]; t[1] = s_pose[1][lane]; t[2] = s_pose[2][lane];
        q[0] = s_pose[3][lane]; q[1] = s_pose[4][lane]; q[2] = s_pose[5][lane];
        q[3] = s_pose[6][lane];
    }
    if (wave == 0 && i < N) {
        normalize_quat(q[0], q[1], q[2], q[3]);
        a.pose[i] = t[0]; a.pose[N + i] = t[1]; a.pose[2 * N + i] = t[2];
        a.pose[3 * N + i] = q[0]; a.pose[4 * N + i] = q[1]; a.pose[5 * N + i] = q[2];
        a.pose[6 * N + i] = q[3];
    }
}

// ---------------------------------------------------------------------------
// Small kernels: scan packing, grid records, prediction
// ---------------------------------------------------------------------------

// Packs M x 3 points into float4.  A point with a non-finite or huge
// coordinate becomes (1e30, 1e30, 1e30): outside every grid, with finite
// products in the kernels, so it contributes exactly like an outside point.
__global__ void k_pack_scan(const float *__restrict__ s3, float4 *__restrict__ s4, int M)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const float x = s3[3 * j], y = s3[3 * j + 1], z = s3[3 * j + 2];
    const bool ok = fabsf(x) <= 1e30f && fabsf(y) <= 1e30f && fabsf(z) <= 1e30f;
    s4[j] = ok ? make_float4(x, y, z, 0.0f) : make_float4(1e30f, 1e30f, 1e30f, 0.0f);
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
    const int cxn = nx - 1, cyn = ny - 1, czn = nz - 1;
    const size_t n_cells = (size_t)cxn * cyn * czn;
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_cells) return;
    const int i = (int)(r % cxn);
    const int j = (int)((r / cxn) % cyn);
    const int k = (int)(r / ((size_t)cxn * cyn));
    float c[8];
    for (int s = 0; s < 8; ++s) {
        const int a = s & 1, b = (s >> 1) & 1, cc = s >> 2;
        c[s] = grid[(size_t)(i + a) + (size_t)nx * ((size_t)(j + b) + (size_t)ny * (k + cc))];
    }
    if (dtype == 0) {
        float4 *o = reinterpret_cast<float4 *>(cells) + 2 * r;
        o[0] = make_float4(c[0], c[1], c[2], c[3]);
        o[1] = make_float4(c[4], c[5], c[6], c[7]);
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

struct Pose7 { float v[7]; };

// T_i <- T_i * dT * Exp(delta_i)  (Eq. 1).
__global__ void k_predict(float *__restrict__ pose, int N, Pose7 dT,
                          const float *__restrict__ noise)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float t[3] = {pose[i], pose[N + i], pose[2 * N + i]};
    float q[4] = {pose[3 * N + i], pose[4 * N + i], pose[5 * N + i], pose[6 * N + i]};
    normalize_quat(q[0], q[1], q[2], q[3]);
    float R[9];
    rot_of_quat(q[0], q[1], q[2], q[3], R);
    const float *d = dT.v;
    t[0] += R[0] * d[0] + R[1] * d[1] + R[2] * d[2];
    t[1] += R[3] * d[0] + R[4] * d[1] + R[5] * d[2];
    t[2] += R[6] * d[0] + R[7] * d[1] + R[8] * d[2];
    float bw = d[3], bx = d[4], by = d[5], bz = d[6];
    normalize_quat(bw, bx, by, bz);
    float nw = q[0] * bw - q[1] * bx - q[2] * by - q[3] * bz;
    float nx = q[0] * bx + q[1] * bw + q[2] * bz - q[3] * by;
    float ny = q[0] * by - q[1] * bz + q[2] * bw + q[3] * bx;
    float nz = q[0] * bz + q[1] * by - q[2] * bx + q[3] * bw;
    normalize_quat(nw, nx, ny, nz);
    q[0] = nw; q[1] = nx; q[2] = ny; q[3] = nz;
    if (noise) {
        const float rho[3] = {noise[6 * (size_t)i], noise[6 * (size_t)i + 1], noise[6 * (size_t)i + 2]};
        const float phi[3] = {noise[6 * (size_t)i + 3], noise[6 * (size_t)i + 4], noise[6 * (size_t)i + 5]};
        right_exp(t, q, rho, phi);
    }
    pose[i] = t[0]; pose[N + i] = t[1]; pose[2 * N + i] = t[2];
    pose[3 * N + i] = q[0]; pose[4 * N + i] = q[1]; pose[5 * N + i] = q[2]; pose[6 * N + i] = q[3];
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

__device__ __forceinline__ bool arrive_last(unsigned int *counter)
{
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        s_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    const bool last = s_last != 0;
    if (last) __threadfence();
    return last;
}

__global__ __launch_bounds__(kWeightBlock) void k_weights(WeightArgs a)
{
    constexpr int B = kWeightBlock;
    __shared__ double sh[B];
    __shared__ int shi[B];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * B + tid;
    const int N = a.N;
    double lw = -INFINITY;
    if (i < N) {
        lw = a.logw[i] + a.beta * (double)a.loglik[i];
        a.logw[i] = lw;
    }
    double m = lw;
    int am = i < N ? i : INT_MAX;
    block_argmax<B>(m, am, sh, shi);
    const double e = (i < N && m > -INFINITY) ? exp(lw - m) : 0.0;
    const double S = block_sum<B>(e, sh);
    const double Q = block_sum<B>(e * e, sh);
    if (tid == 0) {
        double *p = a.part + 4 * (size_t)blockIdx.x;
        p[0] = m; p[1] = S; p[2] = Q; p[3] = (double)am;
    }
    if (!arrive_last(a.counter)) return;

    // Last block: combine the per-block (max, sums) in block order.
    const int nb = gridDim.x;
    double gm = -INFINITY;
    int gam = INT_MAX;
    for (int bk = tid; bk < nb; bk += B) {
        const double bm = a.part[4 * (size_t)bk];
        const int bi = (int)a.part[4 * (size_t)bk + 3];
        if (bm > gm || (bm == gm && bi < gam)) { gm = bm; gam = bi; }
    }
    block_argmax<B>(gm, gam, sh, shi);
    double s = 0.0, q = 0.0;
    if (gm > -INFINITY) {
        for (int bk = tid; bk < nb; bk += B) {
            const double bm = a.part[4 * (size_t)bk];
            if (bm > -INFINITY) {
                const double f = exp(bm - gm);
                s += a.part[4 * (size_t)bk + 1] * f;
                q += a.part[4 * (size_t)bk + 2] * f * f;
            }
        }
    }
    const double St = block_sum<B>(s, sh);
    const double Qt = block_sum<B>(q, sh);
    if (tid == 0) {
        StepStatsDev *st = a.stats;
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
            st->resampled = (a.policy == 1) || (a.policy == 2 && ess < a.ess_frac * (double)N);
            st->best = gam;
            st->degenerate = 0;
        }
        const int b = degenerate ? 0 : gam;
        for (int c = 0; c < 7; ++c) st->best_pose[c] = a.pose[(size_t)c * N + b];
        __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Normalisation and systematic resampling
// ---------------------------------------------------------------------------

// logw -= L (uniform reset when degenerate); when resampling, the block-local
// inclusive scan of w = exp(logw) and, in the last block, the exclusive
// prefix of the block totals.
__global__ __launch_bounds__(kWeightBlock) void k_normalize_scan(ResampleArgs a)
{
    constexpr int B = kWeightBlock;
    __shared__ double sh[2][B];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * B + tid;
    const int N = a.N;
    const StepStatsDev *st = a.stats;
    const int degenerate = st->degenerate;
    const int resampled = st->resampled;
    const double L = st->lse;
    double lw = -INFINITY;
    if (i < N) {
        lw = degenerate ? -log((double)N) : a.logw[i] - L;
        a.logw[i] = lw;
    }
    if (!resampled) return;
    double v = (i < N) ? exp(lw) : 0.0;
    // Inclusive scan (Hillis-Steele, double-buffered; fixed order).
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
    if (i < N) a.cdf_local[i] = v;
    if (tid == B - 1) a.part[blockIdx.x] = v;
    if (!arrive_last(a.counter)) return;
    if (tid == 0) {
        double off = 0.0;
        for (int bk = 0; bk < (int)gridDim.x; ++bk) {
            const double tot = a.part[bk];
            a.part[bk] = off;
            off += tot;
        }
        __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// a_k = min{i : CDF_i > (u + k)/N} (N - 1 if none) by binary search on
// CDF_i = offset[i / B] + local_i, then gather of the pose rows.
__global__ void k_search_gather(ResampleArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = a.N;
    if (k >= N) return;
    if (!a.stats->resampled) {
        a.parents[k] = k;
        return;
    }
    const double uk = (a.u + (double)k) / (double)N;
    int lo = 0, hi = N;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double c = a.part[mid / kWeightBlock] + a.cdf_local[mid];
        if (c > uk) hi = mid; else lo = mid + 1;
    }
    const int anc = lo < N ? lo : N - 1;
    a.parents[k] = anc;
    for (int c = 0; c < 7; ++c) a.pose_tmp[(size_t)c * N + k] = a.pose[(size_t)c * N + anc];
}

// Keyframe poses of the ancestors: rows r of [K*7][N].
__global__ void k_gather_rows(ResampleArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const int N = a.N;
    if (k >= N || !a.stats->resampled) return;
    const int anc = a.parents[k];
    a.kf_pose_tmp[(size_t)r * N + k] = a.kf_pose[(size_t)r * N + anc];
}

__global__ void k_commit(ResampleArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;              // 0..6 pose rows, then keyframe rows
    const int N = a.N;
    if (k >= N || !a.stats->resampled) return;
    if (r < 7) {
        a.pose[(size_t)r * N + k] = a.pose_tmp[(size_t)r * N + k];
        if (r == 0) a.logw[k] = -log((double)N);
    } else {
        const size_t o = (size_t)(r - 7) * N + k;
        a.kf_pose[o] = a.kf_pose_tmp[o];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_pack_scan(const float *scan3, float4 *scan4, int M, hipStream_t st)
{
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_scan, dim3((M + 255) / 256), dim3(256), 0, st, scan3, scan4, M);
    return hipGetLastError();
}

hipError_t launch_build_cells(const float *grid, void *cells, int nx, int ny, int nz, int dtype,
                              hipStream_t st)
{
    const size_t n = (size_t)(nx - 1) * (ny - 1) * (nz - 1);
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_build_cells, dim3((unsigned)blocks), dim3(256), 0, st, grid, cells, nx,
                       ny, nz, dtype);
    return hipGetLastError();
}

hipError_t launch_predict(float *pose, int N, const float dT[7], const float *noise, hipStream_t st)
{
    Pose7 d;
    for (int c = 0; c < 7; ++c) d.v[c] = dT[c];
    hipLaunchKernelGGL(k_predict, dim3((N + 255) / 256), dim3(256), 0, st, pose, N, d, noise);
    return hipGetLastError();
}

template <int DT, bool BIG>
static hipError_t launch_eval_dt(const EvalArgs &a, hipStream_t st)
{
    constexpr int W = 4, U = 2;
    const unsigned blocks = (unsigned)((a.N + 63) / 64);
    hipLaunchKernelGGL((k_eval_step<DT, BIG, W, U>), dim3(blocks), dim3(64 * W), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_eval_step(const EvalArgs &a, hipStream_t st)
{
    const uint64_t n_rec = (uint64_t)(a.grid.nx - 1) * (a.grid.ny - 1) * (a.grid.nz - 1);
    if ((n_rec << (a.grid.dtype == 0 ? 5 : 4)) >= (1ull << 32)) return hipErrorInvalidValue;
    const bool big = (uint64_t)(a.grid.nx - 1) >= (1u << 24) ||
                     (uint64_t)(a.grid.nx - 1) * (a.grid.ny - 1) >= (1u << 24);
    switch (a.grid.dtype * 2 + (big ? 1 : 0)) {
    case 0: return launch_eval_dt<0, false>(a, st);
    case 1: return launch_eval_dt<0, true>(a, st);
    case 2: return launch_eval_dt<1, false>(a, st);
    case 3: return launch_eval_dt<1, true>(a, st);
    case 4: return launch_eval_dt<2, false>(a, st);
    case 5: return launch_eval_dt<2, true>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kf_eval_step(const KfEvalArgs &, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_weights(const WeightArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_weights, dim3(weight_blocks(a.N)), dim3(kWeightBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_resample(const ResampleArgs &a, hipStream_t st)
{
    const unsigned nb = (unsigned)weight_blocks(a.N);
    hipLaunchKernelGGL(k_normalize_scan, dim3(nb), dim3(kWeightBlock), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_search_gather, dim3(nb), dim3(kWeightBlock), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.K > 0) {
        hipLaunchKernelGGL(k_gather_rows, dim3(nb, 7 * a.K), dim3(kWeightBlock), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_commit, dim3(nb, 7 + 7 * a.K), dim3(kWeightBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace mcs
