/*
 * FP64 CPU oracle for the gradient-guided Monte Carlo SLAM particle update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header, table or constant with the HIP library; both are fed from the
 * seeded generators in the `synth` package.
 *
 * Paper: T. Nakao et al., "Range-based 6-DoF Monte Carlo SLAM with
 * Gradient-guided Particle Filter on GPU" (arXiv 2504.18056).
 *
 * What it computes, per particle i and pose T_i = (t_i, q_i):
 *   prediction   T_i <- T_i * dT * Exp(delta_i)                     (Sec. III-B, Eq. 1)
 *   likelihood   l_i = sum_j ln(G(u_ij) + eps), G trilinear in a
 *                likelihood grid exp(-d^2 / 2 sigma^2) sampled at voxel
 *                centres; u = (R p_j + t - o)/h - 1/2 in index units.
 *                The paper's likelihood is the GICP registration error of
 *                Eq. 2-4 (Sec. III-C.1); the grid likelihood replaces it here
 *                and keeps its structure: a sum of per-point log terms of the
 *                scan transformed by the particle pose, summed over neighbour
 *                keyframes (Eq. 2) when several keyframe grids are used.
 *   gradient     g = d l(T Exp(xi)) / d xi at xi = 0, xi = [rho; phi]
 *                (right perturbation, translation first, as in Eq. 7).
 *   pose step    psi = [a_t g_rho; a_r g_phi], each block clamped in norm,
 *                T <- T Exp(psi)                                    (Sec. III-C.2, Eq. 7)
 *   weighting    logw_i += beta * l_i                               (Sec. III-D, Eq. 11)
 *   normalising  L = logsumexp(logw), logw -= L, ESS = 1 / sum w^2
 *   resampling   systematic: a_k = min{i : CDF_i > (u + k)/N}; compare the
 *                paper's dead-particle pruning (Sec. III-F), which respawns
 *                particles from the weights of the remaining ones.
 *
 * Conventions: quaternions are Hamilton (w, x, y, z), active body-to-world;
 * poses are rows [tx ty tz qw qx qy qz]; grids are x-fastest with samples at
 * origin + (i + 1/2) h; a point is inside the grid when 0 <= u_a < n_a - 1 on
 * every axis (a NaN coordinate is outside).  Every quantity is FP64; FP32
 * inputs (scan, poses, grid values) are promoted exactly and the quaternion is
 * renormalised in FP64.  Sums run in ascending index order.
 *
 * Built with gcc -O2 -fopenmp -ffp-contract=off (no fast-math); OpenMP runs
 * over particles only, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* SO(3) / SE(3)                                                             */
/* ------------------------------------------------------------------------ */

static void quat_normalize(double q[4])
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    q[0] /= n; q[1] /= n; q[2] /= n; q[3] /= n;
}

/* Rotation matrix (row-major) of a unit quaternion. */
static void quat_to_rot(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Hamilton product a (x) b. */
static void quat_mul(const double a[4], const double b[4], double o[4])
{
    double r[4];
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    memcpy(o, r, sizeof r);
}

/* sin(x)/x, exact at 0. */
static double sinc(double x)
{
    if (fabs(x) < 1e-6) return 1.0 - x * x / 6.0;
    return sin(x) / x;
}

/* Unit quaternion of exp([phi]x): [cos(th/2), sin(th/2) phi/th]. */
static void so3_exp_quat(const double phi[3], double q[4])
{
    double th = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    double s = 0.5 * sinc(0.5 * th);          /* sin(th/2)/th */
    q[0] = cos(0.5 * th);
    q[1] = s * phi[0]; q[2] = s * phi[1]; q[3] = s * phi[2];
}

/* Left Jacobian V(phi) = I + a [phi]x + b [phi]x^2 with
 * a = (1 - cos th)/th^2 = (1/2) sinc(th/2)^2 and b = (th - sin th)/th^3. */
static void so3_V(const double phi[3], double V[9])
{
    double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double th = sqrt(th2);
    double sh = sinc(0.5 * th);
    double a = 0.5 * sh * sh;
    double b;
    if (th < 0.1) {
        /* Taylor series of (th - sin th)/th^3; the next term is below 2e-20. */
        b = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0 - th2 * th2 * th2 / 362880.0
            + th2 * th2 * th2 * th2 / 39916800.0;
    } else {
        b = (th - sin(th)) / (th2 * th);
    }
    double K[9] = {0.0, -phi[2], phi[1], phi[2], 0.0, -phi[0], -phi[1], phi[0], 0.0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += K[3 * r + m] * K[3 * m + c];
            K2[3 * r + c] = s;
        }
    for (int e = 0; e < 9; ++e) V[e] = (e % 4 == 0 ? 1.0 : 0.0) + a * K[e] + b * K2[e];
}

static void mat3_vec(const double M[9], const double v[3], double o[3])
{
    double r0 = M[0] * v[0] + M[1] * v[1] + M[2] * v[2];
    double r1 = M[3] * v[0] + M[4] * v[1] + M[5] * v[2];
    double r2 = M[6] * v[0] + M[7] * v[1] + M[8] * v[2];
    o[0] = r0; o[1] = r1; o[2] = r2;
}

static void mat3T_vec(const double M[9], const double v[3], double o[3])
{
    double r0 = M[0] * v[0] + M[3] * v[1] + M[6] * v[2];
    double r1 = M[1] * v[0] + M[4] * v[1] + M[7] * v[2];
    double r2 = M[2] * v[0] + M[5] * v[1] + M[8] * v[2];
    o[0] = r0; o[1] = r1; o[2] = r2;
}

static void cross3(const double a[3], const double b[3], double o[3])
{
    double r0 = a[1] * b[2] - a[2] * b[1];
    double r1 = a[2] * b[0] - a[0] * b[2];
    double r2 = a[0] * b[1] - a[1] * b[0];
    o[0] = r0; o[1] = r1; o[2] = r2;
}

/* T * Exp(psi) for a pose row (t, q): t' = t + R V(phi) rho, q' = q (x) q(phi). */
static void pose_right_exp(const double pose[7], const double psi[6], double out[7])
{
    double q[4] = {pose[3], pose[4], pose[5], pose[6]};
    double R[9], V[9], Vr[3], dt[3], dq[4], qn[4];
    quat_normalize(q);
    quat_to_rot(q, R);
    so3_V(psi + 3, V);
    mat3_vec(V, psi, Vr);
    mat3_vec(R, Vr, dt);
    so3_exp_quat(psi + 3, dq);
    quat_mul(q, dq, qn);
    quat_normalize(qn);
    out[0] = pose[0] + dt[0]; out[1] = pose[1] + dt[1]; out[2] = pose[2] + dt[2];
    out[3] = qn[0]; out[4] = qn[1]; out[5] = qn[2]; out[6] = qn[3];
}

/* A * B for poses (composition of rigid transforms). */
static void pose_mul(const double A[7], const double B[7], double out[7])
{
    double qa[4] = {A[3], A[4], A[5], A[6]}, qb[4] = {B[3], B[4], B[5], B[6]}, R[9], tb[3], q[4];
    quat_normalize(qa); quat_normalize(qb);
    quat_to_rot(qa, R);
    mat3_vec(R, B, tb);
    quat_mul(qa, qb, q);
    quat_normalize(q);
    out[0] = A[0] + tb[0]; out[1] = A[1] + tb[1]; out[2] = A[2] + tb[2];
    out[3] = q[0]; out[4] = q[1]; out[5] = q[2]; out[6] = q[3];
}

static void pose_from_float(const float *p, double o[7])
{
    for (int c = 0; c < 7; ++c) o[c] = (double)p[c];
    double q[4] = {o[3], o[4], o[5], o[6]};
    quat_normalize(q);
    o[3] = q[0]; o[4] = q[1]; o[5] = q[2]; o[6] = q[3];
}

/* Exported SE(3) primitives (used by the pins). */
void oracle_quat_to_rot(const double *q_in, double *R)
{
    double q[4] = {q_in[0], q_in[1], q_in[2], q_in[3]};
    quat_normalize(q);
    quat_to_rot(q, R);
}

/* 4x4 row-major matrix of Exp(xi), xi = [rho; phi]. */
void oracle_se3_exp(const double *xi, double *T)
{
    double q[4], R[9], V[9], t[3];
    so3_exp_quat(xi + 3, q);
    quat_to_rot(q, R);
    so3_V(xi + 3, V);
    mat3_vec(V, xi, t);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) T[4 * r + c] = R[3 * r + c];
        T[4 * r + 3] = t[r];
    }
    T[12] = T[13] = T[14] = 0.0; T[15] = 1.0;
}

/* xi = Log(T) for a 4x4 rigid transform with rotation angle below pi. */
int oracle_se3_log(const double *T, double *xi)
{
    double R[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R[3 * r + c] = T[4 * r + c];
    /* Quaternion of R (Shepperd), then phi = 2 atan2(|v|, w) v/|v| with w >= 0. */
    double q[4], tr = R[0] + R[4] + R[8];
    if (tr > 0.0) {
        double s = 2.0 * sqrt(tr + 1.0);
        q[0] = 0.25 * s; q[1] = (R[7] - R[5]) / s; q[2] = (R[2] - R[6]) / s; q[3] = (R[3] - R[1]) / s;
    } else if (R[0] > R[4] && R[0] > R[8]) {
        double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]);
        q[0] = (R[7] - R[5]) / s; q[1] = 0.25 * s; q[2] = (R[1] + R[3]) / s; q[3] = (R[2] + R[6]) / s;
    } else if (R[4] > R[8]) {
        double s = 2.0 * sqrt(1.0 + R[4] - R[0] - R[8]);
        q[0] = (R[2] - R[6]) / s; q[1] = (R[1] + R[3]) / s; q[2] = 0.25 * s; q[3] = (R[5] + R[7]) / s;
    } else {
        double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]);
        q[0] = (R[3] - R[1]) / s; q[1] = (R[2] + R[6]) / s; q[2] = (R[5] + R[7]) / s; q[3] = 0.25 * s;
    }
    if (q[0] < 0.0) { q[0] = -q[0]; q[1] = -q[1]; q[2] = -q[2]; q[3] = -q[3]; }
    quat_normalize(q);
    double vn = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double th = 2.0 * atan2(vn, q[0]);
    double k = (vn < 1e-300) ? 2.0 : th / vn;
    double phi[3] = {k * q[1], k * q[2], k * q[3]};
    /* rho solves V(phi) rho = t: Gaussian elimination with partial pivoting. */
    double V[9], A[12];
    so3_V(phi, V);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) A[4 * r + c] = V[3 * r + c];
        A[4 * r + 3] = T[4 * r + 3];
    }
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[4 * r + c]) > fabs(A[4 * p + c])) p = r;
        if (A[4 * p + c] == 0.0) return -1;
        for (int e = 0; e < 4; ++e) { double tmp = A[4 * c + e]; A[4 * c + e] = A[4 * p + e]; A[4 * p + e] = tmp; }
        for (int r = c + 1; r < 3; ++r) {
            double f = A[4 * r + c] / A[4 * c + c];
            for (int e = c; e < 4; ++e) A[4 * r + e] -= f * A[4 * c + e];
        }
    }
    double rho[3];
    for (int r = 2; r >= 0; --r) {
        double s = A[4 * r + 3];
        for (int e = r + 1; e < 3; ++e) s -= A[4 * r + e] * rho[e];
        rho[r] = s / A[4 * r + r];
    }
    xi[0] = rho[0]; xi[1] = rho[1]; xi[2] = rho[2];
    xi[3] = phi[0]; xi[4] = phi[1]; xi[5] = phi[2];
    return 0;
}

/* Exported pose composition T * Exp(psi) for single poses (pins). */
void oracle_pose_right_exp(const double *pose, const double *psi, double *out)
{
    pose_right_exp(pose, psi, out);
}

/* ------------------------------------------------------------------------ */
/* Trilinear likelihood grid                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    const float *v;
    int nx, ny, nz;
    double o[3];
    double h;
} grid_t;

/* Per-point log term and its gradient in world units for cell i0 at
 * fractions f (each in [0, 1]); the cell must lie inside the grid. */
static void cell_term(const grid_t *g, double eps, const int i0[3], const double f[3],
                      double *lj, double d[3])
{
    double w[3][2];
    for (int a = 0; a < 3; ++a) {
        w[a][0] = 1.0 - f[a];
        w[a][1] = f[a];
    }
    double G = 0.0, dG[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                size_t idx = (size_t)(i0[0] + a) + (size_t)g->nx * ((size_t)(i0[1] + b) + (size_t)g->ny * (size_t)(i0[2] + c));
                double val = (double)g->v[idx];
                G += val * w[0][a] * w[1][b] * w[2][c];
                dG[0] += val * (2 * a - 1) * w[1][b] * w[2][c];
                dG[1] += val * w[0][a] * (2 * b - 1) * w[2][c];
                dG[2] += val * w[0][a] * w[1][b] * (2 * c - 1);
            }
    double den = G + eps;
    *lj = log(den);
    for (int a = 0; a < 3; ++a) d[a] = dG[a] / (g->h * den);
}

static int cell_inside(const grid_t *g, const int i0[3])
{
    const int n[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; ++a)
        if (i0[a] < 0 || i0[a] > n[a] - 2) return 0;
    return 1;
}

/* Per-point log term and its gradient in world units at index-space point u.
 * Returns 1 when u is inside the grid.  Outside: term ln(eps) (or 0 when
 * oob_skip), zero gradient. */
static int point_term(const grid_t *g, double eps, int oob_skip, const double u[3],
                      double *lj, double d[3])
{
    const int n[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; ++a) {
        if (!(u[a] >= 0.0 && u[a] < (double)(n[a] - 1))) {
            *lj = oob_skip ? 0.0 : log(eps);
            d[0] = d[1] = d[2] = 0.0;
            return 0;
        }
    }
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double fl = floor(u[a]);
        i0[a] = (int)fl;
        f[a] = u[a] - fl;
    }
    cell_term(g, eps, i0, f, lj, d);
    return 1;
}

/* Allowance for a point whose cell (or inside/outside) decision sits within
 * `delta` index units of a cell face: the largest change of the term and of
 * its xi-derivative over the positions the kernel may take within delta on
 * either side of each such face.  Along one axis the term is, in each cell, a
 * ratio of two linear functions of the fraction (monotone), so its extremes
 * on [face - delta, face] and [face, face + delta] are at the ends: the lower
 * cell at fractions 1 - delta and 1, the upper cell at 0 and delta. */
static int point_ambiguity(const grid_t *g, double eps, int oob_skip, const double u[3],
                           const double v[3], const double R[9], double delta,
                           double lj0, const double d0[3], double *amb_l, double amb_g[6])
{
    int axes[3], na = 0;
    double face[3];
    for (int a = 0; a < 3; ++a) {
        if (isnan(u[a])) return 0;
        double r = floor(u[a] + 0.5);          /* nearest integer = nearest face */
        if (fabs(u[a] - r) < delta) { axes[na] = a; face[na] = r; ++na; }
    }
    if (na == 0) return 0;
    double g0x[3], g0r[3], vx[3];
    mat3T_vec(R, d0, g0x);
    cross3(v, d0, vx);
    mat3T_vec(R, vx, g0r);
    int base_i[3];
    double base_f[3];
    for (int a = 0; a < 3; ++a) {
        double fl = floor(u[a]);
        base_i[a] = (int)fl;
        base_f[a] = u[a] - fl;
    }
    /* Per ambiguous axis: (cell offset from the face, fraction). */
    const int cell_off[4] = {-1, -1, 0, 0};
    const double frac[4] = {1.0 - delta, 1.0, 0.0, delta};
    int combos = 1;
    for (int s = 0; s < na; ++s) combos *= 4;
    for (int m = 0; m < combos; ++m) {
        int i0[3] = {base_i[0], base_i[1], base_i[2]};
        double f[3] = {base_f[0], base_f[1], base_f[2]};
        int mm = m;
        for (int s = 0; s < na; ++s) {
            int k = mm % 4;
            mm /= 4;
            i0[axes[s]] = (int)face[s] + cell_off[k];
            f[axes[s]] = frac[k];
        }
        double lj, d[3], gx[3], gr[3];
        if (cell_inside(g, i0)) {
            cell_term(g, eps, i0, f, &lj, d);
        } else {
            lj = oob_skip ? 0.0 : log(eps);
            d[0] = d[1] = d[2] = 0.0;
        }
        mat3T_vec(R, d, gx);
        cross3(v, d, vx);
        mat3T_vec(R, vx, gr);
        double dl = fabs(lj - lj0);
        if (dl > *amb_l) *amb_l = dl;
        for (int c = 0; c < 3; ++c) {
            double e0 = fabs(gx[c] - g0x[c]), e1 = fabs(gr[c] - g0r[c]);
            if (e0 > amb_g[c]) amb_g[c] = e0;
            if (e1 > amb_g[3 + c]) amb_g[3 + c] = e1;
        }
    }
    return 1;
}

typedef struct {
    double ll;         /* l = sum_j l_j */
    double g[6];       /* [g_rho; g_phi] */
    double gabs[6];    /* sum_j |d l_j / d xi_c|: scale of the summation error */
    double amb_l;      /* sum over ambiguous points of the term allowance */
    double amb_g[6];   /* same for the gradient components */
    int n_amb;         /* number of ambiguous points */
} eval_out;

/* Likelihood and right-perturbation gradient of one relative pose (R, t)
 * against one grid, accumulated into `o`.  v_j = R p_j, x_j = v_j + t.  The
 * gradient in xi is g_rho = R^T sum d_j and g_phi = R^T sum (v_j x d_j):
 * d/dphi of R (p + phi x p) + t is -R [p]x, whose transpose maps d to
 * p x (R^T d) = R^T ((R p) x d). */
static void eval_pose_grid(const grid_t *g, double eps, int oob_skip, const float *scan, int M,
                           const double R[9], const double t[3], double delta, eval_out *o)
{
    double L = 0.0, A[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
    double gabs[6] = {0, 0, 0, 0, 0, 0}, amb_g[6] = {0, 0, 0, 0, 0, 0}, amb_l = 0.0;
    int n_amb = 0;
    for (int j = 0; j < M; ++j) {
        double p[3] = {(double)scan[3 * j], (double)scan[3 * j + 1], (double)scan[3 * j + 2]};
        double v[3], u[3], lj, d[3], vxd[3], tx[3], tr[3];
        mat3_vec(R, p, v);
        for (int a = 0; a < 3; ++a) u[a] = (v[a] + t[a] - g->o[a]) / g->h - 0.5;
        if (point_term(g, eps, oob_skip, u, &lj, d)) {
            cross3(v, d, vxd);
        } else {
            /* Outside the grid the whole gradient contribution is zero (also
             * for non-finite points, where v x 0 would not be). */
            vxd[0] = vxd[1] = vxd[2] = 0.0;
        }
        L += lj;
        for (int a = 0; a < 3; ++a) { A[a] += d[a]; B[a] += vxd[a]; }
        mat3T_vec(R, d, tx);
        mat3T_vec(R, vxd, tr);
        for (int c = 0; c < 3; ++c) { gabs[c] += fabs(tx[c]); gabs[3 + c] += fabs(tr[c]); }
        if (delta > 0.0) {
            double al = 0.0, ag[6] = {0, 0, 0, 0, 0, 0};
            if (point_ambiguity(g, eps, oob_skip, u, v, R, delta, lj, d, &al, ag)) {
                ++n_amb;
                amb_l += al;
                for (int c = 0; c < 6; ++c) amb_g[c] += ag[c];
            }
        }
    }
    double gr[3], gp[3];
    mat3T_vec(R, A, gr);
    mat3T_vec(R, B, gp);
    o->ll += L;
    for (int c = 0; c < 3; ++c) { o->g[c] += gr[c]; o->g[3 + c] += gp[c]; }
    for (int c = 0; c < 6; ++c) { o->gabs[c] += gabs[c]; o->amb_g[c] += amb_g[c]; }
    o->amb_l += amb_l;
    o->n_amb += n_amb;
}

static void eval_pose(const grid_t *g, double eps, int oob_skip, const float *scan, int M,
                      const double pose[7], double delta, eval_out *o)
{
    double q[4] = {pose[3], pose[4], pose[5], pose[6]}, R[9];
    quat_normalize(q);
    quat_to_rot(q, R);
    memset(o, 0, sizeof *o);
    eval_pose_grid(g, eps, oob_skip, scan, M, R, pose, delta, o);
}

/* Gradient-guided step: psi = [a_t g_rho; a_r g_phi], each block scaled down
 * to its norm bound when longer, then T <- T Exp(psi) (Eq. 7). */
static void step_vector(const double g[6], double a_t, double a_r, double rho_max,
                        double phi_max, double psi[6])
{
    for (int c = 0; c < 3; ++c) { psi[c] = a_t * g[c]; psi[3 + c] = a_r * g[3 + c]; }
    double nr = sqrt(psi[0] * psi[0] + psi[1] * psi[1] + psi[2] * psi[2]);
    double np = sqrt(psi[3] * psi[3] + psi[4] * psi[4] + psi[5] * psi[5]);
    if (nr > rho_max) for (int c = 0; c < 3; ++c) psi[c] *= rho_max / nr;
    if (np > phi_max) for (int c = 3; c < 6; ++c) psi[c] *= phi_max / np;
}

static void step_pose(const double pose[7], const double g[6], double a_t, double a_r,
                      double rho_max, double phi_max, double out[7])
{
    double psi[6];
    step_vector(g, a_t, a_r, rho_max, phi_max, psi);
    pose_right_exp(pose, psi, out);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

static grid_t make_grid(const float *v, int nx, int ny, int nz, const double *origin, double h)
{
    grid_t g;
    g.v = v; g.nx = nx; g.ny = ny; g.nz = nz;
    g.o[0] = origin[0]; g.o[1] = origin[1]; g.o[2] = origin[2];
    g.h = h;
    return g;
}

/* l_i and g_i for every pose (FP32 rows, promoted).  Optional outputs may be
 * NULL: gabs (N*6), amb_l (N), amb_g (N*6), n_amb (N).  delta <= 0 disables
 * the ambiguity allowance. */
int oracle_eval(const float *grid, int nx, int ny, int nz, const double *origin, double h,
                double eps, int oob_skip, const float *scan, int M, const float *poses, int N,
                double delta, double *loglik, double *grad, double *gabs, double *amb_l,
                double *amb_g, int *n_amb, int nthreads)
{
    if (nx < 2 || ny < 2 || nz < 2 || M < 0 || N < 0 || h <= 0.0) return -1;
    grid_t g = make_grid(grid, nx, ny, nz, origin, h);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < N; ++i) {
        double pose[7];
        eval_out o;
        pose_from_float(poses + 7 * (size_t)i, pose);
        eval_pose(&g, eps, oob_skip, scan, M, pose, delta, &o);
        loglik[i] = o.ll;
        for (int c = 0; c < 6; ++c) grad[6 * (size_t)i + c] = o.g[c];
        if (gabs) for (int c = 0; c < 6; ++c) gabs[6 * (size_t)i + c] = o.gabs[c];
        if (amb_l) amb_l[i] = o.amb_l;
        if (amb_g) for (int c = 0; c < 6; ++c) amb_g[6 * (size_t)i + c] = o.amb_g[c];
        if (n_amb) n_amb[i] = o.n_amb;
    }
    return 0;
}

/* l at FP64 poses (used by the finite-difference pins). */
int oracle_eval_f64(const float *grid, int nx, int ny, int nz, const double *origin, double h,
                    double eps, int oob_skip, const float *scan, int M, const double *poses,
                    int N, double *loglik, double *grad)
{
    if (nx < 2 || ny < 2 || nz < 2 || M < 0 || N < 0 || h <= 0.0) return -1;
    grid_t g = make_grid(grid, nx, ny, nz, origin, h);
    for (int i = 0; i < N; ++i) {
        double pose[7];
        eval_out o;
        memcpy(pose, poses + 7 * (size_t)i, sizeof pose);
        double q[4] = {pose[3], pose[4], pose[5], pose[6]};
        quat_normalize(q);
        pose[3] = q[0]; pose[4] = q[1]; pose[5] = q[2]; pose[6] = q[3];
        eval_pose(&g, eps, oob_skip, scan, M, pose, 0.0, &o);
        loglik[i] = o.ll;
        if (grad) for (int c = 0; c < 6; ++c) grad[6 * (size_t)i + c] = o.g[c];
    }
    return 0;
}

/* One gradient step per pose from a given gradient (FP32 pose rows in, FP64 rows out). */
int oracle_step(const float *poses, const double *grad, int N, double a_t, double a_r,
                double rho_max, double phi_max, double *out)
{
    if (N < 0) return -1;
    for (int i = 0; i < N; ++i) {
        double pose[7];
        pose_from_float(poses + 7 * (size_t)i, pose);
        step_pose(pose, grad + 6 * (size_t)i, a_t, a_r, rho_max, phi_max, out + 7 * (size_t)i);
    }
    return 0;
}

/* Prediction T_i <- T_i * dT * Exp(delta_i) (Eq. 1); delta may be NULL (zero noise). */
int oracle_predict(const float *poses, int N, const double *dT, const float *delta, double *out)
{
    if (N < 0) return -1;
    for (int i = 0; i < N; ++i) {
        double pose[7], tmp[7], dTn[7];
        pose_from_float(poses + 7 * (size_t)i, pose);
        memcpy(dTn, dT, sizeof dTn);
        pose_mul(pose, dTn, tmp);
        if (delta) {
            double xi[6];
            for (int c = 0; c < 6; ++c) xi[c] = (double)delta[6 * (size_t)i + c];
            pose_right_exp(tmp, xi, out + 7 * (size_t)i);
        } else {
            memcpy(out + 7 * (size_t)i, tmp, sizeof tmp);
        }
    }
    return 0;
}

/* Prediction noise drawn from a counter-based generator (the device draws
 * the same numbers).  SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the
 * k-th output (k >= 1) of the stream seeded with s is mix(s + k * gamma), with
 * gamma = 0x9e3779b97f4a7c15 and mix the published finaliser.  The stream of
 * frame f is keyed by the f-th output of the seed's stream; within it,
 * particle i takes uniforms j = 6i .. 6i+5, U_j = (mix(key + (j+1) gamma) >> 11)
 * 2^-53, and Box-Muller turns the pairs (U_{6i+2m}, U_{6i+2m+1}) into
 * normals r cos(theta), r sin(theta) with r = sqrt(-2 ln(1 - U_a)) and
 * theta = 2 pi U_b.  delta_c = sigma_c z_c (translation first, Eq. 1). */
static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static const uint64_t SM64_GAMMA = 0x9e3779b97f4a7c15ULL;

static double sm64_uniform(uint64_t key, uint64_t j)
{
    return (double)(sm64_mix(key + (j + 1) * SM64_GAMMA) >> 11) * (1.0 / 9007199254740992.0);
}

static void rng_normals6(uint64_t seed, uint64_t frame, uint64_t i, double z[6])
{
    const uint64_t key = sm64_mix(seed + (frame + 1) * SM64_GAMMA);
    for (int m = 0; m < 3; ++m) {
        const double ua = sm64_uniform(key, 6 * i + 2 * m);
        const double ub = sm64_uniform(key, 6 * i + 2 * m + 1);
        const double r = sqrt(-2.0 * log(1.0 - ua));
        const double th = 2.0 * M_PI * ub;
        z[2 * m] = r * cos(th);
        z[2 * m + 1] = r * sin(th);
    }
}

/* The raw 64-bit outputs of one SplitMix64 stream (for the known-answer pin). */
void oracle_splitmix64(uint64_t seed, int n, uint64_t *out)
{
    for (int k = 0; k < n; ++k) out[k] = sm64_mix(seed + (uint64_t)(k + 1) * SM64_GAMMA);
}

/* Standard normals (N, 6) of frame `frame`. */
void oracle_rng_normals(uint64_t seed, uint64_t frame, int N, double *out)
{
    for (int i = 0; i < N; ++i) rng_normals6(seed, frame, (uint64_t)i, out + 6 * (size_t)i);
}

/* Prediction with generated noise: T_i <- T_i dT Exp(sigma z_i) (Eq. 1). */
int oracle_predict_rng(const float *poses, int N, const double *dT, uint64_t seed, uint64_t frame,
                       const double *sigma, double *out)
{
    if (N < 0) return -1;
    for (int i = 0; i < N; ++i) {
        double pose[7], tmp[7], dTn[7], z[6], xi[6];
        pose_from_float(poses + 7 * (size_t)i, pose);
        memcpy(dTn, dT, sizeof dTn);
        pose_mul(pose, dTn, tmp);
        rng_normals6(seed, frame, (uint64_t)i, z);
        for (int c = 0; c < 6; ++c) xi[c] = sigma[c] * z[c];
        pose_right_exp(tmp, xi, out + 7 * (size_t)i);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Weights and resampling                                                    */
/* ------------------------------------------------------------------------ */

/* logw_i += beta l_i (Eq. 11), then L = m + ln sum exp(logw - m) with
 * m = max logw, logw -= L, ESS = 1 / sum exp(logw)^2.  Sums run i ascending. */
int oracle_weights(const double *logw_in, const double *loglik, int N, double beta,
                   double *logw_out, double *lse, double *ess)
{
    if (N <= 0) return -1;
    double m = -INFINITY;
    for (int i = 0; i < N; ++i) {
        double lw = logw_in[i] + (loglik ? beta * loglik[i] : 0.0);
        logw_out[i] = lw;
        if (lw > m) m = lw;
    }
    double S = 0.0;
    for (int i = 0; i < N; ++i) S += exp(logw_out[i] - m);
    double L = m + log(S);
    double S2 = 0.0;
    for (int i = 0; i < N; ++i) {
        logw_out[i] -= L;
        double w = exp(logw_out[i]);
        S2 += w * w;
    }
    *lse = L;
    *ess = 1.0 / S2;
    return 0;
}

/* Systematic resampling on normalised log-weights: w_i = exp(logw_i),
 * CDF_i = sum_{m <= i} w_m (sequential, not renormalised),
 * u_k = (u + k)/N, a_k = min{i : CDF_i > u_k} or N - 1 when there is none.
 * margin (optional, N): min over the CDF values of |CDF_i - u_k|, i.e. how
 * close the decision for k was to a tie. */
int oracle_resample(const double *logw, int N, double u, int *ancestors, double *margin)
{
    if (N <= 0) return -1;
    double *cdf = (double *)malloc(sizeof(double) * (size_t)N);
    if (!cdf) return -2;
    double s = 0.0;
    for (int i = 0; i < N; ++i) { s += exp(logw[i]); cdf[i] = s; }
    int i = 0;
    for (int k = 0; k < N; ++k) {
        double uk = (u + (double)k) / (double)N;
        while (i < N && !(cdf[i] > uk)) ++i;      /* u_k is non-decreasing in k */
        int a = (i < N) ? i : N - 1;
        ancestors[k] = a;
        if (margin) {
            double mg = INFINITY;
            if (i < N) mg = fabs(cdf[i] - uk);
            if (i > 0 && fabs(cdf[i - 1] - uk) < mg) mg = fabs(cdf[i - 1] - uk);
            margin[k] = mg;
        }
    }
    free(cdf);
    return 0;
}

/* Dead-particle pruning (Sec. III-F) on normalised log-weights.  A particle
 * is dead when its posterior weight is below tau_post (logw_i < ln tau_post)
 * or its likelihood relative to the best particle of the frame is below
 * tau_lik (l_i - max_j l_j < ln tau_lik).  Each dead slot, in ascending index
 * order d_0 < d_1 < ..., receives a copy of a live particle drawn
 * systematically from the live weights: with C_i = sum of w_m over live
 * m <= i (sequential) and W = C_{N-1}, slot d_k takes
 * a_k = min{i : C_i > (u + k)/D W} (the last live index when there is none).
 * A parent p with c_p copies shares its weight equally with them, and the
 * live mass is renormalised: logw'_p = logw_p - ln(1 + c_p) - ln W for p and
 * each of its copies.  Without dead or without live particles nothing changes.
 * Outputs: parents (identity for live particles), logw_out, *n_dead, and
 * margin (N, optional): for a dead slot, min |C_i - target| over the two CDF
 * values around its decision (how close it was to a tie), else +inf. */
int oracle_prune(const double *logw, const double *loglik, int N, double tau_post, double tau_lik,
                 double u, int *parents, double *logw_out, int *n_dead, double *margin)
{
    if (N <= 0) return -1;
    double lmax = -INFINITY;
    for (int i = 0; i < N; ++i) if (loglik[i] > lmax) lmax = loglik[i];
    const double lp = log(tau_post), ll = log(tau_lik);
    char *dead = (char *)malloc((size_t)N);
    double *cdf = (double *)malloc(sizeof(double) * (size_t)N);
    int *copies = (int *)calloc((size_t)N, sizeof(int));
    if (!dead || !cdf || !copies) { free(dead); free(cdf); free(copies); return -2; }
    int D = 0, last_live = -1;
    double c = 0.0;
    for (int i = 0; i < N; ++i) {
        dead[i] = (logw[i] < lp) || (loglik[i] - lmax < ll);
        if (dead[i]) ++D; else { c += exp(logw[i]); last_live = i; }
        cdf[i] = c;
        parents[i] = i;
        logw_out[i] = logw[i];
        if (margin) margin[i] = INFINITY;
    }
    *n_dead = D;
    const double W = c;
    if (D > 0 && last_live >= 0 && W > 0.0) {
        int k = 0, i = 0;
        for (int slot = 0; slot < N; ++slot) {
            if (!dead[slot]) continue;
            const double target = (u + (double)k) / (double)D * W;
            while (i < N && !(cdf[i] > target)) ++i;   /* targets increase with k */
            const int a = (i < N) ? i : last_live;
            parents[slot] = a;
            copies[a]++;
            if (margin) {
                double mg = INFINITY;
                if (i < N) mg = fabs(cdf[i] - target);
                if (i > 0 && fabs(cdf[i - 1] - target) < mg) mg = fabs(cdf[i - 1] - target);
                margin[slot] = mg;
            }
            ++k;
        }
        const double lW = log(W);
        for (int p = 0; p < N; ++p)
            if (!dead[p]) logw_out[p] = logw[p] - log1p((double)copies[p]) - lW;
        for (int s2 = 0; s2 < N; ++s2)
            if (dead[s2]) logw_out[s2] = logw_out[parents[s2]];
    } else {
        *n_dead = 0;
    }
    free(dead); free(cdf); free(copies);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Keyframe map: sum over neighbour keyframes (Eq. 2)                        */
/* ------------------------------------------------------------------------ */

/* Neighbour keyframes of one particle: the n_nb smallest translation
 * distances |t - t_k| (Sec. III-C.1), ties to the smaller k, ranked on FP64
 * squared distances of the FP32 translations.  *margin receives the smallest
 * relative gap (d_b - d_a) / d_b between consecutive ranks 0 .. n_nb (the
 * last selected and the first left out included) whose translations differ:
 * an implementation that ranks in lower precision can only order such a pair
 * differently when the gap is below its rounding error.  Pairs with bitwise
 * equal translations tie exactly in any precision and are skipped. */
static void select_neighbors(const float *t, const float *kf, int K, int n_nb, int *nb,
                             double *margin)
{
    const int n_rank = n_nb < K ? n_nb + 1 : n_nb;
    char *used = (char *)calloc((size_t)K, 1);
    int rank[65];
    double dist[65];
    for (int s = 0; s < n_rank; ++s) {
        int best = -1;
        double bd = INFINITY;
        for (int k = 0; k < K; ++k) {
            if (used[k]) continue;
            double dx = (double)t[0] - (double)kf[7 * k];
            double dy = (double)t[1] - (double)kf[7 * k + 1];
            double dz = (double)t[2] - (double)kf[7 * k + 2];
            double d = dx * dx + dy * dy + dz * dz;
            if (best < 0 || d < bd) { bd = d; best = k; }
        }
        rank[s] = best;
        dist[s] = bd;
        if (best >= 0) used[best] = 1;
    }
    for (int s = 0; s < n_nb; ++s) nb[s] = rank[s];
    double m = INFINITY;
    for (int s = 0; s + 1 < n_rank; ++s) {
        const float *a = kf + 7 * rank[s], *b = kf + 7 * rank[s + 1];
        if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) continue;
        double gap = dist[s + 1] > 0.0 ? (dist[s + 1] - dist[s]) / dist[s + 1] : 0.0;
        if (gap < m) m = gap;
    }
    *margin = m;
    free(used);
}

/* Sum over the n_nb neighbour keyframes of particle i of the grid
 * log-likelihood of the scan under the relative pose kT = T_k^-1 T
 * (Eq. 2 and 4): R' = R_k^T R, t' = R_k^T (t - t_k).  The keyframe grids
 * share dims; grid k starts at grids + k*nx*ny*nz, origin at origins + 3k,
 * both in the keyframe's own frame.  kf_poses is (N, K, 7).  neighbors
 * (N, n_nb) receives the neighbours used and nb_margin (N) the ranking's
 * smallest relative gap (select_neighbors); a non-NULL nb_force (N, n_nb)
 * evaluates against those keyframes instead of the chosen ones (to check an
 * implementation's likelihood where its choice is one of several valid ones). */
int oracle_kf_eval(const float *grids, int K, int nx, int ny, int nz, const double *origins,
                   double h, double eps, int oob_skip, const float *scan, int M,
                   const float *poses, const float *kf_poses, int N, int n_nb, double delta,
                   const int *nb_force, double *loglik, double *grad, double *gabs,
                   double *amb_l, double *amb_g, int *n_amb, int *neighbors, double *nb_margin,
                   int nthreads)
{
    if (K <= 0 || n_nb <= 0 || n_nb > K || n_nb > 64 || N < 0 || M < 0) return -1;
    size_t gsz = (size_t)nx * ny * nz;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < N; ++i) {
        double pose[7], R[9];
        pose_from_float(poses + 7 * (size_t)i, pose);
        double q[4] = {pose[3], pose[4], pose[5], pose[6]};
        quat_to_rot(q, R);
        const float *kf = kf_poses + (size_t)7 * K * i;
        int nbp[64];
        double margin;
        select_neighbors(poses + 7 * (size_t)i, kf, K, n_nb, nbp, &margin);
        if (nb_margin) nb_margin[i] = margin;
        if (nb_force)
            for (int s = 0; s < n_nb; ++s) nbp[s] = nb_force[(size_t)n_nb * i + s];
        eval_out o;
        memset(&o, 0, sizeof o);
        for (int s = 0; s < n_nb; ++s) {
            int k = nbp[s];
            if (neighbors) neighbors[(size_t)n_nb * i + s] = k;
            double kp[7], Rk[9], Rr[9], dt[3], tr[3];
            pose_from_float(kf + 7 * (size_t)k, kp);
            double qk[4] = {kp[3], kp[4], kp[5], kp[6]};
            quat_to_rot(qk, Rk);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double sacc = 0.0;
                    for (int m = 0; m < 3; ++m) sacc += Rk[3 * m + r] * R[3 * m + c];
                    Rr[3 * r + c] = sacc;
                }
            for (int a = 0; a < 3; ++a) dt[a] = pose[a] - kp[a];
            mat3T_vec(Rk, dt, tr);
            grid_t g = make_grid(grids + gsz * (size_t)k, nx, ny, nz, origins + 3 * (size_t)k, h);
            eval_pose_grid(&g, eps, oob_skip, scan, M, Rr, tr, delta, &o);
        }
        loglik[i] = o.ll;
        for (int c = 0; c < 6; ++c) grad[6 * (size_t)i + c] = o.g[c];
        if (gabs) for (int c = 0; c < 6; ++c) gabs[6 * (size_t)i + c] = o.gabs[c];
        if (amb_l) amb_l[i] = o.amb_l;
        if (amb_g) for (int c = 0; c < 6; ++c) amb_g[6 * (size_t)i + c] = o.amb_g[c];
        if (n_amb) n_amb[i] = o.n_amb;
    }
    return 0;
}

/* Loop-gated state update of the keyframe filter (Sec. III-C.2).
 *
 * A particle detects a loop when one of its neighbour keyframes is old: its
 * index (keyframes are numbered in time order) lies below K - n_recent.  Only
 * then is its state corrected: the current pose by the step psi of its
 * gradient, T <- T Exp(psi) (Eq. 5-7 with the gradient step in place of the
 * Gauss-Newton solve), and every keyframe k from the oldest neighbour o up to
 * the newest by the discounted step psi_k = (d_k / d_t) psi,
 * T_k <- T_k Exp(psi_k) (Eq. 8 and 10).  The path lengths (Eq. 9) run along the
 * particle's own trajectory sampled at its keyframe poses:
 * d_k = sum_{m=o}^{k-1} |t_{m+1} - t_m| and d_t = d_{K-1} + |t - t_{K-1}|
 * with t the particle's current translation before the update.  Keyframes
 * older than o, and every pose of a particle without a loop, are unchanged.
 * When d_t = 0 no keyframe moves.
 * Inputs: poses (N, 7), kf_poses (N, K, 7), grad (N, 6), neighbors (N, n_nb).
 * Outputs: poses_out (N, 7), kf_out (N, K, 7), loop (N; the oldest neighbour o
 * when a loop is detected, else -1), psi (N, 6; may be NULL). */
int oracle_kf_loop_update(const float *poses, const float *kf_poses, const double *grad,
                          const int *neighbors, int N, int K, int n_nb, int n_recent,
                          double a_t, double a_r, double rho_max, double phi_max,
                          double *poses_out, double *kf_out, int *loop, double *psi_out)
{
    if (N < 0 || K <= 0 || n_nb <= 0 || n_nb > K) return -1;
    double *d = (double *)malloc(sizeof(double) * (size_t)K);
    if (!d) return -2;
    for (int i = 0; i < N; ++i) {
        const float *kf = kf_poses + (size_t)7 * K * i;
        double *ko = kf_out + (size_t)7 * K * i;
        double pose[7], psi[6];
        pose_from_float(poses + 7 * (size_t)i, pose);
        for (int k = 0; k < K; ++k) pose_from_float(kf + 7 * (size_t)k, ko + 7 * (size_t)k);
        step_vector(grad + 6 * (size_t)i, a_t, a_r, rho_max, phi_max, psi);
        if (psi_out) memcpy(psi_out + 6 * (size_t)i, psi, sizeof psi);
        int o = K;
        for (int s = 0; s < n_nb; ++s) {
            int k = neighbors[(size_t)n_nb * i + s];
            if (k < o) o = k;
        }
        if (o >= K - n_recent) {
            loop[i] = -1;
            memcpy(poses_out + 7 * (size_t)i, pose, sizeof pose);
            continue;
        }
        loop[i] = o;
        pose_right_exp(pose, psi, poses_out + 7 * (size_t)i);
        d[o] = 0.0;
        for (int k = o + 1; k < K; ++k) {
            double s2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double e = (double)kf[7 * (size_t)k + a] - (double)kf[7 * (size_t)(k - 1) + a];
                s2 += e * e;
            }
            d[k] = d[k - 1] + sqrt(s2);
        }
        double s2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double e = pose[a] - (double)kf[7 * (size_t)(K - 1) + a];
            s2 += e * e;
        }
        double dt = d[K - 1] + sqrt(s2);
        if (!(dt > 0.0)) continue;
        for (int k = o; k < K; ++k) {
            double pk[6], prev[7];
            for (int c = 0; c < 6; ++c) pk[c] = (d[k] / dt) * psi[c];
            memcpy(prev, ko + 7 * (size_t)k, sizeof prev);
            pose_right_exp(prev, pk, ko + 7 * (size_t)k);
        }
    }
    free(d);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* GICP likelihood and Gauss-Newton step (Sec. III-C, Eq. 2-7)                */
/* ------------------------------------------------------------------------ */

/* A keyframe voxel map: nx*ny*nz voxels of edge vs, voxel (i, j, k) covering
 * [o + (i, j, k) vs, o + (i+1, j+1, k+1) vs) in the keyframe's frame, x
 * fastest.  Each voxel holds 12 floats: mean (3), point count, covariance
 * (xx xy xz yy yz zz), 2 unused.  A voxel with count 0 is empty. */
typedef struct {
    const float *vox;
    int nx, ny, nz;
    double o[3];
    double vs;
} voxmap_t;

/* The voxel holding x: 1 and its Gaussian, or 0 when x is outside the map or
 * the voxel is empty.  *amb is set when a coordinate lies within delta voxels
 * of a face (the voxel choice is then a near-tie between two voxels). */
static int vox_lookup(const voxmap_t *m, const double x[3], double delta, double mu[3],
                      double S[6], int *amb)
{
    const int n[3] = {m->nx, m->ny, m->nz};
    int i[3];
    for (int a = 0; a < 3; ++a) {
        const double u = (x[a] - m->o[a]) / m->vs;
        const double f = floor(u);
        if (u - f < delta || f + 1.0 - u < delta) *amb = 1;
        if (!(f >= 0.0 && f < (double)n[a])) return 0;
        i[a] = (int)f;
    }
    const float *r = m->vox + 12 * ((size_t)i[0] + (size_t)m->nx * ((size_t)i[1] + (size_t)m->ny * i[2]));
    if (!(r[3] > 0.0f)) return 0;
    for (int a = 0; a < 3; ++a) mu[a] = r[a];
    for (int a = 0; a < 6; ++a) S[a] = r[4 + a];
    return 1;
}

/* Symmetric 3x3 (xx xy xz yy yz zz) to full and back. */
static void sym_full(const double s[6], double F[9])
{
    F[0] = s[0]; F[1] = s[1]; F[2] = s[2];
    F[3] = s[1]; F[4] = s[3]; F[5] = s[4];
    F[6] = s[2]; F[7] = s[4]; F[8] = s[5];
}

/* Inverse of a symmetric positive definite 3x3 by the adjugate. */
static int inv3(const double A[9], double I[9])
{
    const double c00 = A[4] * A[8] - A[5] * A[7];
    const double c01 = A[5] * A[6] - A[3] * A[8];
    const double c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(det > 0.0)) return 0;
    const double id = 1.0 / det;
    I[0] = c00 * id; I[1] = (A[2] * A[7] - A[1] * A[8]) * id; I[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    I[3] = c01 * id; I[4] = (A[0] * A[8] - A[2] * A[6]) * id; I[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    I[6] = c02 * id; I[7] = (A[1] * A[6] - A[0] * A[7]) * id; I[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return 1;
}

/* Index of H[r][c] (r <= c) in the 21-entry upper triangle, row-major. */
static int tri(int r, int c) { return r * 6 - r * (r - 1) / 2 + (c - r); }

typedef struct {
    double ll, H[21], b[6], habs[21], babs[6];
    int n_corr, n_amb;
} gicp_out;

/* Terms of the scan against one keyframe under the relative pose (R', t')
 * = T_k^-1 T (Eq. 4), accumulated into o.  With x = R' mu + t' and the
 * voxel Gaussian (mu', S') of x, the residual e = mu' - x and
 * Omega = (S' + R' Sigma R'^T)^-1 (Eq. 4; rotation only) are taken in the
 * scan's frame: e_s = R'^T e, Omega_s = R'^T Omega R' = (R'^T S' R' + Sigma)^-1.
 * Per point: l += -e^T Omega e, and with the Jacobian of e under T Exp(xi),
 * J_s = [-I, [mu]x], H += J_s^T Omega_s J_s and b += J_s^T Omega_s e_s
 * (Eq. 6). */
static void gicp_terms(const voxmap_t *m, const double R[9], const double t[3], const float *mu_s,
                       const float *cov_s, int M, double delta, gicp_out *o)
{
    for (int j = 0; j < M; ++j) {
        const double p[3] = {mu_s[3 * j], mu_s[3 * j + 1], mu_s[3 * j + 2]};
        double x[3], mv[3], Sv[6];
        mat3_vec(R, p, x);
        for (int a = 0; a < 3; ++a) x[a] += t[a];
        int amb = 0;
        const int hit = vox_lookup(m, x, delta, mv, Sv, &amb);
        o->n_amb += amb;
        if (!hit) continue;
        double d[3], es[3], Sf[9], T1[9], Ss[9], C[9], Om[9];
        for (int a = 0; a < 3; ++a) d[a] = mv[a] - t[a];
        mat3T_vec(R, d, es);
        for (int a = 0; a < 3; ++a) es[a] -= p[a];
        sym_full(Sv, Sf);
        /* Ss = R^T Sf R */
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Sf[3 * r + k] * R[3 * k + c];
                T1[3 * r + c] = acc;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R[3 * k + r] * T1[3 * k + c];
                Ss[3 * r + c] = acc;
            }
        double Cs[6] = {cov_s[6 * j], cov_s[6 * j + 1], cov_s[6 * j + 2],
                        cov_s[6 * j + 3], cov_s[6 * j + 4], cov_s[6 * j + 5]};
        double Cf[9];
        sym_full(Cs, Cf);
        for (int a = 0; a < 9; ++a) C[a] = Ss[a] + Cf[a];
        if (!inv3(C, Om)) continue;
        double w[3];
        mat3_vec(Om, es, w);
        const double q = es[0] * w[0] + es[1] * w[1] + es[2] * w[2];
        o->ll -= q;
        o->n_corr++;
        /* J_s = [-I, [p]x]: column c of [p]x is p x e_c. */
        double J[3][6];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) J[r][c] = (r == c) ? -1.0 : 0.0;
        const double K[9] = {0.0, -p[2], p[1], p[2], 0.0, -p[0], -p[1], p[0], 0.0};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) J[r][3 + c] = K[3 * r + c];
        double OJ[3][6];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 6; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Om[3 * r + k] * J[k][c];
                OJ[r][c] = acc;
            }
        /* Scales for the checks: each entry of b and H is a sum of products
         * (J^T Omega e, J^T Omega J); its rounding in any evaluation order is
         * bounded in proportion to the sum of those products' magnitudes,
         * |J|^T |Omega| |e| and |J|^T |Omega| |J|, which can be far larger
         * than the entry itself when the products cancel. */
        double aw[3], aOJ[3][6];
        for (int r = 0; r < 3; ++r) {
            aw[r] = 0.0;
            for (int k = 0; k < 3; ++k) aw[r] += fabs(Om[3 * r + k]) * fabs(es[k]);
            for (int c = 0; c < 6; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += fabs(Om[3 * r + k]) * fabs(J[k][c]);
                aOJ[r][c] = acc;
            }
        }
        for (int r = 0; r < 6; ++r) {
            double bb = 0.0, ba = 0.0;
            for (int k = 0; k < 3; ++k) {
                bb += J[k][r] * w[k];
                ba += fabs(J[k][r]) * aw[k];
            }
            o->b[r] += bb;
            o->babs[r] += ba;
            for (int c = r; c < 6; ++c) {
                double hh = 0.0, ha = 0.0;
                for (int k = 0; k < 3; ++k) {
                    hh += J[k][r] * OJ[k][c];
                    ha += fabs(J[k][r]) * aOJ[k][c];
                }
                o->H[tri(r, c)] += hh;
                o->habs[tri(r, c)] += ha;
            }
        }
    }
}

/* GICP likelihood (Eq. 2-4) of each particle summed over its n_nb neighbour
 * keyframes (chosen as for the grid likelihood), with the Gauss-Newton
 * system H (21, upper triangle row-major) and b (6) of Eq. 6.  vox holds the
 * K voxel maps back to back (each nx*ny*nz*12 floats), origins (K, 3) in each
 * keyframe's frame; scan means (M, 3) and covariances (M, 6).  n_corr counts
 * the points with a correspondence, n_amb those within delta of a voxel face.
 * habs (21) and babs (6) per particle: the sums of the magnitudes of the
 * products that make up each entry (|J|^T |Omega| |J|, |J|^T |Omega| |e|),
 * the scale of their rounding (test infrastructure).
 * nb_force (N, n_nb) or NULL, nb_margin (N) or NULL as for oracle_kf_eval. */
int oracle_gicp_eval(const float *vox, int K, int nx, int ny, int nz, const double *origins,
                     double vs, const float *mu, const float *cov, int M, const float *poses,
                     const float *kf_poses, int N, int n_nb, double delta, const int *nb_force,
                     double *loglik, double *H, double *b, double *habs, double *babs,
                     int *neighbors, double *nb_margin, int *n_corr, int *n_amb, int nthreads)
{
    if (K <= 0 || n_nb <= 0 || n_nb > K || n_nb > 64 || N < 0 || M < 0) return -1;
    const size_t vsz = (size_t)nx * ny * nz * 12;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < N; ++i) {
        double pose[7], R[9];
        pose_from_float(poses + 7 * (size_t)i, pose);
        double qq[4] = {pose[3], pose[4], pose[5], pose[6]};
        quat_to_rot(qq, R);
        const float *kf = kf_poses + (size_t)7 * K * i;
        int nbp[64];
        double margin;
        select_neighbors(poses + 7 * (size_t)i, kf, K, n_nb, nbp, &margin);
        if (nb_margin) nb_margin[i] = margin;
        if (nb_force)
            for (int s = 0; s < n_nb; ++s) nbp[s] = nb_force[(size_t)n_nb * i + s];
        gicp_out o;
        memset(&o, 0, sizeof o);
        for (int s = 0; s < n_nb; ++s) {
            const int k = nbp[s];
            if (neighbors) neighbors[(size_t)n_nb * i + s] = k;
            double kp[7], Rk[9], Rr[9], dt[3], tr[3];
            pose_from_float(kf + 7 * (size_t)k, kp);
            double qk[4] = {kp[3], kp[4], kp[5], kp[6]};
            quat_to_rot(qk, Rk);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double acc = 0.0;
                    for (int m2 = 0; m2 < 3; ++m2) acc += Rk[3 * m2 + r] * R[3 * m2 + c];
                    Rr[3 * r + c] = acc;
                }
            for (int a = 0; a < 3; ++a) dt[a] = pose[a] - kp[a];
            mat3T_vec(Rk, dt, tr);
            voxmap_t m;
            m.vox = vox + vsz * (size_t)k;
            m.nx = nx; m.ny = ny; m.nz = nz;
            for (int a = 0; a < 3; ++a) m.o[a] = origins[3 * (size_t)k + a];
            m.vs = vs;
            gicp_terms(&m, Rr, tr, mu, cov, M, delta, &o);
        }
        loglik[i] = o.ll;
        for (int c = 0; c < 21; ++c) H[21 * (size_t)i + c] = o.H[c];
        for (int c = 0; c < 6; ++c) b[6 * (size_t)i + c] = o.b[c];
        if (habs) for (int c = 0; c < 21; ++c) habs[21 * (size_t)i + c] = o.habs[c];
        if (babs) for (int c = 0; c < 6; ++c) babs[6 * (size_t)i + c] = o.babs[c];
        if (n_corr) n_corr[i] = o.n_corr;
        if (n_amb) n_amb[i] = o.n_amb;
    }
    return 0;
}

/* Gauss-Newton step (Eq. 5 and 7): psi = -H^-1 b minimises the quadratic
 * model of sum e^T Omega e (with J the derivative of e, the paper's
 * psi = H^-1 b holds for J taken as -de/dT).  H is solved by Cholesky; when
 * it is not positive definite (pivot <= 1e-12 of its largest diagonal entry)
 * the pose is left as it is.  Each block of psi is clamped as for the
 * gradient step, then T <- T Exp(psi).  Outputs poses (N, 7) and psi (N, 6). */
int oracle_gn_step(const float *poses, const double *H, const double *b, int N, double rho_max,
                   double phi_max, double *out, double *psi_out)
{
    if (N < 0) return -1;
    for (int i = 0; i < N; ++i) {
        double pose[7], A[6][6], L[6][6], y[6], x[6];
        pose_from_float(poses + 7 * (size_t)i, pose);
        const double *h = H + 21 * (size_t)i;
        double dmax = 0.0;
        for (int r = 0; r < 6; ++r)
            for (int c = r; c < 6; ++c) A[r][c] = A[c][r] = h[tri(r, c)];
        for (int r = 0; r < 6; ++r) if (A[r][r] > dmax) dmax = A[r][r];
        int ok = dmax > 0.0;
        memset(L, 0, sizeof L);
        for (int c = 0; c < 6 && ok; ++c) {
            double sdiag = A[c][c];
            for (int k = 0; k < c; ++k) sdiag -= L[c][k] * L[c][k];
            if (!(sdiag > 1e-12 * dmax)) { ok = 0; break; }
            L[c][c] = sqrt(sdiag);
            for (int r = c + 1; r < 6; ++r) {
                double sv = A[r][c];
                for (int k = 0; k < c; ++k) sv -= L[r][k] * L[c][k];
                L[r][c] = sv / L[c][c];
            }
        }
        double ps[6] = {0, 0, 0, 0, 0, 0};
        if (ok) {
            for (int r = 0; r < 6; ++r) {
                double sv = -b[6 * (size_t)i + r];
                for (int k = 0; k < r; ++k) sv -= L[r][k] * y[k];
                y[r] = sv / L[r][r];
            }
            for (int r = 5; r >= 0; --r) {
                double sv = y[r];
                for (int k = r + 1; k < 6; ++k) sv -= L[k][r] * x[k];
                x[r] = sv / L[r][r];
            }
            memcpy(ps, x, sizeof ps);
            const double nr = sqrt(ps[0] * ps[0] + ps[1] * ps[1] + ps[2] * ps[2]);
            const double np = sqrt(ps[3] * ps[3] + ps[4] * ps[4] + ps[5] * ps[5]);
            if (nr > rho_max) for (int c = 0; c < 3; ++c) ps[c] *= rho_max / nr;
            if (np > phi_max) for (int c = 3; c < 6; ++c) ps[c] *= phi_max / np;
        }
        if (psi_out) memcpy(psi_out + 6 * (size_t)i, ps, sizeof ps);
        pose_right_exp(pose, ps, out + 7 * (size_t)i);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole filter step                                                          */
/* ------------------------------------------------------------------------ */

/* One frame: optional prediction, `iters` passes of (likelihood + gradient,
 * pose step) per particle, weighting with the likelihood of the last pass
 * (taken at that pass's pre-step pose; with post_eval != 0 a further
 * likelihood-only pass at the final pose is used instead), normalisation and,
 * when the policy fires (1: always; 2: ESS < ess_frac * N strictly), systematic
 * resampling with logw reset to -ln N.
 * Outputs: poses_out and logw_out (N*7, N), loglik/grad of the last pass,
 * ancestors (identity when not resampled), stats = {L, ESS, resampled}. */
int oracle_filter_step(const float *grid, int nx, int ny, int nz, const double *origin,
                       double h, const float *scan, int M, const float *poses_in,
                       const double *logw_in, int N, int iters, double a_t, double a_r,
                       double rho_max, double phi_max, double eps, double beta, int oob_skip,
                       int post_eval, int policy, double ess_frac, double u, const double *dT,
                       const float *delta, double *poses_out, double *logw_out, double *loglik,
                       double *grad, int *ancestors, double *stats, int nthreads)
{
    if (N <= 0 || M < 0 || iters < 1) return -1;
    grid_t g = make_grid(grid, nx, ny, nz, origin, h);
    set_threads(nthreads);
    double *cur = (double *)malloc(sizeof(double) * 7 * (size_t)N);
    double *lw = (double *)malloc(sizeof(double) * (size_t)N);
    if (!cur || !lw) { free(cur); free(lw); return -2; }
    if (dT) {
        oracle_predict(poses_in, N, dT, delta, cur);
    } else {
        for (int i = 0; i < N; ++i) pose_from_float(poses_in + 7 * (size_t)i, cur + 7 * (size_t)i);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < N; ++i) {
        double *pose = cur + 7 * (size_t)i;
        eval_out o;
        for (int it = 0; it < iters; ++it) {
            double next[7];
            eval_pose(&g, eps, oob_skip, scan, M, pose, 0.0, &o);
            loglik[i] = o.ll;
            for (int c = 0; c < 6; ++c) grad[6 * (size_t)i + c] = o.g[c];
            step_pose(pose, o.g, a_t, a_r, rho_max, phi_max, next);
            memcpy(pose, next, sizeof next);
        }
        if (post_eval) {
            eval_pose(&g, eps, oob_skip, scan, M, pose, 0.0, &o);
            loglik[i] = o.ll;
        }
    }
    double L, ess;
    oracle_weights(logw_in, loglik, N, beta, lw, &L, &ess);
    int resample = (policy == 1) || (policy == 2 && ess < ess_frac * (double)N);
    if (resample) {
        oracle_resample(lw, N, u, ancestors, NULL);
        double lnN = -log((double)N);
        for (int k = 0; k < N; ++k) {
            memcpy(poses_out + 7 * (size_t)k, cur + 7 * (size_t)ancestors[k], 7 * sizeof(double));
            logw_out[k] = lnN;
        }
    } else {
        for (int k = 0; k < N; ++k) {
            ancestors[k] = k;
            memcpy(poses_out + 7 * (size_t)k, cur + 7 * (size_t)k, 7 * sizeof(double));
            logw_out[k] = lw[k];
        }
    }
    stats[0] = L; stats[1] = ess; stats[2] = (double)resample;
    free(cur);
    free(lw);
    return 0;
}
