"""FP64 CPU oracle of the gradient-guided particle update -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and its
binding) never calls it.  The arithmetic lives in ``mcs_oracle.c`` (plain C,
FP64, OpenMP over particles); this module only marshals numpy arrays through
ctypes, plus two storage codecs (FP32 -> FP16 and FP32 -> BF16, round to
nearest even) that produce the quantised grids the oracle is run on.

Each function cites the passage of the paper it follows (T. Nakao et al.,
arXiv 2504.18056).
"""

import ctypes as C
import os

import numpy as np

from .build import ensure_built

_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _opt(kind):
    """ndpointer that also accepts None."""
    base = {"d": _dp, "f": _fp, "i": _ip}[kind]

    class _P(base):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return base.from_param(obj)

    return _P


def lib():
    global _lib
    if _lib is None:
        # MCS_ORACLE_LIB names another build of mcs_oracle.c (the mutation
        # check loads deliberately broken copies to show that the pins fail).
        L = C.CDLL(os.environ.get("MCS_ORACLE_LIB") or ensure_built())
        i32, f64 = C.c_int, C.c_double
        L.oracle_quat_to_rot.argtypes = [_dp, _dp]
        L.oracle_se3_exp.argtypes = [_dp, _dp]
        L.oracle_se3_log.argtypes = [_dp, _dp]
        L.oracle_se3_log.restype = i32
        L.oracle_pose_right_exp.argtypes = [_dp, _dp, _dp]
        L.oracle_eval.argtypes = [_fp, i32, i32, i32, _dp, f64, f64, i32, _fp, i32, _fp, i32,
                                  f64, _dp, _dp, _opt("d"), _opt("d"), _opt("d"), _opt("i"), i32]
        L.oracle_eval.restype = i32
        L.oracle_eval_f64.argtypes = [_fp, i32, i32, i32, _dp, f64, f64, i32, _fp, i32, _dp, i32,
                                      _dp, _opt("d")]
        L.oracle_eval_f64.restype = i32
        L.oracle_step.argtypes = [_fp, _dp, i32, f64, f64, f64, f64, _dp]
        L.oracle_step.restype = i32
        L.oracle_predict.argtypes = [_fp, i32, _dp, _opt("f"), _dp]
        L.oracle_predict.restype = i32
        L.oracle_weights.argtypes = [_dp, _opt("d"), i32, f64, _dp, C.POINTER(f64), C.POINTER(f64)]
        L.oracle_weights.restype = i32
        L.oracle_resample.argtypes = [_dp, i32, f64, _ip, _opt("d")]
        L.oracle_resample.restype = i32
        L.oracle_kf_eval.argtypes = [_fp, i32, i32, i32, i32, _dp, f64, f64, i32, _fp, i32, _fp,
                                     _fp, i32, i32, f64, _opt("i"), _dp, _dp, _opt("d"), _opt("d"),
                                     _opt("d"), _opt("i"), _opt("i"), _opt("d"), i32]
        L.oracle_kf_eval.restype = i32
        u64 = C.c_uint64
        L.oracle_splitmix64.argtypes = [u64, i32, np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")]
        L.oracle_rng_normals.argtypes = [u64, u64, i32, _dp]
        L.oracle_predict_rng.argtypes = [_fp, i32, _dp, u64, u64, _dp, _dp]
        L.oracle_predict_rng.restype = i32
        L.oracle_prune.argtypes = [_dp, _dp, i32, f64, f64, f64, _ip, _dp, C.POINTER(i32), _opt("d")]
        L.oracle_prune.restype = i32
        L.oracle_gicp_eval.argtypes = [_fp, i32, i32, i32, i32, _dp, f64, _fp, _fp, i32, _fp, _fp, i32,
                                       i32, f64, _opt("i"), _dp, _dp, _dp, _opt("d"), _opt("d"),
                                       _opt("i"), _opt("d"), _opt("i"), _opt("i"), i32]
        L.oracle_gicp_eval.restype = i32
        L.oracle_gn_step.argtypes = [_fp, _dp, _dp, i32, f64, f64, _dp, _opt("d")]
        L.oracle_gn_step.restype = i32
        L.oracle_kf_loop_update.argtypes = [_fp, _fp, _dp, _ip, i32, i32, i32, i32, f64, f64, f64,
                                            f64, _dp, _dp, _ip, _opt("d")]
        L.oracle_kf_loop_update.restype = i32
        L.oracle_filter_step.argtypes = [_fp, i32, i32, i32, _dp, f64, _fp, i32, _fp, _dp, i32,
                                         i32, f64, f64, f64, f64, f64, f64, i32, i32, i32, f64,
                                         f64, _opt("d"), _opt("f"), _dp, _dp, _dp, _dp, _ip, _dp,
                                         i32]
        L.oracle_filter_step.restype = i32
        _lib = L
    return _lib


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a if shape is None else a.reshape(shape)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _check(rc, name):
    if rc != 0:
        raise ValueError("%s failed with status %d" % (name, rc))


# ---------------------------------------------------------------------------
# SE(3) (Sec. III-C.2, Eq. 7; Sec. III-B, Eq. 1)
# ---------------------------------------------------------------------------

def quat_to_rot(q):
    R = np.empty(9)
    lib().oracle_quat_to_rot(_f64(q, (4,)), R)
    return R.reshape(3, 3)


def se3_exp(xi):
    """4x4 matrix of Exp(xi), xi = [rho; phi] (translation first)."""
    T = np.empty(16)
    lib().oracle_se3_exp(_f64(xi, (6,)), T)
    return T.reshape(4, 4)


def se3_log(T):
    xi = np.empty(6)
    _check(lib().oracle_se3_log(_f64(T, (16,)), xi), "se3_log")
    return xi


def pose_right_exp(pose, psi):
    """Pose row (t, q) composed on the right with Exp(psi) (Eq. 7)."""
    out = np.empty(7)
    lib().oracle_pose_right_exp(_f64(pose, (7,)), _f64(psi, (6,)), out)
    return out


# ---------------------------------------------------------------------------
# Likelihood and gradient (Sec. III-C.1 structure, grid likelihood)
# ---------------------------------------------------------------------------

def _grid_args(grid, dims, origin):
    nx, ny, nz = (int(v) for v in dims)
    g = _f32(grid).reshape(-1)
    if g.size != nx * ny * nz:
        raise ValueError("grid has %d values, dims give %d" % (g.size, nx * ny * nz))
    return g, nx, ny, nz, _f64(origin, (3,))


def evaluate(grid, dims, origin, h, eps, scan, poses, oob_skip=False, delta=0.0, nthreads=0):
    """Per-particle log-likelihood l (N,) and gradient g (N, 6) at FP32 poses.

    Also returns the per-component scale sum_j |d l_j / d xi| (N, 6) and, for
    delta > 0, the allowance for points within delta index units of a cell
    face: (amb_l (N,), amb_g (N, 6), n_amb (N,)).
    """
    g, nx, ny, nz, o = _grid_args(grid, dims, origin)
    scan = _f32(scan).reshape(-1, 3)
    poses = _f32(poses).reshape(-1, 7)
    N, M = poses.shape[0], scan.shape[0]
    ll, gr, ga = np.empty(N), np.empty((N, 6)), np.empty((N, 6))
    al, ag, na = np.empty(N), np.empty((N, 6)), np.empty(N, np.int32)
    _check(lib().oracle_eval(g, nx, ny, nz, o, float(h), float(eps), int(bool(oob_skip)), scan, M,
                             poses, N, float(delta), ll, gr, ga, al, ag, na, int(nthreads)),
           "oracle_eval")
    return dict(loglik=ll, grad=gr, gabs=ga, amb_l=al, amb_g=ag, n_amb=na)


def evaluate_f64(grid, dims, origin, h, eps, scan, poses, oob_skip=False):
    """l and g at FP64 poses (for finite differences)."""
    g, nx, ny, nz, o = _grid_args(grid, dims, origin)
    scan = _f32(scan).reshape(-1, 3)
    poses = _f64(poses).reshape(-1, 7)
    N = poses.shape[0]
    ll, gr = np.empty(N), np.empty((N, 6))
    _check(lib().oracle_eval_f64(g, nx, ny, nz, o, float(h), float(eps), int(bool(oob_skip)),
                                 scan, scan.shape[0], poses, N, ll, gr), "oracle_eval_f64")
    return ll, gr


def step(poses, grad, alpha_t, alpha_r, rho_max, phi_max):
    """Gradient-guided pose step T <- T Exp(psi) from a given gradient (Eq. 7)."""
    poses = _f32(poses).reshape(-1, 7)
    out = np.empty((poses.shape[0], 7))
    _check(lib().oracle_step(poses, _f64(grad).reshape(-1, 6), poses.shape[0], float(alpha_t),
                             float(alpha_r), float(rho_max), float(phi_max), out), "oracle_step")
    return out


def predict(poses, dT, delta=None):
    """T_i <- T_i dT Exp(delta_i) (Eq. 1)."""
    poses = _f32(poses).reshape(-1, 7)
    out = np.empty((poses.shape[0], 7))
    d = None if delta is None else _f32(delta).reshape(-1, 6)
    _check(lib().oracle_predict(poses, poses.shape[0], _f64(dT, (7,)), d, out), "oracle_predict")
    return out


def weights(logw_in, loglik=None, beta=1.0):
    """logw += beta l (Eq. 11), normalised; returns (logw_norm, L, ESS)."""
    logw_in = _f64(logw_in).reshape(-1)
    N = logw_in.size
    out = np.empty(N)
    L, E = C.c_double(), C.c_double()
    ll = None if loglik is None else _f64(loglik).reshape(-1)
    _check(lib().oracle_weights(logw_in, ll, N, float(beta), out, C.byref(L), C.byref(E)),
           "oracle_weights")
    return out, L.value, E.value


def resample(logw_norm, u):
    """Systematic resampling; returns (ancestors int32 (N,), tie margin (N,))."""
    lw = _f64(logw_norm).reshape(-1)
    a = np.empty(lw.size, np.int32)
    m = np.empty(lw.size)
    _check(lib().oracle_resample(lw, lw.size, float(u), a, m), "oracle_resample")
    return a, m


def _force(neighbors, N, n_nb):
    if neighbors is None:
        return None
    nb = np.ascontiguousarray(neighbors, dtype=np.int32).reshape(N, n_nb)
    return nb


def kf_evaluate(grids, dims, origins, h, eps, scan, poses, kf_poses, n_nb=4, oob_skip=False,
                delta=0.0, nthreads=0, neighbors=None):
    """Sum over the n_nb nearest keyframes (Eq. 2) of the grid log-likelihood
    under the relative pose T_k^-1 T (Eq. 4).  grids (K, nz, ny, nx) in each
    keyframe's frame, origins (K, 3), kf_poses (N, K, 7).  The neighbours are
    ranked on FP64 distances; nb_margin (N,) is the ranking's smallest relative
    gap between consecutive ranks (up to the first keyframe left out).
    neighbors (N, n_nb), if given, replaces the choice."""
    nx, ny, nz = (int(v) for v in dims)
    g = _f32(grids).reshape(-1)
    K = g.size // (nx * ny * nz)
    scan = _f32(scan).reshape(-1, 3)
    poses = _f32(poses).reshape(-1, 7)
    N = poses.shape[0]
    kf = _f32(kf_poses).reshape(N, K, 7)
    ll, gr, ga = np.empty(N), np.empty((N, 6)), np.empty((N, 6))
    al, ag, na = np.empty(N), np.empty((N, 6)), np.empty(N, np.int32)
    nb, mg = np.empty((N, n_nb), np.int32), np.empty(N)
    _check(lib().oracle_kf_eval(g, K, nx, ny, nz, _f64(origins).reshape(-1), float(h), float(eps),
                                int(bool(oob_skip)), scan, scan.shape[0], poses, kf, N, int(n_nb),
                                float(delta), _force(neighbors, N, n_nb), ll, gr, ga, al, ag, na,
                                nb, mg, int(nthreads)), "oracle_kf_eval")
    return dict(loglik=ll, grad=gr, gabs=ga, amb_l=al, amb_g=ag, n_amb=na, neighbors=nb,
                nb_margin=mg)


def splitmix64(seed, n):
    """The first n 64-bit outputs of SplitMix64 seeded with `seed`."""
    out = np.empty(int(n), np.uint64)
    lib().oracle_splitmix64(int(seed) & (2**64 - 1), int(n), out)
    return out


def rng_normals(seed, frame, N):
    """Standard normals (N, 6) of the counter-based prediction-noise stream of one frame."""
    out = np.empty((int(N), 6))
    lib().oracle_rng_normals(int(seed) & (2**64 - 1), int(frame), int(N), out)
    return out


def predict_rng(poses, dT, seed, frame, sigma):
    """Prediction T <- T dT Exp(sigma z) with z from the counter-based stream (Eq. 1)."""
    poses = _f32(poses).reshape(-1, 7)
    out = np.empty((poses.shape[0], 7))
    _check(lib().oracle_predict_rng(poses, poses.shape[0], _f64(dT, (7,)), int(seed) & (2**64 - 1),
                                    int(frame), _f64(sigma, (6,)), out), "oracle_predict_rng")
    return out


def prune(logw, loglik, tau_post, tau_lik, u):
    """Dead-particle pruning (Sec. III-F) on normalised log-weights; returns
    parents, logw, n_dead and the per-slot tie margin."""
    logw = _f64(logw).reshape(-1)
    N = logw.size
    par, lw, mg = np.empty(N, np.int32), np.empty(N), np.empty(N)
    nd = C.c_int(0)
    _check(lib().oracle_prune(logw, _f64(loglik).reshape(-1), N, float(tau_post), float(tau_lik),
                              float(u), par, lw, C.byref(nd), mg), "oracle_prune")
    return dict(parents=par, logw=lw, n_dead=nd.value, margin=mg)


def gicp_evaluate(vox, dims, origins, vs, mu, cov, poses, kf_poses, n_nb=4, delta=0.0, nthreads=0,
                  neighbors=None):
    """GICP likelihood (Eq. 2-4) over the n_nb nearest keyframes with voxel
    correspondences, and the Gauss-Newton system of Eq. 6: H (N, 21) upper
    triangle row-major, b (N, 6).  vox (K, nz, ny, nx, 12) voxel Gaussians in
    each keyframe's frame, origins (K, 3), voxel edge vs; scan means mu (M, 3)
    and covariances cov (M, 6: xx xy xz yy yz zz).  habs, babs: per entry, the
    sum of the magnitudes of the products it is made of (the rounding scale)."""
    nx, ny, nz = (int(v) for v in dims)
    v = _f32(vox).reshape(-1)
    K = v.size // (nx * ny * nz * 12)
    mu = _f32(mu).reshape(-1, 3)
    cov = _f32(cov).reshape(-1, 6)
    poses = _f32(poses).reshape(-1, 7)
    N = poses.shape[0]
    kf = _f32(kf_poses).reshape(N, K, 7)
    ll, H, b = np.empty(N), np.empty((N, 21)), np.empty((N, 6))
    ha, ba = np.empty((N, 21)), np.empty((N, 6))
    nb, mg = np.empty((N, n_nb), np.int32), np.empty(N)
    nc, na = np.empty(N, np.int32), np.empty(N, np.int32)
    _check(lib().oracle_gicp_eval(v, K, nx, ny, nz, _f64(origins).reshape(-1), float(vs), mu, cov,
                                  mu.shape[0], poses, kf, N, int(n_nb), float(delta),
                                  _force(neighbors, N, n_nb), ll, H, b, ha, ba, nb, mg, nc, na,
                                  int(nthreads)), "oracle_gicp_eval")
    return dict(loglik=ll, H=H, b=b, habs=ha, babs=ba, neighbors=nb, nb_margin=mg, n_corr=nc,
                n_amb=na)


def gn_step(poses, H, b, rho_max, phi_max):
    """Gauss-Newton step psi = -H^-1 b (Eq. 5), clamped, T <- T Exp(psi) (Eq. 7)."""
    poses = _f32(poses).reshape(-1, 7)
    N = poses.shape[0]
    out, psi = np.empty((N, 7)), np.empty((N, 6))
    _check(lib().oracle_gn_step(poses, _f64(H).reshape(-1), _f64(b).reshape(-1), N, float(rho_max),
                                float(phi_max), out, psi), "oracle_gn_step")
    return out, psi


def kf_loop_update(poses, kf_poses, grad, neighbors, params, n_recent=3):
    """Loop-gated correction of the current pose and the keyframe poses of each
    particle (Sec. III-C.2, Eq. 5-10, with the gradient step in place of the
    Gauss-Newton solve).  Returns poses (N, 7), kf_poses (N, K, 7), loop (N: the
    oldest neighbour when a loop is detected, else -1) and psi (N, 6)."""
    poses = _f32(poses).reshape(-1, 7)
    N = poses.shape[0]
    kf = _f32(kf_poses).reshape(N, -1, 7)
    K = kf.shape[1]
    nb = np.ascontiguousarray(neighbors, dtype=np.int32).reshape(N, -1)
    n_nb = nb.shape[1]
    out_p, out_k = np.empty((N, 7)), np.empty((N, K, 7))
    loop, psi = np.empty(N, np.int32), np.empty((N, 6))
    p = params
    _check(lib().oracle_kf_loop_update(poses, kf, _f64(grad).reshape(-1), nb, N, K, n_nb,
                                       int(n_recent), p["alpha_t"], p["alpha_r"], p["rho_max"],
                                       p["phi_max"], out_p, out_k, loop, psi),
           "oracle_kf_loop_update")
    return dict(poses=out_p, kf_poses=out_k, loop=loop, psi=psi)


POLICY_NEVER, POLICY_ALWAYS, POLICY_ESS = 0, 1, 2


def filter_step(grid, dims, origin, h, scan, poses, logw, params, u, policy=POLICY_ALWAYS,
                ess_frac=0.5, dT=None, delta=None, oob_skip=False, post_eval=False, nthreads=0):
    """One whole frame: prediction, passes of likelihood/gradient/step, weighting,
    normalisation and systematic resampling (Sec. III-B to III-D)."""
    g, nx, ny, nz, o = _grid_args(grid, dims, origin)
    scan = _f32(scan).reshape(-1, 3)
    poses = _f32(poses).reshape(-1, 7)
    N = poses.shape[0]
    out_p, out_w = np.empty((N, 7)), np.empty(N)
    ll, gr = np.empty(N), np.empty((N, 6))
    anc, st = np.empty(N, np.int32), np.empty(3)
    p = params
    _check(lib().oracle_filter_step(
        g, nx, ny, nz, o, float(h), scan, scan.shape[0], poses, _f64(logw).reshape(-1), N,
        int(p["iters"]), p["alpha_t"], p["alpha_r"], p["rho_max"], p["phi_max"], p["eps"],
        p.get("beta", 1.0), int(bool(oob_skip)), int(bool(post_eval)), int(policy),
        float(ess_frac), float(u), None if dT is None else _f64(dT, (7,)),
        None if delta is None else _f32(delta).reshape(-1, 6), out_p, out_w, ll, gr, anc, st,
        int(nthreads)), "oracle_filter_step")
    return dict(poses=out_p, logw=out_w, loglik=ll, grad=gr, ancestors=anc, lse=st[0], ess=st[1],
                resampled=bool(st[2]))


# ---------------------------------------------------------------------------
# Grid storage codecs (round to nearest, ties to even)
# ---------------------------------------------------------------------------

def quantize_fp16(grid):
    """FP32 -> IEEE binary16 (RNE) -> FP32 values the oracle runs on."""
    return np.asarray(grid, np.float32).astype(np.float16).astype(np.float32)


def bf16_bits(grid):
    """FP32 -> bfloat16 bit patterns, round to nearest even on the dropped 16 bits."""
    b = np.ascontiguousarray(grid, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) & 0xFFFF
    nan = np.isnan(np.asarray(grid, np.float32))
    r = np.where(nan, 0x7FC0, r)
    return r.astype(np.uint16)


def quantize_bf16(grid):
    """FP32 -> bfloat16 (RNE) -> FP32 values the oracle runs on."""
    bits = bf16_bits(grid).astype(np.uint32) << 16
    return bits.view(np.float32).reshape(np.shape(grid))

