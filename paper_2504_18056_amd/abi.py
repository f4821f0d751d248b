"""ctypes binding of include/mcslam.h: same names, argument marshalling only.

Every step of the filter runs in the HIP library libmcslam.so built from
csrc/ (see build.py).  There is no fallback: if the library is missing or
cannot be loaded, loading raises McsError.
"""

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcslam.so")

MCS_OK, MCS_EINVAL, MCS_ENOMEM, MCS_EBUDGET, MCS_ENOTFOUND, MCS_EDEVICE, MCS_EBUSY = \
    0, -1, -2, -3, -4, -5, -6
GRID_FP32, GRID_FP16, GRID_BF16 = 0, 1, 2
RESAMPLE_NEVER, RESAMPLE_ALWAYS, RESAMPLE_ESS, RESAMPLE_PRUNE = 0, 1, 2, 3
NOISE_INPUT, NOISE_DEVICE = 0, 1
OOB_FLOOR, OOB_SKIP = 0, 1
KF_FIXED, KF_LOOP = 0, 1

_STATUS_NAMES = {0: "MCS_OK", -1: "MCS_EINVAL", -2: "MCS_ENOMEM", -3: "MCS_EBUDGET",
                 -4: "MCS_ENOTFOUND", -5: "MCS_EDEVICE", -6: "MCS_EBUSY"}


class McsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (_STATUS_NAMES.get(status, "?"), status, message))
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("origin", C.c_float * 3), ("res", C.c_float), ("dtype", C.c_int32)]


class VoxelDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("origin", C.c_float * 3), ("edge", C.c_float)]


class StepParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("alpha_t", C.c_float), ("alpha_r", C.c_float),
                ("rho_max", C.c_float), ("phi_max", C.c_float), ("eps", C.c_float),
                ("beta", C.c_float), ("oob", C.c_int32), ("post_eval", C.c_int32),
                ("resample", C.c_int32), ("ess_frac", C.c_double), ("u", C.c_double),
                ("predict", C.c_int32), ("delta_T", C.c_float * 7), ("n_neighbors", C.c_int32),
                ("kf_update", C.c_int32), ("n_recent", C.c_int32), ("noise_mode", C.c_int32),
                ("rng_seed", C.c_uint64), ("rng_frame", C.c_uint64), ("noise_sigma", C.c_float * 6),
                ("prune_post", C.c_float), ("prune_lik", C.c_float)]


class StepStats(C.Structure):
    _fields_ = [("lse", C.c_double), ("ess", C.c_double), ("resampled", C.c_int32),
                ("best", C.c_int32), ("best_pose", C.c_float * 7), ("degenerate", C.c_int32),
                ("pruned", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("predict_ms", C.c_double), ("eval_ms", C.c_double), ("weights_ms", C.c_double),
                ("resample_ms", C.c_double), ("steps", C.c_int64), ("evals", C.c_int64)]


class RequestTimes(C.Structure):
    _fields_ = [("submit_ns", C.c_int64), ("launch_ns", C.c_int64), ("done_ns", C.c_int64),
                ("session_id", C.c_int32), ("tick", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("requests", C.c_int64), ("ticks", C.c_int64), ("evals", C.c_int64),
                ("max_batch_seen", C.c_int32), ("pad", C.c_int32)]


SERVE_BATCHED, SERVE_SERIAL, SERVE_CONCURRENT = 0, 1, 2

_lib = None


def lib():
    """The loaded libmcslam.so (raises McsError when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise McsError(MCS_EDEVICE, "HIP library %s is not built; run "
                           "`python -m paper_2504_18056_amd.build`" % LIB_PATH)
        # One HIP runtime per process: PyTorch ships its own copy of the ROCm
        # runtime libraries, and when this library is loaded first (binding the
        # system's copy) a later `import torch` finds no GPU.  So torch, when
        # installed, is imported before the library, and both use its runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        try:
            L = C.CDLL(LIB_PATH)
        except OSError as e:
            raise McsError(MCS_EDEVICE, "cannot load %s: %s" % (LIB_PATH, e))
        vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
        P = C.POINTER
        sig = {
            "mcs_version": (C.c_char_p, []),
            "mcs_last_error": (C.c_char_p, []),
            "mcs_create": (i32, [i32, u64, P(vp)]),
            "mcs_destroy": (i32, [vp]),
            "mcs_memory_in_use": (i32, [vp, P(u64)]),
            "mcs_init_map": (i32, [vp, P(GridDesc), vp, P(i32)]),
            "mcs_load_keyframes": (i32, [vp, i32, P(GridDesc), P(vp), P(i32)]),
            "mcs_release_map": (i32, [vp, i32]),
            "mcs_session_create": (i32, [vp, i32, i32, i32, vp, vp, P(i32)]),
            "mcs_session_destroy": (i32, [vp, i32]),
            "mcs_session_bytes": (i32, [vp, i32, i32, i32, P(u64)]),
            "mcs_set_particles": (i32, [vp, i32, vp, vp, vp]),
            "mcs_filter_step": (i32, [vp, i32, vp, i32, vp, P(StepParams)]),
            "mcs_filter_step_dev": (i32, [vp, i32, vp, i32, vp, P(StepParams), vp]),
            "mcs_get_particles": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, P(StepStats)]),
            "mcs_session_sync": (i32, [vp, i32]),
            "mcs_session_stream": (i32, [vp, i32, P(vp)]),
            "mcs_get_neighbors": (i32, [vp, i32, vp, P(i32)]),
            "mcs_server_create": (i32, [vp, i32, i32, i32, i32, i32, P(vp)]),
            "mcs_server_destroy": (i32, [vp]),
            "mcs_server_submit": (i32, [vp, i32, vp, i32, vp, P(StepParams), P(C.c_int64)]),
            "mcs_server_drain": (i32, [vp]),
            "mcs_server_times": (i32, [vp, C.c_int64, P(RequestTimes)]),
            "mcs_server_stats_get": (i32, [vp, P(ServerStats)]),
            "mcs_session_profile": (i32, [vp, i32, i32]),
            "mcs_session_profile_read": (i32, [vp, i32, P(Profile)]),
            "mcs_load_gicp_keyframes": (i32, [vp, i32, P(VoxelDesc), P(vp), P(i32)]),
            "mcs_create_keyframe_map": (i32, [vp, i32, P(GridDesc), P(i32)]),
            "mcs_append_keyframe": (i32, [vp, i32, P(GridDesc), vp, P(i32)]),
            "mcs_session_add_keyframe": (i32, [vp, i32, P(i32)]),
            "mcs_filter_step_gicp": (i32, [vp, i32, vp, vp, i32, vp, P(StepParams)]),
            "mcs_filter_step_gicp_dev": (i32, [vp, i32, vp, vp, i32, vp, P(StepParams), vp]),
            "mcs_get_gicp_system": (i32, [vp, i32, vp, vp]),
            "mcs_session_info": (i32, [vp, i32, P(i32), P(i32), P(i32), P(i32)]),
            "mcs_gather_floor_dev": (i32, [vp, i32, vp, i32, P(StepParams), vp]),
            "mcs_measure_issue_rates": (i32, [vp, P(C.c_double), i32]),
            "mcs_filter_step_noalloc": (i32, [vp, i32, i32, vp, vp, vp, vp, vp, vp, i32, vp,
                                              P(StepParams), vp, vp]),
            "mcs_session_trace": (i32, [vp, i32, i32]),
            "mcs_get_pass_trace": (i32, [vp, i32, i32, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != MCS_OK:
        raise McsError(status, mcs_last_error())
    return status


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a, shape):
    return np.ascontiguousarray(a, dtype=np.float32).reshape(shape)


# ---------------------------------------------------------------------------
# The C ABI, one function per entry point
# ---------------------------------------------------------------------------

def mcs_version():
    return lib().mcs_version().decode()


def mcs_last_error():
    return lib().mcs_last_error().decode()


def mcs_create(device=0, hbm_budget_bytes=0):
    ctx = C.c_void_p()
    _check(lib().mcs_create(int(device), int(hbm_budget_bytes), C.byref(ctx)))
    return ctx


def mcs_destroy(ctx):
    _check(lib().mcs_destroy(ctx))


def mcs_memory_in_use(ctx):
    v = C.c_uint64()
    _check(lib().mcs_memory_in_use(ctx, C.byref(v)))
    return v.value


def grid_desc(dims, origin, res, dtype=GRID_FP32):
    d = GridDesc()
    d.nx, d.ny, d.nz = (int(v) for v in dims)
    for a in range(3):
        d.origin[a] = float(origin[a])
    d.res = float(res)
    d.dtype = int(dtype)
    return d


def mcs_init_map(ctx, desc, values):
    """values: (nz, ny, nx) or flat FP32, x fastest."""
    v = _f32(values, (-1,))
    mid = C.c_int32()
    _check(lib().mcs_init_map(ctx, C.byref(desc), _ptr(v), C.byref(mid)))
    return mid.value


def mcs_load_keyframes(ctx, descs, values):
    K = len(descs)
    arr = (GridDesc * K)(*descs)
    keep = [_f32(v, (-1,)) for v in values]
    ptrs = (C.c_void_p * K)(*[k.ctypes.data for k in keep])
    mid = C.c_int32()
    _check(lib().mcs_load_keyframes(ctx, K, arr, ptrs, C.byref(mid)))
    return mid.value


def voxel_desc(dims, origin, edge):
    d = VoxelDesc()
    d.nx, d.ny, d.nz = (int(v) for v in dims)
    for a in range(3):
        d.origin[a] = float(origin[a])
    d.edge = float(edge)
    return d


def mcs_load_gicp_keyframes(ctx, descs, voxels):
    """descs: VoxelDesc per keyframe; voxels: per keyframe (nz, ny, nx, 12) FP32."""
    K = len(descs)
    arr = (VoxelDesc * K)(*descs)
    keep = [_f32(v, (-1,)) for v in voxels]
    ptrs = (C.c_void_p * K)(*[k.ctypes.data for k in keep])
    mid = C.c_int32()
    _check(lib().mcs_load_gicp_keyframes(ctx, K, arr, ptrs, C.byref(mid)))
    return mid.value


def mcs_filter_step_gicp(ctx, sid, mu, cov, params, noise=None):
    m = _f32(mu, (-1, 3))
    c = _f32(cov, (-1, 6))
    n = None if noise is None else _f32(noise, (-1, 6))
    p = params if isinstance(params, StepParams) else step_params(params)
    _check(lib().mcs_filter_step_gicp(ctx, int(sid), _ptr(m), _ptr(c), m.shape[0], _ptr(n), C.byref(p)))


def mcs_filter_step_gicp_dev(ctx, sid, mu_dev_ptr, cov_dev_ptr, M, params, noise_dev_ptr=None,
                             stream=None):
    p = params if isinstance(params, StepParams) else step_params(params)
    _check(lib().mcs_filter_step_gicp_dev(
        ctx, int(sid), C.c_void_p(int(mu_dev_ptr)), C.c_void_p(int(cov_dev_ptr)), int(M),
        None if noise_dev_ptr is None else C.c_void_p(int(noise_dev_ptr)), C.byref(p),
        None if stream is None else C.c_void_p(int(stream))))


def mcs_get_gicp_system(ctx, sid, N):
    """(H (N, 21) upper triangle row-major, b (N, 6)) of the last stepping pass."""
    H = np.empty((N, 21), np.float32)
    b = np.empty((N, 6), np.float32)
    _check(lib().mcs_get_gicp_system(ctx, int(sid), _ptr(H), _ptr(b)))
    return H, b


def mcs_create_keyframe_map(ctx, K_cap, desc):
    mid = C.c_int32()
    _check(lib().mcs_create_keyframe_map(ctx, int(K_cap), C.byref(desc), C.byref(mid)))
    return mid.value


def mcs_append_keyframe(ctx, map_id, desc, values):
    v = _f32(values, (-1,))
    k = C.c_int32()
    _check(lib().mcs_append_keyframe(ctx, int(map_id), C.byref(desc), _ptr(v), C.byref(k)))
    return k.value


def mcs_session_add_keyframe(ctx, sid):
    k = C.c_int32()
    _check(lib().mcs_session_add_keyframe(ctx, int(sid), C.byref(k)))
    return k.value


def mcs_release_map(ctx, map_id):
    _check(lib().mcs_release_map(ctx, int(map_id)))


def mcs_session_create(ctx, map_id, poses, M_max, kf_poses=None):
    p = _f32(poses, (-1, 7))
    kf = None if kf_poses is None else _f32(kf_poses, (-1,))
    sid = C.c_int32()
    _check(lib().mcs_session_create(ctx, int(map_id), p.shape[0], int(M_max), _ptr(p), _ptr(kf),
                                    C.byref(sid)))
    return sid.value


def mcs_session_destroy(ctx, sid):
    _check(lib().mcs_session_destroy(ctx, int(sid)))


def mcs_session_bytes(ctx, map_id, N, M_max):
    v = C.c_uint64()
    _check(lib().mcs_session_bytes(ctx, int(map_id), int(N), int(M_max), C.byref(v)))
    return v.value


def mcs_set_particles(ctx, sid, poses=None, logw=None, kf_poses=None):
    p = None if poses is None else _f32(poses, (-1, 7))
    w = None if logw is None else np.ascontiguousarray(logw, dtype=np.float64)
    kf = None if kf_poses is None else _f32(kf_poses, (-1,))
    _check(lib().mcs_set_particles(ctx, int(sid), _ptr(p), _ptr(w), _ptr(kf)))


def step_params(d):
    """StepParams from a dict (keys named as the struct fields)."""
    p = StepParams()
    p.iters = int(d.get("iters", 1))
    p.alpha_t = d["alpha_t"]
    p.alpha_r = d["alpha_r"]
    p.rho_max = d["rho_max"]
    p.phi_max = d["phi_max"]
    p.eps = d["eps"]
    p.beta = d.get("beta", 1.0)
    p.oob = int(d.get("oob", OOB_FLOOR))
    p.post_eval = int(bool(d.get("post_eval", False)))
    p.resample = int(d.get("resample", RESAMPLE_ALWAYS))
    p.ess_frac = float(d.get("ess_frac", 0.5))
    p.u = float(d.get("u", 0.5))
    dT = d.get("delta_T")
    p.predict = int(dT is not None)
    dT = dT if dT is not None else (0, 0, 0, 1, 0, 0, 0)
    for c in range(7):
        p.delta_T[c] = float(dT[c])
    p.n_neighbors = int(d.get("n_neighbors", 4))
    p.kf_update = int(d.get("kf_update", KF_FIXED))
    p.n_recent = int(d.get("n_recent", p.n_neighbors))
    p.noise_mode = int(d.get("noise_mode", NOISE_INPUT))
    p.rng_seed = int(d.get("rng_seed", 0)) & (2**64 - 1)
    p.rng_frame = int(d.get("rng_frame", 0)) & (2**64 - 1)
    sig = d.get("noise_sigma", (0.0,) * 6)
    for c in range(6):
        p.noise_sigma[c] = float(sig[c])
    p.prune_post = float(d.get("prune_post", 1e-8))
    p.prune_lik = float(d.get("prune_lik", 1e-16))
    return p


def mcs_filter_step(ctx, sid, scan, params, noise=None):
    s = _f32(scan, (-1, 3))
    n = None if noise is None else _f32(noise, (-1, 6))
    p = params if isinstance(params, StepParams) else step_params(params)
    _check(lib().mcs_filter_step(ctx, int(sid), _ptr(s), s.shape[0], _ptr(n), C.byref(p)))


def mcs_filter_step_dev(ctx, sid, scan_dev_ptr, M, params, noise_dev_ptr=None, stream=None):
    """Device pointers (ints, e.g. torch tensor .data_ptr()) and an optional hipStream_t."""
    p = params if isinstance(params, StepParams) else step_params(params)
    _check(lib().mcs_filter_step_dev(ctx, int(sid), C.c_void_p(int(scan_dev_ptr)), int(M),
                                     None if noise_dev_ptr is None else C.c_void_p(int(noise_dev_ptr)),
                                     C.byref(p), None if stream is None else C.c_void_p(int(stream))))


NOALLOC_MAX_PARTICLES, NOALLOC_MAX_POINTS = 262144, 16384


def mcs_filter_step_noalloc(ctx, map_id, N, pose_dev, logw_dev, loglik_dev, grad_dev, parents_dev,
                            scan_dev, M, params, noise_dev=None, stats_dev=None, stream=None):
    """Allocation-free step on caller device memory (pointers as ints)."""
    p = params if isinstance(params, StepParams) else step_params(params)
    v = lambda x: None if x is None else C.c_void_p(int(x))  # noqa: E731
    _check(lib().mcs_filter_step_noalloc(ctx, int(map_id), int(N), v(pose_dev), v(logw_dev),
                                         v(loglik_dev), v(grad_dev), v(parents_dev), v(scan_dev),
                                         int(M), v(noise_dev), C.byref(p), v(stats_dev), v(stream)))


def mcs_gather_floor_dev(ctx, sid, scan_dev_ptr, M, params, stream=None):
    """Gather-floor passes over the session's poses (measurement aid)."""
    p = params if isinstance(params, StepParams) else step_params(params)
    _check(lib().mcs_gather_floor_dev(ctx, int(sid), C.c_void_p(int(scan_dev_ptr)), int(M), C.byref(p),
                                      None if stream is None else C.c_void_p(int(stream))))


RATE_CLASSES = ("fp32_fma", "fp64_fma", "fp64_unary", "int24", "trans", "fp32_fp64")


def mcs_measure_issue_rates(ctx):
    """VALU lane-operations per second by instruction class (measurement aid)."""
    r = (C.c_double * len(RATE_CLASSES))()
    _check(lib().mcs_measure_issue_rates(ctx, r, len(RATE_CLASSES)))
    return {k: float(r[i]) for i, k in enumerate(RATE_CLASSES)}


def mcs_session_info(ctx, sid):
    """Sizes of a session: dict(N, K, M_max, last_nb)."""
    v = [C.c_int32() for _ in range(4)]
    _check(lib().mcs_session_info(ctx, int(sid), *[C.byref(x) for x in v]))
    return dict(N=v[0].value, K=v[1].value, M_max=v[2].value, last_nb=v[3].value)


def _sizes(ctx, sid, N, K=None):
    """Output sizes from the session itself; N and K given by the caller must match."""
    info = mcs_session_info(ctx, sid)
    if N is not None and int(N) != info["N"]:
        raise McsError(MCS_EINVAL, "session %d has N=%d, asked for %d" % (sid, info["N"], N))
    if K is not None and int(K) != info["K"]:
        raise McsError(MCS_EINVAL, "session %d has K=%d, asked for %d" % (sid, info["K"], K))
    return info


def mcs_get_particles(ctx, sid, N=None, K=None, poses=True, logw=True, parents=True, loglik=True,
                      grad=True, kf_poses=False, stats=True):
    info = _sizes(ctx, sid, N, K)
    N, K = info["N"], info["K"]
    out = {}
    P = np.empty((N, 7), np.float32) if poses else None
    W = np.empty(N, np.float64) if logw else None
    A = np.empty(N, np.int32) if parents else None
    Lk = np.empty(N, np.float32) if loglik else None
    G = np.empty((N, 6), np.float32) if grad else None
    KF = np.empty((N, K, 7), np.float32) if (kf_poses and K > 0) else None
    st = StepStats()
    _check(lib().mcs_get_particles(ctx, int(sid), _ptr(P), _ptr(W), _ptr(A), _ptr(Lk), _ptr(G),
                                   _ptr(KF), C.byref(st) if stats else None))
    out.update(poses=P, logw=W, parents=A, loglik=Lk, grad=G, kf_poses=KF)
    if stats:
        out["stats"] = dict(lse=st.lse, ess=st.ess, resampled=bool(st.resampled), best=st.best,
                            best_pose=np.array(st.best_pose[:], np.float32),
                            degenerate=bool(st.degenerate), pruned=int(st.pruned))
    return out


def mcs_session_trace(ctx, sid, max_passes):
    _check(lib().mcs_session_trace(ctx, int(sid), int(max_passes)))


def mcs_get_pass_trace(ctx, sid, pass_):
    """Pass `pass_` of the last traced step: dict(poses (N, 7), loglik (N,), grad (N, 6))."""
    N = mcs_session_info(ctx, sid)["N"]
    P = np.empty((N, 7), np.float32)
    Lk = np.empty(N, np.float32)
    G = np.empty((N, 6), np.float32)
    _check(lib().mcs_get_pass_trace(ctx, int(sid), int(pass_), _ptr(P), _ptr(Lk), _ptr(G)))
    return dict(poses=P, loglik=Lk, grad=G)


def mcs_session_sync(ctx, sid):
    _check(lib().mcs_session_sync(ctx, int(sid)))


def mcs_session_stream(ctx, sid):
    s = C.c_void_p()
    _check(lib().mcs_session_stream(ctx, int(sid), C.byref(s)))
    return s.value


def mcs_session_profile(ctx, sid, enable=True):
    _check(lib().mcs_session_profile(ctx, int(sid), int(bool(enable))))


def mcs_session_profile_read(ctx, sid):
    p = Profile()
    _check(lib().mcs_session_profile_read(ctx, int(sid), C.byref(p)))
    return {f: getattr(p, f) for f, _ in Profile._fields_}


def mcs_get_neighbors(ctx, sid, N=None, n_nb=None):
    info = _sizes(ctx, sid, N)
    if n_nb is not None and int(n_nb) != info["last_nb"]:
        raise McsError(MCS_EINVAL, "session used %d neighbours, asked for %d" % (info["last_nb"], n_nb))
    out = np.empty((info["N"], info["last_nb"]), np.int32)
    k = C.c_int32()
    _check(lib().mcs_get_neighbors(ctx, int(sid), _ptr(out), C.byref(k)))
    if k.value != info["last_nb"]:
        raise McsError(MCS_EINVAL, "neighbour count changed from %d to %d" % (info["last_nb"], k.value))
    return out


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------

def mcs_server_create(ctx, mode=SERVE_BATCHED, dtype=GRID_FP16, oob=OOB_FLOOR, max_batch=64,
                      max_items=0):
    s = C.c_void_p()
    _check(lib().mcs_server_create(ctx, int(mode), int(dtype), int(oob), int(max_batch),
                                   int(max_items), C.byref(s)))
    return s


def mcs_server_destroy(srv):
    _check(lib().mcs_server_destroy(srv))


def mcs_server_submit(srv, sid, scan_dev_ptr, M, params, noise_dev_ptr=None):
    p = params if isinstance(params, StepParams) else step_params(params)
    rid = C.c_int64()
    _check(lib().mcs_server_submit(srv, int(sid), C.c_void_p(int(scan_dev_ptr)), int(M),
                                   None if noise_dev_ptr is None else C.c_void_p(int(noise_dev_ptr)),
                                   C.byref(p), C.byref(rid)))
    return rid.value


def mcs_server_drain(srv):
    _check(lib().mcs_server_drain(srv))


def mcs_server_times(srv, rid):
    t = RequestTimes()
    _check(lib().mcs_server_times(srv, C.c_int64(int(rid)), C.byref(t)))
    return {f: getattr(t, f) for f, _ in RequestTimes._fields_}


def mcs_server_stats_get(srv):
    s = ServerStats()
    _check(lib().mcs_server_stats_get(srv, C.byref(s)))
    return {f: getattr(s, f) for f, _ in ServerStats._fields_ if f != "pad"}
