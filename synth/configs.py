"""The synthetic workloads the filter is run, tested and measured on.

Each builder returns a plain dict of numpy arrays and scalars.  Seeds are fixed
per workload (scene = 1000 + workload number, particles = scene + 1, resampling
offsets = scene + 2, prediction noise = scene + 3) and every builder takes an
optional seed override.

Workloads (sizes as named; ``small`` variants keep the same structure at sizes
the FP64 oracle finishes in seconds):

* ``box_room``   -- N = 1,024 particles, M = 512 points, 128^3 grid at 0.2 m:
  20 random boxes on a floor plane in a 25.6 m cube.  One gradient-guided step,
  weight normalisation and an always-on systematic resample.
* ``corridors``  -- N = 100,000, M = 2,048 (32 rings x 64 azimuths, range <= 60 m),
  512 x 512 x 128 grid at 0.2 m over a 102.4 x 102.4 x 25.6 m corridor maze with
  boxes; a 200-frame smooth trajectory, 3 gradient passes per frame, resample
  when ESS < N/2.
* ``keyframes``  -- K = 64 keyframes (16,384 points each) voxelised into local
  128^3 grids; N = 50,000 particles, each with its own pose per keyframe;
  M = 2,048; 4 nearest keyframes per particle.
* ``serving``    -- many concurrent sessions with their own maps, particle
  counts and scan sizes.

Scans come in a spinning LiDAR's firing order (all rings at one azimuth, then
the next azimuth).  Particles start from a Gaussian around the
true pose: translation N(0, 0.5^2 I) m per axis and a body-frame rotation
vector N(0, (5 deg)^2 I).
"""

import math

import numpy as np

from . import geometry as geo
from .rng import splitmix64_uniforms
from .scene import Scene

GRID_FP32, GRID_FP16, GRID_BF16 = 0, 1, 2


# ---------------------------------------------------------------------------
# Scans, particles and step parameters
# ---------------------------------------------------------------------------

def f32(x):
    """x rounded to the nearest FP32 value.  Grid geometry (voxel edge,
    origins) crosses the C ABI as FP32, so the inputs use values that FP32
    holds exactly: both the library and the FP64 oracle then see the same
    numbers."""
    return float(np.float32(x))


def lidar_scan(scene, t, q, elevations_deg, n_az, rmax, noise_sigma, rng, el_range=None,
               column_major=True):
    """Ray-cast a scan of rings x azimuths from pose (t, q); returns (M, 3) FP32, sensor frame.

    Points come in the firing order of a spinning LiDAR: every ring at one
    azimuth, then the next azimuth (column_major=False: ring by ring).
    Rays that miss (nothing within ``rmax`` inside the volume) are re-drawn in
    place from a seeded stream of directions with uniform azimuth and uniform
    elevation in ``el_range``, so the scan always has exactly
    len(elevations) * n_az points.
    """
    R = geo.quat_to_matrix(q)
    els = np.radians(np.asarray(elevations_deg, dtype=np.float64))
    az = 2.0 * np.pi * np.arange(n_az) / n_az
    E, A = np.meshgrid(els, az, indexing="ij")
    if column_major:
        E, A = E.T, A.T
    E, A = E.reshape(-1), A.reshape(-1)
    if el_range is None:
        el_range = (els.min(), els.max())
    else:
        el_range = tuple(np.radians(el_range))
    dirs_s = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)
    rng_dist = scene.raycast(t, dirs_s @ R.T, rmax)
    for _ in range(1000):
        miss = ~np.isfinite(rng_dist)
        if not miss.any():
            break
        k = int(miss.sum())
        a = rng.uniform(0.0, 2.0 * np.pi, k)
        e = rng.uniform(el_range[0], el_range[1], k)
        d_new = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)], -1)
        dirs_s[miss] = d_new
        rng_dist[miss] = scene.raycast(t, d_new @ R.T, rmax)
    else:
        raise RuntimeError("lidar_scan: could not find hits for every ray")
    noisy = rng_dist + rng.normal(0.0, noise_sigma, rng_dist.shape)
    pts_sensor = dirs_s * noisy[:, None]
    return pts_sensor.astype(np.float32)


def gaussian_particles(t_true, q_true, n, sigma_t, sigma_r_deg, rng):
    """(n, 7) FP32 poses [tx ty tz qw qx qy qz] around a true pose (q.w >= 0)."""
    t = np.asarray(t_true)[None, :] + rng.normal(0.0, sigma_t, (n, 3))
    phi = rng.normal(0.0, math.radians(sigma_r_deg), (n, 3))
    q = geo.quat_mul(np.asarray(q_true)[None, :], geo.quat_from_axis_angle(phi))
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    q = np.where(q[:, :1] < 0, -q, q)
    return np.concatenate([t, q], axis=1).astype(np.float32)


def step_params(scan, grid_h, sigma, eps=1e-3, iters=1):
    """Gradient-step constants from the diagonal preconditioner reading.

    A Gaussian likelihood of width sigma has curvature ~1/sigma^2 per point, so
    the translation gain is sigma^2/M; the rotation gain divides by the mean
    squared lever arm r2 = mean |p_j|^2.  Each block is clamped per pass to
    half a voxel of motion (rotation: half a voxel at the RMS range).
    """
    p = np.asarray(scan, dtype=np.float64)
    M = p.shape[0]
    r2 = float(np.mean(np.sum(p * p, axis=1)))
    r_rms = math.sqrt(r2)
    return dict(
        iters=int(iters),
        alpha_t=float(np.float32(sigma * sigma / M)),
        alpha_r=float(np.float32(sigma * sigma / (M * r2))),
        rho_max=float(np.float32(0.5 * grid_h)),
        phi_max=float(np.float32(0.5 * grid_h / r_rms)),
        eps=float(np.float32(eps)),
        beta=1.0,
    )


def random_yaw_pose(rng, lo, hi, z, clearance_fn, min_clear):
    for _ in range(10000):
        xy = rng.uniform(lo, hi, 2)
        t = np.array([xy[0], xy[1], z])
        if clearance_fn(t) > min_clear:
            q = geo.quat_yaw(rng.uniform(0.0, 2.0 * np.pi))
            return t, q
    raise RuntimeError("no free pose found")


# ---------------------------------------------------------------------------
# box_room: 20 boxes + floor in a 25.6 m cube
# ---------------------------------------------------------------------------

def box_room_scene(rng, n_boxes=20, size=25.6, floor_z=1.0):
    sides = rng.uniform(0.5, 4.0, (n_boxes, 3))
    centres = rng.uniform(2.0, size - 2.0, (n_boxes, 2))
    lo = np.stack([centres[:, 0] - sides[:, 0] / 2, centres[:, 1] - sides[:, 1] / 2,
                   np.full(n_boxes, floor_z)], -1)
    hi = np.stack([centres[:, 0] + sides[:, 0] / 2, centres[:, 1] + sides[:, 1] / 2,
                   floor_z + sides[:, 2]], -1)
    return Scene(lo, hi, [floor_z], [0.0, 0.0, 0.0], [size, size, size])


def box_room(N=1024, seed=1001, grid_n=128, h=0.2, sigma=0.1, n_rings=8, n_az=64,
             grid_dtype=GRID_FP32):
    """The single-step box-room workload (N particles, n_rings x n_az point scan)."""
    h = f32(h)
    rng = np.random.default_rng(seed)
    size = grid_n * h
    scene = box_room_scene(rng, size=size)
    t_true, q_true = random_yaw_pose(rng, 2.0, size - 2.0, 2.5, scene.distance, 1.0)
    scan = lidar_scan(scene, t_true, q_true, np.linspace(-20.0, 10.0, n_rings), n_az,
                      rmax=2.0 * size, noise_sigma=0.02, rng=rng)
    grid = scene.likelihood_grid((grid_n,) * 3, (0.0, 0.0, 0.0), h, sigma)
    prng = np.random.default_rng(seed + 1)
    poses = gaussian_particles(t_true, q_true, N, 0.5, 5.0, prng)
    params = step_params(scan, h, sigma, iters=1)
    return dict(
        name="box_room", grid=grid, dims=(grid_n, grid_n, grid_n), origin=(0.0, 0.0, 0.0),
        h=h, sigma=sigma, grid_dtype=grid_dtype, scan=scan, poses=poses,
        logw=np.full(N, -math.log(N)), params=params,
        u=float(splitmix64_uniforms(seed + 2, 1)[0]), t_true=t_true, q_true=q_true,
        scene=scene,
    )


# ---------------------------------------------------------------------------
# corridors: maze of wall slabs + floor/ceiling + boxes, 200-frame trajectory
# ---------------------------------------------------------------------------

def _maze_edges(rng, n, extra_frac=0.12):
    """Random spanning tree (iterative DFS) over an n x n cell lattice plus extra loops."""
    visited = np.zeros((n, n), bool)
    open_e = set()
    stack = [(int(rng.integers(n)), int(rng.integers(n)))]
    visited[stack[0]] = True
    while stack:
        i, j = stack[-1]
        nb = [(i + di, j + dj) for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1))
              if 0 <= i + di < n and 0 <= j + dj < n and not visited[i + di, j + dj]]
        if not nb:
            stack.pop()
            continue
        a = nb[int(rng.integers(len(nb)))]
        visited[a] = True
        open_e.add(frozenset(((i, j), a)))
        stack.append(a)
    all_e = [frozenset(((i, j), (i + 1, j))) for i in range(n - 1) for j in range(n)] + \
            [frozenset(((i, j), (i, j + 1))) for i in range(n) for j in range(n - 1)]
    closed = [e for e in all_e if e not in open_e]
    for k in rng.permutation(len(closed))[: int(extra_frac * len(closed))]:
        open_e.add(closed[k])
    return open_e


def corridor_scene(rng, cells=19, cell=5.0, size_xy=102.4, size_z=25.6, floor_z=1.0,
                   ceil_z=4.0, wall=0.3, n_boxes=80):
    off = 0.5 * (size_xy - cells * cell)
    open_e = _maze_edges(rng, cells)
    lo, hi = [], []
    hw = 0.5 * wall
    # Walls between lattice neighbours that are not connected.
    for i in range(cells):
        for j in range(cells):
            if i + 1 < cells and frozenset(((i, j), (i + 1, j))) not in open_e:
                x = off + (i + 1) * cell
                lo.append([x - hw, off + j * cell - hw, floor_z])
                hi.append([x + hw, off + (j + 1) * cell + hw, ceil_z])
            if j + 1 < cells and frozenset(((i, j), (i, j + 1))) not in open_e:
                y = off + (j + 1) * cell
                lo.append([off + i * cell - hw, y - hw, floor_z])
                hi.append([off + (i + 1) * cell + hw, y + hw, ceil_z])
    # Perimeter.
    a, b = off, off + cells * cell
    lo += [[a - hw, a - hw, floor_z], [b - hw, a - hw, floor_z], [a - hw, a - hw, floor_z],
           [a - hw, b - hw, floor_z]]
    hi += [[a + hw, b + hw, ceil_z], [b + hw, b + hw, ceil_z], [b + hw, a + hw, ceil_z],
           [b + hw, b + hw, ceil_z]]
    n_walls = len(lo)
    # Boxes against the walls of random cells: offset 1.2-1.9 m from the cell centre.
    for _ in range(n_boxes):
        ci, cj = rng.integers(cells, size=2)
        c = np.array([off + (ci + 0.5) * cell, off + (cj + 0.5) * cell])
        side = rng.uniform(0.4, 1.2, 3)
        ang = rng.uniform(0, 2 * np.pi)
        r = rng.uniform(1.2, 0.5 * cell - 0.6)
        p = c + r * np.array([math.cos(ang), math.sin(ang)])
        lo.append([p[0] - side[0] / 2, p[1] - side[1] / 2, floor_z])
        hi.append([p[0] + side[0] / 2, p[1] + side[1] / 2, floor_z + side[2]])
    sc = Scene(lo, hi, [floor_z, ceil_z], [0.0, 0.0, 0.0], [size_xy, size_xy, size_z])
    sc.maze = dict(cells=cells, cell=cell, off=off, open=open_e, n_walls=n_walls)
    return sc


def _catmull_rom(P, samples_per_seg=64):
    P = np.asarray(P, dtype=np.float64)
    P = np.vstack([2 * P[0] - P[1], P, 2 * P[-1] - P[-2]])
    out = []
    s = np.linspace(0.0, 1.0, samples_per_seg, endpoint=False)[:, None]
    for k in range(1, len(P) - 2):
        p0, p1, p2, p3 = P[k - 1], P[k], P[k + 1], P[k + 2]
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * s + (2 * p0 - 5 * p1 + 4 * p2 - p3) * s ** 2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * s ** 3))
    out.append(P[-2][None, :])
    return np.vstack(out)


def maze_trajectory(scene, rng, n_frames=200, step_lo=0.5, step_hi=1.0, z=2.5):
    """Smooth seeded path through connected maze cells; returns (n_frames, 3), (n_frames, 4)."""
    mz = scene.maze
    n, cell, off, open_e = mz["cells"], mz["cell"], mz["off"], mz["open"]
    need = n_frames * step_hi * 1.3
    cur = (int(rng.integers(n)), int(rng.integers(n)))
    path, prev, length = [cur], None, 0.0
    while length < need:
        nb = [(cur[0] + d[0], cur[1] + d[1]) for d in ((1, 0), (-1, 0), (0, 1), (0, -1))]
        nb = [c for c in nb if 0 <= c[0] < n and 0 <= c[1] < n and frozenset((cur, c)) in open_e]
        fwd = [c for c in nb if c != prev]
        nxt = (fwd or nb)[int(rng.integers(len(fwd or nb)))]
        prev, cur = cur, nxt
        path.append(cur)
        length += cell
    way = np.array([[off + (i + 0.5) * cell, off + (j + 0.5) * cell] for i, j in path])
    curve = _catmull_rom(way)
    seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    steps = rng.uniform(step_lo, step_hi, n_frames - 1)
    s = np.concatenate([[0.0], np.cumsum(steps)]) + 0.5 * cell
    s = np.minimum(s, arc[-1] - 1e-6)
    xy = np.stack([np.interp(s, arc, curve[:, 0]), np.interp(s, arc, curve[:, 1])], -1)
    tang = np.stack([np.interp(s + 0.05, arc, curve[:, 0]) - xy[:, 0],
                     np.interp(s + 0.05, arc, curve[:, 1]) - xy[:, 1]], -1)
    yaw = np.arctan2(tang[:, 1], tang[:, 0])
    t = np.concatenate([xy, np.full((n_frames, 1), z)], axis=1)
    return t, geo.quat_yaw(yaw)


def frame_scans(scene, t_traj, q_traj, els, n_az, rmax, noise, seed, workers=8):
    """One scan per trajectory frame; frame f draws from its own stream (seed, 7, f)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(f):
        return lidar_scan(scene, t_traj[f], q_traj[f], els, n_az, rmax, noise,
                          np.random.default_rng([seed, 7, f]))

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return np.stack(list(ex.map(one, range(len(t_traj)))))


def relative_motion(t0, q0, t1, q1):
    """(t, q) of T0^-1 T1."""
    T0, T1 = geo.pose_matrix(t0, q0), geo.pose_matrix(t1, q1)
    return geo.matrix_to_pose(np.linalg.inv(T0) @ T1)


def corridors(N=100000, M_rings=32, n_az=64, n_frames=200, seed=1002, grid=(512, 512, 128),
              h=0.2, sigma=0.1, iters=3, ess_frac=0.5, with_noise=True, grid_dtype=GRID_FP32):
    """The paper-scale corridor workload; per-frame scans, odometry and noise."""
    h = f32(h)
    rng = np.random.default_rng(seed)
    size_xy, size_z = grid[0] * h, grid[2] * h
    scene = corridor_scene(rng, size_xy=size_xy, size_z=size_z)
    t_traj, q_traj = maze_trajectory(scene, rng, n_frames=n_frames)
    els = np.linspace(-15.0, 15.0, M_rings)
    scans = frame_scans(scene, t_traj, q_traj, els, n_az, 60.0, 0.02, seed)
    G = scene.likelihood_grid(grid, (0.0, 0.0, 0.0), h, sigma)
    # Odometry: true relative motion composed with (1 cm, 0.2 deg) noise.
    odo = np.zeros((n_frames, 7), np.float32)
    odo[0] = [0, 0, 0, 1, 0, 0, 0]
    for f in range(1, n_frames):
        dt, dq = relative_motion(t_traj[f - 1], q_traj[f - 1], t_traj[f], q_traj[f])
        dt = dt + rng.normal(0.0, 0.01, 3)
        dq = geo.quat_mul(dq, geo.quat_from_axis_angle(rng.normal(0.0, math.radians(0.2), 3)))
        dq = dq / np.linalg.norm(dq)
        odo[f] = np.concatenate([dt, dq])
    prng = np.random.default_rng(seed + 1)
    poses = gaussian_particles(t_traj[0], q_traj[0], N, 0.5, 5.0, prng)
    params = step_params(scans[0], h, sigma, iters=iters)
    params["ess_frac"] = ess_frac
    out = dict(
        name="corridors", grid=G, dims=tuple(grid), origin=(0.0, 0.0, 0.0), h=h, sigma=sigma,
        grid_dtype=grid_dtype, scans=scans, scan=scans[0], poses=poses,
        logw=np.full(N, -math.log(N)), params=params, odometry=odo,
        u=splitmix64_uniforms(seed + 2, n_frames), t_traj=t_traj, q_traj=q_traj, scene=scene,
        noise_sigma=(0.05, math.radians(1.0)), noise_seed=seed + 3,
    )
    return out


def prediction_noise(N, frame, noise_sigma, seed):
    """(N, 6) FP32 tangent-space noise [rho; phi] for one frame (seeded per frame)."""
    rng = np.random.default_rng([seed, frame])
    d = np.empty((N, 6), np.float32)
    d[:, :3] = rng.normal(0.0, noise_sigma[0], (N, 3))
    d[:, 3:] = rng.normal(0.0, noise_sigma[1], (N, 3))
    return d


# ---------------------------------------------------------------------------
# keyframes: K local grids voxelised from keyframe scans, per-particle
# keyframe poses
# ---------------------------------------------------------------------------

def keyframe_grid(points, grid_n, h, sigma, cutoff_sigmas=6.0):
    """Local likelihood grid of one keyframe in its own frame.

    G(c) = exp(-d_min^2 / 2 sigma^2), d_min the distance from voxel centre c to
    the nearest keyframe point, and 0 beyond cutoff_sigmas * sigma.  The grid
    is centred on the keyframe: origin = -grid_n h / 2 on every axis.
    """
    from scipy.spatial import cKDTree
    half = 0.5 * grid_n * h
    pts = np.asarray(points, np.float64)
    pts = pts[np.all(np.abs(pts) < half + cutoff_sigmas * sigma, axis=1)]
    G = np.zeros((grid_n, grid_n, grid_n), np.float32)
    if pts.shape[0] == 0:
        return G
    rc = cutoff_sigmas * sigma
    # Candidate voxels: those within rc of some point's voxel (dilation of the occupancy).
    r = int(math.ceil(rc / h)) + 1
    idx = np.floor((pts + half) / h).astype(np.int64)
    occ = np.zeros((grid_n + 2 * r,) * 3, bool)
    ii = np.clip(idx + r, 0, grid_n + 2 * r - 1)
    occ[ii[:, 2], ii[:, 1], ii[:, 0]] = True
    from scipy.ndimage import binary_dilation
    cand = binary_dilation(occ, iterations=r)[r:r + grid_n, r:r + grid_n, r:r + grid_n]
    kz, ky, kx = np.nonzero(cand)
    centres = np.stack([kx, ky, kz], -1) * h - half + 0.5 * h
    d, _ = cKDTree(pts).query(centres, distance_upper_bound=rc)
    ok = np.isfinite(d)
    with np.errstate(under="ignore"):
        G[kz[ok], ky[ok], kx[ok]] = np.exp(-d[ok] ** 2 / (2.0 * sigma * sigma)).astype(np.float32)
    return G


def keyframes(N=50000, K=64, kf_points=16384, M_rings=32, n_az=64, grid_n=128, h=0.2,
              sigma=0.1, n_nb=4, seed=1003, kf_drift=(0.05, 0.5), ambiguous=False,
              out_and_back=False, grid_dtype=GRID_FP32, workers=8, gicp=False, vox_n=64,
              vox_edge=0.4):
    """Keyframe-map workload: K keyframes along a corridor trajectory.

    Each keyframe scan (kf_points rays, 64 rings over [-15, 15] deg) is
    voxelised into a local grid_n^3 grid at h in the keyframe frame.  The
    current frame is the trajectory frame just after the last keyframe; its scan
    has M_rings x n_az points.  Every particle carries its own pose per keyframe:
    the true keyframe pose composed with N(0, drift) noise (metres, degrees).
    With ambiguous=True the scene is a row of identical rooms (translated copies).
    With out_and_back=True the path turns round half way and retraces itself, so
    the current frame is back at the start: its neighbour keyframes include the
    oldest ones (a loop) as well as the newest.
    With gicp=True each keyframe is also voxelised into vox_n^3 voxel
    Gaussians of edge vox_edge centred on the keyframe (synth.gicp), and the
    current scan gets per-point covariances (10 nearest neighbours).
    """
    h, vox_edge = f32(h), f32(vox_edge)     # the origins below are then FP32 values too
    rng = np.random.default_rng(seed)
    if ambiguous:
        scene = repeated_rooms_scene(rng)
        n_frames = 3 * K + 1
        t_traj, q_traj = rooms_trajectory(scene, rng, n_frames)
    else:
        scene = corridor_scene(rng)
        n_frames = 3 * K + 1
        t_traj, q_traj = maze_trajectory(scene, rng, n_frames=n_frames)
    if out_and_back:
        half = (n_frames + 1) // 2
        t_traj = np.concatenate([t_traj[:half], t_traj[:n_frames - half][::-1]])
        flip = geo.quat_yaw(np.full(n_frames - half, math.pi))
        q_back = np.stack([geo.quat_mul(q, flip[0]) for q in q_traj[:n_frames - half][::-1]])
        q_traj = np.concatenate([q_traj[:half], q_back])
    kf_frames = np.arange(K) * 3
    cur = n_frames - 1
    n_kf_rings = 64
    kf_az = max(1, kf_points // n_kf_rings)
    els_kf = np.linspace(-15.0, 15.0, n_kf_rings)
    from concurrent.futures import ThreadPoolExecutor

    from . import gicp as gicp_inputs
    vox_origin = -0.5 * vox_n * vox_edge

    def kf_one(k):
        f = kf_frames[k]
        pts = lidar_scan(scene, t_traj[f], q_traj[f], els_kf, kf_az, 60.0, 0.02,
                         np.random.default_rng([seed, 11, k]))
        vox = (gicp_inputs.voxel_gaussians(pts, (vox_n,) * 3, (vox_origin,) * 3, vox_edge)
               if gicp else None)
        return keyframe_grid(pts, grid_n, h, sigma), vox

    with ThreadPoolExecutor(max_workers=workers) as ex:
        made = list(ex.map(kf_one, range(K)))
    grids = np.stack([m[0] for m in made])
    scan = lidar_scan(scene, t_traj[cur], q_traj[cur], np.linspace(-15.0, 15.0, M_rings), n_az,
                      60.0, 0.02, np.random.default_rng([seed, 12]))
    prng = np.random.default_rng(seed + 1)
    poses = gaussian_particles(t_traj[cur], q_traj[cur], N, 0.5, 5.0, prng)
    kf = np.empty((N, K, 7), np.float32)
    for k in range(K):
        f = kf_frames[k]
        kf[:, k, :] = gaussian_particles(t_traj[f], q_traj[f], N, kf_drift[0], kf_drift[1], prng)
    origin = -0.5 * grid_n * h
    params = step_params(scan, h, sigma, iters=3)
    params["n_neighbors"] = n_nb
    extra = {}
    if gicp:
        extra = dict(vox=np.stack([m[1] for m in made]), vox_dims=(vox_n,) * 3,
                     vox_origins=np.full((K, 3), vox_origin), vox_edge=vox_edge,
                     scan_cov=gicp_inputs.point_covariances(scan))
    return dict(
        **extra,
        name="keyframes", grids=grids, dims=(grid_n,) * 3, origins=np.full((K, 3), origin),
        h=h, sigma=sigma, grid_dtype=grid_dtype, scan=scan, poses=poses, kf_poses=kf,
        logw=np.full(N, -math.log(N)), params=params, u=float(splitmix64_uniforms(seed + 2, 1)[0]),
        t_traj=t_traj, q_traj=q_traj, kf_frames=kf_frames, cur=cur, scene=scene,
    )


def repeated_rooms_scene(rng, rooms=6, room=8.0, size_xy=102.4, size_z=25.6, floor_z=1.0,
                         ceil_z=4.0, wall=0.3, door=1.6):
    """A row of identical rooms (translated copies) joined by doors: an ambiguous map."""
    lo, hi = [], []
    hw = 0.5 * wall
    y0, y1 = 40.0, 40.0 + room
    x0 = 0.5 * (size_xy - rooms * room)
    # Furniture of one room, copied into every room.
    furn = []
    for _ in range(5):
        side = rng.uniform(0.5, 1.5, 3)
        p = rng.uniform(1.5, room - 1.5, 2)
        furn.append((p, side))
    for r in range(rooms):
        xa = x0 + r * room
        # Long walls.
        lo += [[xa - hw, y0 - hw, floor_z], [xa - hw, y1 - hw, floor_z]]
        hi += [[xa + room + hw, y0 + hw, ceil_z], [xa + room + hw, y1 + hw, ceil_z]]
        # Cross wall with a centred door (two slabs).
        ym = 0.5 * (y0 + y1)
        lo += [[xa - hw, y0 - hw, floor_z], [xa - hw, ym + 0.5 * door, floor_z]]
        hi += [[xa + hw, ym - 0.5 * door, ceil_z], [xa + hw, y1 + hw, ceil_z]]
        for p, side in furn:
            lo.append([xa + p[0] - side[0] / 2, y0 + p[1] - side[1] / 2, floor_z])
            hi.append([xa + p[0] + side[0] / 2, y0 + p[1] + side[1] / 2, floor_z + side[2]])
    xe = x0 + rooms * room
    lo.append([xe - hw, y0 - hw, floor_z])
    hi.append([xe + hw, y1 + hw, ceil_z])
    sc = Scene(lo, hi, [floor_z, ceil_z], [0.0, 0.0, 0.0], [size_xy, size_xy, size_z])
    sc.rooms = dict(rooms=rooms, room=room, x0=x0, y0=y0, y1=y1)
    return sc


def rooms_trajectory(scene, rng, n_frames, z=2.5):
    """Straight walk along the row of rooms through the doors, 0.5-1 m per frame."""
    rm = scene.rooms
    y = 0.5 * (rm["y0"] + rm["y1"])
    x_start = rm["x0"] + 1.0
    x_end = rm["x0"] + rm["rooms"] * rm["room"] - 1.0
    steps = rng.uniform(0.5, 1.0, n_frames - 1)
    x = x_start + np.concatenate([[0.0], np.cumsum(steps)])
    # Walk back and forth along the row if the path is longer than the row.
    span = x_end - x_start
    ph = np.mod(x - x_start, 2 * span)
    xx = x_start + np.where(ph < span, ph, 2 * span - ph)
    yaw = np.where(ph < span, 0.0, np.pi)
    t = np.stack([xx, np.full(n_frames, y), np.full(n_frames, z)], -1)
    return t, geo.quat_yaw(yaw)


# ---------------------------------------------------------------------------
# serving: many concurrent sessions with their own maps
# ---------------------------------------------------------------------------

def serving_sessions(n_sessions=64, seed=1005, n_scans=8, n_lo=1000, n_hi=200000, m_lo=512,
                     m_hi=4096, sizes=(128, 256, 512), nz=128, h=0.2, sigma=0.1):
    """Per-session descriptions for the serving workload (maps are built lazily).

    Session s: grid (nx, ny, nz) with nx, ny drawn from `sizes`, FP16 storage;
    N = round(exp(U[ln n_lo, ln n_hi])); M = 64 * rings with rings ~ U{m_lo/64 .. m_hi/64};
    n_scans distinct frames along a seeded maze trajectory, cycled.
    """
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_sessions):
        nx, ny = (int(v) for v in rng.choice(sizes, 2))
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        rings = int(rng.integers(m_lo // 64, m_hi // 64 + 1))
        out.append(dict(session=s, dims=(nx, ny, nz), N=N, M=rings * 64, rings=rings,
                        seed=seed * 100 + s, n_scans=n_scans, h=h, sigma=sigma))
    return out


def serving_session_inputs(desc):
    """Map, scans, particles and step parameters of one serving session."""
    nx, ny, nz = desc["dims"]
    h, sigma = f32(desc["h"]), desc["sigma"]
    rng = np.random.default_rng(desc["seed"])
    cell = 5.0
    cx, cy = max(2, int(nx * h // cell) - 1), max(2, int(ny * h // cell) - 1)
    n_cells = min(cx, cy)
    scene = corridor_scene(rng, cells=n_cells, cell=cell, size_xy=min(nx, ny) * h,
                           size_z=nz * h, n_boxes=4 * n_cells)
    scene.volume_hi = np.array([nx * h, ny * h, nz * h])
    t_traj, q_traj = maze_trajectory(scene, rng, n_frames=desc["n_scans"] + 1)
    els = np.linspace(-15.0, 15.0, desc["rings"])
    scans = frame_scans(scene, t_traj[1:], q_traj[1:], els, 64, 60.0, 0.02, desc["seed"], workers=4)
    grid = scene.likelihood_grid((nx, ny, nz), (0.0, 0.0, 0.0), h, sigma)
    poses = gaussian_particles(t_traj[0], q_traj[0], desc["N"], 0.5, 5.0,
                               np.random.default_rng(desc["seed"] + 1))
    params = step_params(scans[0], h, sigma, iters=3)
    params["ess_frac"] = 0.5
    odo = np.zeros((desc["n_scans"], 7), np.float32)
    for f in range(desc["n_scans"]):
        dt, dq = relative_motion(t_traj[f], q_traj[f], t_traj[f + 1], q_traj[f + 1])
        odo[f] = np.concatenate([dt, dq])
    return dict(grid=grid, dims=(nx, ny, nz), origin=(0.0, 0.0, 0.0), h=h, scans=scans,
                poses=poses, params=params, odometry=odo,
                u=splitmix64_uniforms(desc["seed"] + 2, 4096))


def poisson_arrivals(rate_hz, duration_s, rng):
    """Arrival times of a Poisson process on [0, duration_s)."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.array(out)
        out.append(t)


# ---------------------------------------------------------------------------
# repeated floors: a kidnapped start over identical storeys
# ---------------------------------------------------------------------------

def repeated_floors(N=20000, floors=4, true_floor=2, n_frames=80, M_rings=8, n_az=64, seed=1006,
                    grid=(256, 256, 128), h=0.2, sigma=0.1, storey=4.0, feature_frame=0.6,
                    rmax=10.0, min_blind=10, grid_dtype=GRID_FP32):
    """A building of `floors` identical storeys (the same maze level copied every
    `storey` metres), except one box that stands only on the true floor, next
    to the path at the fraction `feature_frame` of the trajectory.  The sensor
    moves on the true floor; the particles start kidnapped: their storey is
    drawn uniformly, the rest is the true start pose with 0.3 m / 3 deg of
    spread.  Until the box comes into view every storey explains the scans
    equally well.  The range sensor reaches rmax metres."""
    h = f32(h)
    rng = np.random.default_rng(seed)
    size_xy, size_z = grid[0] * h, grid[2] * h
    cells = int(size_xy // 5.0) - 1
    level = corridor_scene(rng, cells=cells, cell=5.0, size_xy=size_xy, size_z=size_z, floor_z=1.0,
                           ceil_z=1.0 + storey - 1.0, n_boxes=4 * cells)
    lo, hi, planes = [], [], []
    for f in range(floors):
        dz = f * storey
        lo.append(level.lo + [0.0, 0.0, dz])
        hi.append(level.hi + [0.0, 0.0, dz])
        planes += [1.0 + dz, 1.0 + dz + storey - 1.0]
    z_true = 2.5 + true_floor * storey
    t_traj, q_traj = maze_trajectory(level, rng, n_frames=n_frames, z=z_true)
    # The distinguishing box: beside the path on the true floor only, at the
    # first frame from `feature_frame` on whose box no scan of the first
    # `min_blind` frames sees; `first_seen` is the first frame that does.
    els = np.linspace(-15.0, 15.0, M_rings)
    vol = ([0.0, 0.0, 0.0], [size_xy, size_xy, size_z])
    plain = Scene(np.vstack(lo), np.vstack(hi), planes, *vol)
    scans_plain = frame_scans(plain, t_traj, q_traj, els, n_az, rmax, 0.02, seed)
    base = 1.0 + true_floor * storey
    scene = None
    for cand in range(int(feature_frame * (n_frames - 1)), n_frames - 2):
        side = geo.quat_to_matrix(q_traj[cand])[:, 1]
        c = t_traj[cand, :2] + 1.2 * side[:2] / max(1e-9, np.linalg.norm(side[:2]))
        trial = Scene(np.vstack(lo + [[[c[0] - 0.35, c[1] - 0.35, base]]]),
                      np.vstack(hi + [[[c[0] + 0.35, c[1] + 0.35, base + 1.8]]]), planes, *vol)
        scans = frame_scans(trial, t_traj, q_traj, els, n_az, rmax, 0.02, seed)
        differs = [f for f in range(n_frames) if not np.array_equal(scans[f], scans_plain[f])]
        if differs and differs[0] >= min_blind:
            scene, fk, first_seen = trial, cand, differs[0]
            break
    if scene is None:
        raise ValueError("no place for the distinguishing box that stays unseen; try another seed")
    G = scene.likelihood_grid(grid, (0.0, 0.0, 0.0), h, sigma)
    odo = np.zeros((n_frames, 7), np.float32)
    odo[0] = [0, 0, 0, 1, 0, 0, 0]
    for f in range(1, n_frames):
        dt, dq = relative_motion(t_traj[f - 1], q_traj[f - 1], t_traj[f], q_traj[f])
        dt = dt + rng.normal(0.0, 0.01, 3)
        dq = geo.quat_mul(dq, geo.quat_from_axis_angle(rng.normal(0.0, math.radians(0.2), 3)))
        odo[f] = np.concatenate([dt, dq / np.linalg.norm(dq)])
    prng = np.random.default_rng(seed + 1)
    poses = gaussian_particles(t_traj[0], q_traj[0], N, 0.3, 3.0, prng)
    floor_of = prng.integers(0, floors, N)
    poses[:, 2] += ((floor_of - true_floor) * storey).astype(np.float32)
    params = step_params(scans[0], h, sigma, iters=2)
    return dict(name="repeated_floors", grid=G, dims=tuple(grid), origin=(0.0, 0.0, 0.0), h=h,
                sigma=sigma, grid_dtype=grid_dtype, scans=scans, poses=poses,
                logw=np.full(N, -math.log(N)), params=params, odometry=odo,
                u=splitmix64_uniforms(seed + 2, n_frames), t_traj=t_traj, q_traj=q_traj,
                floors=floors, true_floor=true_floor, storey=storey, feature_frame=fk,
                first_seen=first_seen,
                floor_of_start=floor_of, scene=scene)


def wide_slab(N=33000, M=300, seed=1007, n_xy=4098, h=0.05, sigma=0.1):
    """A grid whose row-by-column slab holds 2^24 or more cells (n_xy = 4098:
    4097^2 cells per slab), three samples thick, with a smooth field in [0.1,
    0.9]; particles near the far corner (cell indices near 3,800-3,900), level
    within 0.1 deg, at mid-slab height; a planar scan of radius <= 5 m."""
    h = f32(h)
    rng = np.random.default_rng(seed)
    i = np.arange(n_xy, dtype=np.float64)
    fx = np.sin(0.07 * i + 0.3)
    fy = np.cos(0.05 * i)
    fz = np.array([-0.1, 0.0, 0.1])
    grid = (0.5 + 0.3 * fy[None, :, None] * fx[None, None, :] + fz[:, None, None]).astype(np.float32)
    r = rng.uniform(0.5, 5.0, M)
    a = rng.uniform(0.0, 2.0 * np.pi, M)
    scan = np.stack([r * np.cos(a), r * np.sin(a), np.zeros(M)], axis=1).astype(np.float32)
    t = np.stack([190.0 + rng.normal(0.0, 0.5, N), 195.0 + rng.normal(0.0, 0.5, N),
                  1.5 * h + rng.normal(0.0, 0.1 * h, N)], axis=1)
    phi = rng.normal(0.0, math.radians(0.1), (N, 3))
    q = geo.quat_mul(np.asarray(geo.quat_yaw(0.7))[None, :], geo.quat_from_axis_angle(phi))
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    q = np.where(q[:, :1] < 0, -q, q)
    poses = np.concatenate([t, q], axis=1).astype(np.float32)
    return dict(name="wide_slab", grid=grid, dims=(n_xy, n_xy, 3), origin=(0.0, 0.0, 0.0), h=h,
                sigma=sigma, scan=scan, poses=poses, params=step_params(scan, h, sigma, iters=1))


def beyond_4gib(N=33000, M=300, seed=1011, n_xy=2048, n_z=34, h=0.05, sigma=0.1):
    """A grid whose FP32 records pass one buffer's 32-bit byte range (2049^2 x 35
    records of 32 B: 4.7 GB), with a smooth field in [0.1, 0.9]; half the
    particles near the top (cell layer 32, records beyond 4 GiB), half near the
    bottom (layer 2), level within 0.1 deg, at (60, 70) m; a planar scan of
    radius <= 5 m."""
    h = f32(h)
    rng = np.random.default_rng(seed)
    i = np.arange(n_xy, dtype=np.float64)
    fx = np.sin(0.07 * i + 0.3)
    fy = np.cos(0.05 * i)
    fz = 0.1 * np.cos(0.4 * np.arange(n_z, dtype=np.float64))
    grid = (0.5 + 0.3 * fy[None, :, None] * fx[None, None, :] + fz[:, None, None]).astype(np.float32)
    r = rng.uniform(0.5, 5.0, M)
    a = rng.uniform(0.0, 2.0 * np.pi, M)
    scan = np.stack([r * np.cos(a), r * np.sin(a), np.zeros(M)], axis=1).astype(np.float32)
    layer = np.where(np.arange(N) < N // 2, 32.5, 2.5)
    t = np.stack([60.0 + rng.normal(0.0, 0.5, N), 70.0 + rng.normal(0.0, 0.5, N),
                  layer * h + rng.normal(0.0, 0.1 * h, N)], axis=1)
    phi = rng.normal(0.0, math.radians(0.1), (N, 3))
    q = geo.quat_mul(np.asarray(geo.quat_yaw(0.7))[None, :], geo.quat_from_axis_angle(phi))
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    q = np.where(q[:, :1] < 0, -q, q)
    poses = np.concatenate([t, q], axis=1).astype(np.float32)
    return dict(name="beyond_4gib", grid=grid, dims=(n_xy, n_xy, n_z), origin=(0.0, 0.0, 0.0), h=h,
                sigma=sigma, scan=scan, poses=poses, params=step_params(scan, h, sigma, iters=1))
