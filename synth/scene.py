"""Analytic scenes: axis-aligned boxes plus horizontal planes.

A scene is a list of boxes ``(lo, hi)`` and horizontal planes ``z = z0``
restricted to the map volume.  Two things are built from it:

* ray-cast range scans (slab test for boxes, plane test for the planes), and
* the likelihood grid ``G(c) = exp(-d(c)^2 / (2 sigma^2))`` sampled at voxel
  centres ``origin + (i + 1/2) h`` (x fastest), where ``d`` is the exact
  Euclidean distance from the voxel centre to the nearest scene surface (inside
  a box: the distance to its nearest face), evaluated in FP64 and rounded to
  FP32.

Distances beyond ``CUTOFF`` metres are not evaluated: with sigma <= 0.1 m the
value there is below half the smallest FP32 subnormal and rounds to zero, so
the FP32 grid is the same as with the full evaluation.
"""

import numpy as np

CUTOFF = 1.6  # metres; exp(-1.6^2 / 0.02) = 2.6e-56 rounds to 0 in FP32


class Scene:
    def __init__(self, lo, hi, planes, volume_lo, volume_hi):
        self.lo = np.asarray(lo, dtype=np.float64).reshape(-1, 3)
        self.hi = np.asarray(hi, dtype=np.float64).reshape(-1, 3)
        self.planes = np.asarray(planes, dtype=np.float64).reshape(-1)
        self.volume_lo = np.asarray(volume_lo, dtype=np.float64)
        self.volume_hi = np.asarray(volume_hi, dtype=np.float64)

    # -- distance -------------------------------------------------------------
    def box_distance(self, p, b):
        """Unsigned distance from points p (..., 3) to the surface of box b."""
        q = np.maximum(self.lo[b] - p, p - self.hi[b])
        qmax = q.max(axis=-1)
        outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
        return np.where(qmax > 0.0, outside, -qmax)

    def distance(self, p):
        """Unsigned distance to the nearest surface for points p (..., 3)."""
        p = np.asarray(p, dtype=np.float64)
        d = np.full(p.shape[:-1], np.inf)
        for z0 in self.planes:
            d = np.minimum(d, np.abs(p[..., 2] - z0))
        for b in range(len(self.lo)):
            d = np.minimum(d, self.box_distance(p, b))
        return d

    # -- likelihood grid --------------------------------------------------------
    def likelihood_grid(self, dims, origin, h, sigma):
        """FP32 array of shape (nz, ny, nx): exp(-d^2/(2 sigma^2)) at voxel centres."""
        nx, ny, nz = (int(v) for v in dims)
        origin = np.asarray(origin, dtype=np.float64)
        cx = origin[0] + (np.arange(nx) + 0.5) * h
        cy = origin[1] + (np.arange(ny) + 0.5) * h
        cz = origin[2] + (np.arange(nz) + 0.5) * h
        d2 = np.full((nz, ny, nx), np.inf)
        for z0 in self.planes:
            kz = np.nonzero(np.abs(cz - z0) < CUTOFF)[0]
            if kz.size:
                dz2 = (cz[kz] - z0) ** 2
                d2[kz] = np.minimum(d2[kz], dz2[:, None, None])

        def window(c, lo, hi):
            return np.nonzero((c > lo - CUTOFF) & (c < hi + CUTOFF))[0]

        for b in range(len(self.lo)):
            lo, hi = self.lo[b], self.hi[b]
            ix, iy, iz = window(cx, lo[0], hi[0]), window(cy, lo[1], hi[1]), window(cz, lo[2], hi[2])
            if not (ix.size and iy.size and iz.size):
                continue
            x0, x1 = ix[0], ix[-1] + 1
            y0, y1 = iy[0], iy[-1] + 1
            z0_, z1 = iz[0], iz[-1] + 1
            P = np.stack(np.meshgrid(cz[z0_:z1], cy[y0:y1], cx[x0:x1], indexing="ij"), axis=-1)[..., ::-1]
            db = self.box_distance(P, b)
            sub = d2[z0_:z1, y0:y1, x0:x1]
            np.minimum(sub, db * db, out=sub)
        with np.errstate(under="ignore"):
            g = np.exp(-d2 / (2.0 * sigma * sigma))
        return g.astype(np.float32)

    # -- ray casting ------------------------------------------------------------
    def raycast(self, origin, dirs, rmax, chunk=2048):
        """Nearest hit distance along unit directions ``dirs`` (R, 3); inf if none.

        Hits outside the map volume or beyond ``rmax`` count as misses.
        """
        d = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
        out = np.empty(d.shape[0])
        for s0 in range(0, d.shape[0], chunk):
            out[s0:s0 + chunk] = self._raycast(origin, d[s0:s0 + chunk], rmax)
        return out

    def _raycast(self, origin, d, rmax):
        o = np.asarray(origin, dtype=np.float64)
        best = np.full(d.shape[0], np.inf)
        # Components of exactly zero are nudged so every slab bound is finite.
        dd = np.where(np.abs(d) < 1e-300, 1e-300, d)
        inv = 1.0 / dd
        for z0 in self.planes:
            s = (z0 - o[2]) * inv[:, 2]
            best = np.where((s > 1e-9) & (s < best), s, best)
        if len(self.lo):
            t1 = (self.lo[None, :, :] - o) * inv[:, None, :]
            t2 = (self.hi[None, :, :] - o) * inv[:, None, :]
            tmin = np.minimum(t1, t2).max(axis=-1)
            tmax = np.maximum(t1, t2).min(axis=-1)
            tmin[(tmax < tmin) | (tmin <= 1e-9)] = np.inf
            best = np.minimum(best, tmin.min(axis=-1))
        fin = np.isfinite(best)
        x = o + np.where(fin, best, 0.0)[:, None] * d
        inside = np.all((x >= self.volume_lo) & (x < self.volume_hi), axis=-1)
        return np.where(fin & inside & (best <= rmax), best, np.inf)
